// Placement probe: how fast a population buffer serves the step kernels'
// memory pattern.  Every population of the buffer is read and written back
// unchanged, 81 values per site, one site per lane, in the sweep order and
// workgroup numbering of the even step.  The step kernels run at the
// rate of that pattern (their arithmetic hides under it), and on MI355X the
// rate depends on where the driver placed the buffer's physical memory (the
// FP64 step time by up to 18 %); timing this probe on candidate buffers
// lets a caller keep the fastest before initialising a simulation in it.
#include "kernels.hpp"
#include "placement.hpp"

namespace lbm81 {
namespace {

// The storage element moved as raw bits of its width.
template <int ST>
using Bits = std::conditional_t<sizeof(typename Store<ST>::T) == 8, uint64_t,
             std::conditional_t<sizeof(typename Store<ST>::T) == 4, uint32_t,
                                uint16_t>>;

template <int ST, int MODE>
__global__ __launch_bounds__(BLOCK) void k_placement(typename Store<ST>::T *F,
                                                     Geom g) {
    using T = typename Store<ST>::T;
    using B = Bits<ST>;
    // the even step's workgroup order
    const uint32_t tile = plain_order<ST, false, false>()
                              ? uint32_t(blockIdx.x)
                              : xcd_tile(blockIdx.x, gridDim.x);
    B v[Q];
    if constexpr (MODE == ROW) {
        const RowSite r = row_site(g, tile);
        if (!r.active) return;
        // the step kernels' addressing, on the storage form's element type
        // (which selects planes or row tiles); the values move as raw bits
        const Addr<T, ROW> ad(F, g, r);
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            v[i] = *reinterpret_cast<const __attribute__((address_space(1))) B *>(
                ad.template own<i>());
        });
        // the empty asm hides that each value is the one just loaded, so the
        // stores are kept
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            asm volatile("" : "+v"(v[i]));
            *reinterpret_cast<__attribute__((address_space(1))) B *>(
                ad.template own<i>()) = v[i];
        });
    } else {
        const uint32_t s = tile * BLOCK + threadIdx.x;
        if (s >= g.nsites) return;
        B *p = reinterpret_cast<B *>(F) + site_el(g, s);
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            v[i] = p[uint64_t(i) * g.ss];
        });
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            asm volatile("" : "+v"(v[i]));
            p[uint64_t(i) * g.ss] = v[i];
        });
    }
}

template <int ST>
void launch(void *f, const Geom &g, hipStream_t stream) {
    auto *F = static_cast<typename Store<ST>::T *>(f);
    const dim3 grid(sweep_blocks(g)), block(BLOCK);
    if (mode_of(g) != SMALL)
        hipLaunchKernelGGL((k_placement<ST, ROW>), grid, block, 0, stream, F, g);
    else
        hipLaunchKernelGGL((k_placement<ST, SMALL>), grid, block, 0, stream, F,
                           g);
}

}  // namespace

bool launch_placement(void *f, const Geom &g, int storage, hipStream_t stream) {
    switch (storage) {
        case LBM_F64: launch<LBM_F64>(f, g, stream); return true;
        case LBM_F32: launch<LBM_F32>(f, g, stream); return true;
        case LBM_F16: launch<LBM_F16>(f, g, stream); return true;
        case LBM_BF16: launch<LBM_BF16>(f, g, stream); return true;
    }
    return false;
}

}  // namespace lbm81
