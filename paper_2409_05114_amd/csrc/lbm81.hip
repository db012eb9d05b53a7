// C ABI of the RD3Q81 lattice Boltzmann library (include/lbm81.h): argument
// checks, simulation handles and dispatch to the per-storage launchers
// (kernels_*.hip).  No device memory is allocated here: every buffer belongs
// to the caller, except the static per-device workspace of
// lbm_create_static, which is loaded with the library.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>

#include "entropic_launch.hpp"
#include "lattice.hpp"
#include "lbm81.h"
#include "placement.hpp"
#include "types.hpp"

// ======================================================================= ABI
using namespace lbm81;

// The workspace of the simulations made by lbm_create_static: one copy per
// device, held from the library's load to the process's end.  In host code
// `scratch` is only a handle of the symbol, never a device address; its
// device address on each device comes from hipGetSymbolAddress (with that
// device current) and is cached per device (static_scratch below).
static __device__ __align__(256) unsigned char scratch[WS_BYTES];

struct lbm_sim {
    int nx, ny, nz, storage;
    Geom g;
    void *f;
    void *ws;
    hipStream_t stream;
    long long step;
    int collision;  // LBM_COLLIDE_BGK, _ENTROPIC or _SERIES
    hipEvent_t order;  // orders lbm_step_batch against `stream` (lazy)
    float *warm;       // per-site start values of the entropic search, or null
};

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

lbm_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return LBM_OK;
    return fail(LBM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t storage_size(int st) {
    switch (st) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        case LBM_F16:
        case LBM_BF16: return 2;
        default: return 0;
    }
}


unsigned *flag_ptr(lbm_sim *s) {
    return reinterpret_cast<unsigned *>(static_cast<char *>(s->ws) + WS_FLAGS);
}

// Call fn with the storage form as an integral constant.
template <class F>
lbm_status with_storage(int storage, F &&fn) {
    switch (storage) {
        case LBM_F64: fn(std::integral_constant<int, LBM_F64>{}); break;
        case LBM_F32: fn(std::integral_constant<int, LBM_F32>{}); break;
        case LBM_F16: fn(std::integral_constant<int, LBM_F16>{}); break;
        case LBM_BF16: fn(std::integral_constant<int, LBM_BF16>{}); break;
        default: return fail(LBM_E_ARG, "unknown storage");
    }
    return hip_check(hipGetLastError(), "kernel launch");
}

bool valid_dims(int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1) return false;
    const unsigned long long n = 2ull * unsigned(nx) * unsigned(ny) * unsigned(nz);
    // sites and (padded) row lengths are indexed with 32-bit integers
    return n < (1ull << 31) && unsigned(nx) <= (1u << 24);
}

uint32_t tiles_per_row(int nx) { return uint32_t((nx + int(TILE) - 1) / int(TILE)); }

// Population layout of each storage form (the strides of types.hpp).
constexpr uint64_t PLANE_PAD_BYTES = 17 * 256;
struct Layout {
    uint64_t ts, rs, ss;
    uint64_t bytes;
};
Layout layout_of(int nx, int ny, int nz, int storage) {
    const uint64_t es = storage_size(storage);
    const uint64_t rows = 2ull * uint64_t(ny) * uint64_t(nz);
    Layout L;
    if (tiled_layout(storage)) {
        const uint64_t tw = nx < int(TILE) ? uint64_t(nx) : TILE;
        L.ts = Q * TILE;
        L.ss = tw;
        L.rs = uint64_t(tiles_per_row(nx)) * Q * tw;
        L.bytes = rows * L.rs * es;
    } else {
        L.ts = TILE;
        L.rs = uint64_t(nx);
        const uint64_t plane = (rows * uint64_t(nx) * es + 255) / 256 * 256;
        L.ss = (plane + PLANE_PAD_BYTES) / es;
        L.bytes = uint64_t(Q) * L.ss * es;
    }
    return L;
}

// Cross-stream ordering of a batch launched on `batch` over simulations
// created on other streams.  before: `batch` waits for the work queued so
// far on each such simulation's stream; after: each such stream waits for
// the batch.  Simulations on `batch` itself need nothing.
lbm_status order_streams(lbm_sim *const *sims, int n, hipStream_t batch,
                         bool before) {
    hipEvent_t done = nullptr;
    for (int k = 0; k < n; ++k) {
        lbm_sim *s = sims[k];
        if (s->stream == batch) continue;
        if (!s->order) {
            lbm_status st = hip_check(
                hipEventCreateWithFlags(&s->order, hipEventDisableTiming),
                "event create");
            if (st != LBM_OK) return st;
        }
        lbm_status st;
        if (before) {
            st = hip_check(hipEventRecord(s->order, s->stream), "event record");
            if (st == LBM_OK)
                st = hip_check(hipStreamWaitEvent(batch, s->order, 0),
                               "stream wait");
        } else {
            if (!done) {
                done = s->order;
                st = hip_check(hipEventRecord(done, batch), "event record");
                if (st != LBM_OK) return st;
            }
            st = hip_check(hipStreamWaitEvent(s->stream, done, 0), "stream wait");
        }
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

// Zero `bytes` (a multiple of 4) bytes at p (4-byte aligned) with a kernel
// rather than hipMemsetAsync, so that the clear is an ordinary kernel node
// when a caller captures the stream into a graph.
__global__ __launch_bounds__(256) void k_zero(uint32_t *p, uint64_t words) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t quads = words / 4;
    uint4 *q = reinterpret_cast<uint4 *>(p);
    if (reinterpret_cast<uintptr_t>(p) % 16 == 0) {
        for (uint64_t k = i; k < quads; k += stride) q[k] = make_uint4(0, 0, 0, 0);
        for (uint64_t k = 4 * quads + i; k < words; k += stride) p[k] = 0;
    } else {
        for (uint64_t k = i; k < words; k += stride) p[k] = 0;
    }
}

lbm_status zero_async(void *p, size_t bytes, hipStream_t stream) {
    if (bytes % 4 || reinterpret_cast<uintptr_t>(p) % 4)
        return fail(LBM_E_ARG, "internal: unaligned clear");
    const uint64_t words = bytes / 4;
    const uint64_t quads = words / 4 > 0 ? words / 4 : 1;
    const uint64_t want = (quads + 255) / 256;
    const unsigned blocks = unsigned(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, stream,
                       static_cast<uint32_t *>(p), words);
    return hip_check(hipGetLastError(), "clear launch");
}

// Flag words of up to LBM_BATCH_MAX simulations, gathered into `out` and
// cleared, by one workgroup (lane k serves simulation k).
struct FlagPtrs {
    unsigned *p[LBM_BATCH_MAX];
};
__global__ __launch_bounds__(64) void k_flags_gather(FlagPtrs f, int n,
                                                     unsigned *out) {
    const int k = int(threadIdx.x);
    if (k < n) {
        out[k] = *f.p[k];
        *f.p[k] = 0u;
    }
}

lbm_status create_sim(int nx, int ny, int nz, int storage, void *populations,
                      void *workspace, void *stream, lbm_sim **out);

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

lbm_status static_scratch(void **out) {
    int dev = -1;
    lbm_status st = hip_check(hipGetDevice(&dev), "current device");
    if (st != LBM_OK) return st;
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(LBM_E_ARG, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                       "static scratch address");
        if (st != LBM_OK) return st;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256)
            return fail(LBM_E_HIP, "static scratch address is not 256-byte aligned");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_population_bytes(int nx, int ny, int nz, int storage) {
    const size_t es = storage_size(storage);
    if (!es || !valid_dims(nx, ny, nz)) return 0;
    return size_t(layout_of(nx, ny, nz, storage).bytes);
}

size_t lbm_workspace_bytes(int nx, int ny, int nz) {
    (void)nx;
    (void)ny;
    (void)nz;
    return WS_BYTES;
}

lbm_status lbm_create(int nx, int ny, int nz, int storage, void *populations,
                      void *workspace, void *stream, lbm_sim **out) {
    return create_sim(nx, ny, nz, storage, populations, workspace, stream, out);
}

lbm_status lbm_create_static(int nx, int ny, int nz, int storage,
                             void *populations, void *stream, lbm_sim **out) {
    if (!out) return fail(LBM_E_ARG, "out is NULL");
    *out = nullptr;
    void *ws = nullptr;
    lbm_status st = static_scratch(&ws);
    if (st != LBM_OK) return st;
    return create_sim(nx, ny, nz, storage, populations, ws, stream, out);
}

}  // extern "C"

namespace {

lbm_status create_sim(int nx, int ny, int nz, int storage, void *populations,
                      void *workspace, void *stream, lbm_sim **out) {
    if (!out) return fail(LBM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!valid_dims(nx, ny, nz))
        return fail(LBM_E_ARG, "grid sizes must be >= 1 with 2 nx ny nz < 2^31");
    const size_t es = storage_size(storage);
    if (!es) return fail(LBM_E_ARG, "unknown storage");
    const Layout L = layout_of(nx, ny, nz, storage);
    if (L.rs * es >= (1ull << 31) || L.ss >= (1ull << 32))
        return fail(LBM_E_ARG, "one x-row of populations must stay below 2 GiB");
    Geom g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.N = uint32_t(uint64_t(nx) * ny * nz);
    g.nsites = 2u * g.N;
    g.wpr = tiles_per_row(nx);
    g.nwaves = 2u * uint32_t(ny) * uint32_t(nz) * g.wpr;
    g.ts = uint32_t(L.ts);
    g.rs = uint32_t(L.rs);
    g.ss = uint32_t(L.ss);
    // a sweep launches one lane per site, or a wavefront per row segment of
    // up to 64 x; a launch holds fewer than 2^32 lanes
    if (uint64_t(sweep_blocks(g)) * BLOCK > 0xFFFFFFFFull)
        return fail(LBM_E_ARG,
                    "too many rows for the x extent: a sweep needs 2^32 lanes "
                    "or more (one wavefront per row segment of up to 64 x)");
    if (!populations || !workspace)
        return fail(LBM_E_ARG, "populations and workspace must be device pointers");
    if (reinterpret_cast<uintptr_t>(populations) % 256 ||
        reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(LBM_E_ARG, "buffers must be 256-byte aligned");
    lbm_sim *s = new (std::nothrow) lbm_sim;
    if (!s) return fail(LBM_E_ARG, "out of host memory");
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->storage = storage;
    s->g = g;
    s->f = populations;
    s->ws = workspace;
    s->stream = static_cast<hipStream_t>(stream);
    s->step = 0;
    s->collision = LBM_COLLIDE_BGK;
    s->order = nullptr;
    s->warm = nullptr;
    lbm_status st = zero_async(workspace, WS_BYTES, s->stream);
    if (st != LBM_OK) {
        delete s;
        return st;
    }
    *out = s;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_destroy(lbm_sim *sim) {
    if (sim && sim->order) (void)hipEventDestroy(sim->order);
    delete sim;
    return LBM_OK;
}

lbm_status lbm_init(lbm_sim *s, const double *rho, const double *u,
                    const double *theta) {
    if (!s || !rho || !u || !theta) return fail(LBM_E_ARG, "NULL argument");
    {
        // padding between planes or in partial tiles is never read; give it
        // a defined value so that copies of the buffer compare equal
        lbm_status z = zero_async(
            s->f, lbm_population_bytes(s->nx, s->ny, s->nz, s->storage),
            s->stream);
        if (z != LBM_OK) return z;
    }
    lbm_status st = with_storage(s->storage, [&](auto ST) {
        Launch<decltype(ST)::value>::init(s->f, s->g, rho, u, theta, flag_ptr(s), s->stream);
    });
    if (st == LBM_OK) s->step = 0;
    return st;
}

lbm_status lbm_step(lbm_sim *s, int nsteps, double tau) {
    if (!s) return fail(LBM_E_ARG, "NULL simulation");
    if (nsteps < 0) return fail(LBM_E_ARG, "nsteps must be >= 0");
    if (!(tau > 0.0) || !std::isfinite(tau))
        return fail(LBM_E_ARG, "tau must be positive and finite");
    // alpha beta with alpha = 2, beta = dt / (2 tau + dt), dt = 1
    const double omega = 2.0 / (2.0 * tau + 1.0);
    for (int k = 0; k < nsteps; ++k) {
        lbm_status st = with_storage(s->storage, [&](auto ST) {
            if (s->collision == LBM_COLLIDE_ENTROPIC)
                launch_step_entropic_warm<decltype(ST)::value>(
                    s->f, s->g, omega, flag_ptr(s), s->step & 1, s->warm,
                    s->stream);
            else
                Launch<decltype(ST)::value>::step(s->f, s->g, omega, flag_ptr(s),
                                                  s->step & 1, s->collision,
                                                  s->stream);
        });
        if (st != LBM_OK) return st;
        s->step++;
    }
    return LBM_OK;
}

lbm_status lbm_moments(lbm_sim *s, double *rho, double *u, double *theta) {
    if (!s) return fail(LBM_E_ARG, "NULL simulation");
    if (!rho && !u && !theta) return LBM_OK;
    return with_storage(s->storage, [&](auto ST) {
        Launch<decltype(ST)::value>::gather(s->f, s->g, s->step & 1, rho, u, theta, nullptr,
                           s->stream);
    });
}

lbm_status lbm_populations(lbm_sim *s, double *f) {
    if (!s || !f) return fail(LBM_E_ARG, "NULL argument");
    return with_storage(s->storage, [&](auto ST) {
        Launch<decltype(ST)::value>::gather(s->f, s->g, s->step & 1, nullptr, nullptr, nullptr,
                           f, s->stream);
    });
}

int lbm_velocities(int *c2, double *w) {
    for (int i = 0; i < Q; ++i) {
        if (c2) {
            c2[3 * i + 0] = DIRS.d[i].x;
            c2[3 * i + 1] = DIRS.d[i].y;
            c2[3 * i + 2] = DIRS.d[i].z;
        }
        if (w) w[i] = shell_weight(DIRS.d[i].shell);
    }
    return Q;
}

lbm_status lbm_flags(lbm_sim *s, unsigned *flags, int clear) {
    if (!s) return fail(LBM_E_ARG, "NULL simulation");
    unsigned v = 0;
    lbm_status st = hip_check(
        hipMemcpyAsync(&v, flag_ptr(s), sizeof v, hipMemcpyDeviceToHost,
                       s->stream),
        "flag read");
    if (st == LBM_OK)
        st = hip_check(hipStreamSynchronize(s->stream), "stream sync");
    if (st == LBM_OK && clear && v)
        st = zero_async(flag_ptr(s), sizeof v, s->stream);
    if (flags) *flags = v;
    return st;
}

lbm_status lbm_flags_async(lbm_sim *s, unsigned *host_flags) {
    if (!s || !host_flags) return fail(LBM_E_ARG, "NULL argument");
    lbm_status st = hip_check(
        hipMemcpyAsync(host_flags, flag_ptr(s), sizeof(unsigned),
                       hipMemcpyDeviceToHost, s->stream),
        "flag read");
    if (st != LBM_OK) return st;
    return zero_async(flag_ptr(s), sizeof(unsigned), s->stream);
}

lbm_status lbm_flags_batch(lbm_sim *const *sims, int n, unsigned *host_flags,
                           void *stream) {
    if (n == 0) return LBM_OK;
    if (!sims || !host_flags || n < 0 || n > LBM_BATCH_MAX)
        return fail(LBM_E_ARG,
                    "need 0 <= n <= LBM_BATCH_MAX sims and a host array");
    FlagPtrs fp;
    for (int k = 0; k < n; ++k) {
        if (!sims[k]) return fail(LBM_E_ARG, "NULL simulation in batch");
        for (int j = 0; j < k; ++j)
            if (sims[j]->ws == sims[k]->ws)
                return fail(LBM_E_ARG, "two simulations share one flag word");
        fp.p[k] = flag_ptr(sims[k]);
    }
    hipStream_t hs = static_cast<hipStream_t>(stream);
    lbm_status st = order_streams(sims, n, hs, true);
    if (st != LBM_OK) return st;
    // staging: the reduction-partials area of the first simulation's
    // workspace (used otherwise only by lbm_totals and lbm_diagnostics)
    unsigned *stage = reinterpret_cast<unsigned *>(
        static_cast<char *>(sims[0]->ws) + WS_PART);
    hipLaunchKernelGGL(k_flags_gather, dim3(1), dim3(64), 0, hs, fp, n, stage);
    st = hip_check(hipGetLastError(), "flag gather launch");
    if (st != LBM_OK) return st;
    st = hip_check(hipMemcpyAsync(host_flags, stage, size_t(n) * sizeof(unsigned),
                                  hipMemcpyDeviceToHost, hs),
                   "flag read");
    if (st != LBM_OK) return st;
    return order_streams(sims, n, hs, false);
}

lbm_status lbm_totals(lbm_sim *s, double out[5], unsigned *flags) {
    if (!s || !out) return fail(LBM_E_ARG, "NULL argument");
    lbm_status st = with_storage(s->storage, [&](auto ST) {
        Launch<decltype(ST)::value>::totals(s->f, s->g, s->step & 1, s->ws, s->stream);
    });
    if (st != LBM_OK) return st;
    st = hip_check(hipMemcpyAsync(out, static_cast<char *>(s->ws) + WS_OUT,
                                  5 * sizeof(double), hipMemcpyDeviceToHost,
                                  s->stream),
                   "totals read");
    if (st != LBM_OK) return st;
    unsigned v = 0;
    st = lbm_flags(s, &v, 1);
    if (flags) *flags = v;
    if (st != LBM_OK) return st;
    if (v & (LBM_FLAG_UNREALIZABLE | LBM_FLAG_NONFINITE))
        return fail(LBM_E_UNREALIZABLE, "unrealizable or non-finite state seen");
    if (v & LBM_FLAG_NEWTON)
        return fail(LBM_E_NEWTON, "equilibrium solve hit its iteration cap");
    return LBM_OK;
}

lbm_status lbm_diagnostics(lbm_sim *s, double *fields, double out[2]) {
    if (!s || !fields || !out) return fail(LBM_E_ARG, "NULL argument");
    const size_t S = s->g.nsites;
    lbm_status st = lbm_moments(s, fields, fields + S, nullptr);
    if (st != LBM_OK) return st;
    launch_diagnostics(s->g, fields, fields + S, s->ws, s->stream);
    st = hip_check(hipGetLastError(), "diagnostics launch");
    if (st != LBM_OK) return st;
    st = hip_check(hipMemcpyAsync(out, static_cast<char *>(s->ws) + WS_OUT,
                                  2 * sizeof(double), hipMemcpyDeviceToHost,
                                  s->stream),
                   "diagnostics read");
    if (st != LBM_OK) return st;
    return hip_check(hipStreamSynchronize(s->stream), "diagnostics sync");
}

lbm_status lbm_step_batch(lbm_sim *const *sims, const int *nsteps,
                          const double *taus, int n, void *stream) {
    if (n == 0) return LBM_OK;
    if (!sims || !nsteps || !taus || n < 0 || n > LBM_BATCH_MAX)
        return fail(LBM_E_ARG,
                    "need 0 <= n <= LBM_BATCH_MAX sims, step counts and taus");
    const int st0 = sims[0] ? sims[0]->storage : -1;
    int most = 0;
    for (int k = 0; k < n; ++k) {
        lbm_sim *s = sims[k];
        if (!s) return fail(LBM_E_ARG, "NULL simulation in batch");
        if (s->storage != st0)
            return fail(LBM_E_ARG, "all simulations of a batch share one storage");
        if (mode_of(s->g) == SMALL)
            return fail(LBM_E_ARG, "batched simulations need nx, ny, nz >= 4");
        if (s->collision != LBM_COLLIDE_BGK)
            return fail(LBM_E_ARG, "batched steps use the BGK collision");
        if (nsteps[k] < 0) return fail(LBM_E_ARG, "nsteps must be >= 0");
        if (!(taus[k] > 0.0) || !std::isfinite(taus[k]))
            return fail(LBM_E_ARG, "tau must be positive and finite");
        for (int j = 0; j < k; ++j)
            if (sims[j] == s || sims[j]->f == s->f)
                return fail(LBM_E_ARG, "a simulation appears twice in a batch");
        most = nsteps[k] > most ? nsteps[k] : most;
    }
    // every launch holds a subset of these tiles, one workgroup each, and a
    // launch holds fewer than 2^32 lanes
    uint64_t all_tiles = 0;
    for (int k = 0; k < n; ++k)
        if (nsteps[k] > 0) all_tiles += sweep_blocks(sims[k]->g);
    if (all_tiles * BLOCK > 0xFFFFFFFFull)
        return fail(LBM_E_ARG, "batch too large: 2^32 lanes or more in one launch");
    if (most == 0) return LBM_OK;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    // Order the batch after the work already queued on each simulation's
    // own stream, and that stream's later work after the batch.
    lbm_status st = order_streams(sims, n, hs, true);
    if (st != LBM_OK) return st;
    for (int step = 0; step < most; ++step) {
        // one launch per group present among the simulations
        // that still have steps to take: even steps; odd steps without the
        // LDS row exchange; odd steps with it (16-bit forms, whole-row
        // workgroups).  The groups run different kernels (k_step_batch).
        const bool xch_form = st0 == LBM_F16 || st0 == LBM_BF16;
        BatchArgs a[3];
        std::memset(a, 0, sizeof a);
        uint64_t tiles[3] = {0, 0, 0};
        for (int k = 0; k < n; ++k) {
            if (step >= nsteps[k]) continue;
            lbm_sim *s = sims[k];
            const bool odd = (s->step & 1) != 0;
            const bool xch = mode_of(s->g) == ROWX;
            const int p = !odd ? 0 : (xch_form && xch ? 2 : 1);
            BatchDesc &d = a[p].d[a[p].n++];
            d.f = s->f;
            d.flags = flag_ptr(s);
            d.g = s->g;
            d.omega = 2.0 / (2.0 * taus[k] + 1.0);
            d.tile0 = uint32_t(tiles[p]);
            d.xch = xch ? 1 : 0;
            tiles[p] += sweep_blocks(s->g);  // bounded by all_tiles
        }
        for (int p = 0; p < 3; ++p) {
            if (!a[p].n) continue;
            a[p].ntiles = uint32_t(tiles[p]);
            st = with_storage(st0, [&](auto ST) {
                Launch<decltype(ST)::value>::batch(a[p], p >= 1, p == 2, hs);
            });
            if (st != LBM_OK) return st;
        }
        for (int k = 0; k < n; ++k)
            if (step < nsteps[k]) sims[k]->step++;
    }
    return order_streams(sims, n, hs, false);
}

lbm_status lbm_set_collision(lbm_sim *s, int collision) {
    if (!s) return fail(LBM_E_ARG, "NULL simulation");
    if (collision != LBM_COLLIDE_BGK && collision != LBM_COLLIDE_ENTROPIC &&
        collision != LBM_COLLIDE_SERIES)
        return fail(LBM_E_ARG, "unknown collision");
    s->collision = collision;
    return LBM_OK;
}

size_t lbm_warm_bytes(int nx, int ny, int nz) {
    if (!valid_dims(nx, ny, nz)) return 0;
    return size_t(2) * size_t(nx) * size_t(ny) * size_t(nz) * sizeof(float);
}

lbm_status lbm_set_warm_start(lbm_sim *s, void *alpha) {
    if (!s) return fail(LBM_E_ARG, "NULL simulation");
    if (reinterpret_cast<uintptr_t>(alpha) % sizeof(float))
        return fail(LBM_E_ARG, "the start-value buffer must be 4-byte aligned");
    s->warm = static_cast<float *>(alpha);
    if (!alpha) return LBM_OK;
    return zero_async(alpha, size_t(s->g.nsites) * sizeof(float), s->stream);
}

lbm_status lbm_probe_placement(lbm_sim *s, int reps, float *ms) {
    if (!s || !ms) return fail(LBM_E_ARG, "NULL argument");
    *ms = 0.0f;
    if (reps < 1 || reps > 1000)
        return fail(LBM_E_ARG, "reps must be in [1, 1000]");
    hipEvent_t e[2] = {nullptr, nullptr};
    lbm_status st = LBM_OK;
    for (int k = 0; k < 2 && st == LBM_OK; ++k)
        st = hip_check(hipEventCreate(&e[k]), "event create");
    // one untimed pass, then `reps` timed ones
    for (int k = 0; k <= reps && st == LBM_OK; ++k) {
        if (k == 1) st = hip_check(hipEventRecord(e[0], s->stream), "event record");
        if (st == LBM_OK && !launch_placement(s->f, s->g, s->storage, s->stream))
            st = fail(LBM_E_ARG, "unknown storage");
        if (st == LBM_OK) st = hip_check(hipGetLastError(), "probe launch");
    }
    if (st == LBM_OK) st = hip_check(hipEventRecord(e[1], s->stream), "event record");
    if (st == LBM_OK) st = hip_check(hipEventSynchronize(e[1]), "event wait");
    float t = 0.0f;
    if (st == LBM_OK) st = hip_check(hipEventElapsedTime(&t, e[0], e[1]), "event time");
    if (st == LBM_OK) *ms = t / float(reps);
    for (int k = 0; k < 2; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
    return st;
}

long long lbm_step_count(const lbm_sim *s) { return s ? s->step : -1; }

lbm_status lbm_set_step_count(lbm_sim *s, long long count) {
    if (!s || count < 0) return fail(LBM_E_ARG, "bad argument");
    s->step = count;
    return LBM_OK;
}

const char *lbm_status_string(int status) {
    switch (status) {
        case LBM_OK: return "ok";
        case LBM_E_ARG: return "invalid argument";
        case LBM_E_HIP: return "HIP runtime error";
        case LBM_E_STATE: return "invalid state";
        case LBM_E_UNREALIZABLE: return "unrealizable state";
        case LBM_E_NEWTON: return "equilibrium solve did not converge";
    }
    return "unknown status";
}

const char *lbm_last_error(void) { return g_err.c_str(); }

int lbm_version(void) { return LBM81_VERSION; }

}  // extern "C"
