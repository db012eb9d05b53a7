// Memory-pattern ceiling of the step kernels, measured without their
// arithmetic.  A measurement program, not part of the library: it allocates
// its own buffers and moves 81 values per site in place (every value read
// once and written back once to the same address), as the even step of the
// in-place streaming does, on the 256^3 grid of the benchmark (2 x 256^3
// sites).  What it reports bounds what the step kernels can reach with the
// same access pattern; it backs the profiles/ summaries.
//
//   pattern_ceiling split     FP64 planes, each site's 81 directions spread
//                             over G = 1, 2, 4, 8 lanes (81/G values per
//                             lane, 64/G sites per wavefront)
//   pattern_ceiling windows   FP64, one site per lane, in eight 21.7-GB
//                             windows of one buffer: direction planes at the
//                             library's stride and at other strides, and
//                             64-site tiles (the FP32 layout)
//   pattern_ceiling tiles     FP64, one site per lane, in the same eight
//                             windows: planes at the library's stride beside
//                             tiles of T = 64 ... 16384 sites (81 runs of T
//                             values each), which keep each direction's
//                             per-wavefront access a 512-byte run while a
//                             wavefront's 81 accesses fall in one tile
//   pattern_ceiling alloc     FP64 planes in the first hipMalloc buffer and
//                             in one allocated as physically contiguous
//   pattern_ceiling windows16 16-bit planes, one site per lane, unshifted
//                             and shifted, at the start of the eight windows
//   pattern_ceiling pairs16   16-bit planes: one site per lane (2-byte
//                             accesses) against two adjacent sites per lane
//                             (4-byte accesses), unshifted and with 32 of
//                             the 81 directions shifted by one element, as
//                             the odd step shifts them
//   pattern_ceiling check     only the host-side bounds checks
//
// Every kernel's index arithmetic is a host/device function that the host
// checks against the buffer bounds for every lane before any launch.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define CHECK(x)                                                            \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_),      \
                   __LINE__);                                               \
            exit(1);                                                        \
        }                                                                   \
    } while (0)

namespace {

constexpr int Q = 81;
constexpr uint32_t NS = 2u * 256 * 256 * 256;  // sites of the 256^3 grid
constexpr uint64_t PAD = 4352;                  // the library's plane padding

template <class T>
using gptr = __attribute__((address_space(1))) T *;
using gchar = __attribute__((address_space(1))) char;

template <class KF>
float time_ms(KF launch, int reps) {
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    launch();
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a));
    for (int r = 0; r < reps; ++r) launch();
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return ms / reps;
}

// Launder a uniform base pointer so that store addresses are formed after
// the loads (as the step kernels do), not kept alive across them.
template <class P>
__device__ __forceinline__ P launder(P p) {
    uint64_t b = uint64_t(p);
    asm volatile("" : "+s"(b));
    return P(b);
}

// ------------------------------------------------------------------ split
// Lane l of a wavefront: group g = l / (64 / G), site s = l % (64 / G);
// it moves directions g, g + G, g + 2G, ... of site wave * 64 / G + s.
template <int G>
__host__ __device__ inline uint32_t split_site(uint32_t wave, uint32_t lane) {
    return wave * (64u / G) + lane % (64u / G);
}
template <int G>
__host__ __device__ inline int split_group(uint32_t lane) {
    return int(lane / (64u / G));
}

template <int G>
__global__ __launch_bounds__(256, 1) void k_split(double *F, uint64_t ss) {
    constexpr int K = (Q + G - 1) / G;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const uint32_t s = split_site<G>(wave, lane);
    if (s >= NS) return;
    const int g = split_group<G>(lane);
    gchar *base = (gchar *)F;
    const uint32_t off = s * 8u;
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int d = g + G * k;
        if (d < Q) v[k] = *(gptr<double>)(base + uint64_t(d) * ss * 8 + off);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) asm volatile("" : "+v"(v[k]));
    base = launder(base);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int d = g + G * k;
        if (d < Q) *(gptr<double>)(base + uint64_t(d) * ss * 8 + off) = v[k];
    }
}

template <int G>
bool check_split(uint64_t ss, uint64_t elems) {
    const uint32_t waves = NS / (64u / G);
    for (uint32_t w = 0; w < waves; w += (w + 1 < waves ? 997u : 1u)) {
        for (uint32_t lane = 0; lane < 64; ++lane) {
            const uint32_t s = split_site<G>(w, lane);
            const int g = split_group<G>(lane);
            if (s >= NS) continue;
            for (int d = g; d < Q; d += G)
                if (uint64_t(d) * ss + s >= elems) return false;
        }
    }
    // the last wavefront of the grid
    for (uint32_t lane = 0; lane < 64; ++lane) {
        const uint32_t s = split_site<G>(waves - 1, lane);
        if (s >= NS || uint64_t(80) * ss + s >= elems) return false;
    }
    return uint64_t(NS) * 8 < (1ull << 32);
}

template <int G>
void run_split(double *F, uint64_t ss) {
    const uint32_t blocks = NS / (64u / G) / 4u;
    const float ms = time_ms(
        [&] { hipLaunchKernelGGL(k_split<G>, dim3(blocks), dim3(256), 0, 0, F, ss); }, 10);
    printf("split  G=%d lanes/site (%2d sites per wavefront, %3d B per direction per load): "
           "%.3f ms, %.0f GB/s\n",
           G, 64 / G, 8 * 64 / G, ms, 2.0 * Q * 8 * NS / (ms * 1e6));
    fflush(stdout);
}

// ---------------------------------------------------------------- windows
struct Offsets {
    uint64_t o[Q];  // byte offset of each direction plane from the window
};

// planes at host-chosen offsets, one site per lane
__global__ __launch_bounds__(256, 1) void k_planes(char *W, Offsets off) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= NS) return;
    gchar *base = (gchar *)W;
    const uint32_t lane = s * 8u;
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = *(gptr<double>)(base + off.o[q] + lane);
#pragma unroll
    for (int q = 0; q < Q; ++q) asm volatile("" : "+v"(v[q]));
    base = launder(base);
#pragma unroll
    for (int q = 0; q < Q; ++q) *(gptr<double>)(base + off.o[q] + lane) = v[q];
}

// 64-site tiles: tile t holds slot 0..80 runs of 64 values each
__host__ __device__ inline uint64_t tile_elem(int q, uint32_t s) {
    return (uint64_t(s / 64u) * Q + uint64_t(q)) * 64u + s % 64u;
}
__global__ __launch_bounds__(256, 1) void k_tiles(char *W) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= NS) return;
    const uint32_t s0 = __builtin_amdgcn_readfirstlane(s & ~63u);
    gchar *base = (gchar *)W + tile_elem(0, s0) * 8;
    const uint32_t lane = (s % 64u) * 8u;
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = *(gptr<double>)(base + q * 512 + lane);
#pragma unroll
    for (int q = 0; q < Q; ++q) asm volatile("" : "+v"(v[q]));
    base = launder(base);
#pragma unroll
    for (int q = 0; q < Q; ++q) *(gptr<double>)(base + q * 512 + lane) = v[q];
}

// tiles of T sites: tile t holds slot 0..80 runs of T values each
template <uint32_t T>
__host__ __device__ inline uint64_t tile_elem_t(int q, uint32_t s) {
    return (uint64_t(s / T) * Q + uint64_t(q)) * T + s % T;
}
template <uint32_t T>
__global__ __launch_bounds__(256, 1) void k_tiles_t(char *W) {
    static_assert(T % 64 == 0, "a wavefront's 64 sites lie in one tile");
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= NS) return;
    const uint32_t s0 = __builtin_amdgcn_readfirstlane(s & ~63u);
    gchar *base = (gchar *)W + tile_elem_t<T>(0, s0) * 8;
    const uint32_t lane = (s % 64u) * 8u;
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q)
        v[q] = *(gptr<double>)(base + uint64_t(q) * T * 8 + lane);
#pragma unroll
    for (int q = 0; q < Q; ++q) asm volatile("" : "+v"(v[q]));
    base = launder(base);
#pragma unroll
    for (int q = 0; q < Q; ++q)
        *(gptr<double>)(base + uint64_t(q) * T * 8 + lane) = v[q];
}
template <uint32_t T>
bool check_tiles_t(uint64_t window_bytes) {
    // the kernel's split base(s0) + q T + s % 64 equals tile_elem_t, and the
    // largest element lies in the window
    for (uint32_t s = 0; s < NS; s += 4093u)
        for (int q = 0; q < Q; ++q)
            if (tile_elem_t<T>(0, s & ~63u) + uint64_t(q) * T + s % 64 !=
                tile_elem_t<T>(q, s))
                return false;
    for (int q = 0; q < Q; ++q)
        if ((tile_elem_t<T>(q, NS - 1) + 1) * 8 > window_bytes) return false;
    return NS % T == 0;
}

bool check_offsets(const Offsets &o, uint64_t window_bytes) {
    const uint64_t plane = uint64_t(NS) * 8;
    for (int q = 0; q < Q; ++q) {
        if (o.o[q] % 256 || o.o[q] + plane > window_bytes) return false;
        for (int p = 0; p < q; ++p)
            if (o.o[p] < o.o[q] + plane && o.o[q] < o.o[p] + plane) return false;
    }
    return true;
}

bool check_tiles(uint64_t window_bytes) {
    // the kernel's split base(s0) + q 64 + s % 64 equals tile_elem, and the
    // largest element lies in the window
    for (uint32_t s = 0; s < NS; s += 4093u)
        for (int q = 0; q < Q; ++q)
            if (tile_elem(0, s & ~63u) + uint64_t(q) * 64 + s % 64 != tile_elem(q, s))
                return false;
    return (tile_elem(Q - 1, NS - 1) + 1) * 8 <= window_bytes;
}

// ---------------------------------------------------------------- pairs16
// Element shift of direction d for access `which` (0: load, 1: store);
// SHIFTED moves the first 32 directions by -1 (loads) and +1 (stores).
template <bool SHIFTED>
__host__ __device__ constexpr int shift16(int d, int which) {
    return (SHIFTED && d < 32) ? (which == 0 ? -1 : 1) : 0;
}
constexpr int MARGIN16 = 256;  // elements before plane 0 and after the last

template <bool PAIR, bool SHIFTED>
__global__ __launch_bounds__(256) void k_16(uint16_t *F, uint64_t ss) {
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    const uint32_t x = PAIR ? 2u * gid : gid;
    if (x >= NS) return;
    // uniform row base F - MARGIN16 + d ss; non-negative lane byte offset
    gchar *base = (gchar *)(F - MARGIN16);
    uint32_t v[Q];
#pragma unroll
    for (int d = 0; d < Q; ++d) {
        gchar *row = base + uint64_t(d) * ss * 2;
        const uint32_t off = uint32_t(int32_t(x) + MARGIN16 + shift16<SHIFTED>(d, 0)) * 2u;
        if (PAIR) {
            uint32_t w;  // 4 bytes, 2-byte aligned where shifted
            __builtin_memcpy(&w, (const void *)(row + off), 4);
            v[d] = w;
        } else {
            v[d] = *(gptr<uint16_t>)(row + off);
        }
    }
#pragma unroll
    for (int d = 0; d < Q; ++d) asm volatile("" : "+v"(v[d]));
    base = launder(base);
#pragma unroll
    for (int d = 0; d < Q; ++d) {
        if (d % 16 == 15) base = launder(base);
        gchar *row = base + uint64_t(d) * ss * 2;
        const uint32_t off = uint32_t(int32_t(x) + MARGIN16 + shift16<SHIFTED>(d, 1)) * 2u;
        if (PAIR) {
            const uint32_t w = v[d];
            __builtin_memcpy((void *)(row + off), &w, 4);
        } else {
            *(gptr<uint16_t>)(row + off) = uint16_t(v[d]);
        }
    }
}

template <bool PAIR, bool SHIFTED>
bool check_16(uint64_t ss, uint64_t total_elems) {
    const uint32_t lanes = PAIR ? NS / 2 : NS;
    for (uint32_t gid = 0; gid < lanes; ++gid) {
        const uint32_t x = PAIR ? 2u * gid : gid;
        for (int d = 0; d < Q; ++d)
            for (int which = 0; which < 2; ++which) {
                const int64_t lane_el = int64_t(x) + MARGIN16 + shift16<SHIFTED>(d, which);
                const int64_t e = int64_t(d) * int64_t(ss) + lane_el;  // from F0
                if (lane_el < 0 || lane_el * 2 + 4 >= (int64_t(1) << 32)) return false;
                if (e < 0 || e + (PAIR ? 2 : 1) > int64_t(total_elems)) return false;
            }
    }
    return true;
}

template <bool PAIR, bool SHIFTED>
void run_16(uint16_t *F, uint64_t ss) {
    const uint32_t lanes = PAIR ? NS / 2 : NS;
    const float ms = time_ms(
        [&] {
            hipLaunchKernelGGL((k_16<PAIR, SHIFTED>), dim3(lanes / 256u), dim3(256), 0, 0, F, ss);
        },
        10);
    printf("pairs16 %s per lane, %s: %.3f ms, %.0f GB/s\n",
           PAIR ? "two sites (4-byte accesses)" : "one site (2-byte accesses)",
           SHIFTED ? "32 directions shifted by one element" : "unshifted", ms,
           2.0 * Q * 2 * NS / (ms * 1e6));
    fflush(stdout);
}

// --------------------------------------------------------------- drivers
struct Windows {
    static constexpr int NV = 5;
    const char *name[NV];
    Offsets off[NV];
    uint64_t span = 0;
    Windows() {
        const uint64_t plane = uint64_t(NS) * 8, mb2 = 1ull << 21;
        const uint64_t strides[4] = {plane + PAD, plane + PAD + mb2, plane + PAD + (1ull << 24),
                                     plane + PAD + (1ull << 27)};
        const char *names[NV] = {"planes, library stride", "stride + 2 MB", "stride + 16 MB",
                                 "stride + 128 MB", "planes + per-plane 2-MB offsets"};
        for (int v = 0; v < 4; ++v)
            for (int q = 0; q < Q; ++q) off[v].o[q] = uint64_t(q) * strides[v];
        for (int q = 0; q < Q; ++q) {
            // a fixed scramble of the plane offsets in 2-MB steps, below the
            // gap left between consecutive planes
            uint32_t h = uint32_t(q + 1) * 2654435761u;
            h ^= h >> 15;
            off[4].o[q] = uint64_t(q) * (plane + 64 * mb2) + uint64_t(h % 64) * mb2;
        }
        for (int v = 0; v < NV; ++v) {
            this->name[v] = names[v];
            for (int q = 0; q < Q; ++q)
                if (off[v].o[q] + plane > span) span = off[v].o[q] + plane;
        }
        span = (span + mb2 - 1) / mb2 * mb2;
    }
};

bool all_checks() {
    bool ok = true;
    const uint64_t ss = (uint64_t(NS) * 8 + PAD) / 8;
    ok = ok && check_split<1>(ss, Q * ss) && check_split<2>(ss, Q * ss) &&
         check_split<4>(ss, Q * ss) && check_split<8>(ss, Q * ss);
    const Windows w;
    for (int v = 0; v < Windows::NV; ++v) ok = ok && check_offsets(w.off[v], w.span);
    ok = ok && check_tiles(w.span);
    ok = ok && check_tiles_t<64>(w.span) && check_tiles_t<256>(w.span) &&
         check_tiles_t<1024>(w.span) && check_tiles_t<4096>(w.span) &&
         check_tiles_t<16384>(w.span);
    const uint64_t ss16 = ((uint64_t(NS) + 2 * MARGIN16) * 2 + 255) / 256 * 256 / 2 + PAD / 2;
    const uint64_t tot16 = uint64_t(Q) * ss16 + 2 * MARGIN16;
    ok = ok && check_16<false, false>(ss16, tot16) && check_16<false, true>(ss16, tot16) &&
         check_16<true, false>(ss16, tot16) && check_16<true, true>(ss16, tot16);
    return ok;
}

void cmd_split() {
    const uint64_t ss = (uint64_t(NS) * 8 + PAD) / 8;
    double *F;
    CHECK(hipMalloc(&F, Q * ss * 8));
    CHECK(hipMemset(F, 0, Q * ss * 8));
    run_split<1>(F, ss);
    run_split<2>(F, ss);
    run_split<4>(F, ss);
    run_split<8>(F, ss);
    CHECK(hipFree(F));
}

void cmd_windows() {
    const Windows w;
    const int nwin = 8;
    char *B;
    CHECK(hipMalloc(&B, nwin * w.span));
    CHECK(hipMemset(B, 0, nwin * w.span));
    CHECK(hipDeviceSynchronize());
    const double alg = 2.0 * Q * 8 * double(NS);
    for (int k = 0; k < nwin; ++k) {
        char *W = B + uint64_t(k) * w.span;
        printf("window %d at %.1f GB:", k, double(k) * w.span / 1e9);
        for (int v = 0; v < Windows::NV; ++v) {
            const Offsets o = w.off[v];
            const float ms = time_ms(
                [&] { hipLaunchKernelGGL(k_planes, dim3(NS / 256u), dim3(256), 0, 0, W, o); }, 8);
            printf("  %s %.0f", w.name[v], alg / (ms * 1e6));
        }
        const float ms = time_ms(
            [&] { hipLaunchKernelGGL(k_tiles, dim3(NS / 256u), dim3(256), 0, 0, W); }, 8);
        printf("  64-site tiles %.0f  (GB/s)\n", alg / (ms * 1e6));
        fflush(stdout);
    }
    CHECK(hipFree(B));
}

template <uint32_t T>
float time_tiles(char *W) {
    return time_ms([&] { hipLaunchKernelGGL(k_tiles_t<T>, dim3(NS / 256u), dim3(256), 0, 0, W); },
                   8);
}

void cmd_tiles() {
    const Windows w;
    const int nwin = 8;
    char *B;
    CHECK(hipMalloc(&B, nwin * w.span));
    CHECK(hipMemset(B, 0, nwin * w.span));
    CHECK(hipDeviceSynchronize());
    const double alg = 2.0 * Q * 8 * double(NS);
    for (int k = 0; k < nwin; ++k) {
        char *W = B + uint64_t(k) * w.span;
        const Offsets o = w.off[0];
        const float mp = time_ms(
            [&] { hipLaunchKernelGGL(k_planes, dim3(NS / 256u), dim3(256), 0, 0, W, o); }, 8);
        printf("window %d at %.1f GB: planes %.0f  tiles of 64 %.0f  256 %.0f  1024 %.0f  "
               "4096 %.0f  16384 %.0f  (GB/s)\n",
               k, double(k) * w.span / 1e9, alg / (mp * 1e6), alg / (time_tiles<64>(W) * 1e6),
               alg / (time_tiles<256>(W) * 1e6), alg / (time_tiles<1024>(W) * 1e6),
               alg / (time_tiles<4096>(W) * 1e6), alg / (time_tiles<16384>(W) * 1e6));
        fflush(stdout);
    }
    CHECK(hipFree(B));
}

// FP64 planes at the library's stride in a buffer from hipMalloc (the
// process's first allocation) and in one allocated with the contiguous flag
// of hipExtMallocWithFlags (reported as refused if the runtime rejects it)
void cmd_alloc() {
    const Windows w;
    const uint64_t bytes = uint64_t(Q) * (uint64_t(NS) * 8 + PAD);
    const Offsets o = w.off[0];
    if (!check_offsets(o, bytes)) {
        printf("alloc: offsets exceed the buffer\n");
        return;
    }
    const double alg = 2.0 * Q * 8 * double(NS);
    auto rate = [&](char *W) {
        const float ms = time_ms(
            [&] { hipLaunchKernelGGL(k_planes, dim3(NS / 256u), dim3(256), 0, 0, W, o); }, 8);
        return alg / (ms * 1e6);
    };
    char *A = nullptr, *Bc = nullptr;
    CHECK(hipMalloc(&A, bytes));
    CHECK(hipMemset(A, 0, bytes));
    printf("alloc: hipMalloc, first allocation (%.1f GB): %.0f GB/s\n", bytes / 1e9, rate(A));
    fflush(stdout);
    const hipError_t e = hipExtMallocWithFlags((void **)&Bc, bytes, hipDeviceMallocContiguous);
    if (e != hipSuccess || !Bc) {
        (void)hipGetLastError();
        printf("alloc: contiguous flag refused (%s)\n", hipGetErrorString(e));
    } else {
        CHECK(hipMemset(Bc, 0, bytes));
        printf("alloc: hipExtMallocWithFlags(contiguous): %.0f GB/s\n", rate(Bc));
        CHECK(hipFree(Bc));
    }
    printf("alloc: hipMalloc again: %.0f GB/s\n", rate(A));
    fflush(stdout);
    CHECK(hipFree(A));
}

// 16-bit planes (one site per lane, unshifted and shifted as the odd step
// shifts them) at the start of each of the eight windows of cmd_windows
void cmd_windows16() {
    const Windows w;
    const int nwin = 8;
    const uint64_t ss16 = ((uint64_t(NS) + 2 * MARGIN16) * 2 + 255) / 256 * 256 / 2 + PAD / 2;
    const uint64_t tot16 = uint64_t(Q) * ss16 + 2 * MARGIN16;
    if (tot16 * 2 > w.span) {
        printf("windows16: the 16-bit planes exceed a window\n");
        return;
    }
    char *B;
    CHECK(hipMalloc(&B, nwin * w.span));
    CHECK(hipMemset(B, 0, nwin * w.span));
    CHECK(hipDeviceSynchronize());
    const double alg = 2.0 * Q * 2 * double(NS);
    for (int k = 0; k < nwin; ++k) {
        uint16_t *F = reinterpret_cast<uint16_t *>(B + uint64_t(k) * w.span) + MARGIN16;
        const float mu = time_ms(
            [&] { hipLaunchKernelGGL((k_16<false, false>), dim3(NS / 256u), dim3(256), 0, 0, F, ss16); }, 10);
        const float msh = time_ms(
            [&] { hipLaunchKernelGGL((k_16<false, true>), dim3(NS / 256u), dim3(256), 0, 0, F, ss16); }, 10);
        printf("window %d at %.1f GB: 16-bit planes unshifted %.0f  shifted %.0f  (GB/s)\n", k,
               double(k) * w.span / 1e9, alg / (mu * 1e6), alg / (msh * 1e6));
        fflush(stdout);
    }
    CHECK(hipFree(B));
}

void cmd_pairs16() {
    const uint64_t ss16 = ((uint64_t(NS) + 2 * MARGIN16) * 2 + 255) / 256 * 256 / 2 + PAD / 2;
    const uint64_t tot16 = uint64_t(Q) * ss16 + 2 * MARGIN16;
    uint16_t *F0;
    CHECK(hipMalloc(&F0, tot16 * 2));
    CHECK(hipMemset(F0, 0, tot16 * 2));
    uint16_t *F = F0 + MARGIN16;
    run_16<false, false>(F, ss16);
    run_16<true, false>(F, ss16);
    run_16<false, true>(F, ss16);
    run_16<true, true>(F, ss16);
    CHECK(hipFree(F0));
}

}  // namespace

int main(int argc, char **argv) {
    const char *cmd = argc > 1 ? argv[1] : "check";
    const bool ok = all_checks();
    printf("host bounds checks: %s\n", ok ? "ok" : "FAILED");
    if (!ok) return 1;
    if (!strcmp(cmd, "split")) cmd_split();
    else if (!strcmp(cmd, "windows")) cmd_windows();
    else if (!strcmp(cmd, "pairs16")) cmd_pairs16();
    else if (!strcmp(cmd, "tiles")) cmd_tiles();
    else if (!strcmp(cmd, "alloc")) cmd_alloc();
    else if (!strcmp(cmd, "windows16")) cmd_windows16();
    else if (strcmp(cmd, "check")) {
        printf("usage: pattern_ceiling [check|split|windows|tiles|alloc|windows16|pairs16]\n");
        return 2;
    }
    return 0;
}
