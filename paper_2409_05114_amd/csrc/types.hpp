// Types shared by the host side of the library and its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbm81.h"

namespace lbm81 {

constexpr int BLOCK = 256;
constexpr int TOT_BLOCKS = 1024;  // fixed grid of the totals reduction
constexpr size_t WS_FLAGS = 0;    // unsigned flag word
constexpr size_t WS_OUT = 64;     // 5 doubles: final totals
constexpr size_t WS_PART = 256;   // TOT_BLOCKS x 5 doubles: block partials
constexpr size_t WS_BYTES = WS_PART + size_t(TOT_BLOCKS) * 5 * sizeof(double);

// Grid of one simulation, passed to the kernels by value.
struct Geom {
    int nx, ny, nz;
    uint32_t N;       // sites per sub-lattice = nx ny nz
    uint32_t nsites;  // 2 N
    uint64_t plane;   // elements per direction plane = 2 N
};

// Addressing modes.  ROW: nx is a multiple of 64, so the 64 lanes of a
// wavefront share (sub, y, z) and differ in x only; all row arithmetic is
// wavefront-uniform (scalar) and a lane adds a 32-bit byte offset.  GEN: any
// grid with nx, ny, nz >= 4, per-lane arithmetic.  SMALL: some side < 4, the
// periodic wrap uses a remainder.
enum Mode { ROW = 0, GEN = 1, SMALL = 2 };

// Descriptors of a batched step (serving): one per simulation, passed by
// value in the kernel arguments.
struct BatchDesc {
    void *f;
    unsigned *flags;
    Geom g;
    double omega;
    uint32_t tile0;  // first tile of this simulation
    int odd;
};

struct BatchArgs {
    int n;
    uint32_t ntiles;
    BatchDesc d[LBM_BATCH_MAX];
};

// Launchers of one storage form, defined in kernels_<storage>.hip.
template <int ST>
struct Launch {
    static void step(void *f, const Geom &g, double omega, unsigned *flags,
                     bool odd, hipStream_t stream);
    static void init(void *f, const Geom &g, const double *rho,
                     const double *u, const double *theta, unsigned *flags,
                     hipStream_t stream);
    static void gather(void *f, const Geom &g, bool odd, double *rho,
                       double *u, double *theta, double *fout,
                       hipStream_t stream);
    static void totals(const void *f, const Geom &g, bool odd, void *ws,
                       hipStream_t stream);
    static void batch(const BatchArgs &a, bool row, hipStream_t stream);
};

inline int mode_of(const Geom &g) {
    if (g.nx < 4 || g.ny < 4 || g.nz < 4) return SMALL;
    return g.nx % 64 == 0 ? ROW : GEN;
}

}  // namespace lbm81
