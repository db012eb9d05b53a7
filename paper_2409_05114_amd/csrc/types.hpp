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
// Population element of direction slot q at x of row r (rows ordered
// (sub, z, y)):  r rs + q ss + (x / TILE) ts + x % TILE.  Two layouts fill
// this formula (the host picks one per storage form):
//   planes: 81 direction planes of 2 nx ny nz sites, x fastest, the plane
//     stride padded (ss = 2 nx ny nz + pad) so that the 81 streams of a
//     wavefront do not start at addresses that agree in all low bits;
//     rs = nx, ts = TILE;
//   tiles: rows of tiles of tw = min(nx, TILE) consecutive x, a tile holding
//     tw values of slot 0, then of slot 1, ..., slot 80 (the last tile of a
//     row padded to TILE when nx > TILE is not a multiple of it);
//     ss = tw, ts = 81 TILE, rs = 81 tw tiles-per-row.
// Strides are 32-bit (a row and a plane stay below 2^31 elements), which
// keeps the scalar address arithmetic of the step kernels short.
constexpr uint32_t TILE = 64;
// FP32 keeps row tiles, the other storage forms planes: on MI355X each ran
// fastest that way (256^3 vortex: row tiles gave FP32 +9 %, FP64 -2 %, 16-bit
// -2 %; the plane padding gave 16-bit +4 %).
constexpr bool tiled_layout(int storage) { return storage == LBM_F32; }
struct Geom {
    int nx, ny, nz;
    uint32_t N;       // sites per sub-lattice = nx ny nz
    uint32_t nsites;  // 2 N
    uint32_t wpr;     // row segments of TILE x (one wavefront each) per row
    uint32_t nwaves;  // row mode: wavefronts per sweep = 2 ny nz wpr
    uint32_t ts;      // elements between consecutive TILE-x segments of a row
    uint32_t rs;      // elements between consecutive rows
    uint32_t ss;      // elements between consecutive direction slots
};

// Addressing modes.  ROW (every side >= 4): each wavefront takes one
// segment of up to 64 consecutive x of one row (fixed sub-lattice, y, z),
// so all row arithmetic is wavefront-uniform (scalar) and a lane only adds
// its x offset; lanes past the end of a row idle.  SMALL (a side below 4):
// one lane per site in site order, per-lane arithmetic with a remainder
// for the periodic wrap.  ROWX: ROW where every workgroup covers whole rows
// with no idle lane (nx = 64, 128 or 256 and a row count divisible by the
// rows per workgroup); kernels may then exchange values between the
// wavefronts of a row through LDS.
enum Mode { ROW = 0, ROWX = 1, SMALL = 2 };

constexpr int WAVES_PER_BLOCK = BLOCK / 64;

// Descriptors of a batched step (serving): one per simulation, passed by
// value in the kernel arguments.
struct BatchDesc {
    void *f;
    unsigned *flags;
    Geom g;
    double omega;
    uint32_t tile0;  // first tile of this simulation
    int xch;         // mode ROWX: odd steps of 16-bit forms use the LDS row
                     // exchange (the host launches those apart)
};

struct BatchArgs {
    int n;
    uint32_t ntiles;
    BatchDesc d[LBM_BATCH_MAX];
};

// Launchers of one storage form, defined in kernels_<storage>.hip.
template <int ST>
struct Launch {
    // collision: LBM_COLLIDE_BGK, _ENTROPIC (alpha from the entropy
    // condition, Eq. delH) or _SERIES (BGK towards the series equilibrium
    // where it is positive)
    static void step(void *f, const Geom &g, double omega, unsigned *flags,
                     bool odd, int collision, hipStream_t stream);
    static void init(void *f, const Geom &g, const double *rho,
                     const double *u, const double *theta, unsigned *flags,
                     hipStream_t stream);
    static void gather(void *f, const Geom &g, bool odd, double *rho,
                       double *u, double *theta, double *fout,
                       hipStream_t stream);
    static void totals(const void *f, const Geom &g, bool odd, void *ws,
                       hipStream_t stream);
    // xch: every simulation of the launch takes the LDS row exchange of the
    // odd step (16-bit forms, whole-row workgroups); odd steps only
    static void batch(const BatchArgs &a, bool odd, bool xch,
                      hipStream_t stream);
};

// Mean kinetic energy and enstrophy of FP64 fields rho[S], u[3][S] into
// the workspace's output slots 0 and 1 (diagnostics.hip).
void launch_diagnostics(const Geom &g, const double *rho, const double *u,
                        void *ws, hipStream_t stream);

template <int ST>
void launch_step_entropic(void *f, const Geom &g, double omega,
                          unsigned *flags, bool odd, hipStream_t stream);
template <int ST>
void launch_step_series(void *f, const Geom &g, double omega,
                        unsigned *flags, bool odd, hipStream_t stream);

inline int mode_of(const Geom &g) {
    if (g.nx < 4 || g.ny < 4 || g.nz < 4) return SMALL;
    const uint32_t rows = 2u * uint32_t(g.ny) * uint32_t(g.nz);
    if ((g.nx == 64 || g.nx == 128 || g.nx == 256) &&
        rows % (uint32_t(BLOCK) / uint32_t(g.nx)) == 0)
        return ROWX;
    return ROW;
}

// Workgroups of one sweep with bs lanes each: ROW mode packs bs / 64 row
// segments per workgroup, SMALL mode bs sites.
inline uint32_t sweep_blocks(const Geom &g, uint32_t bs = BLOCK) {
    if (mode_of(g) != SMALL) {
        const uint32_t wpb = bs / 64;
        return (g.nwaves + wpb - 1) / wpb;
    }
    return (g.nsites + bs - 1) / bs;
}

}  // namespace lbm81
