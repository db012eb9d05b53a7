// Flow diagnostics of the compressible Taylor-Green vortex (Sec. IV.C of
// Atif et al., arXiv:2409.05114): mean kinetic energy <rho u.u / 2> and
// mean enstrophy <rho w.w / 2>, w = curl u, over all sites of the
// body-centred grid (each sub-lattice holds one site per cell volume).
// Every derivative is the second-order central difference between the two
// sites one cell away along that axis on the same sub-lattice (periodic).
//
// Input: FP64 fields rho[S], u[3][S] in site order
// ((sub nz + z) ny + y) nx + x, as lbm_moments writes them.  Deterministic:
// a fixed grid of TOT_BLOCKS workgroups, fixed-order tree sums in FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "types.hpp"

namespace lbm81 {
namespace {

__global__ __launch_bounds__(BLOCK) void k_diag_part(Geom g, const double *rho,
                                                     const double *u,
                                                     double *part) {
    __shared__ double sh[2][BLOCK];
    const uint32_t S = g.nsites;
    const uint32_t nx = uint32_t(g.nx), ny = uint32_t(g.ny), nz = uint32_t(g.nz);
    const uint32_t plane = nx * ny;
    const double *ux = u, *uy = u + S, *uz = u + 2 * size_t(S);
    double ke = 0.0, en = 0.0;
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < S;
         s += TOT_BLOCKS * BLOCK) {
        const uint32_t x = s % nx, r = s / nx;
        const uint32_t y = r % ny, r2 = r / ny;
        const uint32_t z = r2 % nz;
        // neighbours one cell away on the same sub-lattice, periodic
        const uint32_t xp = x + 1 == nx ? s - x : s + 1;
        const uint32_t xm = x == 0 ? s + nx - 1 : s - 1;
        const uint32_t yp = y + 1 == ny ? s - y * nx : s + nx;
        const uint32_t ym = y == 0 ? s + (ny - 1) * nx : s - nx;
        const uint32_t zp = z + 1 == nz ? s - z * plane : s + plane;
        const uint32_t zm = z == 0 ? s + (nz - 1) * plane : s - plane;
        const double wx = 0.5 * (uz[yp] - uz[ym]) - 0.5 * (uy[zp] - uy[zm]);
        const double wy = 0.5 * (ux[zp] - ux[zm]) - 0.5 * (uz[xp] - uz[xm]);
        const double wz = 0.5 * (uy[xp] - uy[xm]) - 0.5 * (ux[yp] - ux[ym]);
        const double r0 = rho[s];
        ke += 0.5 * r0 * (ux[s] * ux[s] + uy[s] * uy[s] + uz[s] * uz[s]);
        en += 0.5 * r0 * (wx * wx + wy * wy + wz * wz);
    }
    sh[0][threadIdx.x] = ke;
    sh[1][threadIdx.x] = en;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < unsigned(w)) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) part[blockIdx.x * 2 + threadIdx.x] = sh[threadIdx.x][0];
}

// out[a] = (sum over blocks of part[b][a]) / S, fixed order.
__global__ __launch_bounds__(BLOCK) void k_diag_final(const double *part,
                                                      uint32_t S, double *out) {
    __shared__ double sh[2][BLOCK];
    double a0 = 0.0, a1 = 0.0;
    for (int b = threadIdx.x; b < TOT_BLOCKS; b += BLOCK) {
        a0 += part[b * 2];
        a1 += part[b * 2 + 1];
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < unsigned(w)) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) out[threadIdx.x] = sh[threadIdx.x][0] / double(S);
}

}  // namespace

void launch_diagnostics(const Geom &g, const double *rho, const double *u,
                        void *ws, hipStream_t stream) {
    char *w = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(w + WS_PART);
    hipLaunchKernelGGL(k_diag_part, dim3(TOT_BLOCKS), dim3(BLOCK), 0, stream, g,
                       rho, u, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(BLOCK), 0, stream,
                       static_cast<const double *>(part), g.nsites,
                       reinterpret_cast<double *>(w + WS_OUT));
}

}  // namespace lbm81
