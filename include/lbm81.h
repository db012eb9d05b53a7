/*
 * lbm81.h -- C ABI of the MI355X (gfx950) RD3Q81 lattice Boltzmann library.
 *
 * The library advances the populations of the 81-velocity transonic lattice
 * Boltzmann model of Atif et al., "Lattice Boltzmann Model for Transonic
 * Flows" (arXiv:2409.05114), on a periodic body-centred-cubic grid:
 *   - velocity set and weights: Table "tab:weights" (Appendix);
 *   - moments rho, rho u, rho u^2 + 3 rho theta: Eq. (conslaws), Sec. II;
 *   - entropic equilibrium f_i = w_i rho exp(mu + zeta.c_i + gamma c_i^2),
 *     multipliers from the 5x5 Newton system of Sec. III;
 *   - update f_i(x + c_i, t + 1) = f_i + alpha beta (f_i^eq - f_i),
 *     alpha = 2, beta = 1 / (2 tau + 1): Eq. (discretelbm), Sec. II;
 *   - optional collisions: the entropic alpha of Eq. (delH), Sec. II, and
 *     the series form of the equilibrium of Sec. III / Appendix B
 *     (lbm_set_collision);
 *   - half-integer links join the cube corners to the cube centres (the
 *     replica grid of Sec. I; Sec. V calls the model body-centred cubic).
 *
 * Grid and layouts.  A grid of nx x ny x nz cubic cells (periodic in all
 * three directions) holds S = 2 nx ny nz sites: sub-lattice 0 at the cube
 * corners (x, y, z) and sub-lattice 1 at the cube centres
 * (x + 1/2, y + 1/2, z + 1/2), in lattice units (dx = dt = 1).  Field
 * buffers are FP64 device arrays in site order
 * s = ((sub * nz + z) * ny + y) * nx + x: rho[S], theta[S], u[3][S]
 * (all x components, then all y, then all z).
 *
 * Ownership.  The caller allocates every device buffer (populations,
 * workspace, fields) and owns the HIP stream; the library never allocates
 * or frees device memory.  Its one device buffer of its own is a static
 * 41216-byte workspace per device (lbm_create_static), loaded with the
 * library and held until the process ends.  All device work is
 * enqueued on the stream given to lbm_create (or to lbm_step_batch); calls
 * return when the work is enqueued unless documented as synchronising.
 *
 * Errors.  Every lbm_status-returning function returns LBM_OK (0) or a
 * negative code; argument errors are detected synchronously and leave the
 * simulation unchanged.  Device-side conditions (unrealizable state,
 * non-converged Newton solve, non-finite values) set bits in a flag word in
 * the workspace; lbm_totals and lbm_flags (both synchronising) report them.
 * lbm_last_error() gives a readable message for the last failure on the
 * calling thread.  No C++ exception crosses this boundary.
 *
 * Threading.  One simulation may be used by one host thread at a time.
 * Different simulations on different streams are independent.
 */
#ifndef LBM81_H
#define LBM81_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM81_VERSION 1

typedef enum {
    LBM_OK = 0,
    LBM_E_ARG = -1,          /* bad argument (size, pointer, storage, tau) */
    LBM_E_HIP = -2,          /* a HIP runtime call failed                  */
    LBM_E_STATE = -3,        /* call not valid in the simulation's state   */
    LBM_E_UNREALIZABLE = -4, /* rho <= 0, theta <= 0 or non-finite seen    */
    LBM_E_NEWTON = -5        /* equilibrium solve did not converge         */
} lbm_status;

/* Population storage.  LBM_F64 stores f_i.  The low-precision forms store
 * the deviation from the rest weights, scaled by them, h_i = f_i / w_i - 1,
 * and compute moments, equilibrium and collision in FP32 (the temperature
 * is recovered from the energy moment in FP64); rounding to storage is
 * round-to-nearest-even. */
typedef enum {
    LBM_F64 = 0,
    LBM_F32 = 1,
    LBM_F16 = 2,
    LBM_BF16 = 3
} lbm_storage;

/* Bits of the device flag word. */
#define LBM_FLAG_UNREALIZABLE 0x1u /* a site had rho <= 0 or theta <= 0; it
                                      kept its populations (no collision) */
#define LBM_FLAG_NEWTON 0x2u       /* a Newton solve hit its iteration cap */
#define LBM_FLAG_NONFINITE 0x4u    /* a non-finite moment was seen        */
#define LBM_FLAG_NEGATIVE 0x8u     /* entropic collision: a site had a
                                      non-positive population and was
                                      relaxed with alpha = 2 */

/* Collision operators (lbm_set_collision). */
#define LBM_COLLIDE_BGK 0       /* alpha = 2: Eq. (discretelbm), Sec. II    */
#define LBM_COLLIDE_ENTROPIC 1  /* alpha from Eq. (delH), Sec. II           */
#define LBM_COLLIDE_SERIES 2    /* alpha = 2 towards the series equilibrium
                                   of Sec. III / Appendix B where positive */

typedef struct lbm_sim lbm_sim;

/* Bytes of the population buffer: 81 * 2 * nx * ny * nz * sizeof(storage)
 * plus a little padding.  Layout (library-private): FP32 keeps x-rows
 * (ordered sub, z, y) of tiles of min(nx, 64) consecutive x, each tile
 * holding its values of direction slot 0, then slot 1, ..., slot 80 (rows
 * longer than 64 padded to a multiple of 64); FP64, FP16 and BF16 keep 81
 * direction planes [sub][z][y][x], each padded by 4352 bytes after rounding
 * up to 256 bytes.  Returns 0 for invalid sizes or storage. */
size_t lbm_population_bytes(int nx, int ny, int nz, int storage);

/* Bytes of the workspace (reduction partials and the flag word); the same
 * for every grid, since the reductions use a fixed number of partials. */
size_t lbm_workspace_bytes(int nx, int ny, int nz);

/* Create a simulation handle over caller-owned device buffers.
 * nx, ny, nz >= 1 with 2 nx ny nz < 2^31 and nx <= 2^24, and fewer than
 * 2^32 lanes per sweep: where every side is >= 4 a sweep runs one 64-lane
 * wavefront per row segment of up to 64 x, i.e. 2 ny nz 64 ceil(nx / 64)
 * lanes (rounded up to 256), which only narrow x extents with very many
 * rows exceed (4 x 8192 x 8192 does; refused with LBM_E_ARG).
 * populations: device pointer, lbm_population_bytes() bytes, 256-byte
 * aligned.  workspace: device pointer, lbm_workspace_bytes() bytes.
 * stream: a hipStream_t (NULL = the default stream).  The step counter
 * starts at 0.  The buffers must outlive the handle. */
lbm_status lbm_create(int nx, int ny, int nz, int storage, void *populations,
                      void *workspace, void *stream, lbm_sim **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as lbm_create, without the workspace argument.  The simulation's
 * workspace (flag word, reduction partials and outputs of lbm_totals and
 * lbm_diagnostics) is instead the library's static per-device scratch, a
 * file-scope device array of exactly lbm_workspace_bytes() = 41216 bytes
 * (the workspace does not grow with the grid, so no grid is too large for
 * it; grid limits are those of lbm_create).  The call allocates no device
 * memory (no hipMalloc, no library allocator): it looks up the scratch's
 * address on the current device once (hipGetSymbolAddress) and clears it
 * with a kernel on `stream`.
 * Sharing: every simulation made this way on one device uses that device's
 * one scratch, which keeps the last call's contents; creating a simulation
 * clears it.  Calls on two such simulations of one device that overlap (on
 * any streams, or interleaved between a create and the last totals or flags
 * read) race on the flag word and the partials: use one at a time per
 * device, or lbm_create with a workspace each.  Errors: as lbm_create, plus
 * LBM_E_HIP if the scratch's address cannot be obtained and LBM_E_ARG for a
 * device index of 64 or more. */
lbm_status lbm_create_static(int nx, int ny, int nz, int storage,
                             void *populations, void *stream, lbm_sim **out);

/* Release the handle (host memory only; caller buffers are untouched). */
lbm_status lbm_destroy(lbm_sim *sim);

/* Set every site to the entropic equilibrium f_eq(rho, u, theta) (Sec. III)
 * of the given FP64 device fields, solved in FP64, and reset the step
 * counter to 0.  Sites with rho <= 0, theta <= 0 or non-finite input set
 * LBM_FLAG_UNREALIZABLE and get the rest weights w_i. */
lbm_status lbm_init(lbm_sim *sim, const double *rho, const double *u,
                    const double *theta);

/* Advance nsteps >= 0 time steps of Eq. (discretelbm) with relaxation time
 * tau > 0 (omega = alpha beta = 2 / (2 tau + 1)).  In-place (AA pattern):
 * one kernel launch per step on the simulation's stream. */
lbm_status lbm_step(lbm_sim *sim, int nsteps, double tau);

/* Per-site moments of the current populations (pre-collision state at
 * the current step) into FP64 device fields: rho[S], u[3][S], theta[S]
 * (Eq. conslaws).  Any output pointer may be NULL to skip it. */
lbm_status lbm_moments(lbm_sim *sim, double *rho, double *u, double *theta);

/* Current populations f_i(x) in FP64 into a device buffer f[81][S], in the
 * library's velocity order (see lbm_velocities). */
lbm_status lbm_populations(lbm_sim *sim, double *f);

/* The library's velocity set: c2[3 * i + a] = 2 c_{i,a} (integers) and
 * w[i] = W_i(theta0) for i = 0..80; host pointers; either may be NULL.
 * Returns 81. */
int lbm_velocities(int *c2, double *w);

/* Domain totals of the conserved densities of Eq. (conslaws), Sec. II --
 * the moments sum f_i, sum f_i c_i and sum f_i c_i^2 summed over all
 * sites -- in FP64 with a deterministic, fixed-order reduction:
 * out[0] = sum rho, out[1..3] = sum rho u, out[4] = sum (rho u^2 +
 * 3 rho theta); host pointers.  Also returns the
 * flag word in *flags (may be NULL) and clears it.  Synchronises the
 * stream.  Returns LBM_E_UNREALIZABLE or LBM_E_NEWTON if the corresponding
 * flag was set, LBM_OK otherwise (the totals are written either way). */
lbm_status lbm_totals(lbm_sim *sim, double out[5], unsigned *flags);

/* Read (and clear if clear != 0) the flag word; synchronises the stream. */
lbm_status lbm_flags(lbm_sim *sim, unsigned *flags, int clear);

/* Enqueue a copy of the flag word into *host_flags (host memory that stays
 * valid until the stream reaches the copy; pinned memory keeps it
 * asynchronous) followed by a clear of the word, without synchronising. */
lbm_status lbm_flags_async(lbm_sim *sim, unsigned *host_flags);

/* The flag words of n <= LBM_BATCH_MAX simulations, in one launch: enqueue
 * on `stream` one kernel that copies each simulation's flag word into a
 * staging area and clears it, then one copy of the n words into
 * host_flags[0..n-1] (host memory that stays valid until the stream reaches
 * the copy; pinned memory keeps it asynchronous).  Same result as
 * lbm_flags_async on each simulation, without 2 n stream operations.  The
 * staging area is the reduction-partials area of sims[0]'s workspace, so
 * lbm_totals and lbm_diagnostics on sims[0] must not run concurrently on
 * another stream.  Simulations created on other streams are ordered by
 * events as in lbm_step_batch.  Simulations sharing one workspace (made by
 * lbm_create_static on one device) are refused. */
lbm_status lbm_flags_batch(lbm_sim *const *sims, int n, unsigned *host_flags,
                           void *stream);

/* Flow diagnostics of the current state (Sec. IV.C, compressible
 * Taylor-Green vortex): out[0] = mean kinetic energy <rho u.u / 2>,
 * out[1] = mean enstrophy <rho w.w / 2>, w = curl u, means over all sites.
 * The paper does not say how the curl is discretised: every derivative is
 * the second-order central difference between the two sites one cell away
 * along that axis on the same sub-lattice (periodic).  fields: caller-owned
 * device buffer of 4 * S doubles that receives rho[S] and u[3][S] on the
 * way (as lbm_moments writes them).  out: host pointer.  Deterministic
 * FP64 reduction; synchronises the stream. */
lbm_status lbm_diagnostics(lbm_sim *sim, double *fields, double out[2]);

/* Advance simulation sims[k] by nsteps[k] >= 0 time steps of
 * Eq. (discretelbm) with relaxation time taus[k] > 0, for k = 0..n-1, with
 * batched kernel launches on `stream` (serving): the r-th launch round
 * covers every simulation with nsteps[k] > r, one launch per streaming
 * parity present among them (16-bit forms: odd steps of whole-row grids
 * apart from the others), with one workgroup per tile of every simulation
 * in it, so simulations drop out of later launches as they finish.  The
 * tiles of one launch hold fewer than 2^32 lanes.  All simulations must use the same storage and
 * the BGK collision, be distinct and have sides >= 4; each keeps its own
 * grid, tau and step parity.  sims, nsteps, taus: host arrays of n entries;
 * n <= LBM_BATCH_MAX.  Step counters advance by nsteps[k].  The work of
 * every simulation is the same per site as with lbm_step, so results do not
 * depend on the batch.
 * Streams: a simulation created on another stream than `stream` is ordered
 * by events: the batch starts after the work already queued on that
 * simulation's stream, and work queued there later starts after the batch.
 * Argument errors are returned before anything is enqueued. */
#define LBM_BATCH_MAX 64
lbm_status lbm_step_batch(lbm_sim *const *sims, const int *nsteps,
                          const double *taus, int n, void *stream);

/* Select the collision of lbm_step: LBM_COLLIDE_BGK (default) relaxes with
 * alpha = 2; LBM_COLLIDE_ENTROPIC takes alpha at every site as the positive
 * root of H[f + alpha (f_eq - f)] = H[f] (Sec. II, Eq. delH), with the
 * entropy H[g] = sum g_i (ln(g_i / w_i) - 1) whose constrained minimiser is
 * f_eq (Sec. III), capped where a population would turn negative; then
 * f* = f + alpha beta (f_eq - f).  alpha -> 2 near equilibrium.  A site
 * with a non-positive population gets alpha = 2 and LBM_FLAG_NEGATIVE.  The
 * search costs two logarithms per direction per Newton iteration in FP64
 * and one with the FP32-arithmetic storage forms (which compute the
 * relative departures (f_eq,i - f_i) / f_i once per site); the step is
 * bound by arithmetic, not by memory.  Where the flow carries tail
 * populations far above their equilibrium (the outer shells downstream of
 * strong gradients), the positivity cap rather than the entropy condition
 * sets alpha: on the 256^3 Taylor-Green vortex at Ma 1.2 it does so at
 * about 96 % of the sites (median alpha 1.26), so there the step is mostly
 * a relaxation with alpha below 2.
 * LBM_COLLIDE_SERIES relaxes with alpha = 2 towards the series form of the
 * equilibrium (Sec. III; Appendix B: the quartic weights of
 * Eq. zeroveleqseries and the velocity terms to third order with their
 * R-bar corrections), accurate to O(u^3, eta^4), eta = theta / theta0 - 1,
 * whose mass, momentum and energy are exactly the fluid's; at a site where
 * any of its 81 values is not positive (from about Mach 0.3, depending on
 * theta and the flow direction) the step solves for f_eq instead.  It is
 * an approximation of the BGK step, not the same result.  Batched steps
 * (lbm_step_batch) use BGK and reject the other collisions. */
lbm_status lbm_set_collision(lbm_sim *sim, int collision);

/* Warm start of the entropic collision's search for alpha (Sec. II,
 * Eq. delH; Sec. III notes that Newton's convergence depends on its initial
 * guess): per-site start values kept between steps.  lbm_warm_bytes gives
 * the size of the buffer, one 4-byte value per site (2 nx ny nz sites, site
 * order [sub][z][y][x]), 0 for invalid sizes.  lbm_set_warm_start(sim,
 * alpha) attaches a caller-owned device buffer of that many bytes, 4-byte
 * aligned (NULL detaches it) and clears it on the simulation's stream (no
 * start values yet).  While attached, each entropic step on a grid whose
 * sides are all >= 4 starts the search at a site from the alpha found there
 * in the previous entropic step (negative where it was capped by
 * positivity, which keeps that check first) and stores the new one; the
 * search's tolerance is unchanged, so results agree with cold starts to
 * within it (FP64: alpha to ~1e-14 relative).  The values are not part of a
 * checkpoint: after a restore the first step starts cold.  The buffer must
 * outlive its attachment.  Errors: LBM_E_ARG for a NULL simulation or a
 * misaligned buffer. */
size_t lbm_warm_bytes(int nx, int ny, int nz);
lbm_status lbm_set_warm_start(lbm_sim *sim, void *alpha);

/* Placement probe (a measurement of the buffer, not of the paper's method;
 * the step kernels are bound by HBM bandwidth, Sec. V): reads every
 * population of the simulation's buffer and writes it back unchanged, 81
 * values per site in the step kernels' sweep, once untimed and then `reps`
 * times, on the simulation's stream, and stores the mean time of one pass in
 * *ms.  The contents are left as they were, so it may run on a live state.
 * The steps move their bytes at this pattern's rate, which depends on where
 * the driver placed the buffer's physical memory (on MI355X the FP64 step
 * time differs by up to 18 % between buffers):
 * a caller can create handles on several candidate buffers, probe each and
 * keep the fastest before lbm_init.  Blocks the calling thread until the
 * passes are done.  Errors: LBM_E_ARG for a NULL argument or reps outside
 * [1, 1000]; LBM_E_HIP from the runtime. */
lbm_status lbm_probe_placement(lbm_sim *sim, int reps, float *ms);

/* Step counter; its parity selects the AA-pattern phase. */
long long lbm_step_count(const lbm_sim *sim);

/* Restore the step counter of populations copied back from a checkpoint
 * taken at that count (the counter's parity must match the saved one). */
lbm_status lbm_set_step_count(lbm_sim *sim, long long count);

const char *lbm_status_string(int status);
const char *lbm_last_error(void);
int lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM81_H */
