/*
 * lbm_mc -- one GPU (MI355X, gfx950) implementation of the explicit
 * velocity-difference (EVD) multicomponent lattice Boltzmann method with
 * forcing of Lourenco, Constantino & Tavares, "Forcing mass transfer approach
 * in multicomponent miscible mixtures using the lattice Boltzmann method",
 * Chem. Eng. Sci. 2025 (arXiv 2504.07059).
 *
 * The problem the interface encodes is the paper's: N species of given molar
 * masses (Sec. 4.1, Table 1) with pair Maxwell-Stefan diffusivities D_ij
 * (Table 2), a viscosity set through tau_1 (Sec. 4 opening), a body force on
 * each species F_i = rho_i g (eq. MS_equation with k_i = g; Sec. 4.1), an
 * initial composition x_i(x) with a total mole number n0 (Sec. 4.1), and
 * impermeable walls (Appendix A) or periodicity on each axis (and, as the
 * paper's comparison case, the equilibrium boundary of Sec. 4.1).  The caller
 * advances the system and observes x_i, rho_i, u and the total mass of every
 * species (Sec. 4.1: region-averaged mole fractions, total mass).
 *
 * Lattice units: dx = dt = 1.  Species must be given in ascending molar mass;
 * masses are normalised internally so that M_1 = 1 and c_1 = 1 (Sec. 4
 * opening), and species i then moves with c_i = sqrt(M_1/M_i)
 * (eq. speed_DLS).
 *
 * Memory.  Population buffers are caller-owned device memory (float32); the
 * library borrows them for the lifetime of a context and never frees them.
 * Their layout, per lattice, is [species][direction][z][y][x] with the x rows
 * padded to a pitch of a multiple of 32 floats; lbm_mc_layout() gives the
 * sizes and offsets.  The Q planes of one species must stay below 2 GiB
 * (pitch * ny * nz * Q * 4 bytes; larger lattices are LBM_MC_ERR_UNSUPPORTED),
 * so a buffer holds up to 8 GiB per lattice with 4 species.  Several lattices (the batched form) are concatenated in
 * one buffer.  Populations are stored post-collision: after lbm_mc_init the
 * "current" buffer holds the state s(0) of f~(0), after t steps s(t) of f~(t).
 * The state s of a population set f~ (per species and node) is
 *     plane 0:       P0  = f~_0                    (rest population)
 *     plane a >= 1:  g_a = f~_a - (w_a/w_0) f~_0
 * with w the lattice weights (D2Q9: w_0 = 4/9; D3Q19: w_0 = 1/3) and the
 * directions in the paper's numbering (Sec. 2 for D2Q9).  The species density
 * is rho_i = P0/w_0 + sum_{a>=1} g_a.  Keeping the small deviations g_a keeps
 * rho_i and the momentum to the float32 precision of the deviations rather
 * than of rho_i.
 *
 * Streams.  Every call that launches work does so asynchronously on the HIP
 * stream given to lbm_mc_init (may be NULL for the null stream).  Calls that
 * return host values synchronise that stream.
 *
 * Errors.  Every entry point returns an lbm_mc_status; on failure
 * lbm_mc_last_error() gives a thread-local message.  No entry point aborts the
 * process.  Calls on one context are not thread-safe; separate contexts are
 * independent.
 */
#ifndef LBM_MC_H
#define LBM_MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_mc_status {
    LBM_MC_OK = 0,
    LBM_MC_ERR_INVALID = 1,     /* an argument is invalid (message says which) */
    LBM_MC_ERR_UNSUPPORTED = 2, /* valid in principle, not provided (N > 4, moving walls on
                                   several axes, ...; the message says which) */
    LBM_MC_ERR_HIP = 3,         /* a HIP runtime call failed (message has the HIP error) */
    LBM_MC_ERR_UNSTABLE = 4,    /* linear stability pre-check of the cross relaxation failed */
    LBM_MC_ERR_NONFINITE = 5    /* a step produced a non-finite population */
} lbm_mc_status;

enum { LBM_MC_D2Q9 = 0, LBM_MC_D3Q19 = 1 };
enum { LBM_MC_PERIODIC = 0, LBM_MC_WALL = 1, LBM_MC_WALL_EQ = 2 };

/* Problem statement of one lattice. */
typedef struct lbm_mc_params {
    int32_t lattice;        /* LBM_MC_D2Q9 (the paper's lattice, Sec. 4 opening) or
                               LBM_MC_D3Q19 (same scheme in 3-D; not in the paper) */
    int32_t nx, ny, nz;     /* fluid nodes per axis; nz = 1 for D2Q9 */
    int32_t n_species;      /* 2..4 */
    int32_t bc[3];          /* per axis x, y, z: LBM_MC_PERIODIC, or LBM_MC_WALL =
                               impermeable halfway walls beyond both ends of the axis
                               (Appendix A).  Walls may close several axes (a channel
                               edge or a box corner): a population of a wall node that
                               would cross several walls returns to the node, in the
                               reversed direction if it moves toward any crossed wall,
                               else in its own (mass conserved; reading of Appendix A
                               for corners).
                               LBM_MC_WALL_EQ = walls at the same place treated with the
                               equilibrium comparison boundary of Sec. 4.1 instead: the
                               solid nodes hold w_a rho_s of the fluid node they face and
                               are interpolated over like fluid nodes, with no Appendix A
                               terms.  A negative control, which does not conserve mass:
                               every walled axis of every lattice uses the same kind,
                               forcing 0, no wall velocity, no force field, no adjoint
                               (else LBM_MC_ERR_UNSUPPORTED); it runs one thread per
                               column (execution variant 0 only). */
    double molar_mass[4];   /* molar masses, non-decreasing; any unit (normalised) */
    double diff[4][4];      /* pair diffusivities D_ij in lattice units, symmetric,
                               > 0 off the diagonal; the diagonal is ignored */
    double tau1;            /* relaxation time of species 1, > 1/2; tau_i follows from
                               a common kinematic viscosity (Sec. 3) */
    double g[3];            /* specific body force (same for every species): F_i = rho_i g */
    double n0;              /* initial total mole number n (Sec. 4.1: rho_i = x_i M_i n);
                               <= 0 selects 1/M_max, i.e. a pure heaviest species would
                               have rho = 1 (Sec. 4 opening) */
    int32_t forcing;        /* 0: the standard forcing term (eq. CE_forcing_term_
                               discretized); 1: plus the diffusion-driven contribution
                               S_diff of eq. (improved_forcing_scheme); 2: that whole
                               equation, - S_p + S_rho + S_diff, its density gradients
                               by central differences of the streamed populations'
                               densities (one-sided second order next to a wall; a
                               wall axis needs >= 3 nodes), about 1.5x the step's
                               traffic.  The same value for every lattice of a batch;
                               other values are rejected */
    int32_t reserved;       /* must be 0 */
    double wall_velocity[2][3]; /* velocity of the wall at the low ([0]) and high ([1]) end
                               of the wall axis, tangential to it (the component along
                               the wall axis must be 0; all 0 without walls; moving
                               walls need walls on exactly one axis, else
                               LBM_MC_ERR_UNSUPPORTED).  A moving
                               wall adds the term of Appendix A's closing remark,
                               -2 omega_a rho_i w_i (e_a.u_w)/c_{s,i}^2 for the reflected
                               direction, with rho_i and the mass fraction w_i of the
                               streamed populations at the wall node */
} lbm_mc_params;

typedef struct lbm_mc_ctx lbm_mc_ctx;

/*
 * Buffer layout of n_lattices lattices (p[0..n_lattices-1]).  Host only.
 *   buffer_floats    out: floats each of the two population buffers must hold.
 *   lattice_offsets  out (may be NULL): n_lattices float offsets of each lattice.
 *   pitch            out (may be NULL): n_lattices row pitches (floats).
 *   field_offsets    out (may be NULL): n_lattices node offsets of each lattice in
 *                    the dense node-field outputs of lbm_mc_moments.
 * Errors: LBM_MC_ERR_INVALID for NULL or invalid parameters.
 */
lbm_mc_status lbm_mc_layout(const lbm_mc_params* p, int32_t n_lattices,
                            int64_t* buffer_floats, int64_t* lattice_offsets,
                            int32_t* pitch, int64_t* field_offsets);

/*
 * Host-only validation of a problem: everything lbm_mc_init checks before it
 * touches the GPU, including the linear-stability pre-check of the cross
 * relaxation (a uniform node relaxes species velocity differences with the
 * matrix I - K, K_ij = -rho_j/(rho tau_ij), K_ii = sum_j rho_j/(rho tau_ij); the
 * check requires every eigenvalue of K in [0, 2) at sampled initial
 * compositions and at points between them and the mean composition).
 *   x0          host float64 initial mole fractions, [lattice][N][nz][ny][nx]
 *               concatenated over lattices; each node must sum to 1 (1e-9) and be >= 0.
 *   lambda_max  out (may be NULL): the largest eigenvalue found.
 * Errors: LBM_MC_ERR_INVALID, LBM_MC_ERR_UNSUPPORTED, LBM_MC_ERR_UNSTABLE.
 */
lbm_mc_status lbm_mc_check(const lbm_mc_params* p, int32_t n_lattices, const double* x0,
                           double* lambda_max);

/*
 * Create a context and write the initial state (Sec. 4.1 and 4.2).
 * rho_i = x_i M_i n0; the species and mixture velocities are zero; the
 * populations are the equilibrium of eq. (feqi0) with u_i^eq replaced by the
 * force-consistent u_i0 = -F_i dt/(2 rho_i) (Sec. 4.2), i.e. f(0); these are
 * collided once so that the current buffer holds f~(0), and f(0) itself is kept
 * in the other buffer for lbm_mc_moments at t = 0.
 *   p, n_lattices  problem(s); a batch (n_lattices > 1) must share lattice type
 *                  and species count.
 *   x0             host float64, as for lbm_mc_check; copied, not retained.
 *   f_a, f_b       distinct caller-owned device float buffers of buffer_floats
 *                  floats each (lbm_mc_layout); borrowed until lbm_mc_destroy.
 *   hip_stream     the hipStream_t all work is queued on (NULL = null stream).
 *   out            the new context.
 * Errors: those of lbm_mc_check, plus LBM_MC_ERR_INVALID for buffers that are
 * NULL, equal or too small, and LBM_MC_ERR_HIP.  On error *out is NULL.
 */
lbm_mc_status lbm_mc_init(const lbm_mc_params* p, int32_t n_lattices, const double* x0,
                          float* f_a, float* f_b, int64_t buffer_floats, void* hip_stream,
                          lbm_mc_ctx** out);

/*
 * lbm_mc_init with a position-dependent specific force k(x) in place of the
 * constant g: F_i = rho_i k(x) for every species, in the force shift of the
 * equilibrium velocity (eq. first_order_moment_force), the forcing term and
 * the force-consistent initial velocity u_i0 = -k(x)/2 -- the setting of the
 * paper's centrifugal case (Sec. 4.2, F_i = rho_i omega_u^2 r).
 *   accel   device float, caller-owned, borrowed until lbm_mc_destroy (it is
 *           read by every step, so it must stay valid and may be updated
 *           between steps): dense node fields [lattice][d][nz][ny][nx],
 *           d = 2 (D2Q9) or 3 (D3Q19), lattice l starting at
 *           d * field_offsets[l] (lbm_mc_layout); 4-byte aligned.
 *   p[l].g  must be 0 for every lattice.
 * Other arguments as for lbm_mc_init.  Adds about 4 d bytes per node and step
 * of reads.  The adjoint entry points reject such a context
 * (LBM_MC_ERR_UNSUPPORTED).  Errors: those of lbm_mc_init, plus
 * LBM_MC_ERR_INVALID for a NULL or misaligned accel or a nonzero g.
 */
lbm_mc_status lbm_mc_init_field(const lbm_mc_params* p, int32_t n_lattices, const double* x0,
                                const float* accel, float* f_a, float* f_b,
                                int64_t buffer_floats, void* hip_stream, lbm_mc_ctx** out);

/*
 * Advance every lattice by n_steps time steps (asynchronous).  One step is the
 * paper's lattice Boltzmann equation with forcing, eq. (LBE_forcing): stream
 * the post-collision populations with the second-order interpolation of eq.
 * (Second_order_spatial_interpolation) and the impermeable-wall scheme of
 * Appendix A, take the moments (eqs. zeroth_order_moment,
 * first_order_moment_force, Sirovich_mixture_density, Sirovich_mixture_velocity),
 * solve the cross-relaxation times from eq. (relation_tauij_diff_coeff), and
 * collide (eqs. BGK_self_collision, Cross_collision_Sirovich, feqi0,
 * CE_forcing_term_discretized).  The two buffers swap roles every step.
 * n_steps = 0 is a no-op.  Errors: LBM_MC_ERR_INVALID (NULL ctx, n_steps < 0),
 * LBM_MC_ERR_HIP.  A non-finite population is reported by the next
 * lbm_mc_sync or lbm_mc_moments.
 */
lbm_mc_status lbm_mc_step(lbm_mc_ctx* ctx, int64_t n_steps);

/*
 * lbm_mc_step replays captured step sequences (graphs) and captures each on
 * first use, which costs host time while the GPU waits.  lbm_mc_prepare does
 * that capture ahead of time for the sequences a following
 * lbm_mc_step(ctx, n_steps) will replay, and enqueues no work (the state and
 * the step counter are unchanged).  Optional.  Errors: LBM_MC_ERR_INVALID
 * (NULL ctx, n_steps < 0), LBM_MC_ERR_HIP.
 */
lbm_mc_status lbm_mc_prepare(lbm_mc_ctx* ctx, int64_t n_steps);

/* Wait for the context's stream; LBM_MC_ERR_NONFINITE if any step so far
 * produced a non-finite population (the flag is sticky). */
lbm_mc_status lbm_mc_sync(lbm_mc_ctx* ctx);

/*
 * Observables of the post-stream state f(t) at the current step t (Sec. 2:
 * moments are taken after streaming and boundary conditions).  f(t) is
 * re-gathered from f~(t-1), which is still in the other buffer (at t = 0 it is
 * f(0) itself).  Every pointer may be NULL.
 *   rho   device float [lattice][N][nz][ny][nx]: species densities rho_i.
 *   x     device float, same layout: mole fractions x_i = rho_i/(M_i n).
 *   u     device float [lattice][d][nz][ny][nx]: mixture velocity
 *         u = sum_i w_i u_i^eq with the force-shifted u_i^eq (d = 2 or 3;
 *         eq. Sirovich_mixture_velocity).
 *   ueq   device float [lattice][N][d][nz][ny][nx]: the force-shifted
 *         equilibrium velocity u_i^eq of every species (eq.
 *         first_order_moment_force; a species with rho_i = 0 at a node takes
 *         g/2 there).
 *   us    device float, same layout: the real species velocity
 *         u_i = u_i^eq - Theta_i/(2 rho_i) (eq. CE_EQ83, dt = 1), Theta_i of
 *         eq. (CE_theta_definition) with the cross-relaxation times of the
 *         step; Theta_i/rho_i = sum_j rho_j/(rho tau_ij)(u_i^eq - u_j^eq), which
 *         is also its value where rho_i = 0.
 *   mass      host double [lattice][N]: total mass of each species (FP64 sum).
 *   momentum  host double [lattice][d]: total sum_x rho u (FP64 sum).
 * Node-field offsets of each lattice: lbm_mc_layout field_offsets (times N,
 * d or N*d).  Requesting mass or momentum synchronises the stream.  Errors:
 * LBM_MC_ERR_INVALID, LBM_MC_ERR_HIP, LBM_MC_ERR_NONFINITE (as lbm_mc_sync).
 */
lbm_mc_status lbm_mc_moments(lbm_mc_ctx* ctx, float* rho, float* x, float* u, float* ueq,
                             float* us, double* mass, double* momentum);

/* Current buffers and step: *cur holds f~(t), *prev holds f~(t-1) (f(0) at t = 0).
 * Any out pointer may be NULL. */
lbm_mc_status lbm_mc_state(lbm_mc_ctx* ctx, float** cur, float** prev, int64_t* t);

/*
 * Checkpoint restore: copy caller buffers (device, buffer_floats each) into the
 * context's buffers on its stream and set the step counter to t.  cur must hold
 * f~(t); prev must hold f~(t-1), or f(0) when t = 0, for lbm_mc_moments to be
 * exact (it may be NULL, then moments are unavailable until the next step).
 * A run resumed this way is bitwise identical to an uninterrupted one.
 */
lbm_mc_status lbm_mc_restore(lbm_mc_ctx* ctx, const float* cur, const float* prev, int64_t t);

/*
 * Discrete adjoint (reverse mode of the time stepping; single-lattice
 * contexts).  With Phi the map s(t-1) -> s(t) of one lbm_mc_step on the stored
 * states (stream with walls, collide, store), the adjoint of a loss L is
 * lam(t) = dL/ds(t), a buffer of the population layout, and
 * lam(t-1) = (dPhi/ds(t-1))^T lam(t).  Parameters theta are the pair
 * diffusivities D_ij, i < j, in row-major order (in the caller's units), and
 * the specific force g (x, y, z): grad is a device double array of
 * n_pairs + 3 entries (n_pairs = N(N-1)/2) that the adjoint calls ADD into.
 * The parameter gradients are summed in FP64 in a fixed order (reproducible);
 * the adjoint fields are float32.  Buffers are device memory of the
 * population layout, caller-owned; the padding between rows is never read.
 *
 * One reverse step at f_prev = s(t-1): lam_out = (dPhi/ds(t-1))^T lam_in and
 * grad += (dPhi/dtheta)^T lam_in.  lam_out must not alias lam_in or f_prev.
 * Uses a context-owned scratch buffer of one population buffer (allocated on
 * first use).  Errors: LBM_MC_ERR_INVALID, LBM_MC_ERR_UNSUPPORTED (batched
 * context, forcing other than 0, a force field, moving walls, walls on
 * several axes), LBM_MC_ERR_HIP.
 */
lbm_mc_status lbm_mc_adjoint_step(lbm_mc_ctx* ctx, const float* f_prev, const float* lam_in,
                                  float* lam_out, double* grad);

/*
 * Adjoint of the initialisation s(0) = store(C(f(0; g))) of lbm_mc_init
 * (f(0) built from the initial mole fractions with u_i0 = -g/2, Sec. 4.2):
 * grad += (ds(0)/dtheta)^T lam0.  The initial mole fractions are those given
 * to lbm_mc_init (the context keeps a device copy).
 */
lbm_mc_status lbm_mc_adjoint_init(lbm_mc_ctx* ctx, const float* lam0, double* grad);

/*
 * Mole-fraction profile along x of a stored state (single-lattice contexts):
 *     xbar_i(x) = (1/(ny nz)) sum over y, z of x_i(x, y, z),
 * x_i = rho_i/(M_i n), n = sum_j rho_j/M_j (Sec. 3), rho_i = P0/w_0 + sum g_a
 * of the state (the collision conserves rho_i, so this is the profile of the
 * observables at that step).  The region averages that Sec. 4.1 reports for
 * the two halves of the tube are the means of xbar_i over x < nx/2 and over
 * x >= nx/2 (regions of equal node counts).
 * Evaluated in FP64 with a fixed-order reduction (reproducible).
 *   state  device float, population layout (buffer_floats), e.g. a buffer of
 *          lbm_mc_state or a checkpoint; read only.
 *   xbar   device double [N][nx], written.
 * Uses a context-owned scratch array of FP64 partial sums (allocated on first
 * use, a few MB at most).  Errors: LBM_MC_ERR_INVALID (NULL pointers),
 * LBM_MC_ERR_UNSUPPORTED (batched context), LBM_MC_ERR_HIP.
 */
lbm_mc_status lbm_mc_profile(lbm_mc_ctx* ctx, const float* state, double* xbar);

/*
 * lbm_mc_profile for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same profile, computed with the same kernels, whose FP64 partial sums live
 * in a fixed device array of the library (4 MiB on each GPU it runs on, held
 * until the process ends) instead of context memory.  The call allocates and
 * frees nothing.  The array holds N * nx partial sums per chunk of rows:
 * N * nx above 524288 is rejected (LBM_MC_ERR_INVALID) before any device
 * work; below that the rows are split into at most 524288 / (N nx) chunks
 * (the chunks of lbm_mc_profile whenever they fit, then the results are
 * bit-identical to it).  Every context on one GPU shares that GPU's array, so
 * calls that overlap in time on one GPU (different streams) race; calls in
 * one stream are ordered.  Nothing in the array needs clearing between calls.
 * Arguments and other errors as lbm_mc_profile.
 */
lbm_mc_status lbm_mc_profile_static(lbm_mc_ctx* ctx, const float* state, double* xbar);

/*
 * Vector-Jacobian product of lbm_mc_profile at `state`: given
 * dxbar = dL/dxbar (device double [N][nx]), writes lam = dL/dstate (device
 * float, population layout) at every node: with d_i = dxbar_i(x),
 *   dL/drho_j = (d_j - sum_i d_i x_i) / (ny nz M_j n),
 *   lam(P0_j) = dL/drho_j / w_0,   lam(g_{j,a}) = dL/drho_j   (a >= 1).
 * This is the adjoint lam(T) that starts the reverse sweep of a loss of the
 * final profile.  The row padding of lam is not touched; lam must not alias
 * state.  Errors as lbm_mc_profile.
 */
lbm_mc_status lbm_mc_profile_vjp(lbm_mc_ctx* ctx, const float* state, const double* dxbar,
                                 float* lam);

/*
 * Recompute n steps from the state src into a state sequence: slot k of
 * `states` (device, at a stride of `stride` floats >= buffer_floats, a
 * multiple of 4, 16-byte aligned) receives the state k+1 steps after src.  The
 * context's own buffers and step counter are not touched.  src may not be
 * slot 0.  Bitwise identical to lbm_mc_step.
 */
lbm_mc_status lbm_mc_replay(lbm_mc_ctx* ctx, const float* src, int64_t n, float* states,
                            int64_t stride);

/*
 * n reverse steps through a stored sequence: states[k] = s(t0 + k) for
 * k = 0..n-1 (layout as lbm_mc_replay), lam_in = lam(t0 + n); on return
 * lam_out = lam(t0) and grad has the n steps' parameter terms added.
 * The arithmetic of n lbm_mc_adjoint_step calls; the transposed stream of
 * each reverse step runs in one pass with the collision VJP of the step
 * before it, so between steps the adjoint stays in population space (lam_f)
 * instead of going through the storage transform and back, and the results
 * agree with the single steps to FP32 rounding (a one-step run: identical).
 * Uses one more context-owned buffer.  lam_out must not alias lam_in.
 */
lbm_mc_status lbm_mc_adjoint_run(lbm_mc_ctx* ctx, const float* states, int64_t stride,
                                 int64_t n, const float* lam_in, float* lam_out, double* grad);

/*
 * Execution shape of the fused step.  A tile is block_x x block_y
 * cross-section columns (x, and y in 3-D) by `rows` layers of the slowest axis
 * (y in 2-D, z in 3-D); block_x is 8..256 (a multiple of 8), block_y is 1 in
 * 2-D, and block_x * block_y is 64, 128, 192 or 256.  persistent: 0 = one
 * work-group per tile, > 0 = that many resident work-groups looping over the
 * tile list.  variant: 0 = one thread per column carrying every species;
 * 1 = one wavefront per species over each segment of 64 columns, the species
 * exchanging their moments through LDS: block_x * block_y = 64 (one segment),
 * or W = block_x * block_y / 64 segments (block_x a multiple of 64: W pieces
 * of an x row, or W rows in 3-D) marching in step, with N * W <= 12.  Both
 * variants give the same results.
 * Rebuilds the tile list and drops captured graphs.  0 for block_x, block_y
 * or rows, and -1 for persistent, keep the current value; variant -1 keeps
 * the current variant if the new shape allows it, else selects variant 0.
 * The default shape uses variant 1.
 * Errors: LBM_MC_ERR_INVALID for a shape outside these limits.
 */
lbm_mc_status lbm_mc_set_tuning(lbm_mc_ctx* ctx, int32_t block_x, int32_t block_y,
                                int32_t rows, int32_t persistent, int32_t variant);

/* Query the execution shape in use (any pointer may be NULL). */
lbm_mc_status lbm_mc_get_tuning(lbm_mc_ctx* ctx, int32_t* block_x, int32_t* block_y,
                                int32_t* rows, int32_t* persistent, int32_t* variant);

/*
 * Autotuner: time `reps` steps of each candidate execution shape, both
 * variants (state is not advanced: candidates read the current buffer and
 * write the other one) and keep the fastest.  Results are cached per shape class for the process.
 * best_us (may be NULL) receives the best time per step in microseconds.
 */
lbm_mc_status lbm_mc_autotune(lbm_mc_ctx* ctx, int32_t reps, double* best_us);

/*
 * Batched contexts only: 1 = advance all lattices with one persistent launch per
 * step (default), 0 = one launch per lattice per step (the single-lattice
 * kernel applied lattice by lattice, for comparison).
 */
lbm_mc_status lbm_mc_set_batched_mode(lbm_mc_ctx* ctx, int32_t one_launch);

/* Release the context's own device tables, scratch and graphs (not f_a, f_b). */
lbm_mc_status lbm_mc_destroy(lbm_mc_ctx* ctx);

/* Thread-local message of the last failing call ("" if none). */
const char* lbm_mc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_MC_H */
