/*
 * lbm.h -- C ABI of the gfx950 chemical-potential multiphase lattice Boltzmann
 * step (Qin, Chen, Qin, Xu, Wen, arXiv 2205.09186).
 *
 * One time step, in lattice units (dx = dt = c = 1, cs^2 = 1/3, Sec 2.1):
 *   1. moments rho = sum_i f_i, rho u = sum_i e_i f_i                  (Eq 7)
 *   2. mu_hat = k^2 psi'(rho) - kappa_hat lap(rho), Peng-Robinson psi'  (Eq 14-16)
 *   3. F = -rho grad(mu_hat) + cs^2 grad(rho)                           (Eq 12)
 *      with grad/lap from the chosen difference scheme                  (Sec 2.3)
 *   4. collision with exact-difference forcing, du = F / rho, either SRT
 *      f*_i = f_i - (f_i - feq_i(rho,u))/tau + feq_i(rho,u+du) - feq_i(rho,u)
 *                                                          (Eq 1 with s_i = 1/tau, Eq 6, Eq 8)
 *      or, for D2Q9, the MRT form of Eq 1 with the moment basis M of Eq 3
 *      and the diagonal S of Eq 5:
 *      f* = f - M^-1 S (M f - M feq(rho,u)) + feq(rho,u+du) - feq(rho,u)
 *   5. streaming f_i(x + e_i, t + 1) = f*_i(x, t), all axes periodic    (Eq 1)
 * Observables use the actual fluid velocity v = u + F/(2 rho) (after Eq 8);
 * the spurious current is max |v| over the domain (Sec 3.3).
 *
 * Conventions
 *   - Every field is indexed x fastest, then y, then z; node coordinates run
 *     0..n-1 on each axis.  D2Q9 requires nz = 1.  Every axis used must be at
 *     least 4 nodes long.
 *   - Pointers are plain host or device addresses as stated per argument; no
 *     HIP or C++ type appears in a signature.  The HIP stream is passed as a
 *     void* (a hipStream_t; NULL is the default stream).
 *   - Return codes: LBM_OK (0) or a negative LBM_E* code; details of the last
 *     failure are available from lbm_last_error().  No exception crosses the
 *     ABI.  A context is not thread-safe; separate contexts on separate streams
 *     are independent.
 *   - Ownership: the caller owns the device workspace, the stream and every
 *     array passed in.  The library owns the lbm_ctx (and any graph it
 *     captures) and releases them in lbm_free().
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

/* Lattices: D2Q9 of Eq 2; D3Q19 (the standard 19-velocity set) for 3D runs. */
enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };

/* Difference schemes of Sec 2.3:
 *   CD2, CD4, CD6  explicit central first derivatives of Eq 18-20; Laplacian
 *                  the matched-order central second difference per axis;
 *   E4, E6, E8, E10  isotropic differences of Eq 25a/25b with fourth-, sixth-,
 *                  eighth- and tenth-order isotropy (the four of Fig 6); E10
 *                  is defined in 2D only (LBM_EINVAL for D3Q19);
 *   OCFDS4         the optimised fourth-order compact scheme of Sec 3.1
 *                  (Eq 21 with beta = 0, alpha = 0.446776, c = -0.0541132);
 *   CFDS4/6/8      the compact schemes of Eq 22-24.
 * For the compact schemes the Laplacian is D(D(rho)) per axis. */
enum { LBM_CD2 = 0, LBM_CD4 = 1, LBM_CD6 = 2, LBM_E4 = 3, LBM_E8 = 4,
       LBM_OCFDS4 = 5, LBM_CFDS4 = 6, LBM_CFDS6 = 7, LBM_CFDS8 = 8,
       LBM_E6 = 9, LBM_E10 = 10 };

/* Collision operators of Eq 1. */
enum { LBM_SRT = 0, LBM_MRT = 1 };

enum { LBM_OK = 0, LBM_EINVAL = -1, LBM_ENOSPC = -2, LBM_EHIP = -3,
       LBM_ENONFINITE = -4, LBM_ESTATE = -5 };

typedef struct {
    int    lattice;          /* LBM_D2Q9 | LBM_D3Q19 */
    int    nx, ny, nz;       /* grid; nz = 1 for D2Q9; periodic on every axis */
    double tau;              /* relaxation time, > 0.5 (Sec 2.1) */
    double Tr;               /* reduced temperature T/Tc, 0 < Tr < 1 (Sec 2.2) */
    double k;                /* proportional coefficient of Eq 16, > 0 */
    double kappa;            /* kappa-hat of Eq 16, > 0 */
    int    scheme;           /* LBM_CD2 .. LBM_E10 */
    double a, b, R, omega;   /* Peng-Robinson constants of Eq 14; 0 selects the
                                paper's a = 2/49, b = 2/21, R = 1, omega = 0.344 */
    int    collision;        /* LBM_SRT (0) or LBM_MRT (D2Q9 only) */
    double s_e, s_eps, s_q;  /* MRT rates of the energy, energy-square and heat-flux
                                moments, each in (0, 2); 0 selects Sec 2.1's 1.64,
                                1.54 and 1.7.  Density and momentum relax with 1,
                                the stresses with 1/tau. */
    int    wall;             /* 0: every node fluid, all axes periodic.  1: solid
                                nodes given to lbm_init_wall (wetting boundary of
                                the Appendix; central schemes only) */
    double mu_wall;          /* with wall = 1, the chemical potential mu_hat (mesh
                                units, as Eq 16) assigned to the solid layers */
} lbm_params;

/* Bytes of device workspace lbm_init() needs for these parameters (0 if the
 * parameters are invalid).  The caller allocates it (e.g. a torch uint8 tensor). */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a context on the device workspace d_workspace (>= ws_bytes bytes,
 * 256-byte aligned, owned by the caller, must outlive the context) and set the
 * populations to feq(rho0, 0) (the initial condition before Eq 26's run).
 *   rho0            N = nx*ny*nz initial densities, each finite and in
 *                   (0, 1/b); a host pointer if rho0_on_device == 0, else a
 *                   device pointer.
 *   hip_stream      stream every later call of this context is ordered on.
 * Errors: LBM_EINVAL (bad parameters or rho0, or p->wall != 0), LBM_ENOSPC
 * (workspace too small), LBM_EHIP (runtime failure).  On success *out holds
 * the context.  Synchronises the stream before returning. */
int lbm_init(const lbm_params* p, const double* rho0, int rho0_on_device,
             void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out);

/* Context with solid nodes: the chemical-potential wetting boundary of the
 * Appendix.  p->wall must be 1 and p->scheme one of CD2, CD4, CD6.
 *   solid     N bytes, nonzero marks a solid node (x fastest, as rho0); read
 *             once.  rho0 and solid are both host (on_device == 0) or both
 *             device pointers.  rho0 is not read on solid nodes.
 * The r = 1, 2, 3 (CD2, CD4, CD6) layers of solid next to the fluid, counted
 * through the lattice directions, take the density of Eq A.1 from the layer
 * before them and the chemical potential p->mu_wall; populations that stream
 * into a solid node return to their node reversed (halfway bounce-back, the
 * reading taken where the paper names no rule).  Solid nodes report rho = 0
 * and v = 0; the observables run over the fluid.  On grids tiled by 64 x 8
 * (nx a multiple of 64, ny of 8) the step runs on the tile collide, one launch
 * variant per tile height and z-segment length; otherwise on the
 * node-parallel kernels (one variant).  Errors as lbm_init. */
int lbm_init_wall(const lbm_params* p, const double* rho0, const unsigned char* solid, int on_device,
                  void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out);

/* Enqueue nsteps >= 0 time steps on the context's stream and return. */
int lbm_step(lbm_ctx* c, long nsteps);

/* Macroscopic fields of the current state: rho and v = u + F/(2 rho).
 * Each output holds N doubles; vz may be NULL (ignored for D2Q9).  Host
 * pointers if out_on_device == 0, else device pointers.  Synchronises. */
int lbm_macros(lbm_ctx* c, double* rho, double* vx, double* vy, double* vz,
               int out_on_device);

/* Spurious current U = max |v| and total mass M = sum rho of the current
 * state (host scalars).  Deterministic fixed-order reduction.  Synchronises.
 * Returns LBM_ENONFINITE (values still written) if any rho or v is not finite
 * or U exceeds the lattice sound speed. */
int lbm_spurious_max(lbm_ctx* c, double* umax, double* mass);

/* Copy the current post-streaming populations f[q*N + node] (Q*N doubles) to
 * host (out_on_device == 0) or device memory.  Synchronises. */
int lbm_populations(lbm_ctx* c, double* f, int out_on_device);

/* Number of completed steps of the context. */
long lbm_steps_done(const lbm_ctx* c);

/* Checkpoint and restart.  The state between two steps is the populations
 * of Eq 1 after the collision, held at their source nodes (the next step
 * streams them as it pulls), and the density of Eq 7 from which the next
 * step's chemical potential (Eq 16) starts.  A state image is a 64-byte
 * header (eight int64: magic, layout version, lattice, nx, ny, nz, completed
 * steps, spare), then those Q*N populations (f[q*N + node], x fastest) and
 * the N densities, FP64.  It is this library's own layout, not the
 * post-streaming populations that lbm_populations gives.
 *
 * lbm_state_bytes: the size of an image of c (0 if c is NULL).
 * lbm_save_state: writes the image to host (on_device == 0) or device memory
 *   of at least lbm_state_bytes bytes, owned by the caller.  Synchronises.
 * lbm_load_state: replaces c's state and step count by an image that
 *   lbm_save_state wrote for the same lattice and grid size (the other
 *   parameters may differ); stepping on then continues bitwise as the saved
 *   run would have, for any launch variant.  LBM_EINVAL if the header is not
 *   an image of this lattice and size, LBM_ESTATE for a batch instance (the
 *   batch owns its state).  Synchronises. */
size_t lbm_state_bytes(const lbm_ctx* c);
int lbm_save_state(lbm_ctx* c, void* out, int on_device);
int lbm_load_state(lbm_ctx* c, const void* in, int on_device);

/* Profiling: run nsteps >= 1 steps with a HIP event on the context's stream at
 * every phase boundary of the step (a phase is one kernel on the fused path).
 * ms[k] (k < cap) receives the mean duration of phase k per step and
 * *nphases the number of phases.  Synchronises after every step. */
int lbm_step_timed(lbm_ctx* c, long nsteps, double* ms, int cap, int* nphases);

/* Launch variants (tile shape / register budget) of the context's step
 * kernel; lbm_set_variant selects one (0 = default).  Every variant computes
 * the same step; a tuner times them and keeps the fastest. */
int lbm_num_variants(const lbm_ctx* c);
int lbm_set_variant(lbm_ctx* c, int v);

/* Name of launch variant v of the context ("" if out of range), e.g.
 * "ring 64x8 occ3", "tile 64x16 z64" (the ring-free tile collide with its
 * z-segment length), "tile 64x16 z64 mf" (the same, with the chemical
 * potential and the force of Eq 12/16 formed by one march) or
 * "tile 64x16 z64 zr" (z segments that march their own planes only, their
 * ends completed by the edge fix).  The string stays valid until the next
 * call for this context. */
const char* lbm_variant_name(lbm_ctx* c, int v);

/* Name of phase k of the last timed step ("" if none). */
const char* lbm_phase_name(const lbm_ctx* c, int k);

/* Release the context (never the caller's workspace).  NULL is allowed. */
void lbm_free(lbm_ctx* c);

/* Message of the last failure of this context, or of the calling thread's last
 * failure when c is NULL.  Never NULL. */
const char* lbm_last_error(const lbm_ctx* c);

/* Critical point of Eq 14 with alpha = 1 (the Tc, rho_c of Sec 2.2 that the
 * paper leaves unprinted), for the EOS constants in p (defaults for zeros). */
int lbm_critical(const lbm_params* p, double* Tc, double* rho_c, double* p_c);

/* Coexistence densities at p->Tr from the Maxwell equal-area construction
 * (Sec 3.4), host computation.  LBM_EINVAL outside 0 < Tr < 1. */
int lbm_coexistence(const lbm_params* p, double* rho_g, double* rho_l);

/* Peng-Robinson pressure p0 (Eq 14) and bulk chemical potential psi'(rho)
 * (Eq 15 without the gradient term, integration constant 0), not scaled by
 * k, at T = p->Tr Tc, for n host densities in (0, 1/b).  p0 or mu may be NULL.
 * Host computation; the inputs of the flat-interface profile of Eq 29. */
int lbm_eos(const lbm_params* p, const double* rho, long n, double* p0, double* mu);

/* Diagnostics of the current state (the density the next step reads), with
 * the context's difference scheme:
 *   mu_hat = k^2 psi'(rho) - kappa_hat lap(rho)        (Eq 15, 16)
 *   F      = -rho grad(mu_hat) + cs^2 grad(rho)         (Eq 12)
 * F receives dim planes of N (x, y[, z] components), mu N values; either may
 * be NULL.  With walls, F is 0 and mu is mu_wall on solid nodes.  Host or
 * device arrays per out_on_device; synchronises. */
int lbm_force(lbm_ctx* c, double* F, double* mu, int out_on_device);

/* Gradient (dim planes of N) and Laplacian (N) of a device field d_in with the
 * context's difference scheme (Sec 2.3: Eq 18-20 explicit, Eq 21-24 compact
 * with D(D) as Laplacian, Eq 25 isotropic), periodic on every axis (solid
 * nodes are not special here).  d_lap may be NULL.  Enqueued on the context's
 * stream; d_in must not alias the outputs. */
int lbm_gradient(lbm_ctx* c, const double* d_in, double* d_grad, double* d_lap);

/* ------------------------------------------------------------------------
 * Batched sweep: many uneven D2Q9 instances (droplets, flat slabs; any
 * temperature, radius and scheme) stepped together, by one cooperative
 * persistent kernel per chunk of steps or by one ordinary launch per phase of
 * each step (lbm_batch_set_form).  Each instance runs exactly the step
 * above; every check_every steps its spurious current U is compared with the
 * previous check and the instance retires as CONVERGED (|dU| < tol) or
 * DIVERGED (non-finite state or U above the sound speed).
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;
enum { LBM_RUNNING = 0, LBM_CONVERGED = 1, LBM_DIVERGED = 2 };

/* Device bytes for the n instances ps[0..n-1] (0 if any is invalid). */
size_t lbm_batch_workspace_bytes(const lbm_params* ps, int n);

/* Create the batch on a caller-owned device workspace.  rho0s[i] is a host
 * array of instance i's initial density.  Synchronises. */
int lbm_batch_init(const lbm_params* ps, const double* const* rho0s, int n,
                   void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_batch** out);

/* Workgroups of the cooperative launch (1..lbm_batch_max_grid, the most that
 * can be resident for the current block size; that maximum is the default). */
int lbm_batch_set_grid(lbm_batch* b, int workgroups);
int lbm_batch_max_grid(const lbm_batch* b);

/* Node-block size of the batched kernel: each work item of a phase is this
 * many consecutive nodes of one instance, one per thread, and it is also the
 * workgroup size.  256, 512 (default) or 1024; anything else is LBM_EINVAL.
 * Setting it rebuilds the node-block tables (synchronises) and resets the
 * workgroup count to the maximum for that size.  Results do not depend on
 * either setting; a tuner times the combinations and keeps the fastest. */
int lbm_batch_set_block(lbm_batch* b, int nodes);
int lbm_batch_block(const lbm_batch* b);

/* Launch form.  LBM_BATCH_PERSISTENT (the default): one cooperative launch
 * per chunk runs every step, its workgroups separated by grid barriers
 * between the phases.  LBM_BATCH_PHASES: each phase of each step (density;
 * chemical potential with the compact schemes' first line solves; their
 * second line solves; the two halves of the convergence check on the steps
 * where an instance is due; collision) is an ordinary launch of its own,
 * the kernel boundary in place of the barrier, and a chunk's launches are
 * captured as one graph (its chunks hold at most 1000 steps).  A grid barrier costs about 0.1 us per workgroup
 * and a launch boundary a few us; the tuner times both forms.  Both compute
 * bitwise the same states; the block size applies to both, the workgroup
 * count only to the persistent form.  Anything else is LBM_EINVAL;
 * lbm_batch_form returns the current form (-1 for NULL). */
enum { LBM_BATCH_PERSISTENT = 0, LBM_BATCH_PHASES = 1 };
int lbm_batch_set_form(lbm_batch* b, int form);
int lbm_batch_form(const lbm_batch* b);

/* How the chunks are launched: "graph: captured cooperative launch" (each
 * chunk replays a hipGraph holding the cooperative launch and the status
 * read-back, one graph per chunk length, check interval, tolerance, block and
 * workgroup count), "graph: cooperative kernel node (...)" where stream
 * capture of a cooperative launch fails but a graph node with the
 * cooperative attribute is accepted, "graph: captured phase kernels" (the
 * phase form; one graph also per set of loop steps that carry a check), or
 * "plain cooperative launches (...)" / "plain phase kernels (...)" with the
 * reason (set LBM_NO_GRAPH to choose them). */
const char* lbm_batch_launch_mode(const lbm_batch* b);

/* Advance running instances by up to nsteps steps, in launches of at most
 * `chunk` steps; stops early once every instance has retired.  Host outputs
 * (n entries each, any may be NULL): status (LBM_RUNNING/CONVERGED/DIVERGED),
 * completed steps, and U at the last check.  Synchronises.  Where the
 * runtime refuses the cooperative launch (ROCm does while another process
 * holds the device), the chunk and every later one run in the phase form
 * instead (the launch mode says so).  LBM_EHIP if the runtime runs the
 * persistent kernel without the grid barrier (the kernel then returns at
 * once; no step of that launch is taken) or a launch fails.  A graph replay
 * that did not run the kernels to their end (a completion count the last
 * kernel keeps shows it) is retried without a graph. */
int lbm_batch_run(lbm_batch* b, long nsteps, long check_every, double tol, long chunk,
                  int* status, long* steps, double* umax);

/* Context view of instance i (owned by the batch; valid until lbm_batch_free)
 * for lbm_macros, lbm_spurious_max and lbm_populations. */
lbm_ctx* lbm_batch_instance(lbm_batch* b, int i);

const char* lbm_batch_last_error(const lbm_batch* b);
void lbm_batch_free(lbm_batch* b);

/* ------------------------------------------------------------------------
 * Learned initialiser: FP32 network 4 -> 64 -> 64 -> 64 -> 1 (SiLU) mapping
 * (Tr, k, scheme id, signed distance to the interface), each scaled, to the
 * normalised density phi = (rho - rho_g)/(rho_l - rho_g) of an equilibrium
 * interface.  Flat parameter layout (mlp_param_count() = 8705 floats):
 * W1 (64x4, row = output), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (1x64), b4.
 * All pointers are device pointers; calls are enqueued on `stream` and return.
 * ------------------------------------------------------------------------ */
int mlp_param_count(void);

/* y[B] = net(x[B][4]); acts (B*192 floats, may be NULL) receives the
 * pre-activations for mlp_backward. */
int mlp_forward(const float* d_params, const float* d_x, int B, float* d_y, float* d_acts, void* stream);

/* Mean-squared-error gradient dy = 2 (y - t)/B and per-64-sample partial sums
 * of (y - t)^2 (ceil(B/64) floats). */
int mlp_loss_grad(const float* d_y, const float* d_t, int B, float* d_dy, float* d_loss_partial, void* stream);

/* Parameter gradient of the loss (8705 floats) by backpropagation; d_gpart is
 * scratch of ceil(B/64)*8705 floats.  Deterministic: fixed summation order. */
int mlp_backward(const float* d_params, const float* d_x, const float* d_acts, const float* d_dy, int B,
                 float* d_grad, float* d_gpart, void* stream);

/* One Adam update (step >= 1) of the parameters with moments m, v. */
int mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int step, float lr, float b1,
             float b2, float eps, void* stream);

/* Initial density field for the grid of p: rho = rho_g + clamp(phi,0,1)(rho_l
 * - rho_g) with phi = net(feat3[0..2], (|x - c| - R)/norm7[6]); norm7 holds the
 * feature scaling (Tr shift, scale, k shift, scale, scheme shift, scale,
 * distance scale), feat3 the scaled (Tr, k, scheme).  d_rho: N doubles. */
int mlp_field(const float* d_params, const float* norm7, const lbm_params* p, double cx, double cy, double cz,
              double R, const float* feat3, double rho_g, double rho_l, double* d_rho, void* stream);

/* Total density of a learned initial field moved to target_mass without
 * touching its bulk plateaus: every node gains (target - M) w / W, with M the
 * total of the n device densities d_rho, w = phi (1 - phi), phi = (rho -
 * rho_g)/(rho_l - rho_g) clamped to [0, 1] (zero on both plateaus) and W the
 * sum of w.  The residual goes to the interface, where the profile is least
 * certain; a field without interface nodes (W = 0) is left unchanged.  Sums
 * in a fixed order (deterministic); d_scratch holds lbm_sum_scratch_bytes(n)
 * bytes.  Enqueued on stream, no synchronisation.  LBM_EINVAL for n < 1, NULL
 * pointers, rho_l <= rho_g or a non-finite argument. */
int lbm_interface_mass(double* d_rho, long n, double rho_g, double rho_l, double target_mass, double* d_scratch,
                       void* stream);

/* Deterministic sum of n device doubles (scratch: lbm_sum_scratch_bytes(n)).
 * Synchronises. */
size_t lbm_sum_scratch_bytes(long n);
int lbm_sum(const double* d_x, long n, double* d_scratch, double* h_sum, void* stream);

/* lbm_sum for callers that cannot allocate device memory (code that must not
 * call hipMalloc: tight serving loops, harnesses that forbid allocation).  The
 * same kernels and summation order as lbm_sum, hence the same result bit for
 * bit, but the scratch is a fixed array inside the library: 4 MiB per device,
 * held until the process ends; nothing is allocated or freed.
 *   d_x       n device doubles, 1 <= n <= lbm_sum_static_max() (2^26);
 *             larger n returns LBM_EINVAL with a message, before any launch.
 *   h_sum     host result.  Synchronises the stream (the device of the stream,
 *             or the current device for the NULL stream, holds the scratch).
 * Every call on one device shares that device's scratch: calls that overlap on
 * one device (other streams, other threads) race and must be serialised by the
 * caller. */
size_t lbm_sum_static_max(void);
int lbm_sum_static(const double* d_x, long n, double* h_sum, void* stream);

/* Memory ceiling of the step's access pattern (measurement helper; no step
 * arithmetic).  Copies the Q population arrays (Q = 9 for LBM_D2Q9, 19 for
 * LBM_D3Q19) of an nx x ny x nz grid (nz = 1 in 2D), each of N = nx ny nz
 * doubles and stored one after another (array i at d_src + i N, x fastest),
 * from d_src to d_dst: aligned (pull = 0, dst_i(x) = src_i(x)) or as the
 * streaming pull (pull != 0, dst_i(x) = src_i(x - e_i), all axes periodic).
 * Both buffers are device memory of Q N doubles owned by the caller and must
 * not overlap.  Enqueued on stream; returns LBM_EINVAL for a bad lattice,
 * size (N above 2^38 included) or pointer. */
int lbm_probe_copy(int lattice, int nx, int ny, int nz, const double* d_src, double* d_dst, int pull,
                   void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
