/*
 * turret.h -- C ABI of the MI355X (gfx950) settling-particle time step:
 * D3Q27 recursive-regularized lattice Boltzmann with fused pull streaming,
 * immersed-boundary multi-direct forcing, stress-integral force and torque,
 * the leapfrog / predictor-corrector rigid-body update and the falling-frame
 * window, after arXiv 2408.15115 ("Palabos Turret"), Sec. 2.
 *
 * Conventions
 *   - Lattice units: dx = dt = rho_0 = rho_f = 1.  z is vertical; gravity
 *     points along -z.  x and y are periodic (Sec. 2.5).
 *   - Direction i = 9*(xi_z+1) + 3*(xi_y+1) + (xi_x+1); opposite(i) = 26 - i.
 *   - Device populations are stored as deviations g_i = f_i - w_i from the
 *     lattice weights, structure of arrays: for case c the block
 *     [27][nz][ny][nx] starts at element offset pop_offset(c) of each of the
 *     two population buffers.  The z index is a ring: physical row z lives at
 *     slot (z + z0) mod nz, z0 being moved by window_shift.  FP16/BF16 storage
 *     keeps s_i * g_i with s_i = 2^(14 + 2 |xi_i|^2) (the first power of two
 *     at or above 4096 / w_i), rounded to nearest even.
 *   - Every call returns LBM_OK (0) or a negative LBM_E* code; no C++
 *     exception crosses the boundary.  lbm_last_error() gives the message.
 *   - Ownership: the caller allocates all device memory (sizes from
 *     lbm_required_bytes) and keeps it alive until lbm_destroy; the library
 *     allocates no device memory on the step path.  With moment storage,
 *     lbm_get_populations and lbm_set_populations allocate a temporary buffer
 *     of one case's populations for the duration of the call;
 *     lbm_get_populations_noalloc allocates nothing.  Host arrays passed to lbm_init
 *     are copied.  The stream is the caller's; every call is asynchronous on
 *     it except lbm_get_populations, lbm_set_populations, body_get_state,
 *     lbm_save and lbm_load, which synchronize it.  A context must not be
 *     used from two threads at once.
 */
#ifndef TURRET_H
#define TURRET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument (checked before any launch) */
    LBM_ENOMEM = -2,     /* a caller buffer is smaller than required */
    LBM_EHIP = -3,       /* HIP runtime or launch error */
    LBM_EUNSTABLE = -4,  /* a marker stencil left the box, or NaN/overflow seen */
    LBM_ESTATE = -5      /* call out of order (see the step sequence below) */
};

enum { LBM_F32 = 0, LBM_F16 = 1, LBM_BF16 = 2, LBM_MOM = 3 };      /* population storage */
enum { LBM_BC_PERIODIC = 0, LBM_BC_FREESLIP = 1, LBM_BC_NOSLIP = 2, LBM_BC_PRESSURE = 3 }; /* z walls */

/* One settling case (Sec. 2.5 and Table 2).
 *   nx, ny, nz      lattice cells, each >= 8; x, y periodic
 *   bc_zlo, bc_zhi  LBM_BC_*: walls halfway below z = 0 and above z = nz-1;
 *                   free-slip = specular reflection, no-slip = bounce-back,
 *                   pressure = constant density 1 (Sec. 3 domain top): the
 *                   entering populations by anti-bounce-back,
 *                   f_i = -C_opp(i) + 2 w_i, velocity terms of O(u^2) dropped
 *   sponge_cells    0, or >= 2: tau rises linearly from tau to 1 over the top
 *                   sponge_cells rows (Sec. 2.5)
 *   tau             relaxation time > 0.5 (nu = (tau - 1/2)/3, Sec. 2.1)
 *   gravity         magnitude of g along -z
 *   h_ini, h_end    falling-frame window (Sec. 2.5): when the body centre
 *                   drops below h_end, the whole content moves up by
 *                   round(h_ini - h_end) rows; h_end <= 0 disables it
 *   u_wall          x velocity of the bottom and top wall, |u| <= 0.2; non-zero
 *                   only on a no-slip wall, which then moves in its own plane
 *                   (the shear flow of the rotation case of Sec. 3.1):
 *                   bounce-back adds the wall's momentum,
 *                   f_i = C_opp(i) + 6 w_i (xi_i . u_wall) at density 1.
 *                   Zero for a resting wall (the settling cases) */
typedef struct {
    int32_t nx, ny, nz;
    int32_t bc_zlo, bc_zhi;
    int32_t sponge_cells;
    double tau;
    double gravity;
    double h_ini, h_end;
    double u_wall[2];
} lbm_case;

/* The rigid particle of a case (Sec. 2.2 markers, Sec. 2.3 body).
 *   n_markers       surface markers (0 = no particle)
 *   x_body, n_body  host, n_markers x 3 row-major: marker positions about the
 *                   centre of mass and outward normals, body frame
 *   dS              host, n_markers: marker areas
 *   kappa, volume   density ratio rho_p / rho_f and particle volume
 *   J_over_m        body-frame inertia per unit mass, 3 x 3 row-major
 *   r0, d0, v0, w0  centre, orientation rows d_0..d_2 (3 x 3 row-major),
 *                   velocity v(-1/2) and angular velocity w(-1/2)
 *   force_offset    0: the force and torque are the stress integral at the
 *                   markers, as written in Sec. 2.2 (the default);
 *                   delta > 0: the same integral on the parallel surface at
 *                   distance delta outside them, points X_k + delta n_k with
 *                   the same normals and areas dS_offset.  The 4-point kernel
 *                   at a marker averages the outer flow with the rigidly
 *                   moving fluid inside the surface; from delta = 2 on the
 *                   stencils see only the outer flow, and in steady flow the
 *                   integral there equals the force the body exerts through
 *                   the immersed forcing.  The particle region grows by delta.
 *   dS_offset       host, n_markers: marker areas of that parallel surface
 *                   (required when force_offset > 0; ignored otherwise)
 *   torque          constant external torque, lab frame, added to the fluid
 *                   torque in the angular update of Sec. 2.3 (App. B spins a
 *                   sphere up from rest this way); zeros for settling */
typedef struct {
    int32_t n_markers;
    const double *x_body;
    const double *n_body;
    const double *dS;
    double kappa, volume;
    double J_over_m[9];
    double r0[3], d0[9], v0[3], w0[3];
    double force_offset;
    const double *dS_offset;
    double torque[3];
} lbm_body;

/* Options.
 *   storage     LBM_F32, LBM_F16 or LBM_BF16: the 27 populations as deviations
 *               from the weights, in that precision;
 *               LBM_MOM: moment storage.  The recursive-regularized
 *               post-collision state of a cell depends only on rho, u and the
 *               off-equilibrium stress P1 (App. A), so each cell stores ten
 *               FP32 numbers instead of 27 populations: rho - 1, rho u and
 *               (1 - 1/tau) P1 (xx, yy, zz, xy, xz, yz), layout
 *               [10][nz][ny][nx] per case.  The step reconstructs the
 *               populations it pulls and gives the same result as LBM_F32 up to
 *               rounding.  A forced cell (Sec. 2.2) keeps its equilibrium
 *               shift tau h beside the moments for the next step, in a box over
 *               the particle region.  Lattice 27, collision 0 and schedule 0
 *               only.  lbm_get_populations / lbm_set_populations then allocate
 *               a temporary device buffer of one case's 27 planes for the call
 *               (the step calls allocate nothing).  lbm_get_populations returns
 *               the reconstructed populations; lbm_set_populations keeps the
 *               regularized part of what it is given (exact for a
 *               post-collision state of this collision)
 *   ibm_cycles  multi-direct forcing cycles n (the paper uses 4), 1..16
 *               (0 = default 4)
 *   block       threads per block of the lattice kernel, which is also the
 *               tile size in cells: 64, 128 or 256 (0 = default 256)
 *   schedule    lattice kernel schedule over the tile table:
 *               0 = one workgroup per tile;
 *               1 = one workgroup per tile, consecutive tiles grouped on one
 *                   XCD (workgroups are dealt round-robin over the 8 XCDs);
 *               2 = persistent: persist_wgs workgroups stride over the table;
 *               3 = persistent work queue: persist_wgs workgroups take tiles
 *                   from a device counter (dynamic balance across uneven
 *                   cases; the counter is reset by a kernel, graph-safe);
 *                   the table is split in 8 contiguous segments, one per XCD
 *               4 = as 3, with the 8 segments interleaved chunk by chunk,
 *                   so that the XCDs work through the table side by side
 *   persist_wgs workgroups of schedules 2, 3 and 4 (0 = 2048)
 *   tile_order  0 = case after case; 1 = tiles of all cases interleaved
 *               round-robin; 2 = largest case first
 *   ibm_diag    1 = keep the residual max |U_k - I[u* + H](X_k)| after every
 *               multi-direct forcing cycle (lbm_ibm_stats), 0 = only the last
 *   forcing     0 = the forced collision of Sec. 2.2 as printed,
 *               f0(p, u + tau h) + (1 - 1/tau) f1: f1 carries no momentum, so
 *               each step adds tau rho h (the default);
 *               1 = momentum-exact variant: the first-order Hermite term of
 *               the shift is reduced by (tau - 1) rho h, so each step adds
 *               rho h, the velocity correction the multi-direct forcing
 *               computes; mass and second moment as in 0
 *   serial_ibm  0 = ibm_couple runs the coupling on a second stream beside
 *               the step's lattice kernel (the default); 1 = on the context
 *               stream after it (to time the coupling alone)
 *   collision   0 = the recursive-regularized collision of Sec. 2.1 / App. A
 *               (the default); 1 = BGK for comparison: the same rule with the
 *               raw off-equilibrium f - f0(p, u) in place of f1 (all its
 *               moments relax by 1 - 1/tau); runs with schedule 0
 *   lattice     0 or 27 = D3Q27 (Sec. 2.1, the default); 19 = D3Q19, the
 *               lattice the paper compares its choice with for stability:
 *               the same collision construction on the Hermite
 *               polynomials D3Q19 carries (third order through the
 *               orthogonal pairs H_xxy +- H_yzz, H_yyz +- H_xxz,
 *               H_zzx +- H_xyy; no fourth order).  Fluid-only contexts
 *               (no markers), FP32 storage, periodic z, no sponge,
 *               schedule 0; populations are then [19][nz][ny][nx] with
 *               the D3Q27 direction order, corners left out
 *   fine_box    FP16/BF16 storage only: 1 = keep a box around each body in
 *               FP32 (the particle region of the coupling plus a one-cell
 *               rim, at most the case's size per axis).  After the lattice
 *               kernel, the box cells are stepped again from FP32 sources
 *               wherever those lie in the previous step's box; the
 *               reduced-precision store still holds the rounding of every
 *               cell, and the forced-collision correction rounds the box
 *               cells once.  The stress, the interpolations and the forcing
 *               then see FP32 populations near the body, while the rest of
 *               the lattice moves half the bytes.  0 = none (the default).
 *               The boxes (two per case, one per population buffer) live in
 *               aux; population copies and checkpoints include them. */
typedef struct {
    int32_t storage;
    int32_t ibm_cycles;
    int32_t block;
    int32_t schedule;
    int32_t persist_wgs;
    int32_t tile_order;
    int32_t ibm_diag;
    int32_t forcing;
    int32_t serial_ibm;
    int32_t collision;
    int32_t lattice;
    int32_t fine_box;
} lbm_options;

/* Caller-owned device buffers (byte sizes from lbm_required_bytes):
 *   pop_a, pop_b  the two population buffers (ping-pong); with LBM_MOM they hold
 *                 the ten moment planes per case instead
 *   aux           descriptors, body states, markers, IBM region fields; with
 *                 LBM_MOM also the forcing shifts of the particle region and its
 *                 collided populations (region plus a one-cell rim) */
typedef struct {
    void *pop_a;
    void *pop_b;
    void *aux;
} lbm_buffers;

/* Byte sizes of the three device buffers for n_cases cases.
 * out_bytes[0] = pop_a, out_bytes[1] = pop_b, out_bytes[2] = aux.
 * cases and bodies are arrays of n_cases entries (bodies may be NULL: no
 * particles).  Errors: LBM_EINVAL for invalid cases or options. */
int32_t lbm_required_bytes(const lbm_case *cases, const lbm_body *bodies, int32_t n_cases,
                           const lbm_options *opt, int64_t out_bytes[3]);

/* Set up a context over caller buffers (Table 1 event (0)): fluid at rest
 * (g = 0, i.e. f = w), immersed force 0, F = T = 0, body state from bodies.
 * buf_bytes are the caller's sizes of the three buffers (checked against
 * lbm_required_bytes: LBM_ENOMEM if smaller).  hip_stream is a hipStream_t
 * (NULL = default stream).  Errors: LBM_EINVAL (tau <= 0.5, a dimension < 8,
 * sponge_cells == 1, a region wider than the box, markers closer than two
 * cells to a z wall, NULL buffers), LBM_ENOMEM, LBM_EHIP. */
int32_t lbm_init(const lbm_case *cases, const lbm_body *bodies, int32_t n_cases,
                 const lbm_options *opt, const lbm_buffers *buf, const int64_t buf_bytes[3],
                 void *hip_stream, lbm_ctx **out);

/* Step sequence of one time iteration (Table 1, Sec. 2.4), each call
 * asynchronous on the context stream:
 *     body_advance -> lbm_step -> ibm_couple -> window_shift
 * Without particles only lbm_step is needed.  ibm_couple without a preceding
 * lbm_step, or lbm_step twice without ibm_couple while particles exist,
 * return LBM_ESTATE.
 * The coupling of a step reads the body state and the populations the
 * lattice kernel reads, never its output, so ibm_couple runs everything up to
 * h(t+1) on a second stream the library owns, concurrently with that step's
 * lattice kernel (an event recorded on the context stream just before the
 * lattice kernel starts it); the forced correction and every later call wait
 * for it on the context stream.  Work on the context stream therefore stays
 * ordered as the calls are made, and graph capture on it takes the second
 * stream along. */

/* Table 1 event (2), Sec. 2.3: advance every body with F(t), T(t):
 * a = g + F/(kappa V); v += a; r += v; w += M^-1 (J/m)^-1 M T/(kappa V);
 * d_pred = d + w x d; d += w x (d + d_pred)/2, in FP64. */
int32_t body_advance(lbm_ctx *ctx);

/* Table 1 event (1), Sec. 2.1 evolution rule: pull streaming from the
 * current buffer, recursive-regularized collision (App. A) without immersed
 * force, written to the other buffer, which becomes current. */
int32_t lbm_step(lbm_ctx *ctx);

/* Table 1 events (3)-(4), Sec. 2.2: markers at the new body state, stress
 * and u* from the streamed populations, F(t+1), T(t+1) from the stress
 * integral (FP64 reductions), n-cycle multi-direct forcing, and the forced
 * collision of Sec. 2.2 (f^(0) at u + tau h) applied to the current buffer. */
int32_t ibm_couple(lbm_ctx *ctx);

/* Sec. 2.5 re-injection, decided on the device: if the body centre is below
 * h_end, move the content up by round(h_ini - h_end) rows (ring origin
 * shift; the rows entering at the bottom restart at rest) and the body with
 * it.  A no-op otherwise. */
int32_t window_shift(lbm_ctx *ctx);

/* The four calls above, nsteps times. */
int32_t lbm_run(lbm_ctx *ctx, int32_t nsteps);

/* Change the lattice kernel's launch schedule (block, schedule, persist_wgs,
 * tile_order of opt; storage and ibm_cycles must equal the context's) on a
 * live context, e.g. from an autotuner.  Rebuilds the tile table
 * (synchronizing) and drops a captured graph.  Results are bitwise
 * independent of the schedule.  Errors: LBM_EINVAL, LBM_ESTATE (between
 * lbm_step and ibm_couple), LBM_EHIP. */
int32_t lbm_set_schedule(lbm_ctx *ctx, const lbm_options *opt);

/* Capture steps_per_graph (even, >= 2) full steps into a HIP graph, and
 * replay it.  The graph reads all changing state from device memory, so one
 * capture serves any number of replays. */
int32_t lbm_graph_capture(lbm_ctx *ctx, int32_t steps_per_graph);
int32_t lbm_graph_launch(lbm_ctx *ctx);

/* Host copies (synchronizing).  Populations are f = w + g in FP64, layout
 * [27][nz][ny][nx] in physical z order, of the current post-collision state
 * of case case_id. */
int32_t lbm_get_populations(lbm_ctx *ctx, int32_t case_id, double *host_out);
int32_t lbm_set_populations(lbm_ctx *ctx, int32_t case_id, const double *host_in);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): the populations
 * of lbm_get_populations, written as f = w + g in FP64, layout
 * [q][nz][ny][nx] in physical z order, into the caller's DEVICE buffer
 * dev_out (q * nx * ny * nz doubles), asynchronously on the context's stream,
 * with no allocation and no synchronization.  The values equal
 * lbm_get_populations's bit for bit.  Moment storage rebuilds the
 * populations in a fixed device scratch of 64 MiB that the library holds on
 * each GPU until the process ends: cases whose q * plane * 4 bytes exceed it
 * (about 600k cells) return LBM_EINVAL with a message.  Calls that overlap
 * on one GPU (from two threads or streams) share that scratch and race.  The
 * unstable flag is not reported here (body_get_state reports it). */
int32_t lbm_get_populations_noalloc(lbm_ctx *ctx, int32_t case_id, double *dev_out);

/* Body state of a case (synchronizing), out[32]:
 *   r(3) d(9) v(3) w(3) F(3) T(3) F_pressure(3) ibm_residual steps shifts
 *   z0 err.  F, T are the latest stress-integral force and torque
 *   (Sec. 2.2); F_pressure is the -pI part of F.  err is a bit set: 1 = a
 *   marker stencil left the box in z, 2 = a non-finite or huge IBM value,
 *   4 = non-finite density or |u| > 0.5 in the lattice kernel.  A case with
 *   err != 0 is masked: its populations and body are frozen while the other
 *   cases of the batch go on; the call then returns LBM_EUNSTABLE. */
int32_t body_get_state(lbm_ctx *ctx, int32_t case_id, double out[32]);

/* Step log (synchronizing): at the end of every step (in window_shift)
 * each case appends its state, the 32 values of body_get_state in the same
 * layout (Sec. 2.2 force and torque, Sec. 2.3 motion, Sec. 2.5 window), to
 * a device ring of 1024 records.  lbm_log_read copies the records of case
 * case_id not read before, oldest first, at most max_records of them, into
 * host_out (max_records x 32 doubles), and sets *n_read to their number.
 * Records overwritten before they were read are skipped; their number goes
 * to *n_lost (which may be NULL).  Records left over stay for the next call.
 * After lbm_load only records of later steps are readable.  Errors:
 * LBM_EINVAL (bad case, negative count, NULL n_read, NULL host_out with
 * max_records > 0), LBM_EHIP. */
int32_t lbm_log_read(lbm_ctx *ctx, int32_t case_id, double *host_out, int32_t max_records, int32_t *n_read,
                     int64_t *n_lost);

/* Checkpoint: populations (storage format), body states, ring origins and
 * step counters; lbm_load needs a context created with the same cases. */
int32_t lbm_save(lbm_ctx *ctx, const char *path);
int32_t lbm_load(lbm_ctx *ctx, const char *path);

/* Element offset of a case's population block inside pop_a / pop_b, the
 * element stride between its direction planes (its cell count rounded up to
 * 128, plus 1 KB: 256 elements of 4 bytes or 512 of 2), and the device
 * pointer of the current buffer (for tests that read raw storage).  -1 /
 * NULL for a bad case or context. */
int64_t lbm_pop_offset(const lbm_ctx *ctx, int32_t case_id);
int64_t lbm_plane_stride(const lbm_ctx *ctx, int32_t case_id);
void *lbm_current_buffer(const lbm_ctx *ctx);

/* ------------------------------------------------------------------------
 * Learned warm start of the multi-direct forcing.
 *
 * A network (16 -> 64 -> 64 -> 3, SiLU hidden layers) maps each marker's
 * features to a correction of the start of the multi-direct forcing.  The
 * features (LBM_MLP_IN of them) are the plain l = 0 start
 * h0_k(t) = U_k - I[u*](X_k) of Sec. 2.2, the previous step's final force
 * h_k(t-1), its last change h_k(t-1) - h_k(t-2) and the change of the plain
 * start h0_k(t) - h0_k(t-1), each divided by the marker scale
 * s_k = |h0_k(t)| + |h_k(t-1)|, then the normal n_k and the area dS_k.  The start is
 * s_k (h_k(t-1) / s_k + output): the network predicts the change of h from
 * the previous step's final value (a zero network gives the previous-h
 * start; h0 and U enter as their difference, which keeps it out of
 * cancellation; the per-marker scale makes the map independent of the
 * case's velocity scale).
 * From that start the solver runs cycles until the case's residual
 * max_k |U_k - I[u* + H](X_k)| is at or below its gate
 * (lbm_set_ibm_gate, default 1e-6), at most `cycles` of them; a case that
 * does not get there reruns the plain ibm_cycles cycles from the plain
 * start.  All decisions are made on the device, so graphs stay valid.  The
 * network is trained on samples of the solver's own plain runs
 * (lbm_ibm_samples) by the library's forward/backward kernels (FP16
 * weights, FP32 operands and accumulation) and Adam; inference (the warm
 * start and mlp_forward) runs on the matrix cores with FP16 weights and
 * operands and FP32 accumulation.
 *
 * Flat FP32 parameter layout (LBM_MLP_PARAMS = 5443 values): W1[64][16]
 * b1[64] W2[64][64] b2[64] W3[3][64] b3[3].
 * ---------------------------------------------------------------------- */
enum { LBM_MLP_IN = 16, LBM_MLP_PARAMS = 5443 };
typedef struct lbm_mlp lbm_mlp;

/* Device bytes of a network object able to train on batches of up to
 * max_batch samples (1..2^20).  Errors: LBM_EINVAL. */
int32_t mlp_required_bytes(int32_t max_batch, int64_t *out_bytes);

/* Network over a caller device buffer (zeroed here; synchronizing).  Errors:
 * LBM_EINVAL, LBM_ENOMEM (buffer too small), LBM_EHIP. */
int32_t mlp_create(void *dev_buf, int64_t bytes, int32_t max_batch, void *hip_stream, lbm_mlp **out);

/* Parameters from / to host FP32 arrays of LBM_MLP_PARAMS values (synchronizing).
 * Setting them rounds the FP16 compute copy (nearest even) and resets Adam. */
int32_t mlp_set_params(lbm_mlp *m, const float *host_params);
int32_t mlp_get_params(lbm_mlp *m, float *host_params);

/* Inference (matrix cores, FP16 operands): device arrays X (n x LBM_MLP_IN
 * FP32) -> Y (n x 3 FP32), on the network's stream. */
int32_t mlp_forward(lbm_mlp *m, const float *dev_x, int32_t n, float *dev_y);

/* Loss L = 1/(2n) sum |Y - T|^2 and its gradient (LBM_MLP_PARAMS FP32 values), into
 * device arrays (either may be NULL); n <= max_batch.  The gradient is
 * bitwise reproducible (fixed-order sums). */
int32_t mlp_grad(lbm_mlp *m, const float *dev_x, const float *dev_t, int32_t n, float *dev_grad, float *dev_loss);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the batch (X, T); the loss
 * before the step goes to dev_loss when not NULL. */
int32_t mlp_train_step(lbm_mlp *m, const float *dev_x, const float *dev_t, int32_t n, float lr, float *dev_loss);

int32_t mlp_destroy(lbm_mlp *m);
const char *mlp_last_error(const lbm_mlp *m);

/* Start of ibm_couple's multi-direct forcing: LBM_WARM_NONE (the plain
 * l = 0 start of Sec. 2.2), LBM_WARM_PREVIOUS (the previous step's final
 * h_k, a control without network) or LBM_WARM_MLP (network m), with at
 * most `cycles` (1..8) gated cycles from that start before the plain
 * fallback.  Gate 0 never accepts: the run is then the plain run, with the
 * warm start's residuals after each of its cycles recorded (a diagnostic).
 * Drops a captured graph. */
enum { LBM_WARM_NONE = 0, LBM_WARM_PREVIOUS = 1, LBM_WARM_MLP = 2 };
int32_t lbm_set_warm_start(lbm_ctx *ctx, int32_t mode, const lbm_mlp *m, int32_t cycles);

/* Gate of a case's learned start (residual threshold, >= 0; synchronizing). */
int32_t lbm_set_ibm_gate(lbm_ctx *ctx, int32_t case_id, double threshold);

/* Samples of the last ibm_couple, to caller device arrays: features
 * (markers x LBM_MLP_IN FP32) and the training target, the final force
 * h_k(t) minus the previous step's, over the marker scale s_k (markers x 3),
 * written on the context's stream, markers of
 * all cases in case order (lbm_marker_count of them; inside a case in the
 * library's own marker order).  Take them from plain runs (no warm start). */
int32_t lbm_ibm_samples(lbm_ctx *ctx, float *dev_features, float *dev_targets);
int32_t lbm_marker_count(const lbm_ctx *ctx);

/* IBM statistics of a case (synchronizing), out[24]: [0] last residual,
 * [1..8] residual after each cycle of the first sequence (of the last step
 * that ran that cycle), [9..16] the same for the fallback sequence, [17]
 * learned starts accepted, [18] rejected, [19] whether the last step fell
 * back, [20] cycles used by the accepted learned starts (summed), [21..23]
 * zero. */
int32_t lbm_ibm_stats(lbm_ctx *ctx, int32_t case_id, double out[24]);

/* Measurement helper: copy `bytes` (a multiple of 16) from src to dst, both
 * device pointers, with a plain streaming kernel on hip_stream (NULL =
 * default).  It gives the achievable HBM copy bandwidth and calibrates the
 * hardware byte counters; it is not part of the time step.  Errors:
 * LBM_EINVAL for NULL pointers or a bad size, LBM_EHIP. */
int32_t lbm_stream_copy(void *dst, const void *src, int64_t bytes, void *hip_stream);

int32_t lbm_destroy(lbm_ctx *ctx);
const char *lbm_last_error(const lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TURRET_H */
