/*
 * aafwi — Anderson-accelerated acoustic FWI / LSRTM hot path for MI355X (gfx950).
 *
 * C ABI of libaafwi.so.  Every entry point takes plain pointers and sizes.
 * Pointers documented as "device" are HIP device pointers the caller owns
 * (contiguous, 4-byte aligned, at least 16-byte aligned recommended); "host"
 * pointers are read synchronously during the call.  Work is enqueued on the
 * stream given at creation and is asynchronous with respect to the host
 * unless stated otherwise: the caller keeps device buffers alive until that
 * stream has drained.  Outputs are overwritten, never accumulated.
 *
 * Errors: every function returns 0 (AAFWI_OK) or a negative code below;
 * aafwi_last_error() returns a thread-local message for the last failure.
 * Argument validation is synchronous; asynchronous HIP failures surface at
 * the next call.  No C++ exception crosses this boundary.
 *
 * Discretisation (shared by all wave-equation calls; the paper's Section
 * "FWI and LSRTM", eq. FWD, eq. FWI, eq. Born, eq. FWI_adj, eq. adj_grad1):
 *   - model m = 1/c^2 [s^2/m^2] on an interior grid nz x nx, row-major with x
 *     fastest, spacing h (dx = dz); extended by edge replication into nb
 *     sponge cells on all four sides (padded grid nz+2nb by nx+2nb);
 *   - centred 8th-order Laplacian, field zero outside the padded grid;
 *   - sponge: sigma = smax*(xi_x^2 + xi_z^2), xi = depth into the layer in
 *     cells / nb, smax = 3 vref ln(1/refl) / (2 nb h); st = sigma dt/2,
 *     A = 1/(1+st), B = (1-st)/(1+st);
 *   - leapfrog u^{n+1} = 2A u^n - B u^{n-1} + A dt^2/m (Lap u^n + s^n),
 *     u^0 = u^{-1} = 0, n = 0..nt-1;
 *   - point source s^n = wavelet[n] / h^2 at (src_iz+nb, src_ix+nb);
 *   - data d[s][n][r] = u_s^{n+1} at (rec_iz+nb, rec_ix+nb), layout [S][nt][R];
 *   - misfit J = 1/2 sum (d - d_obs)^2 (plain Euclidean sum);
 *   - gradient: the exact discrete adjoint of the above, imaged with
 *     q^n = (Lap u^n + s^n)/m and folded back onto the interior (transpose of
 *     the edge replication).
 */
#ifndef AAFWI_H
#define AAFWI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AAFWI_OK            0
#define AAFWI_E_INVALID    (-1) /* bad argument or geometry                        */
#define AAFWI_E_CFL        (-2) /* vmax_bound*dt/h above the 2D stability limit    */
#define AAFWI_E_NOMEM      (-3) /* device allocation failed                        */
#define AAFWI_E_HIP        (-4) /* HIP runtime error                               */
#define AAFWI_E_NONFINITE  (-5) /* a model value was non-positive or non-finite    */
#define AAFWI_E_STATE      (-6) /* call order violated (e.g. no kept checkpoints)  */

typedef struct aafwi_ctx aafwi_ctx;
typedef struct aafwi_aa aafwi_aa;
/* hipStream_t passed opaquely; NULL is the null stream. */
typedef void* aafwi_stream;

/* Acquisition and grid description.  All array pointers are host memory,
 * copied by aafwi_create. */
typedef struct aafwi_geometry {
    int32_t nz, nx;        /* interior grid (rows = depth, columns = x)           */
    int32_t nb;            /* sponge width in cells (each side), >= 4            */
    float h;               /* grid spacing dx = dz [m]                            */
    float dt;              /* time step [s]                                       */
    int32_t nt;            /* number of time steps = samples per trace            */
    float vref;            /* velocity used for the sponge strength [m/s]         */
    float refl;            /* nominal sponge reflection coefficient; >= 1 = off   */
    float vmax_bound;      /* largest velocity the scheme runs (CFL check); see   */
                           /* the stable domain below                             */
    int32_t nshots;        /* S                                                   */
    int32_t nrec;          /* R receivers per shot                                */
    const int32_t* src_iz; /* [S] interior row of each shot's source node         */
    const int32_t* src_ix; /* [S] interior column                                 */
    const int32_t* rec_iz; /* [S*R] receiver rows, shot-major                     */
    const int32_t* rec_ix; /* [S*R] receiver columns                              */
    const float* wavelet;  /* [nt] source time function sampled at n*dt           */
    int32_t ckpt_every;    /* checkpoint interval in steps; 0 = library default   */
} aafwi_geometry;

/* Stable domain.  The leapfrog scheme is stable only for velocities up to
 * vmax_bound, so every call runs it on m_eff = max(m, 1/vmax_bound^2): a model
 * with faster cells is modelled with those cells at the bound, and the
 * misfit stays finite for every positive model.  Gradients (and the Born
 * adjoint image) are those of the map m -> m_eff -> data: zero at cells where
 * m < 1/vmax_bound^2 (taken from above at the floor itself); Born modelling
 * ignores dm there.  Inside the bound nothing changes.  The Algorithm 2
 * drivers keep their iterates at or above the floor (aafwi_floor). */

/* ---- context -------------------------------------------------------------- */

/* Validate and copy the geometry, allocate all device scratch (wavefields,
 * checkpoints, segment buffer, per-shot images).  Fails with AAFWI_E_CFL if
 * vmax_bound*dt/h > 0.55 (the 2D limit of this scheme is 0.5547). */
int aafwi_create(const aafwi_geometry* g, aafwi_stream stream, aafwi_ctx** out);

/* Synchronise the context's stream and free everything it owns. */
int aafwi_destroy(aafwi_ctx* ctx);

/* Bytes of device memory the context holds. */
int aafwi_device_bytes(const aafwi_ctx* ctx, int64_t* bytes);

/* Synchronise the stream and report a model-validity flag raised by an
 * earlier call (AAFWI_E_NONFINITE if some m was <= 0 or not finite; the flag
 * is then cleared). */
int aafwi_sync(aafwi_ctx* ctx);

/* ---- forward modelling: f(m) = R F(m)  (eq. FWD, eq. FWI) ------------------ */

/* m: device [nz][nx]; d: device [S][nt][R], overwritten.  If keep_ckpt != 0,
 * the run is kept (wavefield checkpoints, or q-hat of every step with full
 * storage, see aafwi_set_full_storage) so that aafwi_adjoint_from_residual
 * can run the backward pass without a second forward. */
int aafwi_forward_model(aafwi_ctx* ctx, const float* m, float* d, int keep_ckpt);

/* r = d - d_obs (device [S][nt][R]; r may alias d) and J = 1/2 sum r^2 written
 * as one double to device memory J (FP64 accumulation, deterministic order). */
int aafwi_residual_misfit(aafwi_ctx* ctx, const float* d, const float* d_obs, float* r,
                          double* J);

/* The same residual and misfit for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc), with no context: r = d - d_obs over n device floats (r
 * may alias d) and J = 1/2 sum r^2 as one device double, with the same
 * kernels and summation order as aafwi_residual_misfit (bitwise equal
 * results for the same n).  The FP64 partial sums live in a static device
 * array of 1024 doubles (8 KiB), one per GPU, held until the process ends;
 * its device address is looked up on the first call on each device.  Nothing
 * is allocated and nothing needs to start at zero.  Work is enqueued on
 * `stream`, which must belong to the current device.  Calls that overlap on
 * one GPU (on different streams, or from different threads) share the array
 * and race.  Errors: AAFWI_E_INVALID for NULL pointers or n outside
 * [1, 2^40]; AAFWI_E_HIP if the array's address cannot be found. */
int aafwi_residual_misfit_noalloc(aafwi_stream stream, int64_t n, const float* d, const float* d_obs,
                                  float* r, double* J);

/* ---- adjoint-state gradient (eq. FWI_adj, eq. adj_grad1) ------------------- */

/* Forward (with checkpoints) + residual + adjoint + zero-lag imaging + fold.
 * m, d_obs: device inputs; grad: device [nz][nx] = dJ/dm; J: device double. */
int aafwi_adjoint_gradient(aafwi_ctx* ctx, const float* m, const float* d_obs, float* grad,
                           double* J);

/* Backward pass only: grad = J'(m)^T r for a data-space vector r [S][nt][R],
 * where m is the model of the last forward run with kept checkpoints (the
 * context holds a copy of it).  AAFWI_E_STATE if no checkpoints are kept. */
int aafwi_adjoint_from_residual(aafwi_ctx* ctx, const float* r, float* grad);

/* Storage layout of the forward wavefield the backward pass images against
 * (eq. adj_grad1 needs the forward field of every step).  Off (the layout at
 * creation): checkpoints every ckpt_every steps, and the backward pass
 * recomputes each segment's forward steps from its checkpoint.  On (full
 * storage): a forward run with kept checkpoints writes q-hat of every step
 * (nt field planes of all shots, nt * nshots * (nz+2nb) * pitch floats, pitch
 * = nx+2nb rounded up to 64) and the backward pass reads them, recomputing
 * nothing.  Gradients, images and traces are bitwise the same in both.  The
 * switch drops kept state (aafwi_adjoint_from_residual needs a new forward
 * run with keep_ckpt=1) and synchronises the stream.  AAFWI_E_NOMEM if the
 * device cannot hold the full layout; the previous layout is kept then. */
int aafwi_set_full_storage(aafwi_ctx* ctx, int enable);
/* enabled: 1 with full storage, 0 with checkpoints. */
int aafwi_get_full_storage(const aafwi_ctx* ctx, int* enabled);

/* ---- Born modelling and its adjoint (eq. Born, eq. LSRTM) ------------------ */

/* d_scat = L dm at background m0 (device [nz][nx] each; d_scat [S][nt][R]). */
int aafwi_born(aafwi_ctx* ctx, const float* m0, const float* dm, float* d_scat);

/* image = L^T y at background m0 (y device [S][nt][R]; image device [nz][nx]).
 * The RTM image of the LSRTM section is aafwi_born_adjoint(m0, d_r).  When
 * the context keeps checkpoints of a forward run whose model is bitwise m0
 * (checked on the device, one host synchronisation), the background forward
 * is not repeated; otherwise it runs with checkpoints kept.  aafwi_born does
 * not discard kept checkpoints. */
int aafwi_born_adjoint(aafwi_ctx* ctx, const float* m0, const float* y, float* image);

/* ---- Anderson acceleration for gradient descent (Algorithm 2, Steps 1-3) --- */

/* State for vectors of n FP32 values with memory parameter M (1 <= M <= 31):
 * a device ring of the last M+1 accepted iterates and gradients, the FP64
 * Gram matrix of consecutive gradient differences, and gamma.  cond_max is
 * the largest 2-norm condition number of A_k kept: older columns are
 * dropped (for good) while cond_2(A_k) > cond_max. */
int aafwi_aa_create(int64_t n, int32_t M, double cond_max, aafwi_stream stream, aafwi_aa** out);
int aafwi_aa_reset(aafwi_aa* aa);
int aafwi_aa_destroy(aafwi_aa* aa);

/* Push the accepted iterate p_k (device [n]) and its gradient g_k (device
 * [n]) and compute, with f_i = -eta g_i and G(p) = p - eta grad J(p) (eq. GD):
 *   p_bar   = G(p_k)                                  (Step 1)
 *   gamma   = argmin ||A_k gamma - f_k||_2            (Step 2, eq. AAopt2),
 *             A_k = [f_{i+1} - f_i] over the window, solved in FP64 from the
 *             Gram matrix by a Jacobi eigen-decomposition
 *   p_tilde = G(p_k) - sum_i gamma_i [G(p_{i+1}) - G(p_i)]   (Step 3, eq. AA2_update)
 * p_bar and p_tilde are device [n] outputs.  gamma (device double [M]) and
 * mk (device int32) receive gamma and M_k if non-NULL.  On the first call
 * after create/reset, p_tilde = p_bar = G(p_0). */
int aafwi_aa_step(aafwi_aa* aa, const float* p_k, const float* g_k, float eta, float* p_bar,
                  float* p_tilde, double* gamma, int32_t* mk);

/* Least-squares solver of Step 2.  AAFWI_AA_GRAM (default): FP64 normal
 * equations of the exact gradient differences, solved by a Jacobi
 * eigen-decomposition (parallel ordering).  AAFWI_AA_QR:
 * the rank-updated QR factorisation of the paper's Step 2 (columns appended
 * by Gram-Schmidt with reorthogonalisation, the oldest removed by Givens
 * rotations; Q is n x M doubles on the device, allocated on first use);
 * its accuracy degrades with cond(A_k), not cond(A_k)^2.  Both apply the
 * same drop rule.  Switching clears the history.  Synchronises the stream. */
#define AAFWI_AA_GRAM 0
#define AAFWI_AA_QR   1
int aafwi_aa_set_solver(aafwi_aa* aa, int solver);

/* Damping beta > 0 of the mixed step (eq. AAupdate0; default 1):
 * p_tilde = xbar + beta fbar with xbar = p_k - sum gamma_i (p_{i+1} - p_i) and
 * fbar = f_k - sum gamma_i (f_{i+1} - f_i); p_bar stays G(p_k).  Takes effect
 * at the next step. */
int aafwi_aa_set_damping(aafwi_aa* aa, float beta);

/* Weighted l2 norm for the least-squares problem of Step 2:
 * min || W^(1/2) (A_k gamma - f_k) || with w (device, n positive floats, kept
 * by reference until replaced; NULL = unweighted).  The drop rule then uses
 * cond_2(W^(1/2) A_k).  Clears the history.  Synchronises the stream. */
int aafwi_aa_set_weights(aafwi_aa* aa, const float* w);

/* Condition number of A_k found by the last step (device double), for logs. */
int aafwi_aa_last_cond(aafwi_aa* aa, double* cond_dev);

/* ---- batched Anderson step (Algorithm 2, Steps 1-3, per instance) ---------- */

/* Anderson state of `count` independent instances (instance i holds vectors
 * of n[i] values; all share the depth M, 1..31, and the drop rule cond_max)
 * whose steps run together: one launch prepares every window, one computes
 * every new Gram row and right-hand side (kReduceBlocks partial sums per
 * instance), one workgroup per instance solves its FP64 system, and one
 * launch mixes every instance.  Each instance's arithmetic and summation
 * order are those of aafwi_aa_step with the Gram solver (no damping, no
 * weights), so its gamma, p_bar and p_tilde are bitwise the same.  The
 * library owns the rings (2 (M+1) n[i] floats per instance), the FP64
 * states and partial sums; all are allocated here.  Errors: AAFWI_E_INVALID
 * for a bad count, n, M or cond_max; AAFWI_E_NOMEM. */
typedef struct aafwi_batch_aa aafwi_batch_aa;
int aafwi_batch_aa_create(int32_t count, const int64_t* n, int32_t M, double cond_max,
                          aafwi_stream stream, aafwi_batch_aa** out);

/* One step for every active instance i (active: host [count] mask, or NULL
 * for all): p_bar[i] = G(p_k[i]) = p_k[i] - eta[i] g_k[i] and p_tilde[i] from
 * the instance's window (eq. AA2_update); on an instance's first step (or
 * after a reset) p_tilde[i] = p_bar[i].  p_k, g_k, p_bar, p_tilde: host
 * arrays of device pointers (n[i] floats each; inactive entries may be
 * NULL); eta: host array.  Inactive instances are left untouched. */
int aafwi_batch_aa_step(aafwi_batch_aa* b, const float* const* p_k, const float* const* g_k,
                        const float* eta, float* const* p_bar, float* const* p_tilde,
                        const uint8_t* active);

/* Clear the windows of the instances selected by `which` (host [count]
 * mask, or NULL for all). */
int aafwi_batch_aa_reset(aafwi_batch_aa* b, const uint8_t* which);

/* Copy every instance's last gamma (device [count][M] doubles) and window
 * size M_k (device [count] int32) out; either pointer may be NULL. */
int aafwi_batch_aa_state(aafwi_batch_aa* b, double* gamma, int32_t* mk);

int aafwi_batch_aa_destroy(aafwi_batch_aa* b);

/* out = lambda*p_tilde + (1-lambda)*p_bar (Algorithm 2, Step 5), formed in
 * FP64 and rounded once; device [n]; out may alias either input. */
int aafwi_blend(aafwi_stream stream, int64_t n, float lambda, const float* p_tilde,
                const float* p_bar, float* out);

/* Number of doubles of device workspace the reductions below need. */
#define AAFWI_DOT_WORKSPACE 1024

/* *out = sum_i x_i y_i in FP64 (device [n] inputs, device double output),
 * summed in a fixed order (bitwise reproducible).  workspace: device memory
 * of AAFWI_DOT_WORKSPACE doubles owned by the caller; calls that may overlap
 * must use different workspaces. */
int aafwi_dot(aafwi_stream stream, int64_t n, const float* x, const float* y, double* out,
              double* workspace);

/* *out = sum_i g_i (a_i - b_i) in FP64 with a_i - b_i formed exactly; the
 * Armijo test of the line search.  workspace as for aafwi_dot. */
int aafwi_dot_diff(aafwi_stream stream, int64_t n, const float* g, const float* a,
                   const float* b, double* out, double* workspace);

/* y = a*x + y in FP32 (device [n]); x may alias y. */
/* Laplacian-filtered RTM image (Section "Numerical Example", the LSRTM
 * comparison): out = -Lap_h image on an nz x nx interior image (device,
 * row-major), 8th-order second differences with zero outside the image,
 * spacing h.  out must not alias image. */
int aafwi_laplacian_filter(aafwi_stream stream, int32_t nz, int32_t nx, float h, const float* image, float* out);

int aafwi_axpy(aafwi_stream stream, int64_t n, float a, const float* x, float* y);

/* x = max(x, floor) in place (device [n], caller-owned), asynchronous on
 * stream: keeps an iterate in the model's stable domain (floor =
 * 1/vmax_bound^2; see the stable domain above).  A NaN entry becomes floor.
 * AAFWI_E_INVALID for n <= 0, a NULL x or a non-finite floor. */
int aafwi_floor(aafwi_stream stream, int64_t n, float floor, float* x);

/* out = a*x in FP32 (device [n]); out may alias x. */
int aafwi_scale(aafwi_stream stream, int64_t n, float a, const float* x, float* out);

/* ---- batches of uneven inversion instances ---------------------------------- */

/* N independent instances (each its own grid, spacing, time step, record
 * length, shots and receivers) advanced together: every stepping launch covers
 * the tiles of all active instances, and each instance derives its own time
 * step, buffer parity and checkpoint slot from the launch's step counter.
 * Each instance reads its model and observed data from, and writes its
 * residual and gradient to, caller-owned device buffers fixed at creation
 * (kept alive until the batch is destroyed), so its launch sequences can be
 * captured once as HIP graphs and replayed (aafwi_batch_use_graphs).
 * geoms, io: host arrays of ninst entries; ckpt_every: checkpoint interval
 * shared by all instances (0 = 50).  Memory is the sum of the instances'
 * needs. */
typedef struct aafwi_batch aafwi_batch;
typedef struct aafwi_batch_io {
    float* m;            /* [nz][nx] model, read by aafwi_batch_forward           */
    const float* d_obs;  /* [S][nt][R] observed data                               */
    float* r;            /* [S][nt][R] residual f(m) - d_obs, written by forward   */
    float* grad;         /* [nz][nx] gradient, written by aafwi_batch_backward      */
} aafwi_batch_io;
int aafwi_batch_create(const aafwi_geometry* geoms, const aafwi_batch_io* io, int32_t ninst,
                       int32_t ckpt_every, aafwi_stream stream, aafwi_batch** out);
int aafwi_batch_destroy(aafwi_batch* b);

/* Copy the misfit J of each instance's last forward run into J (device, N
 * doubles), stream-ordered. */
int aafwi_batch_misfits(aafwi_batch* b, double* J);

/* Host mask of N bytes (NULL = all active).  Masked instances are skipped by
 * every following call; their kept checkpoints, residuals and gradients stay
 * as they were.  Synchronises the batch stream. */
int aafwi_batch_set_active(aafwi_batch* b, const uint8_t* active);

/* For every active instance: r = f(m) - d_obs and J = 1/2 |r|^2 (eq. FWI),
 * keeping wavefield checkpoints when keep_ckpt != 0. */
int aafwi_batch_forward(aafwi_batch* b, int keep_ckpt);

/* For every active instance: grad = J'(m)^T r from its kept checkpoints
 * (eq. FWI_adj, eq. adj_grad1).  AAFWI_E_STATE if one has none. */
int aafwi_batch_backward(aafwi_batch* b);

/* Capture each launch sequence (forward with/without checkpoints, backward)
 * as a HIP graph on first use and replay it afterwards (needs a non-NULL
 * stream).  Masks are read on the device, so replays honour them. */
int aafwi_batch_use_graphs(aafwi_batch* b, int enable);

int aafwi_batch_device_bytes(const aafwi_batch* b, int64_t* bytes);
int aafwi_batch_set_tile(aafwi_batch* b, int32_t kernel_id, int32_t rows_per_wave);

/* Strip height of one instance for stepping kernel kernel_id (or -1 for all):
 * rows per wave in [1, 120], or 0 to follow aafwi_batch_set_tile.  Instances
 * of different grid classes can so take the heights the autotuner chose for
 * their class while sharing every launch (the launch mode, one or two steps
 * per launch, stays common to the batch).  Results do not depend on it
 * (bitwise); captured graphs are rebuilt on their next use. */
int aafwi_batch_set_instance_tile(aafwi_batch* b, int32_t inst, int32_t kernel_id, int32_t rows_per_wave);
int aafwi_batch_kernel_timing(aafwi_batch* b, int every);
int aafwi_batch_kernel_timing_read(aafwi_batch* b, int kernel_id, double* mean_ms, int64_t* count);

/* ---- learned preconditioner -------------------------------------------------
 * A variant of the fixed-point map of the Method section, G(p) = p - eta g
 * (eq. GD), with the gradient replaced by a learned direction
 *   d = softplus(z) * g,   z = CNN([g / rms(g), (m - mean m) / std m]),
 * so d = 0 exactly where g = 0 (G's fixed points are kept) and <d, g> > 0.
 * CNN: four 3x3 zero-padded cross-correlations without bias, channels
 * 2 -> 32 -> 32 -> 32 -> 1, ReLU after the first three; bf16 activations and
 * weights, FP32 accumulation on the matrix cores, FP32 master weights.
 * Weights (host, AAFWI_CNN_PARAMS floats): per layer [C_out][C_in][3][3],
 * layers concatenated; w[co][ci][a][b] multiplies x[ci][i + a - 1][j + b - 1].
 * Training loss of a batch of (g, m, s): mean over images of
 * mean((d / rms(d) + s / rms(s))^2), s being a step p_{k+1} - p_k that an
 * optimiser took; Adam (beta 0.9, 0.999, eps 1e-8) on it.
 * All image arrays are device buffers of B images [B][nz][nx] FP32, on the
 * stream given at creation.  The network owns its weights and activation
 * buffers (about 196 bytes per pixel of max_batch images). */
#define AAFWI_CNN_PARAMS 19296
typedef struct aafwi_cnn aafwi_cnn;

/* weights: host, AAFWI_CNN_PARAMS floats (copied).  max_batch * nz * nx must
 * stay below 2^31 and nz * nx below 2^25 (AAFWI_E_INVALID otherwise). */
int aafwi_cnn_create(int32_t nz, int32_t nx, int32_t max_batch, const float* weights, aafwi_stream stream,
                     aafwi_cnn** out);
int aafwi_cnn_destroy(aafwi_cnn* c);

/* Replace the weights (host) and reset the Adam state; copy them out (host).
 * Both synchronise the network's stream. */
int aafwi_cnn_set_weights(aafwi_cnn* c, const float* weights);
int aafwi_cnn_get_weights(aafwi_cnn* c, float* weights);

/* Inference on B images (1 <= B <= max_batch): z (optional, may be NULL) the
 * network output, d (optional) the direction softplus(z) * g. */
int aafwi_cnn_forward(aafwi_cnn* c, int32_t B, const float* g, const float* m, float* z, float* d);

/* Evaluate the second and third convolutions in one kernel (on, the
 * default: their intermediate activation stays in on-chip memory during
 * inference and is written once for the backward pass during training) or
 * as two kernels (off).  The results are bitwise the same either way. */
int aafwi_cnn_set_fused(aafwi_cnn* c, int32_t on);

/* Weight gradient (device, AAFWI_CNN_PARAMS floats, host weight layout) of
 * the batch loss; loss: device double, optional.  Weights are unchanged. */
int aafwi_cnn_gradients(aafwi_cnn* c, int32_t B, const float* g, const float* m, const float* s, float* grad,
                        double* loss);

/* One Adam step (learning rate lr > 0) on the batch loss; loss (device
 * double, optional) receives the loss before the step. */
int aafwi_cnn_train_step(aafwi_cnn* c, int32_t B, const float* g, const float* m, const float* s, float lr,
                         double* loss);

/* ---- instrumentation ------------------------------------------------------- */

/* HBM stream probe: one launch of a plain streaming kernel over device
 * buffers of `bytes` bytes each (a positive multiple of 16), 256-thread
 * workgroups, blocks_per_cu (1..64) per compute unit of 256.  kind 0 reads a
 * (b receives nothing for finite data but must be a device buffer of 16
 * bytes or more), 1 writes b, 2 copies a to b, 3 writes b = a + 2 c (two
 * reads, one write: the read/write ratio of the two-step adjoint).  Not part
 * of the method: it sets the rates of simple streams beside those of the
 * stepping kernels.  Enqueued on stream, no synchronisation; the caller
 * times it.  Buffers belong to the caller. */
int aafwi_stream_probe(aafwi_stream stream, int32_t kind, int64_t bytes, int32_t blocks_per_cu, const void* a,
                       void* b, const void* c);

/* Kernel ids for aafwi_kernel_timing. */
#define AAFWI_K_FWD_STEP   0 /* forward time step (with injection and sampling)   */
#define AAFWI_K_REC_STEP   1 /* recompute step that stores q for imaging          */
#define AAFWI_K_ADJ_STEP   2 /* adjoint step with imaging                         */
#define AAFWI_K_BORN_STEP  3 /* background + scattered pair step                  */

/* Enable (every > 0) or disable (0) event timing of every `every`-th launch
 * of each stepping kernel on the context's stream; the counters are reset.
 * Event pairs are read back and reused once their launch has completed, so
 * the sample covers every `every`-th launch of a run of any length (a
 * launch is skipped only while all 4096 pairs are still in flight). */
int aafwi_kernel_timing(aafwi_ctx* ctx, int every);

/* Synchronise and return the mean duration in ms and the number of timed
 * launches of kernel `kernel_id`. */
int aafwi_kernel_timing_read(aafwi_ctx* ctx, int kernel_id, double* mean_ms, int64_t* count);

/* Set the z-strip height (rows per wave, 0..120; 0 picks the default; the
 * one-step kernels use at most 64) of
 * stepping kernel kernel_id (an AAFWI_K_* id, or -1 for all of them).  Used
 * by the tile autotuner; results do not depend on it (bitwise). */
int aafwi_set_tile(aafwi_ctx* ctx, int32_t kernel_id, int32_t rows_per_wave);

/* Order of the wave tiles of stepping kernel kernel_id (or -1 for all) in
 * its launch: 0 = the x-tiles of one strip are adjacent (default), 1 = the
 * strips of one tile column are adjacent, G in 2..64 = the same tile of G
 * consecutive shots is adjacent (x-tiles of a strip next, then strips).
 * Adjacent tiles run at about the same time on one XCD, so the order decides
 * whether the x-halo, the strip-overlap or the shared Kp re-reads hit in L2.
 * Results do not depend on it (bitwise). */
int aafwi_set_tile_order(aafwi_ctx* ctx, int32_t kernel_id, int32_t order);

/* Current strip height of stepping kernel kernel_id. */
int aafwi_get_tile(const aafwi_ctx* ctx, int32_t kernel_id, int32_t* rows_per_wave);

/* Time blocking of the forward, recompute and adjoint steps: each launch
 * advances two time levels of a wave tile, evaluating the first level also on
 * the 4-cell frame the second one needs, so every field plane is read and
 * written once per two steps.  Traces, images and gradients are bitwise the
 * same with it on or off (off: one step per launch).  Default at creation:
 * on when two wavefield planes of all shots (of all instances) exceed
 * 256 MB, off otherwise.  Synchronises the stream; drops captured batch
 * graphs. */
int aafwi_set_time_blocking(aafwi_ctx* ctx, int enable);
/* The same for one kernel (AAFWI_K_FWD_STEP, _REC_STEP or _ADJ_STEP): the
 * three choices are independent. */
int aafwi_set_time_blocking_kernel(aafwi_ctx* ctx, int32_t kernel_id, int enable);
/* mask: bit k set when kernel k advances two steps per launch. */
int aafwi_get_time_blocking(const aafwi_ctx* ctx, int* mask);
int aafwi_batch_set_time_blocking(aafwi_batch* b, int enable);
/* mask of the batch's launch modes, as for aafwi_get_time_blocking. */
int aafwi_batch_get_time_blocking(const aafwi_batch* b, int* mask);

/* Thread-local message for the last non-zero return on this thread. */
const char* aafwi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AAFWI_H */
