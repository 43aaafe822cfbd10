/*
 * mera.h - C ABI of the MI355X scale-invariant binary MERA hot path.
 *
 * The operations follow Ganahl, Milsted, Leichenauer, Hidary and Vidal,
 * "TensorNetwork on TensorFlow: Entanglement Renormalization for quantum
 * critical lattice models" (arXiv:1906.12030):
 *   ascending / descending superoperators  - Sec. II.B, Fig. 4(a,b)
 *   environments of w (6 terms) and u (4)   - Sec. II.C, Fig. 4(c,d), Fig. A1
 *   SVD (polar) update                      - Sec. II.C, Fig. 5
 *   fixed-point density of the scale-invariant layer by iteration - Sec. II.B
 *   energy tr(h rho)                        - Sec. II.B
 *
 * Conventions shared by every call
 *   - Every pointer whose name ends in _d is a DEVICE pointer (HIP global
 *     memory) owned by the caller.  The library never allocates, frees or keeps
 *     caller memory; the caller keeps buffers alive until the stream has
 *     finished the work.
 *   - All tensors are float64, dense, row-major (C order), no padding.
 *       u[a,b,c,d]  disentangler, din^4:  (a,b) lower (finer) legs, (c,d) upper;
 *                   sum_ab u[ab,cd] u[ab,c'd'] = delta (Eq. unitarity).
 *       w[a,b,c]    isometry, din*din*dout: (a,b) lower legs, c upper leg;
 *                   sum_ab w[ab,c] w[ab,c'] = delta (Eq. iso).
 *       three-site operators / densities: (d^3 x d^3) matrices stored as
 *                   [i1,i2,i3, j1,j2,j3] (rows = ket legs, columns = bra legs).
 *   - Geometry: coarse site k owns an isometry on intermediate sites (2k,2k+1);
 *     disentanglers act on intermediate pairs (2k+1,2k+2).  A fine three-site
 *     window sits in two positions under the coarse window (k-1,k,k+1):
 *     LEFT = fine sites 2k-1..2k+1, RIGHT = 2k..2k+2.  AVG = (LEFT+RIGHT)/2,
 *     the translation-averaged superoperator.
 *   - `precision` selects the internal contraction arithmetic only; inputs and
 *     outputs stay float64.  MERA_FP64: FP64 MFMA.  MERA_FP32: operands rounded
 *     to FP32, FP32 MFMA.  MERA_BF16X3: operands rounded to FP32 and split into
 *     bf16 hi+lo pairs, products hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32
 *     accumulation.
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = default stream)
 *     and is asynchronous unless a call says otherwise.
 *   - `ws_d`/`ws_bytes`: caller-provided device workspace of at least
 *     mera_workspace_bytes(...) bytes, 256-byte aligned.  It must not overlap
 *     any input or output.  Inputs and outputs must not overlap each other.
 *   - Errors: the return value is a mera_status.  All argument and shape checks
 *     happen on the host before any HIP call, so an invalid call enqueues
 *     nothing and leaves outputs untouched.  MERA_EDEVICE reports a failed HIP
 *     call (its text via mera_last_error()).  Nothing throws across the ABI.
 *   - Thread safety: calls keep no state between them (apart from the
 *     thread-local last-error text) and may be made from several threads on
 *     different streams with different workspaces.
 */
#ifndef MERA_H
#define MERA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MERA_OK = 0,
  MERA_EINVAL = 1,      /* null pointer, enum out of range, bad count */
  MERA_ESHAPE = 2,      /* inconsistent dimensions (e.g. dout > din^2, rows < cols) */
  MERA_EWORKSPACE = 3,  /* workspace smaller than mera_workspace_bytes() */
  MERA_EDEVICE = 4,     /* a HIP call failed */
  MERA_ENUMERIC = 5,    /* non-finite data, or a polar iteration that did not converge */
  MERA_ENOTCONV = 6     /* a tolerance was not reached within the iteration budget */
} mera_status;

typedef enum { MERA_LEFT = 0, MERA_RIGHT = 1, MERA_AVG = 2 } mera_placement;
typedef enum { MERA_FP64 = 0, MERA_FP32 = 1, MERA_BF16X3 = 2 } mera_precision;

typedef enum {
  MERA_OP_ASCEND = 0,
  MERA_OP_DESCEND = 1,
  MERA_OP_ENV_U = 2,
  MERA_OP_ENV_W = 3,
  MERA_OP_POLAR = 4,        /* din = rows, dout = cols of the blocked environment */
  MERA_OP_FIXED_POINT = 5,  /* din = dout = d of the scale-invariant layer */
  MERA_OP_ENERGY = 6,
  MERA_OP_TREE_ASCEND = 7,   /* binary tree network calls (mera_tree_*) */
  MERA_OP_TREE_DESCEND = 8,
  MERA_OP_TREE_ENV_W = 9,
  MERA_OP_POLAR_NEAR = 10   /* mera_polar_update_near; din = rows, dout = cols */
} mera_op;

/* One MERA layer: disentangler u (din^4) and isometry w (din*din*dout), both
 * device pointers.  1 <= dout <= din*din. */
typedef struct {
  int32_t din;
  int32_t dout;
  const double* u_d;
  const double* w_d;
} mera_layer;

/* Allocation-free descend, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes exactly what mera_descend computes, with the same
 * kernels, but takes its workspace from a static device array of
 * MERA_NOALLOC_SCRATCH_MIB MiB inside the library instead of a caller buffer;
 * every device the library runs on holds that array until the process ends.
 * The chi^7 intermediates are sliced over an open leg until they fit; calls that
 * need more than the array even then (mera_workspace_bytes_min(MERA_OP_DESCEND,
 * ...) above it; for din = dout = chi: chi >= 14 in FP64, chi >= 15 in FP32,
 * chi = 13 and chi >= 15 in split bf16) return MERA_EWORKSPACE before any HIP
 * call.  hip_stream must belong to
 * the calling thread's current device.  The call allocates nothing and keeps no
 * result in the array that a later call depends on (every buffer taken from it
 * is written before it is read), but all calls on one device share the array:
 * calls that overlap in time on one device (several streams or host threads)
 * race and must be serialised by the caller.  Per-launch profiling records are
 * not taken for this call.  Asynchronous. */
#define MERA_NOALLOC_SCRATCH_MIB 256
int mera_descend_noalloc(const mera_layer* layer, const double* rho_in_d, double* rho_out_d,
                         int placement, int precision, void* hip_stream);

/* Ascending superoperator (Sec. II.B, Fig. 4a): h_out = A_P(h_in).
 * h_in_d: din^6 operator on the fine window; h_out_d: dout^6 operator on the
 * coarse window.  A_P is the adjoint of D_P: tr(A_P(o) rho) = tr(o D_P(rho)). */
int mera_ascend(const mera_layer* layer, const double* h_in_d, double* h_out_d, int placement,
                int precision, void* ws_d, size_t ws_bytes, void* hip_stream);

/* Descending superoperator (Sec. II.B, Fig. 4b): rho_out = D_P(rho_in).
 * rho_in_d: dout^6 coarse density; rho_out_d: din^6 fine density. */
int mera_descend(const mera_layer* layer, const double* rho_in_d, double* rho_out_d, int placement,
                 int precision, void* ws_d, size_t ws_bytes, void* hip_stream);

/* Environment of the disentangler (Sec. II.C, Fig. 4d, Fig. A1b):
 * env_u = d e / d(ket copies of u), e = tr(h D_P(rho)).  With MERA_AVG this is
 * the sum of the four contributions (two placements x two disentanglers) with
 * the 1/2 of the averaged superoperator.  h_d: din^6, rho_d: dout^6,
 * env_u_d: din^4.  Euler: <env_u, u> = 2e. */
int mera_env_u(const mera_layer* layer, const double* h_d, const double* rho_d, double* env_u_d,
               int placement, int precision, void* ws_d, size_t ws_bytes, void* hip_stream);

/* Environment of the isometry (Sec. II.C, Fig. 4c, Fig. A1a): the six
 * contributions (two placements x three isometries) for MERA_AVG.
 * env_w_d: din*din*dout.  Euler: <env_w, w> = 3e. */
int mera_env_w(const mera_layer* layer, const double* h_d, const double* rho_d, double* env_w_d,
               int placement, int precision, void* ws_d, size_t ws_bytes, void* hip_stream);

/* SVD update (Sec. II.C, Fig. 5): out = -U V^T where env = U S V^T is the
 * environment blocked as a rows x cols matrix (rows = lower legs, cols = upper
 * legs; rows >= cols), i.e. minus the orthogonal polar factor of env.
 * FP64 only, computed on the device by the Newton-Schulz polar iteration
 * X <- X (3 I - X^T X) / 2 from env / ||env||_F; the host reads the change per
 * iteration in batches of four (one stream synchronisation per batch).
 * sv_d (device, nullable, cols doubles) receives the singular values of env,
 * largest first: the eigenvalues of the symmetric positive semidefinite X^T env
 * at convergence (Householder tridiagonalisation and bisection on the device);
 * needs cols <= 4080 (MERA_ESHAPE otherwise).
 * Synchronises `hip_stream`.  Returns MERA_ENUMERIC for a zero or non-finite
 * env, or when the iteration does not reach an isometry within 100 steps
 * (rank-deficient env: the polar factor is not unique); `out_d` (and sv_d) are
 * still written. */
int mera_polar_update(const double* env_d, int64_t rows, int64_t cols, double* out_d, double* sv_d,
                      void* ws_d, size_t ws_bytes, void* hip_stream);

/* SVD update (Sec. II.C, Fig. 5) that stays defined for a rank-deficient
 * environment.  The paper's update minimises tr(env^T x) over isometries x;
 * when env has zero singular values that minimiser is not unique and
 * mera_polar_update returns MERA_ENUMERIC.  This call first runs
 * mera_polar_update on env; if that reports MERA_ENUMERIC it runs it again on
 * env - t * prev with t = tie * ||env||_F / ||prev||_F (FP64 reductions and
 * axpy on the device), which among those minimisers picks (up to O(tie)) the
 * one closest to prev, the tensor being updated.  Full-rank environments give
 * exactly the output of mera_polar_update.
 * prev_d: device, rows x cols doubles, same blocking as env_d (not modified).
 * tie: finite, > 0 (the optimiser uses 1e-10).  Workspace:
 * mera_workspace_bytes(MERA_OP_POLAR_NEAR, rows, cols, 0, 0) (the polar
 * workspace plus rows * cols doubles for the shifted environment).  Returns
 * MERA_EINVAL for a null prev_d or a bad tie, MERA_ENUMERIC when the shifted
 * environment fails too (or env or prev is zero); otherwise as
 * mera_polar_update.  Synchronises `hip_stream`. */
int mera_polar_update_near(const double* env_d, const double* prev_d, int64_t rows, int64_t cols,
                           double tie, double* out_d, double* sv_d, void* ws_d, size_t ws_bytes,
                           void* hip_stream);

/* Fixed point of the scale-invariant descending superoperator by iteration
 * (Sec. II.B): power-iteration steps rho <- D_AVG(rho), rho <- (rho + rho^T)/2,
 * rho <- rho/tr(rho), with the symmetrisation and renormalisation in FP64.
 * MERA_FP64 runs exactly that.  MERA_FP32 / MERA_BF16X3 run it in
 * iterative-refinement form, in cycles of up to 30 steps: one FP64 residual
 * r = D(rho) - rho, then delta <- D_lp(delta) + r with the reduced-precision D,
 * then rho <- normalise(sym(rho + delta)).  In exact arithmetic a cycle of L
 * steps equals L power-iteration steps; the reduced-precision error is
 * proportional to ||delta|| rather than ||rho||, so repeated calls converge to
 * the FP64 fixed point.  rho_d (d^6) holds the warm start on entry and the
 * result on exit.  layer->din must equal layer->dout.
 * Residual: res(rho) = ||D(rho) - rho||_F / ||rho||_F with D in FP64.
 * tol = 0: exactly `iters` steps, fully asynchronous.
 * tol > 0: at most `iters` steps; res is measured at every FP64 descend of the
 *   current density (every step in MERA_FP64, at the start of every cycle
 *   otherwise) and the call returns that density as soon as res <= tol; if the
 *   budget runs out, one more FP64 descend measures the density returned and
 *   the call returns MERA_ENOTCONV when res > tol (rho_d still holds the last
 *   iterate).  Synchronises the stream at every measurement.
 * resid_d (device, nullable, 1 double) receives res of the density returned
 * (with tol = 0 this costs one more FP64 descend).
 * Errors: MERA_EINVAL also for a negative or non-finite tol. */
int mera_fixed_point_rho(const mera_layer* si, double* rho_d, int32_t iters, double tol, int precision,
                         double* resid_d, void* ws_d, size_t ws_bytes, void* hip_stream);

/* Binary tree network (Sec. I, Fig. 1a): a layer of isometries w only, the
 * binary MERA with identity disentanglers (u[a,b,c,d] = delta_ac delta_bd).
 * Same conventions as the MERA calls: w[a,b,c] (din*din*dout, lower legs
 * first), three-site operators/densities [i1,i2,i3, j1,j2,j3], windows LEFT
 * (the right child of the left isometry and both children of the centre one)
 * and RIGHT (both children of the centre isometry and the left child of the
 * right one) under the coarse window, AVG = (LEFT + RIGHT)/2.  Equal to
 * mera_descend / mera_ascend / mera_env_w with u = identity (the isometry whose
 * children are both traced enters through w^T w, also off the isometry
 * manifold), at O(din^6 dout) work per call instead of O(din^6 dout^3).
 * Workspace: mera_workspace_bytes(MERA_OP_TREE_*, din, dout, precision,
 * placement).  Errors and asynchrony as for mera_descend. */
int mera_tree_descend(int32_t din, int32_t dout, const double* w_d, const double* rho_in_d,
                      double* rho_out_d, int placement, int precision, void* ws_d, size_t ws_bytes,
                      void* hip_stream);
int mera_tree_ascend(int32_t din, int32_t dout, const double* w_d, const double* h_in_d,
                     double* h_out_d, int placement, int precision, void* ws_d, size_t ws_bytes,
                     void* hip_stream);
/* env_w_d (din*din*dout) = d tr(h D_P(rho)) / d(ket copies of w): three
 * contributions per window (left, centre and right isometry), halved and summed
 * for AVG.  Euler: <env_w, w> = 3 e. */
int mera_tree_env_w(int32_t din, int32_t dout, const double* w_d, const double* h_d,
                    const double* rho_d, double* env_w_d, int placement, int precision, void* ws_d,
                    size_t ws_bytes, void* hip_stream);

/* Energy (Sec. II.B): e = tr(h rho) = sum_ij h_ij rho_ji for n x n matrices
 * (n = d^3), FP64 with a fixed reduction order (bitwise reproducible).
 * e_d: device pointer to one double.  Needs no workspace. */
int mera_energy(const double* h_d, const double* rho_d, int64_t n, double* e_d, void* hip_stream);

/* Three-site Hamiltonian density of the transverse-field Ising chain
 * (Sec. II, Eq. ham; three-site regrouping of Sec. II.B):
 *   h2 = -X(x)X - (g/2)(Z(x)1 + 1(x)Z),  h3 = (h2(x)1 + 1(x)h2)/2,
 * with the field g split evenly over the two bonds of each site.  Writes the
 * shifted density h3 - c*1 (8x8, row-major, host memory) and c = lambda_max(h3),
 * so that the written operator is negative semidefinite.  Pure host function. */
int mera_tfim_hamiltonian(double field, double* h_host /* 64 doubles */, double* shift_host);

/* Workspace in bytes needed by `op` for the given shape, precision and
 * placement (placement is ignored where it does not matter).  For
 * MERA_OP_POLAR and MERA_OP_POLAR_NEAR, din = rows and dout = cols.  Returns 0 for invalid
 * arguments.  Pure host function. */
size_t mera_workspace_bytes(int op, int32_t din, int32_t dout, int precision, int placement);

/* Per-launch timing of the contraction kernels, for profiling and roofline
 * accounting.  mera_profile_begin() starts recording (on this thread) a pair
 * of HIP events around every contraction launch; mera_profile_end() waits for
 * the recorded events, copies up to max_entries records into out (host
 * memory), stores their count in *n_out and stops recording.  Recording adds
 * two event records per launch and does not change any result. */
typedef struct {
  char step[48];    /* "la,lb->lc" leg labels of the contraction */
  int32_t arith;    /* mera_precision of the launch */
  int32_t op;       /* mera_op of the call that issued it; -1 for mera_contract */
  double flops;     /* 2*M*N*K of the launch */
  double ms;        /* device time between the two events */
} mera_profile_entry;
int mera_profile_begin(void);
int mera_profile_end(mera_profile_entry* out, int32_t max_entries, int32_t* n_out);

/* Smallest workspace with which `op` still runs: for MERA_OP_DESCEND and
 * MERA_OP_FIXED_POINT the chi^7 intermediates can be processed in slices of
 * an open leg (fine site 3 for the left window, site 2 for the right one);
 * given less than mera_workspace_bytes() but at least this much, those calls
 * pick the smallest slice count that fits.  Equal to mera_workspace_bytes()
 * for the other ops.  Pure host function. */
size_t mera_workspace_bytes_min(int op, int32_t din, int32_t dout, int precision, int placement);

/* General contraction through the same engine as the calls above (diagnostic
 * and test entry point): C[lc] = alpha * sum over the legs shared by A and B of
 * A[la] * B[lb] + beta * C[lc].  la, lb, lc: leg labels (one character per leg,
 * 1..6 legs each, no repeats within an operand); every output leg comes from
 * exactly one operand and every summed leg appears in both (no batch legs).
 * labels / sizes: the extent (1 .. 2^30) of every label used.  A, B, C: device
 * float64, dense row-major in the order of their labels.  precision selects the
 * internal arithmetic (MERA_FP64 / MERA_FP32 / MERA_BF16X3, operands converted in
 * the workspace) and, through the shapes, the kernel (the large-tile split-bf16
 * kernel takes operands contiguous along k with a k-run that is a multiple of
 * 32, M >= 256, N >= 192).  Workspace: ws_bytes >= 8 (|A| + |B|) + 8 min(16 |C|,
 * 2^24) + 1024 always suffices (MERA_EWORKSPACE with the exact need in
 * mera_last_error otherwise).  Errors: MERA_EINVAL (null argument, precision),
 * MERA_ESHAPE (labels, sizes; checked before any HIP call), MERA_EDEVICE.  Async. */
int mera_contract(const char* la, const double* a_d, const char* lb, const double* b_d, const char* lc,
                  double* c_d, const char* labels, const int64_t* sizes, double alpha, double beta,
                  int precision, void* ws_d, size_t ws_bytes, void* hip_stream);

/* Measured matrix-core throughput of this device in TFLOP/s, the peak the
 * contraction kernels are compared against: kind 0 = v_mfma_f32_16x16x32_bf16,
 * 1 = v_mfma_f32_16x16x4_f32, 2 = v_mfma_f64_16x16x4_f64, each with eight
 * independent accumulator chains per wave and register operands only, 8
 * waves per SIMD on every CU; best of three timed launches after a warm-up.
 * scratch_d: caller-owned device buffer of at least 2 MiB (written).
 * Synchronous on the default stream.  Diagnostic, not part of the hot path.
 * Errors: MERA_EINVAL (kind, null pointers), MERA_EWORKSPACE (scratch too
 * small; checked before any HIP call), MERA_EDEVICE. */
int mera_mfma_peak(int kind, void* scratch_d, size_t scratch_bytes, double* tflops_out);

/* Static text for a status code. */
const char* mera_strerror(int status);

/* Text of the last error seen on this thread (HIP error string or argument
 * check), empty if none. */
const char* mera_last_error(void);

/* Double-precision flops of the schedule executed by `op` (multiply-add = 2),
 * for throughput accounting; 0 for invalid arguments.  Pure host function. */
double mera_flops(int op, int32_t din, int32_t dout, int placement);

/* Diagnostic: the contraction schedule of `op` (ascend, descend, env_u,
 * env_w, or one fixed-point iteration) for these sizes, one line per
 * contraction, "la,lb->lc <kernel> m=M n=N k=K tiles=TMxTN splits=S store=..."
 * with <kernel> one of f64, f32, b3 (128 x 128 split-bf16 kernel) and b3x192
 * / b3x256 / b3x288 (large-tile split-bf16 kernel), and store= n8 (16-byte
 * halves of whole 8-column split groups along the output's n legs), n4 / n2 /
 * n1 (vector / FP64 pair / element stores along n) or m4 / m1 (along its m
 * legs), and for a
 * large-tile contraction whose last wave of tiles fills at most a quarter of
 * the GPU, tail=RxS: its last R tile rows run as a second launch split S ways
 * along k (partial sums reduced in a fixed order).
 * Writes at most out_bytes bytes (NUL-terminated) into out (host memory,
 * nullable) and the full size including the NUL into *needed (nullable).
 * The unsliced schedule, with the full workspace.  Returns MERA_EINVAL /
 * MERA_ESHAPE for bad arguments.  Pure host function. */
int mera_schedule_plan(int op, int32_t din, int32_t dout, int precision, int placement, char* out,
                       size_t out_bytes, size_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* MERA_H */
