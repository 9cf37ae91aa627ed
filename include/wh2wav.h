/*
 * wh2wav: fast products with the Walsh-Hadamard-to-wavelet change-of-basis
 * section and its adjoint, on AMD Instinct MI355X (gfx950).
 *
 * Operation (Antun, "Recovering wavelet coefficients from binary samples
 * using fast transforms"):
 *
 *   forward   y = P_Omega A x
 *   adjoint   x = A^T P_Omega^T y
 *
 * A is the N x M section <r_c, w_n> of the change-of-basis matrix between
 * the sequency-ordered Walsh functions w_n (Def. 3.1) and the multiscale
 * Daubechies basis C_{psi,j} on [0,1] with vanishing-moment-preserving
 * boundary functions (Sec. 3.2).  In one dimension M = 2^j and N = 2^{j+q};
 * in two dimensions A acts on M x M coefficient arrays and produces N x N
 * Walsh samples (Sec. 5, Algorithm 2), so the section is N^2 x M^2.  Sec. 5
 * notes that the splitting holds for any d-fold tensor product: in three
 * dimensions A maps M^3 coefficients to N^3 samples.  With the tensor basis
 * the axes may have their own sizes M_a = 2^{j_a}, N_a = 2^{j_a + q} (the
 * 1D section of each axis; Sec. 4 reaches other sizes by padding).  The
 * product is computed in O(N log N) (Algorithm 1 and Lemma 3.3) without
 * forming A: inverse DWT C_{psi,j} -> B_{phi,j} (Remark on compressive
 * sensing), a product with O(2^q) tables of Walsh coefficients of the
 * scaling function (the operators D_l of Sec. 4.1 and Prop. 4.2), a
 * sequency-ordered fast Walsh-Hadamard transform, and the gather onto
 * Omega (P_Omega, Notation).  Everything is real (Algorithm 1 works in R),
 * so the adjoint is the transpose.
 *
 * Layouts
 *   x   1D: M values in C_{psi,j} order [a_{J0} | d_{J0} | ... | d_{j-1}].
 *       2D: M x M row-major array in the quadtree (square / isotropic)
 *       layout: the scaling block at [0, 2^{J0})^2 and, for each level
 *       k = J0..j-1, the bands [0,2^k) x [2^k,2^{k+1}) (phi (x) psi),
 *       [2^k,2^{k+1}) x [0,2^k) (psi (x) phi), [2^k,2^{k+1})^2 (psi (x) psi);
 *       the first array index belongs to the first coordinate.  With
 *       basis2d = WH2WAV_TENSOR, x[c1][c2] is the coefficient of
 *       r_{c1} (x) r_{c2}, c1 and c2 in 1D C_{psi,j} order (M_1 x M_2).
 *       3D: M_1 x M_2 x M_3 row-major.  Isotropic (equal sides): the scaling
 *       block [0, 2^{J0})^3 and, per level k, the 7 blocks at offset 2^k
 *       along the axes a with beta_a = 1 (beta in {0,1}^3, not all zero),
 *       holding psi along those axes and phi along the others.  Tensor:
 *       x[c1][c2][c3] is the coefficient of r_{c1} (x) r_{c2} (x) r_{c3}.
 *   y   m = |Omega| values in increasing order of the sequency index n
 *       (1D) or of the row-major linear index of (n1, ..., n_d) over the
 *       N_1 x ... x N_d array (2D, 3D), n1 the first coordinate.
 *   Element type is float or double as chosen by the plan (dtype).
 *
 * Ownership and errors
 *   Plans are created on the host and own their device tables; a plan is
 *   immutable after creation and may be used from several streams at once
 *   as long as each call has its own workspace.  x, y and ws are caller-
 *   owned device pointers; x, y and ws must not overlap.  Calls are
 *   asynchronous on `stream` (a hipStream_t, or NULL for the null stream).
 *   Every function returns WH2WAV_OK (0) or a negative status; nothing
 *   throws across this interface (a failed host allocation inside a call
 *   returns WH2WAV_ENOMEM, any other internal exception WH2WAV_EINTERNAL).
 *   Argument errors are detected on the host before any launch.  A plan or
 *   batch handle that was destroyed, or never returned by a plan call, is
 *   refused with WH2WAV_EINVAL before it is dereferenced (destroying NULL is
 *   a no-op).  wh2wav_last_error() returns a thread-local message for the
 *   last failure on the calling thread.
 */
#ifndef WH2WAV_H
#define WH2WAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WH2WAV_OK = 0,
  WH2WAV_EINVAL = -1,        /* bad argument or descriptor */
  WH2WAV_EUNSUPPORTED = -2,  /* valid but not implemented (e.g. size limits) */
  WH2WAV_ENOMEM = -3,        /* host or device allocation failed */
  WH2WAV_EHIP = -4,          /* a HIP runtime call or launch failed */
  WH2WAV_EINTERNAL = -5      /* plan construction failed a self-check */
};

enum { WH2WAV_F32 = 0, WH2WAV_F64 = 1 };
enum {
  WH2WAV_DB = 0,                      /* Daubechies, minimum phase (Sec. 3.2) */
  WH2WAV_SYM = 1                      /* symlets: least-asymmetric spectral factor (Sec. 3.2, Table 1);
                                         the root choice of least phase deviation from linear */
};
enum {
  WH2WAV_BD = 0,                      /* vanishing-moment-preserving boundary functions (Sec. 3.2) */
  WH2WAV_PER = 1                      /* periodic extension (Sec. 3.2, Prop. 4.2 "per"): each
                                         function crossing an end is periodised with period 1 */
};

/* Wavelet basis in 2D and 3D.  ISOTROPIC: at each level the scaling block
 * splits into phi (x) psi, psi (x) phi, psi (x) psi (the quadtree layout
 * below; in 3D the 7 products with at least one psi).  TENSOR: the products
 * r_{c1} (x) r_{c2} (x) ... of the 1D bases C_{psi,j_a} of the axes, x in 1D
 * order along each index; by Fubini (Sec. 5) its section is the Kronecker
 * product of the 1D sections of the axes. */
enum { WH2WAV_ISOTROPIC = 0, WH2WAV_TENSOR = 1 };

typedef struct wh2wav_plan_s* wh2wav_plan_t;

typedef struct {
  int dim;              /* 1, 2 or 3 */
  int j;                /* M = 2^j per dimension, j0 <= j */
  int q;                /* N = 2^{j+q} per dimension, q >= 1 (Sec. 4: q > 0) */
  int j0;               /* coarsest level J0: 2^{J0} >= 2 nu for nu >= 2 (Sec. 3.2) */
  int nu;               /* vanishing moments, 1 (Haar) .. 10 */
  int family;           /* WH2WAV_DB or WH2WAV_SYM */
  int boundary;         /* WH2WAV_BD or WH2WAV_PER */
  int dtype;            /* WH2WAV_F32 or WH2WAV_F64 */
  int64_t m;            /* |Omega|; with omega == NULL, m must equal N_1 ... N_dim (all samples) */
  const int64_t* omega; /* host array of m strictly increasing linear indices in
                           [0, N_1 ... N_dim), or NULL; copied during wh2wav_plan */
  int basis2d;          /* dim 2 and 3: WH2WAV_ISOTROPIC (0) or WH2WAV_TENSOR (1) */
  int j_axes[3];        /* dim 2 and 3: j_a of axis a (M_a = 2^{j_a}, N_a = 2^{j_a + q}); 0 takes j;
                           entries at a >= dim must be 0; unequal sides need WH2WAV_TENSOR */
} wh2wav_desc;

/* Build a plan: host-side tables (Sec. 3.2, Sec. 4.1, Prop. 4.2) and their
 * upload to the current HIP device.  *out receives the handle. */
int wh2wav_plan(const wh2wav_desc* desc, wh2wav_plan_t* out);

/* Bytes of device workspace a forward or adjoint call needs (may be 0). */
int wh2wav_workspace_size(wh2wav_plan_t plan, size_t* bytes);

/* y = P_Omega A x.  x: M_1 ... M_dim elements, y: m elements (device pointers). */
int wh2wav_forward(wh2wav_plan_t plan, const void* x, void* y, void* ws, void* stream);

/* x = A^T P_Omega^T y.  y: m elements, x: M_1 ... M_dim elements (device pointers). */
int wh2wav_adjoint(wh2wav_plan_t plan, const void* y, void* x, void* ws, void* stream);

/* Staged execution, for callers that time or interleave the stages (for
 * example with events recorded between them on the same stream).  Running
 * stages 0 .. count-1 in order on one stream with one workspace is exactly
 * wh2wav_forward / wh2wav_adjoint.  Forward (direction 0): 0 = inverse DWT
 * (C_{psi,j} -> B_{phi,j}), 1 = column pass (2D; the whole line transform in
 * 1D), 2 = row pass with the gather onto Omega (2D).  Adjoint (direction 1):
 * 0 = row pass with the scatter from Omega (2D; the whole line transform in
 * 1D), 1 = column pass (2D; nothing in 1D), 2 = forward DWT.  The workspace
 * carries the intermediates between stages. */
int wh2wav_stage_count(wh2wav_plan_t plan, int direction, int* count);
int wh2wav_forward_stage(wh2wav_plan_t plan, int stage, const void* x, void* y, void* ws, void* stream);
int wh2wav_adjoint_stage(wh2wav_plan_t plan, int stage, const void* y, void* x, void* ws, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): exactly
 * wh2wav_forward, but the workspace is a fixed array of
 * WH2WAV_NOALLOC_MAX_WORKSPACE bytes inside the library, one per GPU, held
 * until the process ends; the call allocates nothing.  The caller still
 * passes x and y (device pointers, as for wh2wav_forward).  The plan's device
 * must be current.  Plans whose wh2wav_workspace_size exceeds the array are
 * refused with WH2WAV_EUNSUPPORTED.  Every call on one GPU uses the same
 * array, so calls that overlap in time on one GPU (on different streams or
 * from different host threads) race: the caller must order them, for example
 * on one stream. */
#define WH2WAV_NOALLOC_MAX_WORKSPACE (32u << 20)
int wh2wav_forward_noalloc(wh2wav_plan_t plan, const void* x, void* y, void* stream);

/* Release the plan and its device memory.  NULL is accepted. */
int wh2wav_destroy(wh2wav_plan_t plan);

/* Message describing the last failure on this thread ("" if none). */
const char* wh2wav_last_error(void);

/* ------------------------------------------------------------------ batches
 * Many independent operators of the kind above (each with its own size,
 * wavelet order, q, element type and Omega) computed together: the
 * reconstructions in the paper solve one problem per image, and a serving
 * loop or a parameter sweep runs many at once.  Every instance computes
 * exactly what wh2wav_forward / wh2wav_adjoint compute for its descriptor.
 *
 * Each wh2wav_forward_batch / wh2wav_adjoint_batch call is ONE hipGraph
 * launch on `stream`: the graph forks into B concurrent branches, the
 * instances' kernels are dealt to the branches in the schedule's order, and
 * the branches join before the graph ends.  The graph for a given set of
 * pointers (xs, ys, ws) is captured on its first use and replayed afterwards;
 * the batch keeps the graphs of its 8 most recent pointer sets.
 *
 * Ownership and errors follow the single-plan rules: descriptors are copied,
 * pointer arrays are read during the call only (the device buffers they name
 * must stay valid while a graph that captured them may be replayed), one
 * batch must not be used from two threads at once, and instance i uses bytes
 * [off_i, off_i + size_i) of ws (sizes rounded up to 256 B). */
typedef struct wh2wav_batch_s* wh2wav_batch_t;

/* Plan `count` instances; *out receives the handle.  Fails (and releases every
 * plan made so far) if any descriptor fails; the message names the instance. */
int wh2wav_plan_batch(const wh2wav_desc* descs, int count, wh2wav_batch_t* out);

/* Bytes of device workspace the batch needs (sum of the instances'). */
int wh2wav_batch_workspace_size(wh2wav_batch_t b, size_t* bytes);

/* ys[i] = P_Omega_i A_i xs[i] for every instance (arrays of `count` device pointers). */
int wh2wav_forward_batch(wh2wav_batch_t b, const void* const* xs, void* const* ys, void* ws, void* stream);

/* xs[i] = A_i^T P_Omega_i^T ys[i] for every instance. */
int wh2wav_adjoint_batch(wh2wav_batch_t b, const void* const* ys, void* const* xs, void* ws, void* stream);

/* Schedule: `branches` concurrent graph branches (1..8) and instance `order`
 * (0: as given, 1: largest first).  Default 4 and 1. */
int wh2wav_batch_schedule(wh2wav_batch_t b, int* branches, int* order);
int wh2wav_batch_set_schedule(wh2wav_batch_t b, int branches, int order);

/* Execution mode.  BRANCHES (default): every instance runs its own stage
 * kernels in the graph branches.  FUSED: the small instances -- 1D lines of
 * at most 1024 values and square 2D arrays of at most 512^2, isotropic basis,
 * boundary-corrected or periodic, at least one sample -- run as fused
 * launches over (instance, stage, tile) work items: one launch per round of
 * their stages (round r = stage r of every such instance), inside the same
 * graph beside the branches, which keep the other instances.  Its results
 * equal the single plans' to rounding (other summation orders), not bit for
 * bit. */
enum { WH2WAV_BATCH_BRANCHES = 0, WH2WAV_BATCH_FUSED = 1 };
int wh2wav_batch_set_mode(wh2wav_batch_t b, int mode);

/* The mode; *fused_instances (may be NULL) receives how many instances the
 * fused launches take in that mode, *fused_launches (may be NULL) how many
 * launches they make per forward call. */
int wh2wav_batch_mode(wh2wav_batch_t b, int* mode, int* fused_instances, int* fused_launches);

/* Autotuner: times forward(xs -> ys) followed by adjoint(ys -> xa), `reps`
 * times per candidate schedule (branches 1, 2, 4, 8 x both orders) on
 * `stream`, keeps the fastest schedule and writes its time per pair of graph
 * launches in ms to *best_ms (may be NULL).  Synchronises `stream`. */
int wh2wav_batch_tune(wh2wav_batch_t b, const void* const* xs, void* const* ys, void* const* xa, void* ws,
                      void* stream, int reps, float* best_ms);

/* Release the batch, its graphs and its plans.  NULL is accepted. */
int wh2wav_destroy_batch(wh2wav_batch_t b);

/* Host-side introspection (no GPU needed): the float64 tables a plan for
 * `desc` would upload.  `which` selects the table; at most `capacity`
 * values are written to `out` and the full length goes to *count.
 *   WH2WAV_TABLE_H, _G        filter taps h_c, g_c, c = -nu+1 .. nu
 *   WH2WAV_TABLE_T            interior table T[l][s], l = -nu+1..nu-1, s < 2^q
 *   WH2WAV_TABLE_BAND_L, _R   boundary bands of Prop. 4.2 (layout in planner.h)
 *   WH2WAV_TABLE_SYN_L, _R    boundary blocks of the one-level synthesis matrix
 *   WH2WAV_TABLE_ROWPTR       Omega row offsets (as doubles) */
enum {
  WH2WAV_TABLE_H = 0, WH2WAV_TABLE_G = 1, WH2WAV_TABLE_T = 2,
  WH2WAV_TABLE_BAND_L = 3, WH2WAV_TABLE_BAND_R = 4,
  WH2WAV_TABLE_SYN_L = 5, WH2WAV_TABLE_SYN_R = 6, WH2WAV_TABLE_ROWPTR = 7
};
int wh2wav_host_table(const wh2wav_desc* desc, int which, double* out, size_t capacity,
                      size_t* count);

#ifdef __cplusplus
}
#endif

#endif /* WH2WAV_H */
