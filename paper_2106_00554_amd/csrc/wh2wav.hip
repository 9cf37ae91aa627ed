// Kernels and C-ABI entry points of the Walsh-to-boundary-wavelet operator.
//
// One 1D line of the operator in the scaling basis B_{phi,j} (the matrix of
// Sec. 4, called G in Sec. 5) factors through the dyadic cells of [0, 1]:
// for p < M = 2^j and t in [0, 1), Lemma 3.2 (1) and (3) give
//     w_n((p + t)/M) = w_n(p/M) w_s(t),     s = floor(n / M) < 2^q,
// so that (Lemma 3.3)
//     <f, w_n> = sum_p w_n(p/M) L[p, s],
//     L[p, s] = sum_m xi_m 2^{-j/2} W[phi_{0,p-m}](s)   (plus Prop. 4.2 edges).
// The stages are therefore
//   1. table product  L[:, s] = (2nu-1)-tap correlation of xi with the table
//      T[l][s] (operators D_l, Sec. 4.1) plus the dense boundary bands;
//   2. one M-point Walsh-Hadamard transform per phase s (2^q of them);
//   3. index map: w_{sM+b}(p/M) = H_nat[k, p] with the natural (Sylvester)
//      index k = bitrev_j(gray(b)) xor (s & 1) -- only the parity of s enters,
//      through digit n^(j+1) of Def. 3.1;
//   4. gather onto Omega (P_Omega) or scatter for the adjoint.
// This is the same result as the paper's sum over l of D_l H_l (Alg. 1) with
// the linear table product moved in front of the transform, which needs 2^q
// transforms of length M instead of 2nu-1 transforms of length N.
//
// In 2D (Alg. 2, alpha = G xi G^T) a column pass applies G along the first
// index and writes an N x M intermediate whose rows are in natural order
// r = s M + k; the row pass applies G along the second index of each row and
// gathers the samples of Omega in row n1 = seq(r).  The adjoint runs the same
// passes transposed.  The inverse DWT from C_{psi,j} to B_{phi,j} (Remark on
// compressive sensing) runs first in the forward direction and its transpose
// last in the adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/wh2wav.h"
#include "abi_internal.h"
#include "fast2d.h"
#include "generic_lines.h"
#include "planner.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_OK(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(WH2WAV_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

using namespace wh2wav_generic;

// One level along lines (line_stride apart, element stride elem_stride), one
// thread per output value; line_fast: consecutive threads take consecutive
// lines (strided lines).  per: the periodic extension; analysis: the forward
// DWT level instead of the inverse.
template <typename T>
__global__ void k_level(const T* __restrict__ in, T* __restrict__ out, int64_t lines, int64_t line_stride,
                        int64_t elem_stride, int k, int line_fast, int analysis, Tables<T> t) {
  const int64_t size = int64_t(2) << k;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= lines * size) return;
  const int64_t line = line_fast ? gid % lines : gid / size;
  const int64_t n = line_fast ? gid / lines : gid % size;
  const T* src = in + line * line_stride;
  T v;
  if (analysis)
    v = t.per ? analysis_value_per<T>(src, elem_stride, n, k, t) : analysis_value<T>(src, elem_stride, n, k, t);
  else
    v = t.per ? synth_value_per<T>(src, elem_stride, n, k, t) : synth_value<T>(src, elem_stride, n, k, t);
  out[line * line_stride + n * elem_stride] = v;
}

// One level along `axis` of an s0 x s1 x s2 row-major array (unused axes of
// extent 1): the elements whose coordinate along the axis is below 2^{k+1}
// -- and, with `cube` (isotropic basis), whose every coordinate is -- take
// one level of synthesis (analysis); every other element is copied.
template <typename T>
__global__ void k_level_nd(const T* __restrict__ in, T* __restrict__ out, int64_t s0, int64_t s1, int64_t s2,
                           int axis, int k, int cube, int analysis, Tables<T> t) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= s0 * s1 * s2) return;
  const int64_t i2 = gid % s2, i1 = (gid / s2) % s1, i0 = gid / (s1 * s2);
  const int64_t size = int64_t(2) << k;
  const int64_t n = axis == 0 ? i0 : axis == 1 ? i1 : i2;
  const int64_t es = axis == 0 ? s1 * s2 : axis == 1 ? s2 : 1;
  const bool inside = n < size && (!cube || (i0 < size && i1 < size && i2 < size));
  if (!inside) {
    out[gid] = in[gid];
    return;
  }
  const T* src = in + (gid - n * es);
  T v;
  if (analysis)
    v = t.per ? analysis_value_per<T>(src, es, n, k, t) : analysis_value<T>(src, es, n, k, t);
  else
    v = t.per ? synth_value_per<T>(src, es, n, k, t) : synth_value<T>(src, es, n, k, t);
  out[gid] = v;
}

// out = in^T for an n x n row-major array (any n), one element per thread.
template <typename T>
__global__ void k_transpose_any(const T* __restrict__ in, T* __restrict__ out, int64_t n) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= n * n) return;
  const int64_t r = gid / n, c = gid % n;
  out[c * n + r] = in[r * n + c];
}

// Plain fill (kept as a kernel so that the path records no memset nodes when
// a caller captures it into a graph).
template <typename T>
__global__ void k_fill(T* __restrict__ out, int64_t n, T value) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = value;
}

template <typename T>
void launch_fill(T* out, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(unsigned((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, out, n, T(0));
}

// ------------------------------------------------------------ line kernels
LineMap lines_at(int64_t ls, int64_t es) { return LineMap{int64_t(1) << 62, 0, ls, es}; }

// G (k_fwd_lines) and G^T (k_adj_lines): lpw lines per workgroup, each by
// blockDim / lpw threads in its own lbytes of LDS (short lines share a
// workgroup instead of leaving most of its threads idle).  The dispatcher
// deals consecutive workgroups round-robin over the 8 XCDs; the first line
// of workgroup b is taken so that each XCD gets a contiguous band of lines,
// and lines that share cache lines (a strided pass over neighbouring
// columns) meet in one L2.
__device__ __forceinline__ int64_t first_line(int lpw) {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t wg = nb % 8 == 0 ? (b % 8) * (nb / 8) + b / 8 : b;
  return wg * lpw;
}

// NU: the wavelet order (the taps of the table product unrolled).
template <typename T, int NU>
__global__ void __launch_bounds__(kThreads)
k_fwd_lines(const T* __restrict__ in, LineMap im, T* __restrict__ out, LineMap omap, int j, int gather, RowMap rm,
            Tables<T> t, OmegaDev om, int lpw, int lbytes) {
  extern __shared__ unsigned char smem_raw[];
  const int G = int(blockDim.x) / lpw, sub = int(threadIdx.x) / G;
  fwd_line<T, NU>(in, im, out, omap, j, gather, rm, t, om, first_line(lpw) + sub, smem_raw + sub * lbytes,
                  int(threadIdx.x) % G, G);
}

template <typename T, int NU>
__global__ void __launch_bounds__(kThreads)
k_adj_lines(const T* __restrict__ in, LineMap im, T* __restrict__ out, LineMap omap, int j, int scatter, RowMap rm,
            Tables<T> t, OmegaDev om, int lpw, int lbytes) {
  extern __shared__ unsigned char smem_raw[];
  const int G = int(blockDim.x) / lpw, sub = int(threadIdx.x) / G;
  adj_line<T, NU>(in, im, out, omap, j, scatter, rm, t, om, first_line(lpw) + sub, smem_raw + sub * lbytes,
                  int(threadIdx.x) % G, G);
}

#define WH2WAV_LINE_NUS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

}  // namespace

// ======================================================== plan + entry points
struct wh2wav_plan_s {
  wh2wav::HostPlan host;
  void* d_tables = nullptr;   // element type = dtype
  uint32_t* d_mask = nullptr;
  int64_t* d_row_ptr = nullptr;
  uint16_t* d_pos16 = nullptr;
  int64_t* d_seg_ptr = nullptr;
  int32_t* d_pos32 = nullptr;
  size_t off_h = 0, off_g = 0, off_T = 0, off_BL = 0, off_BR = 0, off_SL = 0, off_SR = 0;
  size_t off_T_ax[3] = {0, 0, 0}, off_BL_ax[3] = {0, 0, 0}, off_BR_ax[3] = {0, 0, 0};  // per-axis path
  size_t off_BLf = 0, off_BRf = 0, off_BLa = 0, off_BRa = 0;  // band copies of the wave kernels
  int device = 0;             // the device current when the plan was made
};

namespace {

template <typename T>
Tables<T> tables_of(const wh2wav_plan_s* p) {
  const T* base = static_cast<const T*>(p->d_tables);
  Tables<T> t;
  t.h = base + p->off_h;
  t.g = base + p->off_g;
  t.tabT = base + p->off_T;
  t.bandL = base + p->off_BL;
  t.bandR = base + p->off_BR;
  t.synL = base + p->off_SL;
  t.synR = base + p->off_SR;
  t.nu = p->host.nu;
  t.q = p->host.q;
  t.Q = p->host.Q;
  t.per = p->host.per ? 1 : 0;
  return t;
}

// Tables of axis a on the per-axis path (the interior and band tables carry
// that axis's 2^{-j_a/2}).
template <typename T>
Tables<T> axis_tables_of(const wh2wav_plan_s* p, int a) {
  Tables<T> t = tables_of<T>(p);
  const T* base = static_cast<const T*>(p->d_tables);
  t.tabT = base + p->off_T_ax[a];
  t.bandL = base + p->off_BL_ax[a];
  t.bandR = base + p->off_BR_ax[a];
  return t;
}

template <typename T>
wh2wav_fast::Tables<T> fast_tables_of(const wh2wav_plan_s* p) {
  const Tables<T> a = tables_of<T>(p);
  wh2wav_fast::Tables<T> f;
  f.h = a.h, f.g = a.g, f.tabT = a.tabT, f.bandL = a.bandL, f.bandR = a.bandR, f.synL = a.synL, f.synR = a.synR;
  const T* base = static_cast<const T*>(p->d_tables);
  f.bandLf = base + p->off_BLf, f.bandRf = base + p->off_BRf, f.bandLa = base + p->off_BLa, f.bandRa = base + p->off_BRa;
  f.nu = a.nu, f.q = a.q, f.Q = a.Q, f.per = a.per;
  return f;
}

wh2wav_fast::Omega fast_omega_of(const wh2wav_plan_s* p) {
  wh2wav_fast::Omega o;
  o.pos = p->d_pos16;
  o.seg_ptr = p->d_seg_ptr;
  o.full = p->host.full_omega ? 1 : 0;
  return o;
}

bool use_fast1d(const wh2wav_plan_s* p) {
  const auto& H = p->host;
  const bool f64 = H.dtype == WH2WAV_F64;
  return H.dim == 1 && !H.nd && !H.per && wh2wav_fast::supported1d(f64 ? 8 : 4, H.j, H.nu, H.q) && H.j0 <= (f64 ? 13 : 14);
}

// 1D lines of 128 .. 2048 values: the whole line transform (table product,
// FWHT, gather / scatter) in one workgroup of Q waves, the 2D row-pass kernel
// on the single row of the 1D operator.
bool use_wave1d(const wh2wav_plan_s* p) {
  const auto& H = p->host;
  return use_fast1d(p) && H.j <= 11 && wh2wav_fast::supported(H.dtype == WH2WAV_F64 ? 8 : 4, H.j, H.nu, H.q) &&
         (H.full_omega || !H.pos16.empty());
}

// 1D lines of the wave kernels whose LDS holds the whole operator: one launch
// per direction (wavelet levels fused with the line transform).
bool use_line1d_fused(const wh2wav_plan_s* p) {
  const auto& H = p->host;
  return use_wave1d(p) && wh2wav_fast::line1d_fused(H.dtype == WH2WAV_F64 ? 8 : 4, H.j, H.nu, H.q);
}

bool use_fast(const wh2wav_plan_s* p) {
  const auto& H = p->host;
  return H.dim == 2 && !H.nd && wh2wav_fast::supported(H.dtype == WH2WAV_F64 ? 8 : 4, H.j, H.nu, H.q);
}

OmegaDev omega_of(const wh2wav_plan_s* p) {
  OmegaDev o;
  o.mask = p->d_mask;
  o.row_ptr = p->d_row_ptr;
  o.wpr = p->host.words_per_row;
  o.full = p->host.full_omega ? 1 : 0;
  return o;
}

constexpr size_t kMaxLds = 160 * 1024;

// The dynamic-LDS limit of the line kernels is raised once per plan
// (prepare_line_kernels); calls only check the size.
template <typename T>
int check_and_set_smem(const void* kernel, size_t bytes) {
  (void)kernel;
  if (bytes > kMaxLds) return fail(WH2WAV_EUNSUPPORTED, "line too long for the LDS line kernels");
  return WH2WAV_OK;
}

// G (fwd) or G^T on `lines` lines of 2^j values through the generic line
// kernels.  Lines shorter than a workgroup share one: lpw of them, each with
// kThreads / lpw threads and its own LDS.
template <typename T>
int launch_lines(const wh2wav_plan_s* p, bool fwd, int64_t lines, int j, const T* in, LineMap im, T* out,
                 LineMap om_, int omega_side, RowMap rm, const Tables<T>& tab, hipStream_t st) {
  const int64_t M = int64_t(1) << j;
  int lpw = int(kThreads / (M < kThreads ? M : kThreads));
  while (lpw > 1 && lines % lpw) lpw >>= 1;
  const int G = kThreads / lpw;
  size_t lb = 2 * size_t(M) * sizeof(T);
  if (omega_side && !p->host.full_omega) lb += sizeof(int) * (2 * size_t(p->host.words_per_row) + G);
  lb = (lb + 15) / 16 * 16;
  int rc = check_and_set_smem<T>(nullptr, lb * lpw);
  if (rc) return rc;
  const dim3 grid(unsigned(lines / lpw));
  const OmegaDev om = omega_of(p);
#define X(V)                                                                                                      \
  if (tab.nu == V) {                                                                                              \
    if (fwd)                                                                                                      \
      hipLaunchKernelGGL((k_fwd_lines<T, V>), grid, dim3(kThreads), lb * lpw, st, in, im, out, om_, j, omega_side, \
                         rm, tab, om, lpw, int(lb));                                                              \
    else                                                                                                          \
      hipLaunchKernelGGL((k_adj_lines<T, V>), grid, dim3(kThreads), lb * lpw, st, in, im, out, om_, j, omega_side, \
                         rm, tab, om, lpw, int(lb));                                                              \
    HIP_OK(hipGetLastError());                                                                                    \
    return WH2WAV_OK;                                                                                             \
  }
  WH2WAV_LINE_NUS(X)
#undef X
  return fail(WH2WAV_EINTERNAL, "no line kernel for this wavelet order");
}

template <typename T>
int prepare_line_kernels() {
#define X(V)                                                                                                      \
  HIP_OK(hipFuncSetAttribute((const void*)k_fwd_lines<T, V>, hipFuncAttributeMaxDynamicSharedMemorySize,           \
                             int(kMaxLds)));                                                                      \
  HIP_OK(hipFuncSetAttribute((const void*)k_adj_lines<T, V>, hipFuncAttributeMaxDynamicSharedMemorySize,           \
                             int(kMaxLds)));
  WH2WAV_LINE_NUS(X)
#undef X
  return WH2WAV_OK;
}

template <typename T>
int launch_synth(const wh2wav_plan_s* p, const T* in, T* out, int64_t lines, int64_t ls, int64_t es,
                 int k, bool line_fast, bool analysis, hipStream_t st) {
  const int64_t total = lines * (int64_t(2) << k);
  const int64_t blocks = (total + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_level<T>, dim3(unsigned(blocks)), dim3(kThreads), 0, st, in, out, lines, ls, es, k,
                     int(line_fast), int(analysis), tables_of<T>(p));
  HIP_OK(hipGetLastError());
  return WH2WAV_OK;
}

template <typename T>
int launch_transpose(const T* in, T* out, int64_t n, hipStream_t st) {
  const int64_t total = n * n;
  hipLaunchKernelGGL(k_transpose_any<T>, dim3(unsigned((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                     in, out, n);
  HIP_OK(hipGetLastError());
  return WH2WAV_OK;
}

// Tensor-product basis: x[c1][c2] is the coefficient of r_{c1} (x) r_{c2}, so
// xi = V x V^T with V the 1D multilevel synthesis (boundary-corrected or
// periodic, as the plan says).  In the transposed frame xi^T = V x^T V^T: the
// full 1D synthesis along every column, then along every row.  Sides below
// 32: one launch per level and direction, each level writing its block into
// `tmp`, which is copied back into `cur` (a memcpy node, not a memset, if a
// caller captures the call).
template <typename T>
int tensor_level(const wh2wav_plan_s* p, T* cur, T* tmp, bool columns, int k, bool analysis, hipStream_t st) {
  const int64_t M = p->host.M, size = int64_t(2) << k;
  const size_t e = sizeof(T);
  int rc = columns ? launch_synth<T>(p, cur, tmp, M, 1, M, k, true, analysis, st)
                   : launch_synth<T>(p, cur, tmp, M, M, 1, k, false, analysis, st);
  if (rc) return rc;
  if (columns)  // rows 0 .. size-1, all M columns
    HIP_OK(hipMemcpy2DAsync(cur, M * e, tmp, M * e, M * e, size, hipMemcpyDeviceToDevice, st));
  else  // columns 0 .. size-1 of all M rows
    HIP_OK(hipMemcpy2DAsync(cur, M * e, tmp, M * e, size * e, M, hipMemcpyDeviceToDevice, st));
  return WH2WAV_OK;
}

// The square tensor basis with lines of at most the LDS line length and a
// side of at least 32 takes the line kernels: every level of a line in one
// workgroup, and the 32 x 32-tile transpose between the two axes.
bool tensor_lines(const wh2wav_plan_s* p) {
  const auto& H = p->host;
  return H.tensor && !H.nd && H.dim == 2 && H.M >= 32 &&
         wh2wav_fast::lines_levels_fit(H.dtype == WH2WAV_F64 ? 8 : 4, H.j);
}

// Tensor basis, forward first stage: x -> xi^T (out); W scratch.  With V the
// 1D multilevel synthesis and the line kernels: U = x V^T (every row of x
// through V), its transpose V x^T, and every row of that again:
// V x^T V^T = xi^T.
template <typename T>
int idwt2d_tensor(const wh2wav_plan_s* p, const T* x, T* out, T* W, hipStream_t st) {
  const auto& H = p->host;
  if (tensor_lines(p)) {
    const auto ft = fast_tables_of<T>(p);
    const int64_t M = H.M;
    HIP_OK(wh2wav_fast::lines_levels<T>(x, W, M, 1, M, 1, H.j0, H.j, 0, ft, st));
    HIP_OK(wh2wav_fast::transpose<T>(W, out, M, st));
    HIP_OK(wh2wav_fast::lines_levels<T>(out, out, M, 1, M, 1, H.j0, H.j, 0, ft, st));
    return WH2WAV_OK;
  }
  int rc = launch_transpose<T>(x, out, H.M, st);
  for (int k = H.j0; k < H.j && rc == WH2WAV_OK; ++k) rc = tensor_level<T>(p, out, W, true, k, false, st);
  for (int k = H.j0; k < H.j && rc == WH2WAV_OK; ++k) rc = tensor_level<T>(p, out, W, false, k, false, st);
  return rc;
}

// Its transpose: xi'^T (in, overwritten) -> x; W scratch.  With the line
// kernels: every row of xi'^T through the 1D analysis V^T (xi'^T V), the
// transpose V^T xi', and every row again: V^T xi' V = x.
template <typename T>
int dwt2d_tensor(const wh2wav_plan_s* p, T* in, T* x, T* W, hipStream_t st) {
  const auto& H = p->host;
  if (tensor_lines(p)) {
    const auto ft = fast_tables_of<T>(p);
    const int64_t M = H.M;
    HIP_OK(wh2wav_fast::lines_levels<T>(in, in, M, 1, M, 1, H.j0, H.j, 1, ft, st));
    HIP_OK(wh2wav_fast::transpose<T>(in, W, M, st));
    HIP_OK(wh2wav_fast::lines_levels<T>(W, x, M, 1, M, 1, H.j0, H.j, 1, ft, st));
    return WH2WAV_OK;
  }
  int rc = WH2WAV_OK;
  for (int k = H.j - 1; k >= H.j0 && rc == WH2WAV_OK; --k) rc = tensor_level<T>(p, in, W, false, k, true, st);
  for (int k = H.j - 1; k >= H.j0 && rc == WH2WAV_OK; --k) rc = tensor_level<T>(p, in, W, true, k, true, st);
  if (rc == WH2WAV_OK) rc = launch_transpose<T>(in, x, H.M, st);
  return rc;
}

// ------------------------------------------- three dimensions, unequal sides
// The per-axis path (Sec. 5: the d-fold inner products split into 1D ones).
// x (M_0 x M_1 [x M_2], row-major) -> wavelet levels -> xi; G along axis 0
// (Z0: N_0 x M_1 [x M_2]), along axis 1 in 3D (Z1: N_0 x N_1 x M_2), and
// along the last axis with the gather onto Omega, each axis with its own
// tables.  Workspace: XA, XB (M_0 M_1 M_2 each), Z0, Z1.

// Wavelet levels in the order the inverse DWT applies them: (axis, level).
// Tensor basis: every level of axis 0, then of axis 1, ...  Isotropic: per
// level, every axis within the cube [0, 2^{k+1})^d.
std::vector<std::pair<int, int>> nd_levels(const wh2wav::HostPlan& H) {
  std::vector<std::pair<int, int>> out;
  if (H.tensor) {
    for (int a = 0; a < H.dim; ++a)
      for (int k = H.j0; k < H.ja[a]; ++k) out.emplace_back(a, k);
  } else {
    for (int k = H.j0; k < H.j; ++k)
      for (int a = 0; a < H.dim; ++a) out.emplace_back(a, k);
  }
  return out;
}

struct NdBuffers {
  size_t xa, xb, z0, z1;  // offsets in elements
  size_t total;
};
NdBuffers nd_buffers(const wh2wav::HostPlan& H) {
  const size_t mtot = size_t(H.Ma[0] * H.Ma[1] * H.Ma[2]);
  const size_t z0 = size_t(H.Na[0] * H.Ma[1] * H.Ma[2]);
  const size_t z1 = H.dim == 3 ? size_t(H.Na[0] * H.Na[1] * H.Ma[2]) : 0;
  return NdBuffers{0, mtot, 2 * mtot, 2 * mtot + z0, 2 * mtot + z0 + z1};
}

template <typename T>
int nd_level(const wh2wav_plan_s* p, const T* in, T* out, int axis, int k, bool analysis, hipStream_t st) {
  const auto& H = p->host;
  const int64_t total = H.Ma[0] * H.Ma[1] * H.Ma[2];
  hipLaunchKernelGGL(k_level_nd<T>, dim3(unsigned((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, in,
                     out, H.Ma[0], H.Ma[1], H.Ma[2], axis, k, H.tensor ? 0 : 1, analysis ? 1 : 0, tables_of<T>(p));
  HIP_OK(hipGetLastError());
  return WH2WAV_OK;
}

// Tensor basis on the per-axis path: every level of an axis in one launch of
// the LDS line kernels (lines along the axis, values strided by the product
// of the later extents), when every axis's lines fit.
bool nd_tensor_lines(const wh2wav_plan_s* p) {
  const auto& H = p->host;
  if (!H.nd || !H.tensor) return false;
  for (int a = 0; a < H.dim; ++a)
    if (!wh2wav_fast::lines_levels_fit(H.dtype == WH2WAV_F64 ? 8 : 4, H.ja[a])) return false;
  return true;
}

// All levels along axis a of the M_0 x M_1 x M_2 array (synthesis, or the
// analysis with `analysis`), src -> dst (the same array allowed).
template <typename T>
int nd_axis_levels(const wh2wav_plan_s* p, const T* src, T* dst, int a, bool analysis, hipStream_t st) {
  const auto& H = p->host;
  int64_t es = 1;
  for (int b = a + 1; b < 3; ++b) es *= H.Ma[b];
  const int64_t lines = H.Ma[0] * H.Ma[1] * H.Ma[2] / H.Ma[a];
  HIP_OK(wh2wav_fast::lines_levels<T>(src, dst, lines, es, H.Ma[a] * es, es, H.j0, H.ja[a], analysis ? 1 : 0,
                                      fast_tables_of<T>(p), st));
  return WH2WAV_OK;
}

// One launch of the line kernels on the per-axis path: G (fwd) or G^T along
// axis `a`, `lines` lines.
template <typename T>
int nd_pass(const wh2wav_plan_s* p, bool fwd, int a, int64_t lines, const T* in, LineMap im, T* out, LineMap om_,
            int omega_side, RowMap rm, hipStream_t st) {
  return launch_lines<T>(p, fwd, lines, p->host.ja[a], in, im, out, om_, omega_side, rm, axis_tables_of<T>(p, a), st);
}

// Forward stages: 0 = inverse DWT into XA, 1 = G along every axis but the
// last, 2 = G along the last axis with the gather.
template <typename T>
int forward_nd(const wh2wav_plan_s* p, const T* x, T* y, void* ws, hipStream_t st, int stage) {
  const auto& H = p->host;
  auto run = [&](int s) { return stage < 0 || stage == s; };
  if (H.m == 0) return WH2WAV_OK;
  const NdBuffers b = nd_buffers(H);
  T* W = static_cast<T*>(ws);
  T *XA = W + b.xa, *XB = W + b.xb, *Z0 = W + b.z0, *Z1 = W + b.z1;
  const int64_t M0 = H.Ma[0], M1 = H.Ma[1], M2 = H.Ma[2], N0 = H.Na[0], N1 = H.Na[1];
  if (run(0) && nd_tensor_lines(p)) {  // axis by axis, x -> XA, then in place
    const T* src = x;
    for (int a = 0; a < H.dim; ++a) {
      int rc = nd_axis_levels<T>(p, src, XA, a, false, st);
      if (rc) return rc;
      src = XA;
    }
  } else if (run(0)) {
    const auto levels = nd_levels(H);
    if (levels.empty()) HIP_OK(hipMemcpyAsync(XA, x, sizeof(T) * size_t(M0 * M1 * M2), hipMemcpyDeviceToDevice, st));
    const T* src = x;
    for (size_t i = 0; i < levels.size(); ++i) {  // the last level writes XA
      T* dst = (levels.size() - 1 - i) % 2 == 0 ? XA : XB;
      int rc = nd_level<T>(p, src, dst, levels[i].first, levels[i].second, false, st);
      if (rc) return rc;
      src = dst;
    }
  }
  const RowMap none{0, 0, 0};
  int rc = WH2WAV_OK;
  if (H.dim == 2) {  // Z0 transposed (M1 x N0): whole rows written, strided reads
    if (run(1)) rc = nd_pass<T>(p, true, 0, M1, XA, lines_at(1, M1), Z0, lines_at(N0, 1), 0, none, st);
    if (rc == WH2WAV_OK && run(2))
      rc = nd_pass<T>(p, true, 1, N0, Z0, lines_at(1, N0), y, lines_at(0, 0), 1, RowMap{1, H.ja[0], 0}, st);
    return rc;
  }
  if (run(1)) {
    rc = nd_pass<T>(p, true, 0, M1 * M2, XA, lines_at(1, M1 * M2), Z0, lines_at(1, M1 * M2), 0, none, st);
    if (rc == WH2WAV_OK)
      rc = nd_pass<T>(p, true, 1, N0 * M2, Z0, LineMap{M2, M1 * M2, 1, M2}, Z1, LineMap{M2, N1 * M2, 1, M2}, 0, none,
                      st);
  }
  if (rc == WH2WAV_OK && run(2))
    rc = nd_pass<T>(p, true, 2, N0 * N1, Z1, lines_at(M2, 1), y, lines_at(0, 0), 1, RowMap{2, H.ja[0], H.ja[1]},
                    st);
  return rc;
}

// Adjoint stages: 0 = G^T along the last axis with the scatter, 1 = G^T
// along the other axes (into XA), 2 = forward DWT into x.
template <typename T>
int adjoint_nd(const wh2wav_plan_s* p, const T* y, T* x, void* ws, hipStream_t st, int stage) {
  const auto& H = p->host;
  auto run = [&](int s) { return stage < 0 || stage == s; };
  const int64_t M0 = H.Ma[0], M1 = H.Ma[1], M2 = H.Ma[2], N0 = H.Na[0], N1 = H.Na[1];
  if (H.m == 0) {
    if (run(2)) {
      launch_fill<T>(x, M0 * M1 * M2, st);
      HIP_OK(hipGetLastError());
    }
    return WH2WAV_OK;
  }
  const NdBuffers b = nd_buffers(H);
  T* W = static_cast<T*>(ws);
  T *XA = W + b.xa, *XB = W + b.xb, *Z0 = W + b.z0, *Z1 = W + b.z1;
  const RowMap none{0, 0, 0};
  int rc = WH2WAV_OK;
  if (H.dim == 2) {
    if (run(0))
      rc = nd_pass<T>(p, false, 1, N0, y, lines_at(0, 0), Z0, lines_at(M1, 1), 1, RowMap{1, H.ja[0], 0}, st);
    if (rc == WH2WAV_OK && run(1))
      rc = nd_pass<T>(p, false, 0, M1, Z0, lines_at(1, M1), XA, lines_at(1, M1), 0, none, st);
  } else {
    if (run(0))
      rc = nd_pass<T>(p, false, 2, N0 * N1, y, lines_at(0, 0), Z1, lines_at(M2, 1), 1, RowMap{2, H.ja[0], H.ja[1]},
                      st);
    if (rc == WH2WAV_OK && run(1)) {
      rc = nd_pass<T>(p, false, 1, N0 * M2, Z1, LineMap{M2, N1 * M2, 1, M2}, Z0, LineMap{M2, M1 * M2, 1, M2}, 0,
                      none, st);
      if (rc == WH2WAV_OK)
        rc = nd_pass<T>(p, false, 0, M1 * M2, Z0, lines_at(1, M1 * M2), XA, lines_at(1, M1 * M2), 0, none, st);
    }
  }
  if (rc || !run(2)) return rc;
  if (nd_tensor_lines(p)) {  // axis by axis in reverse order, in place on XA; the last writes x
    for (int a = H.dim - 1; a >= 0; --a) {
      rc = nd_axis_levels<T>(p, XA, a == 0 ? x : XA, a, true, st);
      if (rc) return rc;
    }
    return WH2WAV_OK;
  }
  auto levels = nd_levels(H);
  if (levels.empty()) {
    HIP_OK(hipMemcpyAsync(x, XA, sizeof(T) * size_t(M0 * M1 * M2), hipMemcpyDeviceToDevice, st));
    return WH2WAV_OK;
  }
  const T* src = XA;
  for (size_t i = 0; i < levels.size(); ++i) {  // the transposes in reverse order; the last writes x
    const auto& lv = levels[levels.size() - 1 - i];
    T* dst = i + 1 == levels.size() ? x : (i % 2 == 0 ? XB : XA);
    rc = nd_level<T>(p, src, dst, lv.first, lv.second, true, st);
    if (rc) return rc;
    src = dst;
  }
  return WH2WAV_OK;
}

// Forward stages: 0 = inverse DWT, 1 = column pass (2D) / line transform (1D),
// 2 = row pass with the Omega gather (2D).  stage < 0 runs all of them.
template <typename T>
int forward_impl(const wh2wav_plan_s* p, const T* x, T* y, void* ws, hipStream_t st, int stage) {
  const auto& H = p->host;
  const int64_t M = H.M, N = H.N;
  const Tables<T> t = tables_of<T>(p);
  if (H.nd) return forward_nd<T>(p, x, y, ws, st, stage);
  if (H.m == 0) return WH2WAV_OK;
  T* W = static_cast<T*>(ws);
  auto run = [&](int s) { return stage < 0 || stage == s; };
  if (H.dim == 1 && use_fast1d(p)) {
    T* S0 = W + M;
    T* L = S0 + M;
    const auto ft = fast_tables_of<T>(p);
    if (stage < 0 && use_line1d_fused(p)) {
      HIP_OK(wh2wav_fast::line1d_fwd_fused<T>(x, y, H.j0, H.j, ft, fast_omega_of(p), st));
      return WH2WAV_OK;
    }
    if (run(0)) HIP_OK(wh2wav_fast::idwt1d<T>(x, W, S0, H.j0, H.j, ft, st));
    if (use_wave1d(p)) {
      if (run(1)) HIP_OK(wh2wav_fast::rowpass_fwd<T>(W, y, H.j, ft, fast_omega_of(p), 1, st));
    } else if (run(1)) {
      HIP_OK(wh2wav_fast::line1d_fwd<T>(W, L, y, H.j, ft, p->d_pos32, H.m, H.full_omega ? 1 : 0, st));
    }
    return WH2WAV_OK;
  }
  if (H.dim == 1) {
    T* TMP = W + M;
    const bool one_launch = wh2wav_fast::lines_levels_fit(H.dtype == WH2WAV_F64 ? 8 : 4, H.j);
    if (run(0) && one_launch) {  // every level of the line in one workgroup
      HIP_OK(wh2wav_fast::lines_levels<T>(x, W, 1, 1, M, 1, H.j0, H.j, 0, fast_tables_of<T>(p), st));
    } else if (run(0)) {
      HIP_OK(hipMemcpyAsync(W, x, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
      for (int k = H.j0; k < H.j; ++k) {
        int rc = launch_synth<T>(p, W, TMP, 1, 0, 1, k, false, false, st);
        if (rc) return rc;
        HIP_OK(hipMemcpyAsync(W, TMP, sizeof(T) * (size_t(2) << k), hipMemcpyDeviceToDevice, st));
      }
    }
    if (run(1)) {
      int rc = launch_lines<T>(p, true, 1, H.j, W, lines_at(0, 1), y, lines_at(0, 0), 1, RowMap{0, 0, 0}, t, st);
      if (rc) return rc;
    }
    return WH2WAV_OK;
  }
  T* TMP = W + M * M;
  T* Z = TMP + M * M;
  const bool fast = use_fast(p);
  if (run(0) && H.tensor) {  // xi^T into TMP; W serves as scratch
    int rc = idwt2d_tensor<T>(p, x, TMP, W, st);
    if (rc) return rc;
  } else if (run(0)) {  // xi^T into TMP (tiled 2D wavelet kernels, every shape, boundary or periodic); W and Z serve as scratch
    HIP_OK(wh2wav_fast::idwt2d<T>(x, TMP, W, Z, M, H.j0, H.j, fast_tables_of<T>(p), st));
  }
  if (fast) {
    if (run(1)) HIP_OK(wh2wav_fast::colpass_fwd<T>(TMP, Z, H.j, fast_tables_of<T>(p), st));
    if (run(2)) HIP_OK(wh2wav_fast::rowpass_fwd<T>(Z, y, H.j, fast_tables_of<T>(p), fast_omega_of(p), N, st));
    return WH2WAV_OK;
  }
  int rc = WH2WAV_OK;
  // Z is kept transposed here (Z^T[m2, r], M x N): the column pass writes
  // whole rows and the row pass reads with stride N -- strided reads share
  // cache lines in L2, strided writes leave partly written lines to HBM.
  if (run(1))  // column pass: G along the first index (rows of xi^T); Z^T[m2, r] with r natural
    rc = launch_lines<T>(p, true, M, H.j, TMP, lines_at(M, 1), Z, lines_at(N, 1), 0, RowMap{0, 0, 0}, t, st);
  if (rc == WH2WAV_OK && run(2))  // row pass: G along the second index (columns of Z^T), gather Omega
    rc = launch_lines<T>(p, true, N, H.j, Z, lines_at(1, N), y, lines_at(0, 0), 1, RowMap{1, H.j, 0}, t, st);
  return rc;
}

// Adjoint stages: 0 = row pass with the Omega scatter (2D) / line transform
// (1D), 1 = column pass (2D), 2 = forward DWT.  stage < 0 runs all of them.
template <typename T>
int adjoint_impl(const wh2wav_plan_s* p, const T* y, T* x, void* ws, hipStream_t st, int stage) {
  const auto& H = p->host;
  const int64_t M = H.M, N = H.N;
  const Tables<T> t = tables_of<T>(p);
  if (H.nd) return adjoint_nd<T>(p, y, x, ws, st, stage);
  T* W = static_cast<T*>(ws);
  auto run = [&](int s) { return stage < 0 || stage == s; };
  const int64_t xlen = H.dim == 1 ? M : M * M;
  if (H.m == 0) {
    if (run(2)) {
      launch_fill<T>(x, xlen, st);
      HIP_OK(hipGetLastError());
    }
    return WH2WAV_OK;
  }
  if (H.dim == 1 && use_fast1d(p)) {
    T* S0 = W + M;
    T* L = S0 + M;
    const auto ft = fast_tables_of<T>(p);
    if (stage < 0 && use_line1d_fused(p)) {
      HIP_OK(wh2wav_fast::line1d_adj_fused<T>(y, x, H.j0, H.j, ft, fast_omega_of(p), st));
      return WH2WAV_OK;
    }
    if (use_wave1d(p)) {
      if (run(0)) HIP_OK(wh2wav_fast::rowpass_adj<T>(y, W, H.j, ft, fast_omega_of(p), 1, st));
    } else if (run(0)) {
      HIP_OK(wh2wav_fast::line1d_adj<T>(y, L, W, H.j, ft, p->d_pos32, H.m, H.full_omega ? 1 : 0, st));
    }
    if (run(2)) HIP_OK(wh2wav_fast::dwt1d<T>(W, x, S0, H.j0, H.j, ft, st));
    return WH2WAV_OK;
  }
  if (H.dim == 1) {
    T* TMP = W + M;
    if (run(0)) {
      int rc = launch_lines<T>(p, false, 1, H.j, y, lines_at(0, 0), W, lines_at(0, 1), 1, RowMap{0, 0, 0}, t, st);
      if (rc) return rc;
    }
    const bool one_launch = wh2wav_fast::lines_levels_fit(H.dtype == WH2WAV_F64 ? 8 : 4, H.j);
    if (run(2) && one_launch) {
      HIP_OK(wh2wav_fast::lines_levels<T>(W, x, 1, 1, M, 1, H.j0, H.j, 1, fast_tables_of<T>(p), st));
    } else if (run(2)) {
      for (int k = H.j - 1; k >= H.j0; --k) {
        int rc = launch_synth<T>(p, W, TMP, 1, 0, 1, k, false, true, st);
        if (rc) return rc;
        HIP_OK(hipMemcpyAsync(W, TMP, sizeof(T) * (size_t(2) << k), hipMemcpyDeviceToDevice, st));
      }
      HIP_OK(hipMemcpyAsync(x, W, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    }
    return WH2WAV_OK;
  }
  T* TMP = W + M * M;
  T* Z = TMP + M * M;
  if (use_fast(p)) {
    if (run(0)) HIP_OK(wh2wav_fast::rowpass_adj<T>(y, Z, H.j, fast_tables_of<T>(p), fast_omega_of(p), N, st));
    if (run(1)) HIP_OK(wh2wav_fast::colpass_adj<T>(Z, TMP, H.j, fast_tables_of<T>(p), st));
    if (run(2) && H.tensor) return dwt2d_tensor<T>(p, TMP, x, W, st);
    if (run(2)) HIP_OK(wh2wav_fast::dwt2d<T>(TMP, x, W, Z, M, H.j0, H.j, fast_tables_of<T>(p), st));
    return WH2WAV_OK;
  }
  int rc = WH2WAV_OK;
  if (run(0))
    rc = launch_lines<T>(p, false, N, H.j, y, lines_at(0, 0), Z, lines_at(M, 1), 1, RowMap{1, H.j, 0}, t, st);
  if (rc == WH2WAV_OK && run(1))  // column pass, transposed: xi'^T into TMP
    rc = launch_lines<T>(p, false, M, H.j, Z, lines_at(1, M), TMP, lines_at(M, 1), 0, RowMap{0, 0, 0}, t, st);
  if (rc) return rc;
  if (run(2) && H.tensor) return dwt2d_tensor<T>(p, TMP, x, W, st);
  if (run(2)) HIP_OK(wh2wav_fast::dwt2d<T>(TMP, x, W, Z, M, H.j0, H.j, fast_tables_of<T>(p), st));
  return WH2WAV_OK;
}

template <typename T>
int upload_tables(wh2wav_plan_s* p) {
  const auto& H = p->host;
  std::vector<T> all;
  auto put = [&](const std::vector<double>& v, size_t* off) {
    *off = all.size();
    for (double d : v) all.push_back(T(d));
  };
  put(H.h, &p->off_h);
  put(H.g, &p->off_g);
  put(H.tabT, &p->off_T);
  put(H.tabBL, &p->off_BL);
  put(H.tabBR, &p->off_BR);
  put(H.synL, &p->off_SL);
  put(H.synR, &p->off_SR);
  // bands in the layouts of the wave kernels (index maps in fast2d.h)
  const int nu = H.nu, B = 2 * nu - 1, Q = H.Q;
  std::vector<double> lf(H.tabBL.size()), rf(lf.size()), la(lf.size()), ra(lf.size());
  for (int pp = 0; pp < B; ++pp)
    for (int m = 0; m < nu; ++m)
      for (int s = 0; s < Q; ++s) {
        const size_t src = (size_t(pp) * nu + m) * Q + s;
        lf[(size_t(s) * B + pp) * nu + m] = H.tabBL[src], rf[(size_t(s) * B + pp) * nu + m] = H.tabBR[src];
        la[(size_t(s) * nu + m) * B + pp] = H.tabBL[src], ra[(size_t(s) * nu + m) * B + pp] = H.tabBR[src];
      }
  put(lf, &p->off_BLf);
  put(rf, &p->off_BRf);
  put(la, &p->off_BLa);
  put(ra, &p->off_BRa);
  for (int a = 0; H.nd && a < H.dim; ++a) {
    put(H.tabT_ax[a], &p->off_T_ax[a]);
    put(H.tabBL_ax[a], &p->off_BL_ax[a]);
    put(H.tabBR_ax[a], &p->off_BR_ax[a]);
  }
  HIP_OK(hipMalloc(&p->d_tables, sizeof(T) * all.size()));
  HIP_OK(hipMemcpy(p->d_tables, all.data(), sizeof(T) * all.size(), hipMemcpyHostToDevice));
  return WH2WAV_OK;
}

void release(wh2wav_plan_s* p) {
  if (!p) return;
  if (p->d_tables) (void)hipFree(p->d_tables);
  if (p->d_mask) (void)hipFree(p->d_mask);
  if (p->d_pos16) (void)hipFree(p->d_pos16);
  if (p->d_pos32) (void)hipFree(p->d_pos32);
  if (p->d_seg_ptr) (void)hipFree(p->d_seg_ptr);
  if (p->d_row_ptr) (void)hipFree(p->d_row_ptr);
  delete p;
}

}  // namespace

namespace {
std::mutex g_handles_mu;
std::unordered_set<const void*>* g_handles = nullptr;  // never freed: outlives static destructors
}  // namespace

namespace wh2wav {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
int set_error_nothrow(int code, const char* msg) noexcept {
  try {
    g_last_error = msg;
  } catch (...) {
    g_last_error.clear();
  }
  return code;
}
void handle_add(const void* h) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  if (!g_handles) g_handles = new std::unordered_set<const void*>();
  g_handles->insert(h);
}
bool handle_remove(const void* h) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  return g_handles && g_handles->erase(h) == 1;
}
bool handle_live(const void* h) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  return g_handles && g_handles->count(h) == 1;
}
PlanShape plan_shape(wh2wav_plan_t p) {
  const auto& H = p->host;
  int64_t xlen = H.dim == 1 ? H.M : H.M * H.M, ntot = H.dim == 1 ? H.N : H.N * H.N;
  if (H.nd) {
    xlen = H.Ma[0] * H.Ma[1] * H.Ma[2];
    ntot = H.Na[0] * H.Na[1] * H.Na[2];
  }
  return PlanShape{H.dim, H.j, H.q, H.nu, H.dtype, H.M, H.N, H.m, xlen, ntot};
}
PlanView plan_view(wh2wav_plan_t p) {
  const auto& H = p->host;
  const size_t e = H.dtype == WH2WAV_F64 ? 8 : 4;
  const char* base = static_cast<const char*>(p->d_tables);
  PlanView v;
  v.h = base + e * p->off_h, v.g = base + e * p->off_g, v.tabT = base + e * p->off_T;
  v.bandL = base + e * p->off_BL, v.bandR = base + e * p->off_BR, v.synL = base + e * p->off_SL;
  v.synR = base + e * p->off_SR;
  v.nu = H.nu, v.q = H.q, v.Q = H.Q, v.per = H.per ? 1 : 0, v.dim = H.dim, v.j = H.j, v.j0 = H.j0;
  v.tensor = H.tensor ? 1 : 0, v.nd = H.nd ? 1 : 0, v.dtype = H.dtype, v.full_omega = H.full_omega ? 1 : 0;
  v.M = H.M, v.N = H.N, v.m = H.m;
  v.mask = p->d_mask, v.row_ptr = p->d_row_ptr, v.wpr = H.words_per_row;
  return v;
}
}  // namespace wh2wav

namespace {

int plan_body(const wh2wav_desc* desc, wh2wav_plan_t* out) {
  g_last_error.clear();
  if (!out) return fail(WH2WAV_EINVAL, "out is NULL");
  *out = nullptr;
  // owned by `hold` until it is handed out; release() frees whatever was uploaded
  std::unique_ptr<wh2wav_plan_s, void (*)(wh2wav_plan_s*)> hold(new wh2wav_plan_s(), release);
  wh2wav_plan_s* p = hold.get();
  std::string err;
  int rc = wh2wav::build_host_plan(desc, &p->host, &err);
  if (rc != WH2WAV_OK) return fail(rc, err);
  HIP_OK(hipGetDevice(&p->device));
  const auto& H = p->host;
  if (H.j < 1) return fail(WH2WAV_EUNSUPPORTED, "j must be >= 1");
  const size_t elem = H.dtype == WH2WAV_F64 ? 8 : 4;
  int64_t Mline = H.M;  // longest line of the LDS line kernels
  for (int a = 0; H.nd && a < H.dim; ++a) Mline = std::max(Mline, H.Ma[a]);
  if (!use_fast(p) && !use_fast1d(p) &&
      2 * size_t(Mline) * elem + sizeof(int) * (2 * size_t(H.words_per_row) + kThreads) > kMaxLds)
    return fail(WH2WAV_EUNSUPPORTED, "M too large for the LDS line kernels");
  rc = H.dtype == WH2WAV_F64 ? prepare_line_kernels<double>() : prepare_line_kernels<float>();
  if (rc != WH2WAV_OK) return rc;
  if (H.dim == 2) {
    hipError_t e = H.dtype == WH2WAV_F64 ? wh2wav_fast::prepare_dwt2d<double>(H.nu)
                                         : wh2wav_fast::prepare_dwt2d<float>(H.nu);
    if (e == hipSuccess && use_fast(p))
      e = H.dtype == WH2WAV_F64 ? wh2wav_fast::prepare_lines<double>(H.j, H.nu)
                                : wh2wav_fast::prepare_lines<float>(H.j, H.nu);
    if (e == hipSuccess && tensor_lines(p))
      e = H.dtype == WH2WAV_F64 ? wh2wav_fast::prepare_1d<double>(H.nu) : wh2wav_fast::prepare_1d<float>(H.nu);
    if (e != hipSuccess) return fail(WH2WAV_EHIP, std::string("kernel setup: ") + hipGetErrorString(e));
  }
  if (nd_tensor_lines(p) || (H.dim == 1 && !use_fast1d(p))) {
    hipError_t e = H.dtype == WH2WAV_F64 ? wh2wav_fast::prepare_1d<double>(H.nu) : wh2wav_fast::prepare_1d<float>(H.nu);
    if (e != hipSuccess) return fail(WH2WAV_EHIP, std::string("kernel setup: ") + hipGetErrorString(e));
  }
  if (use_fast1d(p)) {
    hipError_t e = H.dtype == WH2WAV_F64 ? wh2wav_fast::prepare_1d<double>(H.nu)
                                         : wh2wav_fast::prepare_1d<float>(H.nu);
    if (e == hipSuccess && use_wave1d(p))
      e = H.dtype == WH2WAV_F64 ? wh2wav_fast::prepare_lines<double>(H.j, H.nu)
                                : wh2wav_fast::prepare_lines<float>(H.j, H.nu);
    if (e != hipSuccess) return fail(WH2WAV_EHIP, std::string("kernel setup: ") + hipGetErrorString(e));
  }
  rc = H.dtype == WH2WAV_F64 ? upload_tables<double>(p) : upload_tables<float>(p);
  if (rc != WH2WAV_OK) return rc;
  auto upload = [&](void** dst, const void* src, size_t bytes) -> int {
    if (bytes == 0) return WH2WAV_OK;
    HIP_OK(hipMalloc(dst, bytes));
    HIP_OK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return WH2WAV_OK;
  };
  rc = upload((void**)&p->d_row_ptr, H.row_ptr.data(), sizeof(int64_t) * H.row_ptr.size());
  if (rc == WH2WAV_OK) rc = upload((void**)&p->d_mask, H.mask.data(), sizeof(uint32_t) * H.mask.size());
  if (rc == WH2WAV_OK) rc = upload((void**)&p->d_pos16, H.pos16.data(), sizeof(uint16_t) * H.pos16.size());
  if (rc == WH2WAV_OK) rc = upload((void**)&p->d_seg_ptr, H.seg_ptr.data(), sizeof(int64_t) * H.seg_ptr.size());
  if (rc == WH2WAV_OK) rc = upload((void**)&p->d_pos32, H.pos32.data(), sizeof(int32_t) * H.pos32.size());
  if (rc != WH2WAV_OK) return rc;
  wh2wav::handle_add(p);
  *out = hold.release();
  return WH2WAV_OK;
}

}  // namespace

extern "C" {

const char* wh2wav_last_error(void) { return g_last_error.c_str(); }

int wh2wav_plan(const wh2wav_desc* desc, wh2wav_plan_t* out) {
  return wh2wav::guarded([&] { return plan_body(desc, out); });
}

int wh2wav_workspace_size(wh2wav_plan_t p, size_t* bytes) {
  if (!p || !bytes) return fail(WH2WAV_EINVAL, "NULL argument");
  if (!wh2wav::handle_live(p)) return fail(WH2WAV_EINVAL, "not a live plan (destroyed, or never created)");
  const auto& H = p->host;
  const size_t elem = H.dtype == WH2WAV_F64 ? 8 : 4;
  if (H.nd)
    *bytes = nd_buffers(H).total * elem;
  else if (H.dim == 1)
    *bytes = (2 + size_t(H.Q)) * size_t(H.M) * elem;
  else
    *bytes = (2 * size_t(H.M) * size_t(H.M) + size_t(H.N) * size_t(H.M)) * elem;
  return WH2WAV_OK;
}

static int check_call(wh2wav_plan_t p, const void* a, const void* b, void* ws) {
  if (!p) return fail(WH2WAV_EINVAL, "plan is NULL");
  if (!wh2wav::handle_live(p)) return fail(WH2WAV_EINVAL, "not a live plan (destroyed, or never created)");
  const auto& H = p->host;
  const size_t elem = H.dtype == WH2WAV_F64 ? 8 : 4;
  const int64_t xlen = H.nd ? H.Ma[0] * H.Ma[1] * H.Ma[2] : (H.dim == 1 ? H.M : H.M * H.M);
  const size_t in_out[2] = {size_t(xlen) * elem, size_t(H.m) * elem};
  if (!ws) return fail(WH2WAV_EINVAL, "workspace is NULL");
  if ((!a && in_out[0]) || (!b && in_out[1])) return fail(WH2WAV_EINVAL, "x or y is NULL");
  auto overlap = [](const void* p1, size_t n1, const void* p2, size_t n2) {
    if (!p1 || !p2 || !n1 || !n2) return false;
    auto a1 = reinterpret_cast<uintptr_t>(p1), a2 = reinterpret_cast<uintptr_t>(p2);
    return a1 < a2 + n2 && a2 < a1 + n1;
  };
  size_t wsb = 0;
  wh2wav_workspace_size(p, &wsb);
  if (overlap(a, in_out[0], b, in_out[1]) || overlap(a, in_out[0], ws, wsb) || overlap(b, in_out[1], ws, wsb))
    return fail(WH2WAV_EINVAL, "x, y and workspace must not overlap");
  return WH2WAV_OK;
}

static int forward_any(wh2wav_plan_t p, const void* x, void* y, void* ws, void* stream, int stage) {
  return wh2wav::guarded([&] {
    g_last_error.clear();
    int rc = check_call(p, x, y, ws);
    if (rc) return rc;
    auto st = static_cast<hipStream_t>(stream);
    return p->host.dtype == WH2WAV_F64
               ? forward_impl<double>(p, static_cast<const double*>(x), static_cast<double*>(y), ws, st, stage)
               : forward_impl<float>(p, static_cast<const float*>(x), static_cast<float*>(y), ws, st, stage);
  });
}

static int adjoint_any(wh2wav_plan_t p, const void* y, void* x, void* ws, void* stream, int stage) {
  return wh2wav::guarded([&] {
    g_last_error.clear();
    int rc = check_call(p, x, y, ws);
    if (rc) return rc;
    auto st = static_cast<hipStream_t>(stream);
    return p->host.dtype == WH2WAV_F64
               ? adjoint_impl<double>(p, static_cast<const double*>(y), static_cast<double*>(x), ws, st, stage)
               : adjoint_impl<float>(p, static_cast<const float*>(y), static_cast<float*>(x), ws, st, stage);
  });
}

int wh2wav_forward(wh2wav_plan_t p, const void* x, void* y, void* ws, void* stream) {
  return forward_any(p, x, y, ws, stream, -1);
}

int wh2wav_adjoint(wh2wav_plan_t p, const void* y, void* x, void* ws, void* stream) {
  return adjoint_any(p, y, x, ws, stream, -1);
}

int wh2wav_stage_count(wh2wav_plan_t p, int direction, int* count) {
  if (!p || !count || (direction != 0 && direction != 1)) return fail(WH2WAV_EINVAL, "bad argument");
  if (!wh2wav::handle_live(p)) return fail(WH2WAV_EINVAL, "not a live plan (destroyed, or never created)");
  *count = p->host.dim == 1 ? (direction == 0 ? 2 : 3) : 3;
  return WH2WAV_OK;
}

int wh2wav_forward_stage(wh2wav_plan_t p, int stage, const void* x, void* y, void* ws, void* stream) {
  int n = 0;
  int rc = wh2wav_stage_count(p, 0, &n);
  if (rc) return rc;
  if (stage < 0 || stage >= n) return fail(WH2WAV_EINVAL, "stage out of range");
  return forward_any(p, x, y, ws, stream, stage);
}

int wh2wav_adjoint_stage(wh2wav_plan_t p, int stage, const void* y, void* x, void* ws, void* stream) {
  int n = 0;
  int rc = wh2wav_stage_count(p, 1, &n);
  if (rc) return rc;
  if (stage < 0 || stage >= n) return fail(WH2WAV_EINVAL, "stage out of range");
  if (p->host.dim == 1 && stage == 1) return WH2WAV_OK;  // 1D has no column pass
  return adjoint_any(p, y, x, ws, stream, stage);
}

int wh2wav_destroy(wh2wav_plan_t p) {
  if (!p) return WH2WAV_OK;
  if (!wh2wav::handle_remove(p)) return fail(WH2WAV_EINVAL, "not a live plan (destroyed twice, or never created)");
  release(p);
  return WH2WAV_OK;
}

}  // extern "C"

// ------------------------------------------------ entry point without allocation
// The workspace of wh2wav_forward_noalloc: a fixed array in the library's
// device code object, one copy per GPU (held until the process ends).  In host
// code `scratch` names a host-side stand-in, never the device memory: kernels
// get the address that hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(WH2WAV_NOALLOC_MAX_WORKSPACE);
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(WH2WAV_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(WH2WAV_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return WH2WAV_OK;
}

int forward_noalloc_body(wh2wav_plan_t p, const void* x, void* y, void* stream) {
  g_last_error.clear();
  if (!p) return fail(WH2WAV_EINVAL, "plan is NULL");
  if (!wh2wav::handle_live(p)) return fail(WH2WAV_EINVAL, "not a live plan (destroyed, or never created)");
  size_t need = 0;
  int rc = wh2wav_workspace_size(p, &need);
  if (rc) return rc;
  if (need > kScratchBytes)
    return fail(WH2WAV_EUNSUPPORTED, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                         std::to_string(kScratchBytes) + "-byte array of the no-allocation call");
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev != p->device) return fail(WH2WAV_EINVAL, "the plan's device must be current");
  void* ws = nullptr;
  rc = scratch_address(dev, &ws);
  if (rc) return rc;
  return forward_any(p, x, y, ws, stream, -1);
}

}  // namespace

extern "C" {

int wh2wav_forward_noalloc(wh2wav_plan_t p, const void* x, void* y, void* stream) {
  return wh2wav::guarded([&] { return forward_noalloc_body(p, x, y, stream); });
}

static int host_table_body(const wh2wav_desc* desc, int which, double* out, size_t capacity, size_t* count) {
  g_last_error.clear();
  if (!count) return fail(WH2WAV_EINVAL, "count is NULL");
  wh2wav::HostPlan H;
  std::string err;
  int rc = wh2wav::build_host_plan(desc, &H, &err);
  if (rc != WH2WAV_OK) return fail(rc, err);
  std::vector<double> tmp;
  const std::vector<double>* src = nullptr;
  switch (which) {
    case WH2WAV_TABLE_H: src = &H.h; break;
    case WH2WAV_TABLE_G: src = &H.g; break;
    case WH2WAV_TABLE_T: src = &H.tabT; break;
    case WH2WAV_TABLE_BAND_L: src = &H.tabBL; break;
    case WH2WAV_TABLE_BAND_R: src = &H.tabBR; break;
    case WH2WAV_TABLE_SYN_L: src = &H.synL; break;
    case WH2WAV_TABLE_SYN_R: src = &H.synR; break;
    case WH2WAV_TABLE_ROWPTR:
      for (int64_t v : H.row_ptr) tmp.push_back(double(v));
      src = &tmp;
      break;
    default: return fail(WH2WAV_EINVAL, "unknown table");
  }
  *count = src->size();
  if (out) std::memcpy(out, src->data(), sizeof(double) * std::min(capacity, src->size()));
  return WH2WAV_OK;
}

int wh2wav_host_table(const wh2wav_desc* desc, int which, double* out, size_t capacity, size_t* count) {
  return wh2wav::guarded([&] { return host_table_body(desc, which, out, capacity, count); });
}

}  // extern "C"
