// One-dimensional operator on gfx950 (M = 2^j, 6 <= j <= 17).
//
//   forward  x --IDWT--> xi --table product--> L[s][p] --H_M--> natural order
//            --index map, gather onto Omega--> y
//   adjoint  the transpose of each step, in reverse order.
//
// * IDWT / DWT (C_{psi,j} <-> B_{phi,j}, Sec. 3.2): levels whose line fits in
//   LDS run in one workgroup; each finer level is one launch over runs of
//   output pairs (the same one-level helpers as the 2D kernels).
// * Table product (operators D_l of Sec. 4.1 with the boundary terms of
//   Prop. 4.2): one thread per position p computes all 2^q phases from one
//   window of xi held in registers.
// * Natural-order Walsh-Hadamard transform of length M = M1 * M2 per phase,
//   H_M = H_M1 (x) H_M2: rows of M2 = min(M, 2048) contiguous values in one
//   wave each (register, DPP and swizzle stages), then columns of M1 values
//   (stride M2) in registers, one thread per column.
// * Gather / scatter: sample i of y sits at flat natural index pos[i] =
//   s M + bitrev(gray(b)) xor (s & 1) (n = s M + b, Lemma 3.2), so both are
//   coalesced over i.
// * Many lines at once (k_lines_levels): every wavelet level of one line per
//   workgroup, the lines being rows or a strided axis of an array -- the
//   wavelet stage of the tensor-product basis and of the 1D lines outside
//   the kernels above.
#include "dwt_lines.h"
#include "fast2d.h"
#include "wave_ops.h"

namespace wh2wav_fast {
namespace {

using namespace lines;
using namespace wave;

// log2 of the longest line the one-workgroup wavelet kernels keep in LDS
// (two buffers of it).
template <typename T>
constexpr int lds_line_log() {
  return sizeof(T) == 4 ? 14 : 13;
}

// ------------------------------------------------------------- wavelets
// Synthesis levels j0 .. kc-1 on the line x[0, 2^kc) in one workgroup.
template <typename T, int NU>
__global__ void __launch_bounds__(1024) k_synth1d_coarse(const T* __restrict__ x, T* __restrict__ out, int j0, int kc,
                                                         Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const TileLds<T> tl = load_tables<T, NU>(t, tab_lds, hr, gr);
  const int S = 1 << kc, tid = int(threadIdx.x);
  T* a = reinterpret_cast<T*>(smem_raw);  // [a_k | d_k | d_{k+1} ...]
  T* b = a + S;
  for (int i = tid; i < S; i += 1024) a[i] = x[i];
  __syncthreads();
  synth_levels_lds<T, NU>(a, b, j0, kc, tl, hr, gr);
  for (int i = tid; i < S; i += 1024) out[i] = a[i];
}

// Every wavelet level of `lines` lines of 2^j values, one line per
// workgroup in LDS: line r starts at (r / inner) os + r % inner and its
// values are es apart, in `in` and in `out` alike (rows of a row-major array:
// inner 1, os the row length, es 1; an axis of a d-dimensional array: inner
// and es the product of the later extents, os 2^j times that).  Synthesis
// (levels j0 .. j-1, C_{psi,j} order to the scaling coefficients at level
// j) or, with ANALYSIS, its transpose; boundary-corrected or periodic as the
// tables say.  in and out may be the same array (each workgroup reads its
// whole line before it writes).
template <typename T, int NU, bool ANALYSIS>
__global__ void __launch_bounds__(256) k_lines_levels(const T* in, T* out, int64_t inner, int64_t os, int64_t es,
                                                      int j0, int j, Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const TileLds<T> tl = load_tables<T, NU>(t, tab_lds, hr, gr);
  const int S = 1 << j, tid = int(threadIdx.x);
  T* a = reinterpret_cast<T*>(smem_raw);
  T* b = a + S;
  const int64_t r = blockIdx.x, base = (r / inner) * os + r % inner;
  for (int i = tid; i < S; i += 256) a[i] = in[base + i * es];
  __syncthreads();
  if (t.per) {
    if constexpr (ANALYSIS)
      analysis_levels_lds_per<T, NU>(a, b, j0, j, hr, gr);
    else
      synth_levels_lds_per<T, NU>(a, b, j0, j, hr, gr);
  } else {
    if constexpr (ANALYSIS)
      analysis_levels_lds<T, NU>(a, b, j0, j, tl, hr, gr);
    else
      synth_levels_lds<T, NU>(a, b, j0, j, tl, hr, gr);
  }
  for (int i = tid; i < S; i += 256) out[base + i * es] = a[i];
}

// Analysis levels kc-1 .. j0 of the line in[0, 2^kc) in one workgroup; writes
// [a_j0 | d_j0 | ... | d_{kc-1}] to x[0, 2^kc).
template <typename T, int NU>
__global__ void __launch_bounds__(1024) k_analysis1d_coarse(const T* __restrict__ in, T* __restrict__ x, int j0, int kc,
                                                            Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const TileLds<T> tl = load_tables<T, NU>(t, tab_lds, hr, gr);
  const int S = 1 << kc, tid = int(threadIdx.x);
  T* a = reinterpret_cast<T*>(smem_raw);
  T* b = a + S;
  for (int i = tid; i < S; i += 1024) a[i] = in[i];
  __syncthreads();
  analysis_levels_lds<T, NU>(a, b, j0, kc, tl, hr, gr);
  for (int i = tid; i < S; i += 1024) x[i] = a[i];
}

// One synthesis level k (2^k >= 2^13): a(m) = lo[m], d(m) = det[m], m < 2^k;
// out[0, 2^{k+1}).  One thread per run of P pairs.
template <typename T, int NU, int P>
__global__ void __launch_bounds__(256) k_synth1d_level(const T* __restrict__ lo, const T* __restrict__ det,
                                                       T* __restrict__ out, int k, Tables<T> t) {
  const int half = 1 << k;
  const int i0 = (int(blockIdx.x) * 256 + int(threadIdx.x)) * P;
  if (i0 >= half) return;
  T hr[2 * NU], gr[2 * NU];
#pragma unroll
  for (int c = 0; c < 2 * NU; ++c) hr[c] = t.h[c], gr[c] = t.g[c];
  constexpr int LO = synth_lo<NU>();
  T e[P], o[P];
  if (pair_is_interior<NU>(i0, half) && pair_is_interior<NU>(i0 + P - 1, half))
    synth_run<T, NU, P>(lo + i0 + LO, det + i0 + LO, 1, hr, gr, e, o);
  else
    synth_run_edge<T, NU, P>(lo, det, 1, 0, half - 1, i0, half, hr, gr, t.synL, t.synR, e, o);
#pragma unroll
  for (int p = 0; p < P; ++p) out[2 * (i0 + p)] = e[p], out[2 * (i0 + p) + 1] = o[p];
}

// One analysis level k: in[0, 2^{k+1}) -> lo[0, 2^k) (scaling), det[0, 2^k) (wavelets).
template <typename T, int NU, int P>
__global__ void __launch_bounds__(256) k_analysis1d_level(const T* __restrict__ in, T* __restrict__ lo,
                                                          T* __restrict__ det, int k, Tables<T> t) {
  const int half = 1 << k;
  const int m0 = (int(blockIdx.x) * 256 + int(threadIdx.x)) * P;
  if (m0 >= half) return;
  T hr[2 * NU], gr[2 * NU];
#pragma unroll
  for (int c = 0; c < 2 * NU; ++c) hr[c] = t.h[c], gr[c] = t.g[c];
  T a[P], d[P];
  if (m0 >= NU && m0 + P - 1 < half - NU)
    analysis_run<T, NU, P>(in + 2 * m0 - NU + 1, 1, hr, gr, a, d);
  else
    analysis_run_edge<T, NU, P>(in, 1, 0, 2 * half - 1, m0, half, hr, gr, t.synL, t.synR, a, d);
#pragma unroll
  for (int p = 0; p < P; ++p) lo[m0 + p] = a[p], det[m0 + p] = d[p];
}

// ------------------------------------------------------- table product
// L[s M + p] = sum_l T_l[s] xi[p - l] over interior coefficients, plus the
// boundary bands at both ends (Prop. 4.2), for every phase s.
template <typename T, int NU>
__global__ void __launch_bounds__(256) k_table1d(const T* __restrict__ xi, T* __restrict__ L, int M, Tables<T> t) {
  const int p = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (p >= M) return;
  const int Q = t.Q, band = 2 * NU - 1;
  const int right_first = M - NU > NU ? M - NU : NU;
  T w[2 * NU - 1];  // w[li] = xi[p - l], l = li - nu + 1, interior coefficients only
#pragma unroll
  for (int li = 0; li < 2 * NU - 1; ++li) {
    const int m = p - (li - NU + 1);
    const int mc = m < 0 ? 0 : (m > M - 1 ? M - 1 : m);
    const T v = xi[mc];
    w[li] = (m >= NU && m < right_first) ? v : T(0);
  }
  T el[NU], er[NU];
  const bool left = p < band, right = p >= M - band;
  if (left || right) {
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      el[m] = m < M ? xi[m < M ? m : 0] : T(0);
      const int mr = M - 1 - m;
      er[m] = mr >= right_first ? xi[mr >= 0 ? mr : 0] : T(0);
    }
  }
  for (int s = 0; s < Q; ++s) {
    T acc = T(0);
#pragma unroll
    for (int li = 0; li < 2 * NU - 1; ++li) acc = fma(w[li], t.tabT[li * Q + s], acc);
    if (left) {
#pragma unroll
      for (int m = 0; m < NU; ++m) acc = fma(el[m], t.bandL[(p * NU + m) * Q + s], acc);
    }
    if (right) {
      const int i = p - (M - band);
#pragma unroll
      for (int m = 0; m < NU; ++m) acc = fma(er[m], t.bandR[(i * NU + m) * Q + s], acc);
    }
    L[int64_t(s) * M + p] = acc;
  }
}

// Transpose: xi[m] = sum_s sum_p table(p, m, s) L[s M + p].
template <typename T, int NU>
__global__ void __launch_bounds__(256) k_table1d_t(const T* __restrict__ L, T* __restrict__ xi, int M, Tables<T> t) {
  const int m = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (m >= M) return;
  const int Q = t.Q, band = 2 * NU - 1;
  const int right_first = M - NU > NU ? M - NU : NU;
  T acc = T(0);
  if (m >= NU && m < right_first) {
    for (int s = 0; s < Q; ++s) {
      const T* Ls = L + int64_t(s) * M + m;
#pragma unroll
      for (int li = 0; li < 2 * NU - 1; ++li) acc = fma(Ls[li - NU + 1], t.tabT[li * Q + s], acc);
    }
  } else if (m < NU) {
    for (int s = 0; s < Q; ++s)
      for (int p = 0; p < band && p < M; ++p) acc = fma(L[int64_t(s) * M + p], t.bandL[(p * NU + m) * Q + s], acc);
  } else {
    const int mp = M - 1 - m;
    for (int s = 0; s < Q; ++s)
      for (int i = 0; i < band; ++i)
        acc = fma(L[int64_t(s) * M + M - band + i], t.bandR[(i * NU + mp) * Q + s], acc);
  }
  xi[m] = acc;
}

// ------------------------------------------------------------ transforms
// In-place natural-order FWHT of `rows` contiguous lines of M2 = 2^LOG values,
// one wave per line.
template <typename T, int LOG>
__global__ void __launch_bounds__(256) k_fwht_rows(T* __restrict__ L, int64_t rows) {
  constexpr int M2 = 1 << LOG, R = M2 / 64;
  const int lane = lane_id();
  const int64_t row = int64_t(blockIdx.x) * 4 + (int(threadIdx.x) >> 6);
  if (row >= rows) return;
  T v[R];
  T* base = L + row * M2 + lane * R;
  load_line<T, R>(base, v);
  fwht_wave<T, R>(v, lane);
  store_line<T, R>(base, v);
}

// In-place FWHT over the high index bits: for each phase s and column k2 <
// M2, the M1 = 2^LOG1 values L[s M + k1 M2 + k2], one thread per column.
template <typename T, int LOG1>
__global__ void __launch_bounds__(256) k_fwht_cols(T* __restrict__ L, int M2, int64_t cols) {
  constexpr int M1 = 1 << LOG1;
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= cols) return;
  const int64_t s = c / M2, k2 = c % M2;
  T* base = L + s * int64_t(M1) * M2 + k2;
  T v[M1];
#pragma unroll
  for (int i = 0; i < M1; ++i) v[i] = base[int64_t(i) * M2];
  fwht_regs<T, M1>(v);
#pragma unroll
  for (int i = 0; i < M1; ++i) base[int64_t(i) * M2] = v[i];
}

// ------------------------------------------------------ gather / scatter
template <typename T>
__global__ void __launch_bounds__(256) k_gather1d(const T* __restrict__ L, T* __restrict__ y,
                                                  const int32_t* __restrict__ pos, int64_t m) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < m) y[i] = L[pos[i]];
}
template <typename T>
__global__ void __launch_bounds__(256) k_scatter1d(const T* __restrict__ y, T* __restrict__ L,
                                                   const int32_t* __restrict__ pos, int64_t m) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < m) L[pos[i]] = y[i];
}
// Every sample taken: n = s M + b <-> natural index s M + bitrev(gray(b)) xor (s & 1).
template <typename T>
__global__ void __launch_bounds__(256) k_gather1d_full(const T* __restrict__ L, T* __restrict__ y, int j, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t M = int64_t(1) << j, s = i >> j;
  y[i] = L[s * M + natural_of(uint32_t(i & (M - 1)), uint32_t(s), j)];
}
template <typename T>
__global__ void __launch_bounds__(256) k_scatter1d_full(const T* __restrict__ y, T* __restrict__ L, int j,
                                                        int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t M = int64_t(1) << j, s = i >> j;
  L[s * M + natural_of(uint32_t(i & (M - 1)), uint32_t(s), j)] = y[i];
}
template <typename T>
__global__ void __launch_bounds__(256) k_zero1d(T* __restrict__ L, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) L[i] = T(0);
}

unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

// ------------------------------------------------------------- dispatch
template <typename T, int NU>
hipError_t idwt1d_impl(const T* x, T* xi, T* s0, int j0, int j, const Tables<T>& t, hipStream_t st) {
  const int kc = j < lds_line_log<T>() ? j : lds_line_log<T>();
  const int nfine = j - kc;
  T* cur = (nfine % 2 == 0) ? xi : s0;
  const int kc_eff = kc < j0 ? j0 : kc;  // j0 above the LDS limit: no coarse levels
  if (kc_eff > kc) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_synth1d_coarse<T, NU>), dim3(1), dim3(1024), 2 * (size_t(1) << kc) * sizeof(T), st, x, cur,
                     j0, kc, t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int P = 4;
  for (int k = kc; k < j; ++k) {
    T* nxt = cur == xi ? s0 : xi;
    const int half = 1 << k;
    hipLaunchKernelGGL((k_synth1d_level<T, NU, P>), dim3(blocks_for(half / P, 256)), dim3(256), 0, st, cur,
                       x + half, nxt, k, t);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur = nxt;
  }
  return hipSuccess;
}

template <typename T, int NU>
hipError_t dwt1d_impl(T* xi, T* x, T* s0, int j0, int j, const Tables<T>& t, hipStream_t st) {
  const int kc = j < lds_line_log<T>() ? j : lds_line_log<T>();
  if (j0 > kc) return hipErrorInvalidValue;
  constexpr int P = 4;
  T* cur = xi;
  hipError_t e = hipSuccess;
  for (int k = j - 1; k >= kc; --k) {
    T* nxt = cur == xi ? s0 : xi;
    const int half = 1 << k;
    hipLaunchKernelGGL((k_analysis1d_level<T, NU, P>), dim3(blocks_for(half / P, 256)), dim3(256), 0, st, cur, nxt,
                       x + half, k, t);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur = nxt;
  }
  hipLaunchKernelGGL((k_analysis1d_coarse<T, NU>), dim3(1), dim3(1024), 2 * (size_t(1) << kc) * sizeof(T), st, cur,
                     x, j0, kc, t);
  return hipGetLastError();
}

template <typename T>
hipError_t fwht1d(T* L, int j, int Q, hipStream_t st) {
  const int log2r = j < 11 ? j : 11, log1 = j - log2r;
  const int64_t M2 = int64_t(1) << log2r, rows = int64_t(Q) << log1;
  switch (log2r) {
#define ROWS_(LG) \
  case LG: hipLaunchKernelGGL((k_fwht_rows<T, LG>), dim3(blocks_for(rows, 4)), dim3(256), 0, st, L, rows); break;
    ROWS_(6) ROWS_(7) ROWS_(8) ROWS_(9) ROWS_(10) ROWS_(11)
#undef ROWS_
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || log1 == 0) return e;
  const int64_t cols = int64_t(Q) * M2;
  switch (log1) {
#define COLS_(LG) \
  case LG: hipLaunchKernelGGL((k_fwht_cols<T, LG>), dim3(blocks_for(cols, 256)), dim3(256), 0, st, L, int(M2), cols); break;
    COLS_(1) COLS_(2) COLS_(3) COLS_(4) COLS_(5) COLS_(6)
#undef COLS_
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int NU>
hipError_t line1d_fwd_impl(const T* xi, T* L, T* y, int j, const Tables<T>& t, const int32_t* pos, int64_t m,
                           int full, hipStream_t st) {
  const int M = 1 << j;
  hipLaunchKernelGGL((k_table1d<T, NU>), dim3(blocks_for(M, 256)), dim3(256), 0, st, xi, L, M, t);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = fwht1d<T>(L, j, t.Q, st);
  if (e != hipSuccess) return e;
  if (full)
    hipLaunchKernelGGL(k_gather1d_full<T>, dim3(blocks_for(m, 256)), dim3(256), 0, st, L, y, j, m);
  else
    hipLaunchKernelGGL(k_gather1d<T>, dim3(blocks_for(m, 256)), dim3(256), 0, st, L, y, pos, m);
  return hipGetLastError();
}

template <typename T, int NU>
hipError_t line1d_adj_impl(const T* y, T* L, T* xi, int j, const Tables<T>& t, const int32_t* pos, int64_t m,
                           int full, hipStream_t st) {
  const int M = 1 << j;
  const int64_t n = int64_t(M) * t.Q;
  if (full) {
    hipLaunchKernelGGL(k_scatter1d_full<T>, dim3(blocks_for(m, 256)), dim3(256), 0, st, y, L, j, m);
  } else {
    hipLaunchKernelGGL(k_zero1d<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, L, n);
    hipLaunchKernelGGL(k_scatter1d<T>, dim3(blocks_for(m, 256)), dim3(256), 0, st, y, L, pos, m);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = fwht1d<T>(L, j, t.Q, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_table1d_t<T, NU>), dim3(blocks_for(M, 256)), dim3(256), 0, st, L, xi, M, t);
  return hipGetLastError();
}

template <typename T, int NU>
hipError_t lines_levels_impl(const T* in, T* out, int64_t lines, int64_t inner, int64_t os, int64_t es, int j0, int j,
                             int analysis, const Tables<T>& t, hipStream_t st) {
  if (j < 1 || j > lds_line_log<T>() || j0 < 0 || j0 > j || lines < 1 || lines > (int64_t(1) << 30) || inner < 1 ||
      os < 1 || es < 1)
    return hipErrorInvalidValue;
  const size_t smem = 2 * (size_t(1) << j) * sizeof(T);
  if (analysis)
    hipLaunchKernelGGL((k_lines_levels<T, NU, true>), dim3(unsigned(lines)), dim3(256), smem, st, in, out, inner, os,
                       es, j0, j, t);
  else
    hipLaunchKernelGGL((k_lines_levels<T, NU, false>), dim3(unsigned(lines)), dim3(256), smem, st, in, out, inner, os,
                       es, j0, j, t);
  return hipGetLastError();
}

template <typename T, int NU>
hipError_t prepare1d_impl() {
  const int lim = 160 * 1024 - int(tab_lds_size<NU>() * sizeof(T));
  const void* kernels[] = {(const void*)k_synth1d_coarse<T, NU>, (const void*)k_analysis1d_coarse<T, NU>,
                           (const void*)k_lines_levels<T, NU, false>, (const void*)k_lines_levels<T, NU, true>};
  for (const void* f : kernels) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

#define WH2WAV_1D_NUS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

}  // namespace

bool supported1d(int elem_bytes, int logm, int nu, int q) {
  (void)elem_bytes;
  return logm >= 6 && logm <= 17 && nu >= 1 && nu <= 10 && q >= 1 && q <= 4;
}

template <typename T>
hipError_t idwt1d(const T* x, T* xi, T* s0, int j0, int j, const Tables<T>& t, hipStream_t st) {
#define X(V) if (t.nu == V) return idwt1d_impl<T, V>(x, xi, s0, j0, j, t, st);
  WH2WAV_1D_NUS(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t dwt1d(T* xi, T* x, T* s0, int j0, int j, const Tables<T>& t, hipStream_t st) {
#define X(V) if (t.nu == V) return dwt1d_impl<T, V>(xi, x, s0, j0, j, t, st);
  WH2WAV_1D_NUS(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t line1d_fwd(const T* xi, T* L, T* y, int j, const Tables<T>& t, const int32_t* pos, int64_t m, int full,
                      hipStream_t st) {
#define X(V) if (t.nu == V) return line1d_fwd_impl<T, V>(xi, L, y, j, t, pos, m, full, st);
  WH2WAV_1D_NUS(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t line1d_adj(const T* y, T* L, T* xi, int j, const Tables<T>& t, const int32_t* pos, int64_t m, int full,
                      hipStream_t st) {
#define X(V) if (t.nu == V) return line1d_adj_impl<T, V>(y, L, xi, j, t, pos, m, full, st);
  WH2WAV_1D_NUS(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t lines_levels(const T* in, T* out, int64_t lines, int64_t inner, int64_t os, int64_t es, int j0, int j,
                        int analysis, const Tables<T>& t, hipStream_t st) {
#define X(V) if (t.nu == V) return lines_levels_impl<T, V>(in, out, lines, inner, os, es, j0, j, analysis, t, st);
  WH2WAV_1D_NUS(X)
#undef X
  return hipErrorInvalidValue;
}
bool lines_levels_fit(int elem_bytes, int j) { return j >= 1 && j <= (elem_bytes == 4 ? 14 : 13); }
template <typename T>
hipError_t prepare_1d(int nu) {
#define X(V) if (nu == V) return prepare1d_impl<T, V>();
  WH2WAV_1D_NUS(X)
#undef X
  return hipErrorInvalidValue;
}

#define INST_(T)                                                                                                 \
  template hipError_t idwt1d<T>(const T*, T*, T*, int, int, const Tables<T>&, hipStream_t);                      \
  template hipError_t dwt1d<T>(T*, T*, T*, int, int, const Tables<T>&, hipStream_t);                             \
  template hipError_t line1d_fwd<T>(const T*, T*, T*, int, const Tables<T>&, const int32_t*, int64_t, int,         \
                                    hipStream_t);                                                                \
  template hipError_t line1d_adj<T>(const T*, T*, T*, int, const Tables<T>&, const int32_t*, int64_t, int,         \
                                    hipStream_t);                                                                \
  template hipError_t lines_levels<T>(const T*, T*, int64_t, int64_t, int64_t, int64_t, int, int, int,             \
                                      const Tables<T>&, hipStream_t);                                            \
  template hipError_t prepare_1d<T>(int);
INST_(float)
INST_(double)
#undef INST_

}  // namespace wh2wav_fast
