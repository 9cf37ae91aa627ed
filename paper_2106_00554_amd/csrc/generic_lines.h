// Generic device code of the operator: one line of the 1D section per group
// of threads (a workgroup, or a share of one for short lines), in LDS, for
// every shape; the one-level wavelet synthesis and
// analysis (boundary-corrected and periodic); the index maps.  Used by the
// plain kernels of the single-plan path and by the fused batch launches.
//
// One 1D line of the operator in the scaling basis B_{phi,j} (the matrix of
// Sec. 4, called G in Sec. 5) factors through the dyadic cells of [0, 1]:
//   1. table product  L[:, s] = (2nu-1)-tap correlation of xi with the table
//      T[l][s] (operators D_l, Sec. 4.1) plus the dense boundary bands
//      (Prop. 4.2);
//   2. one M-point Walsh-Hadamard transform per phase s (2^q of them);
//   3. index map: w_{sM+b}(p/M) = H_nat[k, p] with the natural (Sylvester)
//      index k = bitrev_j(gray(b)) xor (s & 1);
//   4. gather onto Omega (P_Omega) or scatter for the adjoint.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wh2wav_generic {

constexpr int kThreads = 256;

template <typename T>
struct Tables {
  const T* h;      // 2nu
  const T* g;      // 2nu
  const T* tabT;   // (2nu-1) * Q
  const T* bandL;  // (2nu-1) * nu * Q
  const T* bandR;  // (2nu-1) * nu * Q
  const T* synL;   // (3nu-1) * 2nu
  const T* synR;   // (3nu-1) * 2nu
  int nu, q, Q;
  int per;         // periodic extension (Sec. 3.2): lines wrap around, no boundary functions
};

struct OmegaDev {
  const uint32_t* mask;    // rows * wpr, NULL when every sample is taken
  const int64_t* row_ptr;  // rows + 1
  int64_t wpr;             // words per row
  int full;
};

__device__ __forceinline__ uint32_t bitrev_bits(uint32_t x, int bits) {
  return bits == 0 ? 0u : (__brev(x) >> (32 - bits));
}
__device__ __forceinline__ uint32_t gray_inverse(uint32_t x) {
  x ^= x >> 1;
  x ^= x >> 2;
  x ^= x >> 4;
  x ^= x >> 8;
  x ^= x >> 16;
  return x;
}
// natural position (within phase s) of the sequency index b < M = 2^j
__device__ __forceinline__ uint32_t natural_of(uint32_t b, uint32_t s, int j) {
  return bitrev_bits(b ^ (b >> 1), j) ^ (s & 1u);
}
// sequency index of natural position k of phase s
__device__ __forceinline__ uint32_t sequency_of(uint32_t k, uint32_t s, int j) {
  return gray_inverse(bitrev_bits(k ^ (s & 1u), j));
}

// ------------------------------------------------------------------ IDWT
// One level of the inverse DWT along a line: [a_k | d_k] (2^k + 2^k values,
// element stride es from src) -> output n of the scaling coefficients at
// level k+1 (2^{k+1} values).  Interior columns use the filters
// (phi_{k,m} = sum_c h_c phi_{k+1,2m+c}); boundary columns use the synthesis
// bands.
template <typename T>
__device__ T synth_value(const T* __restrict__ src, int64_t es, int64_t n, int k, const Tables<T>& t) {
  const int64_t half = int64_t(1) << k, size = 2 * half;
  const int nu = t.nu;
  auto A = [&](int64_t m) { return src[m * es]; };
  auto D = [&](int64_t m) { return src[(half + m) * es]; };
  T acc = 0;
  const int64_t right_first = half - nu > nu ? half - nu : nu;  // first right-boundary position
  int64_t mlo = (n - nu + 1) / 2;  // ceil((n - nu) / 2) for n - nu >= -1
  if (n - nu < 0) mlo = 0;
  if (mlo < nu) mlo = nu;
  int64_t mhi = (n + nu - 1) / 2;
  if (mhi > half - nu - 1) mhi = half - nu - 1;
  for (int64_t m = mlo; m <= mhi; ++m) {
    const int c = int(n - 2 * m);
    if (c < -nu + 1 || c > nu) continue;
    acc += A(m) * t.h[c + nu - 1] + D(m) * t.g[c + nu - 1];
  }
  const int rows = 3 * nu - 1;
  if (n < rows)
    for (int cc = 0; cc < nu && cc < half; ++cc)
      acc += t.synL[n * 2 * nu + cc] * A(cc) + t.synL[n * 2 * nu + nu + cc] * D(cc);
  if (n >= size - rows) {
    const int64_t i = n - (size - rows);
    for (int cc = 0; cc < nu; ++cc) {
      const int64_t pos = half - 1 - cc;
      if (pos < right_first) continue;
      acc += t.synR[i * 2 * nu + cc] * A(pos) + t.synR[i * 2 * nu + nu + cc] * D(pos);
    }
  }
  return acc;
}

// Transpose of synth_value (one level of the forward DWT): output o of
// [a_k | d_k] from the 2^{k+1} values of the line.
template <typename T>
__device__ T analysis_value(const T* __restrict__ src, int64_t es, int64_t o, int k, const Tables<T>& t) {
  const int64_t half = int64_t(1) << k, size = 2 * half;
  const int nu = t.nu;
  const int kind = o >= half ? 1 : 0;
  const int64_t m = o - kind * half;
  const int64_t right_first = half - nu > nu ? half - nu : nu;
  const int rows = 3 * nu - 1;
  T acc = 0;
  if (m >= nu && m < right_first) {
    const T* taps = kind ? t.g : t.h;
    for (int c = -nu + 1; c <= nu; ++c) acc += taps[c + nu - 1] * src[(2 * m + c) * es];
  } else if (m < nu) {
    for (int r = 0; r < rows && r < size; ++r) acc += t.synL[r * 2 * nu + kind * nu + m] * src[r * es];
  } else {
    const int64_t cc = half - 1 - m;
    for (int r = 0; r < rows; ++r) acc += t.synR[r * 2 * nu + kind * nu + cc] * src[(size - rows + r) * es];
  }
  return acc;
}

// One level of the inverse DWT of the periodic extension (Sec. 3.2): every
// function is periodised, so output n of a line of 2^{k+1} values is
// sum_c h_c a_m + g_c d_m over the m with n - 2m = c, m taken modulo 2^k.
template <typename T>
__device__ T synth_value_per(const T* __restrict__ src, int64_t es, int64_t n, int k, const Tables<T>& t) {
  const int64_t half = int64_t(1) << k;
  const int nu = t.nu;
  T acc = 0;
  for (int c = -nu + 1; c <= nu; ++c) {
    const int64_t d = n - c;
    if (d & 1) continue;
    const int64_t m = (d >> 1) & (half - 1);  // modulo 2^k, also for d < 0
    acc += src[m * es] * t.h[c + nu - 1] + src[(half + m) * es] * t.g[c + nu - 1];
  }
  return acc;
}

// Its transpose: a_m = sum_c h_c v_{(2m + c) mod 2^{k+1}}, d_m the same with g.
template <typename T>
__device__ T analysis_value_per(const T* __restrict__ src, int64_t es, int64_t o, int k, const Tables<T>& t) {
  const int64_t half = int64_t(1) << k, size = 2 * half;
  const int nu = t.nu;
  const int kind = o >= half ? 1 : 0;
  const int64_t m = o - kind * half;
  const T* taps = kind ? t.g : t.h;
  T acc = 0;
  for (int c = -nu + 1; c <= nu; ++c) acc += taps[c + nu - 1] * src[((2 * m + c) & (size - 1)) * es];
  return acc;
}

// Barrier of a group of nt threads that works on one line.  Groups are
// aligned to waves, and every group of a workgroup has the same size and
// passes the same barriers; a group within one wave (nt <= 64) needs only
// its wave's LDS accesses kept in order, not a workgroup barrier.
__device__ __forceinline__ void group_sync(int nt) {
  if (nt <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Natural-order Walsh-Hadamard transform of buf[0, M) in LDS by a group of
// nthreads threads.  The butterflies of the index bits commute, so they run three
// bits at a time: each work item loads the 8 values whose indices differ in
// bits b .. b+2, applies the three butterfly stages in registers and stores
// them back -- one barrier per three stages.  The last one or two bits, if
// any, run as a radix-2 or radix-4 pass.
template <typename T, int F>
__device__ __forceinline__ void fwht_lds_pass(T* buf, int M, int h, int tid, int nthreads) {
  for (int g = tid; g < M / F; g += nthreads) {
    const int base = (g / h) * F * h + (g % h);
    T v[F];
#pragma unroll
    for (int i = 0; i < F; ++i) v[i] = buf[base + i * h];
#pragma unroll
    for (int hh = 1; hh < F; hh <<= 1)
#pragma unroll
      for (int i = 0; i < F; ++i)
        if ((i & hh) == 0) {
          const T a = v[i], c = v[i + hh];
          v[i] = a + c;
          v[i + hh] = a - c;
        }
#pragma unroll
    for (int i = 0; i < F; ++i) buf[base + i * h] = v[i];
  }
  group_sync(nthreads);
}

template <typename T>
__device__ void fwht_lds(T* buf, int M, int tid, int nthreads) {
  int h = 1;
  for (; h * 8 <= M; h *= 8) fwht_lds_pass<T, 8>(buf, M, h, tid, nthreads);
  if (h * 4 == M) fwht_lds_pass<T, 4>(buf, M, h, tid, nthreads);
  else if (h * 2 == M) fwht_lds_pass<T, 2>(buf, M, h, tid, nthreads);
}

// dst[at(k)] = src(k) for k in [0, n), by nt threads (thread tid): each
// thread issues U global loads before it waits for them and stores the values
// to LDS, instead of one load and one wait per element.
template <int U, typename T, typename Src, typename At>
__device__ __forceinline__ void stage_lds(T* dst, int n, int tid, int nt, Src src, At at) {
  for (int k0 = tid; k0 < n; k0 += U * nt) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * nt;
      v[u] = k < n ? src(k) : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * nt;
      if (k < n) dst[at(k)] = v[u];
    }
  }
}
constexpr int kInFlight = 8;

// Position b (sequency order within a phase) of the u-th element of a line's
// gather or scatter, u = iteration * threads + thread.  In natural order the
// position is bitrev(gray(b)), so the consecutive b that coalesce the global
// accesses all fall into one LDS bank; a wave (64 consecutive u) instead
// takes 8 runs of 8 consecutive b, M / 8 apart: 32-byte global segments and
// 8 distinct low bits of the natural index.  A bijection of [0, M).
__device__ __forceinline__ int spread_pos(int u, int M) {
  if (M < 64) return u;
  return (u & 7) + ((u >> 3) & 7) * (M >> 3) + (u >> 6) * 8;
}
// The same for a sparse Omega, whose samples sit at scattered ranks anyway:
// consecutive u take bit u / W of the mask words u mod W (W = M / 32 words per
// phase), so the lanes of a wave spread over the high bits of b (the low
// bits of the natural index).  A bijection of [0, 2^j).
__device__ __forceinline__ int word_pos(int u, int j) {
  if (j < 5) return u;
  return ((u & ((1 << (j - 5)) - 1)) << 5) | (u >> (j - 5));
}

// The `wpr` mask words of a row into wl[] and the exclusive prefix of their
// popcounts into pre[] (both LDS).
__device__ inline void row_prefix(const uint32_t* __restrict__ words, int64_t wpr, int* pre, uint32_t* wl,
                                  int* scratch, int tid, int nthreads) {
  if (wpr <= 64) {  // a short row: each word's prefix summed directly (two barriers instead of a scan)
    for (int w = tid; w < wpr; w += nthreads) wl[w] = words[w];
    group_sync(nthreads);
    for (int w = tid; w < wpr; w += nthreads) {
      int acc = 0;
      for (int i = 0; i < w; ++i) acc += __popc(wl[i]);
      pre[w] = acc;
    }
    group_sync(nthreads);
    return;
  }
  const int64_t chunk = (wpr + nthreads - 1) / nthreads;
  const int64_t w0 = tid * chunk, w1 = w0 + chunk < wpr ? w0 + chunk : wpr;
  int local = 0;
  for (int64_t w = w0; w < w1; ++w) {
    const uint32_t v = words[w];
    wl[w] = v;
    local += __popc(v);
  }
  scratch[tid] = local;
  group_sync(nthreads);
  for (int off = 1; off < nthreads; off <<= 1) {
    int v = tid >= off ? scratch[tid - off] : 0;
    group_sync(nthreads);
    scratch[tid] += v;
    group_sync(nthreads);
  }
  int run = scratch[tid] - local;
  for (int64_t w = w0; w < w1; ++w) {
    pre[w] = run;
    run += __popc(wl[w]);
  }
  group_sync(nthreads);
}

// L[p, s] for one phase s from xi in LDS (table product with boundary bands).
// NU > 0: the order known at compile time -- the 2 nu - 1 taps of the phase
// in registers and, away from the boundary bands, one unrolled correlation
// per position; NU = 0 takes it from the tables (the fused batch launches
// over instances of different orders).
template <typename T, int NU = 0>
__device__ void table_product(const T* xi, T* L, int M, int s, int tid, int nthreads,
                              const Tables<T>& t) {
  const int nu = NU > 0 ? NU : t.nu, Q = t.Q, band = 2 * nu - 1;
  const int right_first = M - nu > nu ? M - nu : nu;
  constexpr int NT = NU > 0 ? 2 * NU - 1 : 1;
  T tap[NT];
  if constexpr (NU > 0) {
#pragma unroll
    for (int li = 0; li < NT; ++li) tap[li] = t.tabT[li * Q + s];
  }
  if (t.per) {  // periodic extension: the correlation wraps around the line
    for (int p = tid; p < M; p += nthreads) {
      T acc = 0;
      if constexpr (NU > 0) {
#pragma unroll
        for (int li = 0; li < NT; ++li) acc += xi[(p - li + NU - 1) & (M - 1)] * tap[li];
      } else {
        for (int l = -nu + 1; l <= nu - 1; ++l) acc += xi[(p - l) & (M - 1)] * t.tabT[(l + nu - 1) * Q + s];
      }
      L[p] = acc;
    }
    return;
  }
  for (int p = tid; p < M; p += nthreads) {
    T acc = 0;
    if (NU > 0 && p >= 2 * nu - 1 && p <= right_first - nu) {
      // every tap lands on an interior coefficient and no band reaches p
#pragma unroll
      for (int li = 0; li < NT; ++li) acc += xi[p - li + nu - 1] * tap[li];
      L[p] = acc;
      continue;
    }
    for (int l = -nu + 1; l <= nu - 1; ++l) {
      const int m = p - l;
      if (m >= nu && m < right_first) acc += xi[m] * t.tabT[(l + nu - 1) * Q + s];
    }
    if (p < band)
      for (int m = 0; m < nu && m < M; ++m) acc += xi[m] * t.bandL[(p * nu + m) * Q + s];
    if (p >= M - band) {
      const int i = p - (M - band);
      for (int mp = 0; mp < nu; ++mp) {
        const int m = M - 1 - mp;
        if (m < right_first) continue;
        acc += xi[m] * t.bandR[(i * nu + mp) * Q + s];
      }
    }
    L[p] = acc;
  }
}

// xi[m] += sum_p table(p, m, s) R[p] for one phase s (transpose of
// table_product; NU as there).
template <typename T, int NU = 0>
__device__ void table_product_t(const T* R, T* xi, int M, int s, int tid, int nthreads,
                                const Tables<T>& t) {
  const int nu = NU > 0 ? NU : t.nu, Q = t.Q, band = 2 * nu - 1;
  const int right_first = M - nu > nu ? M - nu : nu;
  constexpr int NT = NU > 0 ? 2 * NU - 1 : 1;
  T tap[NT];
  if constexpr (NU > 0) {
#pragma unroll
    for (int li = 0; li < NT; ++li) tap[li] = t.tabT[li * Q + s];
  }
  if (t.per) {
    for (int m = tid; m < M; m += nthreads) {
      T acc = 0;
      if constexpr (NU > 0) {
#pragma unroll
        for (int li = 0; li < NT; ++li) acc += R[(m + li - NU + 1) & (M - 1)] * tap[li];
      } else {
        for (int l = -nu + 1; l <= nu - 1; ++l) acc += R[(m + l) & (M - 1)] * t.tabT[(l + nu - 1) * Q + s];
      }
      xi[m] += acc;
    }
    return;
  }
  for (int m = tid; m < M; m += nthreads) {
    T acc = 0;
    if (m >= nu && m < right_first) {
      if constexpr (NU > 0) {
#pragma unroll
        for (int li = 0; li < NT; ++li) acc += R[m + li - NU + 1] * tap[li];
      } else {
        for (int l = -nu + 1; l <= nu - 1; ++l) acc += R[m + l] * t.tabT[(l + nu - 1) * Q + s];
      }
    } else if (m < nu) {
      for (int p = 0; p < band && p < M; ++p) acc += R[p] * t.bandL[(p * nu + m) * Q + s];
    } else {
      const int mp = M - 1 - m;
      for (int i = 0; i < band; ++i) acc += R[M - band + i] * t.bandR[(i * nu + mp) * Q + s];
    }
    xi[m] += acc;
  }
}

// ------------------------------------------------------------ line kernels
// Addressing of the lines of one launch: line l starts at
// (l / inner) * os + (l % inner) * is, and its elements are es apart.
struct LineMap {
  int64_t inner, os, is, es;
};
__device__ __forceinline__ int64_t line_base(const LineMap& m, int64_t l) {
  return (l / m.inner) * m.os + (l % m.inner) * m.is;
}

// Row of the Omega bitmask that a gathered / scattered line belongs to.  The
// line index encodes `lead` natural indices (0: the single 1D line; 1: line =
// r_0; 2: line = r_0 N_1 + r_1, N_1 = Q 2^{jl1}) of axes with 2^{jl0},
// 2^{jl1} values per phase; the row is the row-major index of their
// sequency indices n = s 2^j + seq(k) (natural r = s 2^j + k).
struct RowMap {
  int lead, jl0, jl1;
};
__device__ __forceinline__ int64_t sequency_row(int64_t r, int jj) {
  const uint32_t s = uint32_t(r >> jj), k = uint32_t(r & ((int64_t(1) << jj) - 1));
  return (int64_t(s) << jj) + sequency_of(k, s, jj);
}
__device__ __forceinline__ int64_t omega_row(int64_t line, const RowMap& rm, int Q) {
  if (rm.lead == 0) return 0;
  if (rm.lead == 1) return sequency_row(line, rm.jl0);
  const int64_t N1 = int64_t(Q) << rm.jl1;
  return sequency_row(line / N1, rm.jl0) * N1 + sequency_row(line % N1, rm.jl1);
}

// Forward G on line `line` of M = 2^j values, by a group of nt threads
// (thread tid of the group; smem: the group's 2 M values and, when gathering
// from a sparse Omega, 2 wpr + nt ints).  Every thread of the workgroup must
// call it, with groups of the same size: its barriers are workgroup-wide
// when a group spans more than one wave, and every group passes the same
// sequence of them.  gather == 0: write the N
// outputs in natural order r = s M + k at element r of output line `line`.
// gather == 1: the samples of the line's Omega row go to y (`out`).
template <typename T, int NU = 0>
__device__ void fwd_line(const T* __restrict__ in, const LineMap& im, T* __restrict__ out, const LineMap& omap, int j,
         int gather, const RowMap& rm,
            const Tables<T>& t, const OmegaDev& om, int64_t line, unsigned char* smem, int tid, int nt) {
  const int M = 1 << j, Q = t.Q;
  T* xi = reinterpret_cast<T*>(smem);
  T* L = xi + M;
  int* pre = reinterpret_cast<int*>(L + M);
  int* scratch = pre + (gather && !om.full ? om.wpr : 0);
  uint32_t* wl = reinterpret_cast<uint32_t*>(scratch + nt);
  const int64_t ib = line_base(im, line);
  stage_lds<kInFlight>(xi, M, tid, nt, [&](int p) { return in[ib + p * im.es]; }, [](int p) { return p; });
  int64_t n1 = 0, base = 0;
  if (gather) {
    n1 = omega_row(line, rm, Q);
    base = om.row_ptr[n1];
    if (!om.full) row_prefix(om.mask + n1 * om.wpr, om.wpr, pre, wl, scratch, tid, nt);
  }
  const int64_t ob = gather ? 0 : line_base(omap, line);
  group_sync(nt);
  for (int s = 0; s < Q; ++s) {
    table_product<T, NU>(xi, L, M, s, tid, nt, t);
    group_sync(nt);
    fwht_lds(L, M, tid, nt);
    if (!gather) {
      for (int k = tid; k < M; k += nt) out[ob + (int64_t(s) * M + k) * omap.es] = L[k];
    } else if (om.full) {
      for (int u = tid; u < M; u += nt) {
        const int b = spread_pos(u, M);
        out[base + int64_t(s) * M + b] = L[natural_of(uint32_t(b), uint32_t(s), j)];
      }
    } else {  // sample n2 = s M + b is number pre[word] + (set bits below it in its word) of the row
      for (int u = tid; u < M; u += nt) {
        const int b = word_pos(u, j);
        const int64_t n2 = int64_t(s) * M + b;
        const uint32_t w = wl[n2 >> 5], bit = uint32_t(n2) & 31u;
        if ((w >> bit) & 1u)
          out[base + pre[n2 >> 5] + __popc(w & ((1u << bit) - 1u))] = L[natural_of(uint32_t(b), uint32_t(s), j)];
      }
    }
    group_sync(nt);
  }
}

// Adjoint G^T on line `line` (the same conventions).  scatter == 0: read the
// N natural-order values of input line `line` (element r at r * im.es).
// scatter == 1: the line's Omega samples come from y (`in`).  The M results
// go to output line `line`.
template <typename T, int NU = 0>
__device__ void adj_line(const T* __restrict__ in, const LineMap& im, T* __restrict__ out, const LineMap& omap, int j,
         int scatter, const RowMap& rm,
            const Tables<T>& t, const OmegaDev& om, int64_t line, unsigned char* smem, int tid, int nt) {
  const int M = 1 << j, Q = t.Q;
  T* xi = reinterpret_cast<T*>(smem);
  T* R = xi + M;
  int* pre = reinterpret_cast<int*>(R + M);
  int* scratch = pre + (scatter && !om.full ? om.wpr : 0);
  uint32_t* wl = reinterpret_cast<uint32_t*>(scratch + nt);
  for (int p = tid; p < M; p += nt) xi[p] = 0;
  int64_t n1 = 0, base = 0;
  if (scatter) {
    n1 = omega_row(line, rm, Q);
    base = om.row_ptr[n1];
    if (!om.full) row_prefix(om.mask + n1 * om.wpr, om.wpr, pre, wl, scratch, tid, nt);
  }
  const int64_t ib = scatter ? 0 : line_base(im, line);
  group_sync(nt);
  for (int s = 0; s < Q; ++s) {
    auto nat = [&](int u) { return int(natural_of(uint32_t(spread_pos(u, M)), uint32_t(s), j)); };
    auto nat_w = [&](int u) { return int(natural_of(uint32_t(word_pos(u, j)), uint32_t(s), j)); };
    if (!scatter) {
      stage_lds<kInFlight>(R, M, tid, nt, [&](int k) { return in[ib + (int64_t(s) * M + k) * im.es]; },
                           [](int k) { return k; });
    } else if (om.full) {
      stage_lds<kInFlight>(R, M, tid, nt, [&](int u) { return in[base + int64_t(s) * M + spread_pos(u, M)]; },
                           nat);
    } else {  // every position of R written once: the sample, or 0 off Omega
      stage_lds<kInFlight>(R, M, tid, nt, [&](int u) {
        const int64_t n2 = int64_t(s) * M + word_pos(u, j);
        const uint32_t w = wl[n2 >> 5], bit = uint32_t(n2) & 31u;
        return (w >> bit) & 1u ? in[base + pre[n2 >> 5] + __popc(w & ((1u << bit) - 1u))] : T(0);
      }, nat_w);
    }
    group_sync(nt);
    fwht_lds(R, M, tid, nt);
    table_product_t<T, NU>(R, xi, M, s, tid, nt, t);
    group_sync(nt);
  }
  const int64_t ob = line_base(omap, line);
  for (int m = tid; m < M; m += nt) out[ob + m * omap.es] = xi[m];
}

}  // namespace wh2wav_generic
