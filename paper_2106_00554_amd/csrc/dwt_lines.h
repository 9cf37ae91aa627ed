// One-level wavelet synthesis and analysis along a line, shared by the 2D
// and 1D wavelet kernels.
//
// Level k -> k+1 of the inverse DWT maps [a_k | d_k] (2^k + 2^k values) to
// the 2^{k+1} scaling coefficients at level k+1.  Interior coefficients use
// the filters at stride 2 (phi_{k,m} = sum_c h_c phi_{k+1,2m+c}, psi likewise
// with g); the nu boundary functions at each end use the dense one-level
// synthesis blocks built by the planner (Sec. 3.2).  Analysis is the
// transpose.  Each helper reads its inputs once into registers ("runs" of P
// consecutive outputs).
#pragma once

#include "fast2d.h"

namespace wh2wav_fast {
namespace lines {

// Synthesis of output n of one line: a(m) = A(m), d(m) = D(m), m < half.
template <typename T, int NU, class FA, class FD>
__device__ __forceinline__ T synth_at(int n, int half, const T* __restrict__ h, const T* __restrict__ g,
                                      const T* __restrict__ synL, const T* __restrict__ synR, FA A, FD D) {
  constexpr int ROWS = 3 * NU - 1;
  const int size = 2 * half;
  const int right_first = half - NU > NU ? half - NU : NU;
  T acc = T(0);
  int mlo = n - NU + 1 > 0 ? (n - NU + 1) >> 1 : 0;
  if (mlo < NU) mlo = NU;
  int mhi = (n + NU - 1) >> 1;
  if (mhi > half - NU - 1) mhi = half - NU - 1;
  for (int m = mlo; m <= mhi; ++m) {
    const int c = n - 2 * m + NU - 1;
    acc = fma(A(m), h[c], acc);
    acc = fma(D(m), g[c], acc);
  }
  if (n < ROWS) {
#pragma unroll
    for (int cc = 0; cc < NU; ++cc) {
      if (cc >= half) break;
      acc = fma(synL[n * 2 * NU + cc], A(cc), acc);
      acc = fma(synL[n * 2 * NU + NU + cc], D(cc), acc);
    }
  }
  if (n >= size - ROWS) {
    const int i = n - (size - ROWS);
#pragma unroll
    for (int cc = 0; cc < NU; ++cc) {
      const int pos = half - 1 - cc;
      if (pos < right_first) continue;
      acc = fma(synR[i * 2 * NU + cc], A(pos), acc);
      acc = fma(synR[i * 2 * NU + NU + cc], D(pos), acc);
    }
  }
  return acc;
}

// Analysis output o of one line (o < half: scaling coefficient, else wavelet).
template <typename T, int NU, class FX>
__device__ __forceinline__ T analysis_at(int o, int half, const T* __restrict__ h, const T* __restrict__ g,
                                         const T* __restrict__ synL, const T* __restrict__ synR, FX X) {
  constexpr int ROWS = 3 * NU - 1;
  const int size = 2 * half;
  const int kind = o >= half ? 1 : 0;
  const int m = o - kind * half;
  const int right_first = half - NU > NU ? half - NU : NU;
  T acc = T(0);
  if (m >= NU && m < right_first) {
    const T* taps = kind ? g : h;
#pragma unroll
    for (int c = 0; c < 2 * NU; ++c) acc = fma(taps[c], X(2 * m + c - NU + 1), acc);
  } else if (m < NU) {
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc = fma(synL[r * 2 * NU + kind * NU + m], X(r), acc);
  } else {
    const int cc = half - 1 - m;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc = fma(synR[r * 2 * NU + kind * NU + cc], X(size - ROWS + r), acc);
  }
  return acc;
}

// Index range of a-part (or d-part) inputs m that synthesis outputs
// [n0, n1) read, boundary columns included.
template <int NU>
__host__ __device__ __forceinline__ void synth_input_range(int n0, int n1, int half, int& lo, int& hi) {
  constexpr int ROWS = 3 * NU - 1;
  lo = n0 - NU > 0 ? (n0 - NU) >> 1 : 0;
  hi = (n1 - 1 + NU) >> 1;
  if (hi > half - 1) hi = half - 1;
  if (n0 < ROWS) lo = 0;
  if (n1 > 2 * half - ROWS) hi = half - 1;
}

// Index range of inputs n that analysis outputs m in [m0, m1) (of either half) read.
template <int NU>
__host__ __device__ __forceinline__ void analysis_input_range(int m0, int m1, int half, int& lo, int& hi) {
  constexpr int ROWS = 3 * NU - 1;
  const int size = 2 * half;
  lo = 2 * m0 - NU + 1;
  hi = 2 * (m1 - 1) + NU;
  if (lo < 0) lo = 0;
  if (hi > size - 1) hi = size - 1;
  if (m0 < NU) lo = 0;
  if (m1 > half - NU) hi = size - 1;
  (void)ROWS;
}

// Periodic extension: the input index ranges of synthesis outputs [n0, n1)
// and of analysis outputs [m0, m1), unclamped (taken modulo the line length
// where they are read).
template <int NU>
__host__ __device__ __forceinline__ void synth_input_range_per(int n0, int n1, int& lo, int& hi) {
  lo = (n0 - NU) >> 1;
  hi = (n1 - 1 + NU) >> 1;
}
template <int NU>
__host__ __device__ __forceinline__ void analysis_input_range_per(int m0, int m1, int& lo, int& hi) {
  lo = 2 * m0 - NU + 1;
  hi = 2 * (m1 - 1) + NU;
}

// Interior synthesis pair i: every filter tap of outputs 2i and 2i+1 lands on
// an interior coefficient (3nu-1 <= 2i and 2i+1 <= size-3nu).
template <int NU>
__device__ __forceinline__ bool pair_is_interior(int i, int half) {
  return 2 * i >= 3 * NU - 1 && 2 * i + 1 <= 2 * half - 3 * NU;
}

// Offsets m - i of the inputs that interior synthesis pair i reads.
template <int NU>
__host__ __device__ constexpr int synth_off(int c) {
  return (((c % 2) + 2) % 2 == 0) ? -c / 2 : -(c - 1) / 2;
}
template <int NU>
__host__ __device__ constexpr int synth_lo() {
  int v = 0;
  for (int c = -NU + 1; c <= NU; ++c) v = synth_off<NU>(c) < v ? synth_off<NU>(c) : v;
  return v;
}
template <int NU>
__host__ __device__ constexpr int synth_hi() {
  int v = 0;
  for (int c = -NU + 1; c <= NU; ++c) v = synth_off<NU>(c) > v ? synth_off<NU>(c) : v;
  return v;
}

// The filter taps of P consecutive synthesis pairs i0 .. i0+P-1 applied to
// a(i0 + lo + u) = a[u], d(i0 + lo + u) = d[u].
template <typename T, int NU, int P>
__device__ __forceinline__ void synth_math(const T (&a)[P + synth_hi<NU>() - synth_lo<NU>()],
                                           const T (&d)[P + synth_hi<NU>() - synth_lo<NU>()],
                                           const T (&hr)[2 * NU], const T (&gr)[2 * NU], T (&e)[P], T (&o)[P]);

// P consecutive interior synthesis pairs i0 .. i0+P-1 of one line.  pa points
// at a(i0 + lo), pd at d(i0 + lo); consecutive m are `stride` elements apart.
// Inputs are read once into registers and reused by every tap.
template <typename T, int NU, int P>
__device__ __forceinline__ void synth_run(const T* __restrict__ pa, const T* __restrict__ pd, int stride,
                                          const T (&hr)[2 * NU], const T (&gr)[2 * NU], T (&e)[P], T (&o)[P]) {
  constexpr int LO = synth_lo<NU>(), L = P + synth_hi<NU>() - LO;
  T a[L], d[L];
#pragma unroll
  for (int u = 0; u < L; ++u) {
    a[u] = pa[u * stride];
    d[u] = pd[u * stride];
  }
  synth_math<T, NU, P>(a, d, hr, gr, e, o);
}

// The same run for the periodic extension (Sec. 3.2), any i0: pa and pd point
// at a(0) and d(0), and the coefficient index is taken modulo half.
template <typename T, int NU, int P>
__device__ __forceinline__ void synth_run_wrap(const T* __restrict__ pa, const T* __restrict__ pd, int stride, int i0,
                                               int half, const T (&hr)[2 * NU], const T (&gr)[2 * NU], T (&e)[P],
                                               T (&o)[P]) {
  constexpr int LO = synth_lo<NU>(), L = P + synth_hi<NU>() - LO;
  T a[L], d[L];
#pragma unroll
  for (int u = 0; u < L; ++u) {
    const int m = (i0 + LO + u) & (half - 1);
    a[u] = pa[m * stride];
    d[u] = pd[m * stride];
  }
  synth_math<T, NU, P>(a, d, hr, gr, e, o);
}

template <typename T, int NU, int P>
__device__ __forceinline__ void synth_math(const T (&a)[P + synth_hi<NU>() - synth_lo<NU>()],
                                           const T (&d)[P + synth_hi<NU>() - synth_lo<NU>()],
                                           const T (&hr)[2 * NU], const T (&gr)[2 * NU], T (&e)[P], T (&o)[P]) {
  constexpr int LO = synth_lo<NU>();
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T ae = T(0), ao = T(0);
#pragma unroll
    for (int c = -NU + 1; c <= NU; ++c) {
      const int idx = p + synth_off<NU>(c) - LO;
      if (((c % 2) + 2) % 2 == 0) {
        ae = fma(a[idx], hr[c + NU - 1], ae);
        ae = fma(d[idx], gr[c + NU - 1], ae);
      } else {
        ao = fma(a[idx], hr[c + NU - 1], ao);
        ao = fma(d[idx], gr[c + NU - 1], ao);
      }
    }
    e[p] = ae;
    o[p] = ao;
  }
}

// The filter taps of P consecutive analysis outputs m0 .. m0+P-1 applied to
// x(2 m0 - nu + 1 + u) = v[u].
template <typename T, int NU, int P>
__device__ __forceinline__ void analysis_math(const T (&v)[2 * P + 2 * NU - 2], const T (&hr)[2 * NU],
                                              const T (&gr)[2 * NU], T (&a)[P], T (&d)[P]);

// P consecutive interior analysis outputs m0 .. m0+P-1 (scaling and wavelet
// coefficient of each); px points at x(2 m0 - nu + 1).
template <typename T, int NU, int P>
__device__ __forceinline__ void analysis_run(const T* __restrict__ px, int stride, const T (&hr)[2 * NU],
                                             const T (&gr)[2 * NU], T (&a)[P], T (&d)[P]) {
  constexpr int L = 2 * P + 2 * NU - 2;
  T v[L];
#pragma unroll
  for (int u = 0; u < L; ++u) v[u] = px[u * stride];
  analysis_math<T, NU, P>(v, hr, gr, a, d);
}

// The same run for the periodic extension, any m0: px points at x(0), and
// the input index is taken modulo size = 2 half.
template <typename T, int NU, int P>
__device__ __forceinline__ void analysis_run_wrap(const T* __restrict__ px, int stride, int m0, int size,
                                                  const T (&hr)[2 * NU], const T (&gr)[2 * NU], T (&a)[P],
                                                  T (&d)[P]) {
  constexpr int L = 2 * P + 2 * NU - 2;
  T v[L];
#pragma unroll
  for (int u = 0; u < L; ++u) v[u] = px[((2 * m0 - NU + 1 + u) & (size - 1)) * stride];
  analysis_math<T, NU, P>(v, hr, gr, a, d);
}

template <typename T, int NU, int P>
__device__ __forceinline__ void analysis_math(const T (&v)[2 * P + 2 * NU - 2], const T (&hr)[2 * NU],
                                              const T (&gr)[2 * NU], T (&a)[P], T (&d)[P]) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T sa = T(0), sd = T(0);
#pragma unroll
    for (int c = 0; c < 2 * NU; ++c) {
      sa = fma(hr[c], v[2 * p + c], sa);
      sd = fma(gr[c], v[2 * p + c], sd);
    }
    a[p] = sa;
    d[p] = sd;
  }
}

// Any run of P synthesis pairs i0 .. i0+P-1, boundary functions included.
// The line's a(m) is pa[(m - wlo) * stride] and d(m) is pd[(m - wlo) * stride]
// for m in the window [wlo, whi], which holds every coefficient the run reads.
// Interior taps see the boundary coefficients as zero; the boundary blocks
// then add the contributions of the nu left and nu right boundary functions.
// HOIST issues the boundary coefficients' loads together with the window's
// (clamped to the window, used only where the boundary blocks apply), so that
// a run near both ends waits on memory once; worth its registers for short
// runs read from global memory.
template <typename T, int NU, int P, bool HOIST = false>
__device__ __forceinline__ void synth_run_edge(const T* __restrict__ pa, const T* __restrict__ pd, int stride, int wlo,
                                               int whi, int i0, int half, const T (&hr)[2 * NU],
                                               const T (&gr)[2 * NU], const T* __restrict__ sL,
                                               const T* __restrict__ sR, T (&e)[P], T (&o)[P]) {
  constexpr int LO = synth_lo<NU>(), L = P + synth_hi<NU>() - LO, ROWS = 3 * NU - 1;
  const int size = 2 * half;
  T hl[NU], hdl[NU], hq[NU], hdq[NU];
  if constexpr (HOIST) {
#pragma unroll
    for (int cc = 0; cc < NU; ++cc) {
      const int pl = cc, pr = half - 1 - cc;
      const int ml = (pl < wlo ? wlo : (pl > whi ? whi : pl)) - wlo;
      const int mr = (pr < wlo ? wlo : (pr > whi ? whi : pr)) - wlo;
      hl[cc] = pa[ml * stride], hdl[cc] = pd[ml * stride];
      hq[cc] = pa[mr * stride], hdq[cc] = pd[mr * stride];
    }
  }
  T a[L], d[L];
#pragma unroll
  for (int u = 0; u < L; ++u) {
    const int m = i0 + LO + u;
    const bool inside = m >= NU && m <= half - NU - 1;
    const int mc = (m < wlo ? wlo : (m > whi ? whi : m)) - wlo;
    const T va = pa[mc * stride], vd = pd[mc * stride];
    a[u] = inside ? va : T(0);
    d[u] = inside ? vd : T(0);
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T ae = T(0), ao = T(0);
#pragma unroll
    for (int c = -NU + 1; c <= NU; ++c) {
      const int idx = p + synth_off<NU>(c) - LO;
      if (((c % 2) + 2) % 2 == 0) {
        ae = fma(a[idx], hr[c + NU - 1], ae);
        ae = fma(d[idx], gr[c + NU - 1], ae);
      } else {
        ao = fma(a[idx], hr[c + NU - 1], ao);
        ao = fma(d[idx], gr[c + NU - 1], ao);
      }
    }
    e[p] = ae;
    o[p] = ao;
  }
  if (2 * i0 < ROWS) {  // left boundary functions, positions 0 .. nu-1
    T bl[NU], bd[NU];
#pragma unroll
    for (int cc = 0; cc < NU; ++cc) {
      T va, vd;
      if constexpr (HOIST) {
        va = hl[cc], vd = hdl[cc];
      } else {
        const int mc = (cc > whi ? whi : cc) - wlo;
        va = pa[mc * stride], vd = pd[mc * stride];
      }
      bl[cc] = cc < half ? va : T(0);
      bd[cc] = cc < half ? vd : T(0);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
      for (int sdx = 0; sdx < 2; ++sdx) {
        const int n = 2 * (i0 + p) + sdx;
        if (n < ROWS) {
          T acc = sdx ? o[p] : e[p];
#pragma unroll
          for (int cc = 0; cc < NU; ++cc) {
            acc = fma(sL[n * 2 * NU + cc], bl[cc], acc);
            acc = fma(sL[n * 2 * NU + NU + cc], bd[cc], acc);
          }
          if (sdx) o[p] = acc; else e[p] = acc;
        }
      }
    }
  }
  if (2 * (i0 + P) > size - ROWS) {  // right boundary functions, positions half-1-cc
    const int right_first = half - NU > NU ? half - NU : NU;
    T br[NU], bd[NU];
#pragma unroll
    for (int cc = 0; cc < NU; ++cc) {
      const int pos = half - 1 - cc;
      T va, vd;
      if constexpr (HOIST) {
        va = hq[cc], vd = hdq[cc];
      } else {
        const int mc = (pos < wlo ? wlo : pos) - wlo;
        va = pa[mc * stride], vd = pd[mc * stride];
      }
      br[cc] = pos >= right_first ? va : T(0);
      bd[cc] = pos >= right_first ? vd : T(0);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
      for (int sdx = 0; sdx < 2; ++sdx) {
        const int n = 2 * (i0 + p) + sdx;
        if (n >= size - ROWS && n < size) {
          const int i = n - (size - ROWS);
          T acc = sdx ? o[p] : e[p];
#pragma unroll
          for (int cc = 0; cc < NU; ++cc) {
            acc = fma(sR[i * 2 * NU + cc], br[cc], acc);
            acc = fma(sR[i * 2 * NU + NU + cc], bd[cc], acc);
          }
          if (sdx) o[p] = acc; else e[p] = acc;
        }
      }
    }
  }
}

// Any run of P analysis outputs m0 .. m0+P-1 (scaling and wavelet coefficient
// of each), boundary functions included.  x(n) is px[(n - wlo) * stride] for
// n in the window [wlo, whi].
template <typename T, int NU, int P>
__device__ __forceinline__ void analysis_run_edge(const T* __restrict__ px, int stride, int wlo, int whi, int m0,
                                                  int half, const T (&hr)[2 * NU], const T (&gr)[2 * NU],
                                                  const T* __restrict__ sL, const T* __restrict__ sR, T (&a)[P],
                                                  T (&d)[P]) {
  constexpr int L = 2 * P + 2 * NU - 2, ROWS = 3 * NU - 1;
  const int size = 2 * half;
  const int right_first = half - NU > NU ? half - NU : NU;
  T v[L];
#pragma unroll
  for (int u = 0; u < L; ++u) {
    const int n = 2 * m0 - NU + 1 + u;
    v[u] = px[((n < wlo ? wlo : (n > whi ? whi : n)) - wlo) * stride];
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T sa = T(0), sd = T(0);
#pragma unroll
    for (int c = 0; c < 2 * NU; ++c) {
      sa = fma(hr[c], v[2 * p + c], sa);
      sd = fma(gr[c], v[2 * p + c], sd);
    }
    a[p] = sa;
    d[p] = sd;
  }
  if (m0 < NU) {  // left boundary functions read x(0 .. 3nu-2)
    T xl[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) xl[r] = px[((r > whi ? whi : r) - wlo) * stride];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int m = m0 + p;
      if (m < NU) {
        T sa = T(0), sd = T(0);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          sa = fma(sL[r * 2 * NU + m], xl[r], sa);
          sd = fma(sL[r * 2 * NU + NU + m], xl[r], sd);
        }
        a[p] = sa;
        d[p] = sd;
      }
    }
  }
  if (m0 + P > right_first) {  // right boundary functions read x(size-3nu+1 .. size-1)
    T xr[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const int n = size - ROWS + r;
      xr[r] = px[((n < wlo ? wlo : n) - wlo) * stride];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int m = m0 + p;
      if (m >= right_first && m >= NU && m < half) {
        const int cc = half - 1 - m;
        T sa = T(0), sd = T(0);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          sa = fma(sR[r * 2 * NU + cc], xr[r], sa);
          sd = fma(sR[r * 2 * NU + NU + cc], xr[r], sd);
        }
        a[p] = sa;
        d[p] = sd;
      }
    }
  }
}

template <typename T>
struct TileLds {
  T* hs;
  T* gs;
  T* sLs;
  T* sRs;
};

// Filters and boundary blocks: taps in registers for the interior runs, a
// copy in LDS for the runtime-indexed boundary outputs.
template <typename T, int NU>
__device__ __forceinline__ TileLds<T> load_tables(const Tables<T>& t, T* tab_lds, T (&hr)[2 * NU], T (&gr)[2 * NU]) {
#pragma unroll
  for (int c = 0; c < 2 * NU; ++c) hr[c] = t.h[c], gr[c] = t.g[c];
  TileLds<T> L;
  L.hs = tab_lds;
  L.gs = L.hs + 2 * NU;
  L.sLs = L.gs + 2 * NU;
  L.sRs = L.sLs + (3 * NU - 1) * 2 * NU;
  for (int e = int(threadIdx.x); e < 2 * NU; e += int(blockDim.x)) L.hs[e] = t.h[e], L.gs[e] = t.g[e];
  for (int e = int(threadIdx.x); e < (3 * NU - 1) * 2 * NU; e += int(blockDim.x))
    L.sLs[e] = t.synL[e], L.sRs[e] = t.synR[e];
  return L;
}

// Synthesis levels j0 .. kc-1 of a line held in LDS by the whole workgroup:
// a = [a_j0 | d_j0 | ... | d_{kc-1}] (2^kc values) becomes the scaling
// coefficients at level kc; b is scratch of 2^kc values.  One output pair per
// work item (twice the items of two-pair runs and half the dependent chain).
// Every level ends with a barrier.
template <typename T, int NU>
__device__ void synth_levels_lds(T* a, T* b, int j0, int kc, const TileLds<T>& tl, const T (&hr)[2 * NU],
                                 const T (&gr)[2 * NU]) {
  const int tid = int(threadIdx.x), nt = int(blockDim.x);
  constexpr int CP = 1, LO = synth_lo<NU>();  // one pair per item: twice the items, half the chain
  for (int k = j0; k < kc; ++k) {
    const int half = 1 << k, runs = (half + CP - 1) / CP;
    for (int item = tid; item < runs; item += nt) {
      const int i0 = item * CP;
      T* yo = b + 2 * i0;
      if (pair_is_interior<NU>(i0, half) && pair_is_interior<NU>(i0 + CP - 1, half)) {
        T e[CP], o[CP];
        synth_run<T, NU, CP>(a + i0 + LO, a + half + i0 + LO, 1, hr, gr, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) yo[2 * p] = e[p], yo[2 * p + 1] = o[p];
      } else if (half >= CP) {
        T e[CP], o[CP];
        synth_run_edge<T, NU, CP>(a, a + half, 1, 0, half - 1, i0, half, hr, gr, tl.sLs, tl.sRs, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) yo[2 * p] = e[p], yo[2 * p + 1] = o[p];
      } else {
        auto A = [&](int m) { return a[m]; };
        auto D = [&](int m) { return a[half + m]; };
        for (int p = 0; p < CP && i0 + p < half; ++p) {
          yo[2 * p] = synth_at<T, NU>(2 * (i0 + p), half, tl.hs, tl.gs, tl.sLs, tl.sRs, A, D);
          yo[2 * p + 1] = synth_at<T, NU>(2 * (i0 + p) + 1, half, tl.hs, tl.gs, tl.sLs, tl.sRs, A, D);
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < 2 * half; i += nt) a[i] = b[i];
    __syncthreads();
  }
}

// Its transpose: analysis levels kc-1 .. j0 of the line a (2^kc values) into
// [a_j0 | d_j0 | ... | d_{kc-1}], in a; b is scratch.  Every level ends with
// a barrier.
template <typename T, int NU>
__device__ void analysis_levels_lds(T* a, T* b, int j0, int kc, const TileLds<T>& tl, const T (&hr)[2 * NU],
                                    const T (&gr)[2 * NU]) {
  const int tid = int(threadIdx.x), nt = int(blockDim.x);
  constexpr int CP = 1;  // one output pair per item
  for (int k = kc - 1; k >= j0; --k) {
    const int half = 1 << k, size = 2 * half, runs = (half + CP - 1) / CP;
    for (int item = tid; item < runs; item += nt) {
      const int m0 = item * CP;
      if (m0 >= NU && m0 + CP - 1 < half - NU) {
        T av[CP], dv[CP];
        analysis_run<T, NU, CP>(a + 2 * m0 - NU + 1, 1, hr, gr, av, dv);
#pragma unroll
        for (int p = 0; p < CP; ++p) b[m0 + p] = av[p], b[half + m0 + p] = dv[p];
      } else if (half >= CP) {
        T av[CP], dv[CP];
        analysis_run_edge<T, NU, CP>(a, 1, 0, size - 1, m0, half, hr, gr, tl.sLs, tl.sRs, av, dv);
#pragma unroll
        for (int p = 0; p < CP; ++p) b[m0 + p] = av[p], b[half + m0 + p] = dv[p];
      } else {
        auto X = [&](int n) { return a[n]; };
        for (int p = 0; p < CP && m0 + p < half; ++p) {
          b[m0 + p] = analysis_at<T, NU>(m0 + p, half, tl.hs, tl.gs, tl.sLs, tl.sRs, X);
          b[half + m0 + p] = analysis_at<T, NU>(half + m0 + p, half, tl.hs, tl.gs, tl.sLs, tl.sRs, X);
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < size; i += nt) a[i] = b[i];
    __syncthreads();
  }
}

// Synthesis levels j0 .. kc-1 with three line buffers of 2^kc values: src
// holds [a_j0 | d_j0 | ... | d_{kc-1}] and is only read (every level reads
// its details there), the approximations alternate between fin and tmp so
// that the last level writes fin.  Every level writes a buffer that it does
// not read: one barrier per level and no copy back.
template <typename T, int NU>
__device__ void synth_levels_lds3(const T* src, T* fin, T* tmp, int j0, int kc, const TileLds<T>& tl,
                                  const T (&hr)[2 * NU], const T (&gr)[2 * NU]) {
  const int tid = int(threadIdx.x), nt = int(blockDim.x);
  constexpr int LO = synth_lo<NU>();
  if (j0 == kc) {
    for (int i = tid; i < (1 << kc); i += nt) fin[i] = src[i];
    __syncthreads();
    return;
  }
  const T* ap = src;  // approximations of the current level
  for (int k = j0; k < kc; ++k) {
    const int half = 1 << k;
    const T* dp = src + half;  // its details
    T* out = ((kc - 1 - k) % 2 == 0) ? fin : tmp;
    for (int i0 = tid; i0 < half; i0 += nt) {
      T e[1], o[1];
      if (pair_is_interior<NU>(i0, half)) {
        synth_run<T, NU, 1>(ap + i0 + LO, dp + i0 + LO, 1, hr, gr, e, o);
      } else {
        synth_run_edge<T, NU, 1>(ap, dp, 1, 0, half - 1, i0, half, hr, gr, tl.sLs, tl.sRs, e, o);
      }
      out[2 * i0] = e[0];
      out[2 * i0 + 1] = o[0];
    }
    __syncthreads();
    ap = out;
  }
}

// Its transpose with three buffers: line (2^kc values, read by the first
// level, then scratch), tmp, and fin, which receives [a_j0 | d_j0 | ... |
// d_{kc-1}]: every level writes its details into fin at their final place
// and its approximations into the buffer it does not read (fin at the last
// level).  One barrier per level.
template <typename T, int NU>
__device__ void analysis_levels_lds3(T* line, T* fin, T* tmp, int j0, int kc, const TileLds<T>& tl,
                                     const T (&hr)[2 * NU], const T (&gr)[2 * NU]) {
  const int tid = int(threadIdx.x), nt = int(blockDim.x);
  if (j0 == kc) {
    for (int i = tid; i < (1 << kc); i += nt) fin[i] = line[i];
    __syncthreads();
    return;
  }
  T* ap = line;
  for (int k = kc - 1; k >= j0; --k) {
    const int half = 1 << k, size = 2 * half;
    T* aout = k == j0 ? fin : (ap == line ? tmp : line);
    for (int m0 = tid; m0 < half; m0 += nt) {
      T av[1], dv[1];
      if (m0 >= NU && m0 < half - NU)
        analysis_run<T, NU, 1>(ap + 2 * m0 - NU + 1, 1, hr, gr, av, dv);
      else
        analysis_run_edge<T, NU, 1>(ap, 1, 0, size - 1, m0, half, hr, gr, tl.sLs, tl.sRs, av, dv);
      aout[m0] = av[0];
      fin[half + m0] = dv[0];
    }
    __syncthreads();
    ap = aout;
  }
}

// The periodic extension (Sec. 3.2): synthesis levels j0 .. kc-1 of a line
// in LDS with every index taken modulo the level's length (no boundary
// functions); layout, scratch and barriers as synth_levels_lds.  Output pair
// i reads a and d at i + synth_off(c) for each tap c.
template <typename T, int NU>
__device__ void synth_levels_lds_per(T* a, T* b, int j0, int kc, const T (&hr)[2 * NU], const T (&gr)[2 * NU]) {
  const int tid = int(threadIdx.x), nt = int(blockDim.x);
  for (int k = j0; k < kc; ++k) {
    const int half = 1 << k;
    for (int i = tid; i < half; i += nt) {
      T e = T(0), o = T(0);
#pragma unroll
      for (int c = -NU + 1; c <= NU; ++c) {
        const int m = (i + synth_off<NU>(c)) & (half - 1);
        const T va = a[m], vd = a[half + m];
        if (((c % 2) + 2) % 2 == 0) {
          e = fma(va, hr[c + NU - 1], e);
          e = fma(vd, gr[c + NU - 1], e);
        } else {
          o = fma(va, hr[c + NU - 1], o);
          o = fma(vd, gr[c + NU - 1], o);
        }
      }
      b[2 * i] = e;
      b[2 * i + 1] = o;
    }
    __syncthreads();
    for (int i = tid; i < 2 * half; i += nt) a[i] = b[i];
    __syncthreads();
  }
}

// Its transpose: a_m = sum_c h_c v((2m + c) mod 2^{k+1}), d_m the same with g,
// levels kc-1 .. j0.
template <typename T, int NU>
__device__ void analysis_levels_lds_per(T* a, T* b, int j0, int kc, const T (&hr)[2 * NU], const T (&gr)[2 * NU]) {
  const int tid = int(threadIdx.x), nt = int(blockDim.x);
  for (int k = kc - 1; k >= j0; --k) {
    const int half = 1 << k, size = 2 * half;
    for (int m = tid; m < half; m += nt) {
      T sa = T(0), sd = T(0);
#pragma unroll
      for (int c = 0; c < 2 * NU; ++c) {
        const T v = a[(2 * m + c - NU + 1) & (size - 1)];
        sa = fma(hr[c], v, sa);
        sd = fma(gr[c], v, sd);
      }
      b[m] = sa;
      b[half + m] = sd;
    }
    __syncthreads();
    for (int i = tid; i < size; i += nt) a[i] = b[i];
    __syncthreads();
  }
}

template <int NU>
constexpr int tab_lds_size() {
  return 4 * NU + 2 * (3 * NU - 1) * 2 * NU;
}

}  // namespace lines
}  // namespace wh2wav_fast
