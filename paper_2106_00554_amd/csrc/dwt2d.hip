// Two-dimensional inverse DWT (C_{psi,j} quadtree -> B_{phi,j} (x) B_{phi,j}) and its
// transpose, for the square (isotropic) 2D basis.
//
// One level k -> k+1 maps the 2^{k+1} x 2^{k+1} block [[LL, LH], [HL, HH]] to
// S X S^T, S the one-level synthesis matrix (interior columns: the filters h, g
// at stride 2; boundary columns: the dense blocks built by the planner).  The
// transpose (the forward DWT) is S^T X S.
//   * The coarse levels run in one workgroup with the block in LDS: output
//     blocks of at most 8 x 8; with nu <= 4 up to 64 x 64, and the whole
//     transform of an FP32 array of at most 128 x 128.
//   * Every larger level is one launch over 2D output tiles (16 x 16 up to
//     64 x 64 by level size).  Synthesis tiles, and analysis tiles of the
//     largest size, filter in two passes: the first reads its lines straight
//     from global memory, the second reads the once-filtered block from LDS.
//     Smaller analysis tiles load their whole input window into LDS first.
//   * The last synthesis level writes xi^T (the layout the column pass reads);
//     the first analysis level reads xi'^T (the layout the adjoint column pass
//     writes) and stores the detail bands straight into x.
#include "dwt_lines.h"

namespace wh2wav_fast {
namespace {

using namespace lines;


// Largest input window (coefficients per direction) of an analysis tile:
// 2 TH + 2nu - 1 inside; at most 2 TH + 3nu at an end when TH < nu.
template <int NU, int TH>
__host__ __device__ constexpr int analysis_window_max() {
  return NU <= TH ? 2 * TH + 2 * NU + 4 : 2 * TH + 3 * NU;
}

// Tile t of an n x n grid: the ring of tiles along the edges (which hold the
// boundary functions and take longest) is dispatched first.
__device__ __forceinline__ void tile_of(int t, int n, int& tr, int& tc) {
  if (n <= 2) {
    tr = t / n;
    tc = t % n;
    return;
  }
  const int E = 4 * n - 4;
  if (t < n) {
    tr = 0, tc = t;
  } else if (t < 2 * n) {
    tr = n - 1, tc = t - n;
  } else if (t < 3 * n - 2) {
    tr = t - 2 * n + 1, tc = 0;
  } else if (t < E) {
    tr = t - (3 * n - 2) + 1, tc = n - 1;
  } else {
    const int r = t - E;
    tr = 1 + r / (n - 2), tc = 1 + r % (n - 2);
  }
}

// ---------------------------------------------------------- tiled levels
// Analysis level k: input xi (size x size; trans: read in^T); output quadrants:
// LL -> ll[a][b], other bands -> det[row][col].  Tile: TH x TH outputs in each
// of the four quadrants at the same (a0, b0); 256 threads; runs of P outputs.
template <typename T, int NU, int TH, int P, bool PER>
__global__ void __launch_bounds__(256) k_analysis2d_tile(const T* __restrict__ in, int64_t ld_in, int trans,
                                                         T* __restrict__ ll, int64_t ld_ll, T* __restrict__ det,
                                                         int64_t ld_det, int k, Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  TileLds<T> tl;
  const int half = 1 << k;
  const int ntile = half / TH;
  int tr, tc;
  tile_of(int(blockIdx.x), ntile, tr, tc);
  const int a0 = tr * TH, b0 = tc * TH;
  int rlo, rhi, clo, chi;
  if constexpr (PER) {
    analysis_input_range_per<NU>(a0, a0 + TH, rlo, rhi);
    analysis_input_range_per<NU>(b0, b0 + TH, clo, chi);
  } else {
    analysis_input_range<NU>(a0, a0 + TH, half, rlo, rhi);
    analysis_input_range<NU>(b0, b0 + TH, half, clo, chi);
  }
  const int nr = rhi - rlo + 1, nc = chi - clo + 1;
  const int W = nc + 1;
  constexpr int YW = 2 * TH + 1;
  T* Xs = reinterpret_cast<T*>(smem_raw);   // nr x W
  T* Ys = Xs + nr * W;                        // nr x YW: a columns then d columns
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
  {
    // outer index over waves, inner over lanes (the contiguous direction of `in`)
    constexpr int MAXR = analysis_window_max<NU, TH>(), OI = (MAXR + 3) / 4, IJ = (MAXR + 63) / 64;
    const int no = trans ? nc : nr, ni = trans ? nr : nc;
    const int64_t ob = trans ? clo : rlo, ib = trans ? rlo : clo;
    T r[OI][IJ];
#pragma unroll
    for (int u = 0; u < OI; ++u) {
      const int a = wave + 4 * u;
#pragma unroll
      for (int v = 0; v < IJ; ++v) {
        const int b = lane + 64 * v;
        // unconditional load (the window's first element when outside it), so
        // that all loads are in flight together; the periodic extension
        // takes the indices modulo the level's size (the window stays
        // unwrapped in LDS, so every run below reads it as an interior run)
        const bool inside = a < no && b < ni;
        int64_t oa = ob + (inside ? a : 0), ibb = ib + (inside ? b : 0);
        if constexpr (PER) oa &= 2 * half - 1, ibb &= 2 * half - 1;
        const T val = in[oa * ld_in + ibb];
        r[u][v] = inside ? val : T(0);
      }
    }
    // the tables load while the window loads are in flight
    tl = load_tables<T, NU>(t, tab_lds, hr, gr);
#pragma unroll
    for (int u = 0; u < OI; ++u) {
      const int a = wave + 4 * u;
#pragma unroll
      for (int v = 0; v < IJ; ++v) {
        const int b = lane + 64 * v;
        if (a < no && b < ni) {
          if (trans)
            Xs[b * W + a] = r[u][v];
          else
            Xs[a * W + b] = r[u][v];
        }
      }
    }
  }
  __syncthreads();
  constexpr int RUNS = TH / P;
  // rows: work item = (window row, run of P outputs m)
  for (int item = int(threadIdx.x); item < nr * RUNS; item += 256) {
    const int i2 = item % nr, u = item / nr;
    const T* xr = Xs + i2 * W;
    const int m0 = b0 + u * P;
    T* yr = Ys + i2 * YW + u * P;
    if (PER || (m0 >= NU && m0 + P - 1 < half - NU)) {
      T a[P], d[P];
      analysis_run<T, NU, P>(xr + 2 * m0 - NU + 1 - clo, 1, hr, gr, a, d);
#pragma unroll
      for (int p = 0; p < P; ++p) yr[p] = a[p], yr[TH + p] = d[p];
    } else {
      T a[P], d[P];
      analysis_run_edge<T, NU, P>(xr, 1, clo, chi, m0, half, hr, gr, tl.sLs, tl.sRs, a, d);
#pragma unroll
      for (int p = 0; p < P; ++p) yr[p] = a[p], yr[TH + p] = d[p];
    }
  }
  __syncthreads();
  // columns: work item = (output column of the a|d row, run of P outputs)
  T* Os = Xs;  // (2 TH) x YW
  for (int item = int(threadIdx.x); item < 2 * TH * RUNS; item += 256) {
    const int oc = item % (2 * TH), u = item / (2 * TH);
    const int m0 = a0 + u * P;
    if (PER || (m0 >= NU && m0 + P - 1 < half - NU)) {
      T a[P], d[P];
      analysis_run<T, NU, P>(Ys + (2 * m0 - NU + 1 - rlo) * YW + oc, YW, hr, gr, a, d);
#pragma unroll
      for (int p = 0; p < P; ++p) Os[(u * P + p) * YW + oc] = a[p], Os[(TH + u * P + p) * YW + oc] = d[p];
    } else {
      T a[P], d[P];
      analysis_run_edge<T, NU, P>(Ys + oc, YW, rlo, rhi, m0, half, hr, gr, tl.sLs, tl.sRs, a, d);
#pragma unroll
      for (int p = 0; p < P; ++p) Os[(u * P + p) * YW + oc] = a[p], Os[(TH + u * P + p) * YW + oc] = d[p];
    }
  }
  __syncthreads();
  for (int rr = wave; rr < 2 * TH; rr += 4) {
    const int o = rr < TH ? a0 + rr : half + a0 + (rr - TH);
    for (int oc = lane; oc < 2 * TH; oc += 64) {
      const int col = oc < TH ? b0 + oc : half + b0 + (oc - TH);
      const T v = Os[rr * YW + oc];
      if (o < half && col < half)
        ll[int64_t(o) * ld_ll + col] = v;
      else
        det[int64_t(o) * ld_det + col] = v;
    }
  }
}

// ------------------------------------------------- direct (two-pass) tiles
// The first filter pass reads its input lines straight from global memory:
// each thread owns one line of the window in the contiguous direction of the
// array (lanes over consecutive columns) and walks it with the row stride.
// Only the once-filtered block goes through LDS, where the second pass reads
// it along the other direction.  Synthesis filters the columns first (S X,
// then (S X) S^T); analysis filters along the array's rows index first.

// Synthesis level k: X[r][c] = (r < half && c < half) ? ll[r][c] : det[r][c]
// (ll and det share the row stride ld); out = S X S^T (trans: out^T).  Tile:
// TS x TS outputs, 256 threads, runs of P output pairs.
template <typename T, int NU, int TS, int P, bool PER>
__global__ void __launch_bounds__(256) k_synth2d_direct(const T* __restrict__ ll, const T* __restrict__ det,
                                                        int64_t ld, T* __restrict__ out, int64_t ld_out, int k,
                                                        int trans, Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const int half = 1 << k, size = 2 * half;
  const int ntile = size / TS;
  int tr, tc;
  tile_of(int(blockIdx.x), ntile, tr, tc);
  const int r0 = tr * TS, c0 = tc * TS;
  int rlo, rhi, clo, chi;
  if constexpr (PER) {
    synth_input_range_per<NU>(r0, r0 + TS, rlo, rhi);
    synth_input_range_per<NU>(c0, c0 + TS, clo, chi);
  } else {
    synth_input_range<NU>(r0, r0 + TS, half, rlo, rhi);
    synth_input_range<NU>(c0, c0 + TS, half, clo, chi);
  }
  const int nc = chi - clo + 1, W2 = 2 * nc;
  const int YW = W2 + 1;                      // odd: conflict-free in both directions
  T* Ys = reinterpret_cast<T*>(smem_raw);     // TS x YW: column-filtered rows r0 .. r0+TS-1
  const TileLds<T> tl = load_tables<T, NU>(t, tab_lds, hr, gr);
  // tiles whose rows reach a boundary read the boundary blocks from LDS
  if (!PER && !(pair_is_interior<NU>(r0 >> 1, half) && pair_is_interior<NU>((r0 >> 1) + TS / 2 - 1, half)))
    __syncthreads();
  constexpr int RUNS = TS / (2 * P), LO = synth_lo<NU>(), HI = synth_hi<NU>(), NT = 256;
  // pass 1, columns: item = (window column j, run u of P output row pairs);
  // the periodic extension reads window column clo + j modulo half, and a
  // run that crosses an end reads its rows modulo half
  for (int item = int(threadIdx.x); item < W2 * RUNS; item += NT) {
    const int j = item % W2, u = item / W2;
    const int col = PER ? (j < nc ? ((clo + j) & (half - 1)) : half + ((clo + j - nc) & (half - 1)))
                        : (j < nc ? clo + j : half + clo + (j - nc));
    const T* ca = (col < half ? ll : det) + col;  // rows 0 .. half-1
    const T* cd = det + int64_t(half) * ld + col;  // rows half .. size-1
    const int i0 = (r0 >> 1) + u * P;
    T e[P], o[P];
    if constexpr (PER) {
      if (i0 + LO >= 0 && i0 + P - 1 + HI <= half - 1) {
        const int64_t off = int64_t(i0 + LO) * ld;
        synth_run<T, NU, P>(ca + off, cd + off, int(ld), hr, gr, e, o);
      } else {
        synth_run_wrap<T, NU, P>(ca, cd, int(ld), i0, half, hr, gr, e, o);
      }
    } else if (pair_is_interior<NU>(i0, half) && pair_is_interior<NU>(i0 + P - 1, half)) {
      const int64_t off = int64_t(i0 + LO) * ld;
      synth_run<T, NU, P>(ca + off, cd + off, int(ld), hr, gr, e, o);
    } else {
      const int64_t off = int64_t(rlo) * ld;
      // FP64 keeps its registers: there the hoisted loads cost a wave per SIMD
      synth_run_edge<T, NU, P, (P <= 2 && sizeof(T) == 4)>(ca + off, cd + off, int(ld), rlo, rhi, i0, half, hr, gr,
                                                           tl.sLs, tl.sRs, e, o);
    }
    T* yc = Ys + 2 * u * P * YW + j;
#pragma unroll
    for (int p = 0; p < P; ++p) yc[2 * p * YW] = e[p], yc[(2 * p + 1) * YW] = o[p];
  }
  __syncthreads();
  // pass 2, rows: item = (output row r, run u of P output column pairs), at
  // most one per thread.  The transposed output is written straight from
  // registers with lanes over r (consecutive addresses).  Otherwise, with
  // short runs, lanes run over u (each row segment written by consecutive
  // lanes); with long runs the tile is staged in LDS and written row by row.
  static_assert(TS * RUNS <= NT, "one row item per thread");
  constexpr bool STAGE = P >= 4;
  const int item = int(threadIdx.x);
  const bool rfast = trans || STAGE;
  const int r = rfast ? item % TS : item / RUNS, u = rfast ? item / TS : item % RUNS;
  T e[P], o[P];
  if (item < TS * RUNS) {
    const T* yr = Ys + r * YW;
    const int i0 = (c0 >> 1) + u * P;
    if (PER || (pair_is_interior<NU>(i0, half) && pair_is_interior<NU>(i0 + P - 1, half)))
      synth_run<T, NU, P>(yr + i0 + LO - clo, yr + nc + i0 + LO - clo, 1, hr, gr, e, o);
    else
      synth_run_edge<T, NU, P>(yr, yr + nc, 1, clo, chi, i0, half, hr, gr, tl.sLs, tl.sRs, e, o);
  }
  if (trans) {
    if (item < TS * RUNS) {
      const int rr = r0 + r, cc = c0 + 2 * u * P;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        out[int64_t(cc + 2 * p) * ld_out + rr] = e[p];
        out[int64_t(cc + 2 * p + 1) * ld_out + rr] = o[p];
      }
    }
    return;
  }
  if constexpr (!STAGE) {
    if (item < TS * RUNS) {
      T* orow = out + int64_t(r0 + r) * ld_out + c0 + 2 * u * P;
#pragma unroll
      for (int p = 0; p < P; ++p) orow[2 * p] = e[p], orow[2 * p + 1] = o[p];
    }
    return;
  }
  constexpr int OW = TS + 1;
  T* Os = Ys;  // TS x OW, fits in Ys (2 nc >= TS)
  __syncthreads();
  if (item < TS * RUNS) {
#pragma unroll
    for (int p = 0; p < P; ++p) Os[r * OW + 2 * u * P + 2 * p] = e[p], Os[r * OW + 2 * u * P + 2 * p + 1] = o[p];
  }
  __syncthreads();
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
  for (int rr = wave; rr < TS; rr += NT / 64)
    for (int cc = lane; cc < TS; cc += 64) out[int64_t(r0 + rr) * ld_out + c0 + cc] = Os[rr * OW + cc];
}

// Analysis level k.  The filters run in the frame of the input array: G =
// S^T in S when trans = 0, and G = S^T in S with in holding xi^T when trans =
// 1, so that the coefficients are G^T (quadrants LH and HL exchange).  Tile:
// TH x TH outputs in each quadrant of G at (A0, B0), 256 threads, runs of P.
template <typename T, int NU, int TH, int P, bool PER>
__global__ void __launch_bounds__(256) k_analysis2d_direct(const T* __restrict__ in, int64_t ld_in, int trans,
                                                           T* __restrict__ ll, int64_t ld_ll, T* __restrict__ det,
                                                           int64_t ld_det, int k, Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const int half = 1 << k;
  const int ntile = half / TH;
  int tr, tc;
  tile_of(int(blockIdx.x), ntile, tr, tc);
  const int A0 = tr * TH, B0 = tc * TH;
  int plo, phi, qlo, qhi;
  if constexpr (PER) {
    analysis_input_range_per<NU>(A0, A0 + TH, plo, phi);
    analysis_input_range_per<NU>(B0, B0 + TH, qlo, qhi);
  } else {
    analysis_input_range<NU>(A0, A0 + TH, half, plo, phi);
    analysis_input_range<NU>(B0, B0 + TH, half, qlo, qhi);
  }
  const int nq = qhi - qlo + 1;
  const int YW = nq + 1;
  T* Ys = reinterpret_cast<T*>(smem_raw);  // 2TH x YW: a rows, then d rows
  const TileLds<T> tl = load_tables<T, NU>(t, tab_lds, hr, gr);
  // tiles whose rows reach a boundary read the boundary blocks from LDS
  if (!PER && !(A0 >= NU && A0 + TH - 1 < half - NU)) __syncthreads();
  constexpr int RUNS = TH / P, NT = 256;
  const int size = 2 * half;
  // pass 1, along the row index of `in`: item = (window column jq, run u);
  // the periodic extension reads window column qlo + jq modulo size, and a
  // run that crosses an end reads its rows modulo size
  for (int item = int(threadIdx.x); item < nq * RUNS; item += NT) {
    const int jq = item % nq, u = item / nq;
    const T* cx = in + (PER ? ((qlo + jq) & (size - 1)) : qlo + jq);
    const int m0 = A0 + u * P;
    T a[P], d[P];
    if (PER && !(2 * m0 - NU + 1 >= 0 && 2 * (m0 + P - 1) + NU <= size - 1))
      analysis_run_wrap<T, NU, P>(cx, int(ld_in), m0, size, hr, gr, a, d);
    else if (PER || (m0 >= NU && m0 + P - 1 < half - NU))
      analysis_run<T, NU, P>(cx + int64_t(2 * m0 - NU + 1) * ld_in, int(ld_in), hr, gr, a, d);
    else
      analysis_run_edge<T, NU, P>(cx + int64_t(plo) * ld_in, int(ld_in), plo, phi, m0, half, hr, gr, tl.sLs,
                                  tl.sRs, a, d);
    T* yc = Ys + u * P * YW + jq;
#pragma unroll
    for (int p = 0; p < P; ++p) yc[p * YW] = a[p], yc[(TH + p) * YW] = d[p];
  }
  __syncthreads();
  // pass 2, along the column index: item = (Ys row rho, run u), at most one
  // per thread.  The result G[g_r][g_c] is coefficient (g_r, g_c) (trans = 0)
  // or (g_c, g_r) (trans = 1).  Lanes run over rho: the transposed case is
  // written straight from registers (consecutive addresses); otherwise the
  // four TH x TH blocks are staged in LDS and written row by row.
  static_assert(2 * TH * RUNS <= NT, "one row item per thread");
  const int item = int(threadIdx.x);
  const int rho = item % (2 * TH), u = item / (2 * TH);
  const int m0 = B0 + u * P;
  T a[P], d[P];
  if (item < 2 * TH * RUNS) {
    const T* yr = Ys + rho * YW;
    if (PER || (m0 >= NU && m0 + P - 1 < half - NU))
      analysis_run<T, NU, P>(yr + 2 * m0 - NU + 1 - qlo, 1, hr, gr, a, d);
    else
      analysis_run_edge<T, NU, P>(yr, 1, qlo, qhi, m0, half, hr, gr, tl.sLs, tl.sRs, a, d);
  }
  const int g_r = rho < TH ? A0 + rho : half + A0 + (rho - TH);
  if (trans) {
    if (item < 2 * TH * RUNS) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int part = 0; part < 2; ++part) {
          const int g_c = (part ? half : 0) + m0 + p;
          const T v = part ? d[p] : a[p];
          if (g_c < half && g_r < half)
            ll[int64_t(g_c) * ld_ll + g_r] = v;
          else
            det[int64_t(g_c) * ld_det + g_r] = v;
        }
      }
    }
    return;
  }
  constexpr int OW = 2 * TH + 1;
  T* Os = Ys;  // 2TH x OW: a columns then d columns; fits in Ys (nq >= 2 TH)
  __syncthreads();
  if (item < 2 * TH * RUNS) {
#pragma unroll
    for (int p = 0; p < P; ++p) Os[rho * OW + u * P + p] = a[p], Os[rho * OW + TH + u * P + p] = d[p];
  }
  __syncthreads();
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
  for (int rr = wave; rr < 2 * TH; rr += NT / 64) {
    const int orow = rr < TH ? A0 + rr : half + A0 + (rr - TH);
    for (int oc = lane; oc < 2 * TH; oc += 64) {
      const int ocol = oc < TH ? B0 + oc : half + B0 + (oc - TH);
      const T v = Os[rr * OW + oc];
      if (orow < half && ocol < half)
        ll[int64_t(orow) * ld_ll + ocol] = v;
      else
        det[int64_t(orow) * ld_det + ocol] = v;
    }
  }
}

// ---------------------------------------------------------- coarse levels
// One workgroup: levels j0 .. kc-1 (output block 2^kc) with the block in LDS.
// Input x (quadtree, row stride ld_x).  Output: the 2^kc block into out
// (trans: transposed).
template <typename T, int NU, bool PER>
__global__ void __launch_bounds__(1024) k_synth2d_coarse(const T* __restrict__ x, int64_t ld_x, T* __restrict__ out,
                                                         int64_t ld_out, int j0, int kc, int trans, Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const TileLds<T> tl = load_tables<T, NU>(t, tab_lds, hr, gr);
  const int S = 1 << kc, P = S + 1;
  T* blk = reinterpret_cast<T*>(smem_raw);  // S x P
  T* tmp = blk + S * P;
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;  // 16 waves
  for (int i0 = 0; i0 < S; i0 += 128) {  // 8 rows per wave per batch, loads first
    T r[8][2];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int i = i0 + wave + 16 * u, c = lane + 64 * v;
        r[u][v] = (i < S && c < S) ? x[int64_t(i) * ld_x + c] : T(0);
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int i = i0 + wave + 16 * u, c = lane + 64 * v;
        if (i < S && c < S) blk[i * P + c] = r[u][v];
      }
  }
  __syncthreads();
  constexpr int CP = 2, LO = synth_lo<NU>(), HI = synth_hi<NU>();
  // the periodic extension: runs that cross an end read modulo half
  auto wraps = [&](int i0, int half) { return i0 + LO < 0 || i0 + CP - 1 + HI > half - 1; };
  for (int k = j0; k < kc; ++k) {
    const int half = 1 << k, size = 2 * half;
    const int runs = (half + CP - 1) / CP;
    // rows: work item = (row, run of CP output pairs); consecutive lanes take consecutive rows
    for (int item = int(threadIdx.x); item < size * runs; item += 1024) {
      const int i = item % size, i0 = (item / size) * CP;
      const T* xr = blk + i * P;
      T* yr = tmp + i * P + 2 * i0;
      if (PER && half < CP) {
        T e[1], o[1];
        synth_run_wrap<T, NU, 1>(xr, xr + half, 1, i0, half, hr, gr, e, o);
        yr[0] = e[0], yr[1] = o[0];
      } else if (PER && wraps(i0, half)) {
        T e[CP], o[CP];
        synth_run_wrap<T, NU, CP>(xr, xr + half, 1, i0, half, hr, gr, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) yr[2 * p] = e[p], yr[2 * p + 1] = o[p];
      } else if (PER || (pair_is_interior<NU>(i0, half) && pair_is_interior<NU>(i0 + CP - 1, half))) {
        T e[CP], o[CP];
        synth_run<T, NU, CP>(xr + i0 + LO, xr + half + i0 + LO, 1, hr, gr, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) yr[2 * p] = e[p], yr[2 * p + 1] = o[p];
      } else if (half >= CP) {
        T e[CP], o[CP];
        synth_run_edge<T, NU, CP>(xr, xr + half, 1, 0, half - 1, i0, half, hr, gr, tl.sLs, tl.sRs, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) yr[2 * p] = e[p], yr[2 * p + 1] = o[p];
      } else {
        auto A = [&](int m) { return xr[m]; };
        auto D = [&](int m) { return xr[half + m]; };
        for (int p = 0; p < CP && i0 + p < half; ++p) {
          yr[2 * p] = synth_at<T, NU>(2 * (i0 + p), half, tl.hs, tl.gs, tl.sLs, tl.sRs, A, D);
          yr[2 * p + 1] = synth_at<T, NU>(2 * (i0 + p) + 1, half, tl.hs, tl.gs, tl.sLs, tl.sRs, A, D);
        }
      }
    }
    __syncthreads();
    // columns: work item = (column, run of CP output row pairs)
    for (int item = int(threadIdx.x); item < size * runs; item += 1024) {
      const int c = item % size, i0 = (item / size) * CP;
      T* oc = blk + 2 * i0 * P + c;
      if (PER && half < CP) {
        T e[1], o[1];
        synth_run_wrap<T, NU, 1>(tmp + c, tmp + half * P + c, P, i0, half, hr, gr, e, o);
        oc[0] = e[0], oc[P] = o[0];
      } else if (PER && wraps(i0, half)) {
        T e[CP], o[CP];
        synth_run_wrap<T, NU, CP>(tmp + c, tmp + half * P + c, P, i0, half, hr, gr, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) oc[2 * p * P] = e[p], oc[(2 * p + 1) * P] = o[p];
      } else if (PER || (pair_is_interior<NU>(i0, half) && pair_is_interior<NU>(i0 + CP - 1, half))) {
        T e[CP], o[CP];
        synth_run<T, NU, CP>(tmp + (i0 + LO) * P + c, tmp + (half + i0 + LO) * P + c, P, hr, gr, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) oc[2 * p * P] = e[p], oc[(2 * p + 1) * P] = o[p];
      } else if (half >= CP) {
        T e[CP], o[CP];
        synth_run_edge<T, NU, CP>(tmp + c, tmp + half * P + c, P, 0, half - 1, i0, half, hr, gr, tl.sLs, tl.sRs, e, o);
#pragma unroll
        for (int p = 0; p < CP; ++p) oc[2 * p * P] = e[p], oc[(2 * p + 1) * P] = o[p];
      } else {
        auto A = [&](int m) { return tmp[m * P + c]; };
        auto D = [&](int m) { return tmp[(half + m) * P + c]; };
        for (int p = 0; p < CP && i0 + p < half; ++p) {
          oc[2 * p * P] = synth_at<T, NU>(2 * (i0 + p), half, tl.hs, tl.gs, tl.sLs, tl.sRs, A, D);
          oc[(2 * p + 1) * P] = synth_at<T, NU>(2 * (i0 + p) + 1, half, tl.hs, tl.gs, tl.sLs, tl.sRs, A, D);
        }
      }
    }
    __syncthreads();
  }
  for (int i = wave; i < S; i += 16)
    for (int c = lane; c < S; c += 64)
      out[int64_t(i) * ld_out + c] = trans ? blk[c * P + i] : blk[i * P + c];
}

// One workgroup: analysis levels kc-1 down to j0 on the 2^kc block read from
// in (trans: in^T); writes the whole 2^kc block of the quadtree into x.
template <typename T, int NU, bool PER>
__global__ void __launch_bounds__(1024) k_analysis2d_coarse(const T* __restrict__ in, int64_t ld_in, int trans,
                                                            T* __restrict__ x, int64_t ld_x, int j0, int kc,
                                                            Tables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const TileLds<T> tl = load_tables<T, NU>(t, tab_lds, hr, gr);
  const int S = 1 << kc, P = S + 1;
  T* blk = reinterpret_cast<T*>(smem_raw);
  T* tmp = blk + S * P;
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
  for (int i0 = 0; i0 < S; i0 += 128) {
    T r[8][2];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int i = i0 + wave + 16 * u, c = lane + 64 * v;
        r[u][v] = (i < S && c < S) ? in[int64_t(i) * ld_in + c] : T(0);
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int i = i0 + wave + 16 * u, c = lane + 64 * v;
        if (i < S && c < S) {
          if (trans)
            blk[c * P + i] = r[u][v];
          else
            blk[i * P + c] = r[u][v];
        }
      }
  }
  __syncthreads();
  constexpr int CP = 2;
  // the periodic extension: runs that cross an end read modulo size
  auto wraps = [&](int m0, int size) { return 2 * m0 - NU + 1 < 0 || 2 * (m0 + CP - 1) + NU > size - 1; };
  for (int k = kc - 1; k >= j0; --k) {
    const int half = 1 << k, size = 2 * half;
    const int runs = (half + CP - 1) / CP;
    // rows: work item = (row, run of CP outputs m)
    for (int item = int(threadIdx.x); item < size * runs; item += 1024) {
      const int i = item % size, m0 = (item / size) * CP;
      const T* xr = blk + i * P;
      T* yr = tmp + i * P + m0;
      if (PER && half < CP) {
        T a[1], d[1];
        analysis_run_wrap<T, NU, 1>(xr, 1, m0, size, hr, gr, a, d);
        yr[0] = a[0], yr[half] = d[0];
      } else if (PER && wraps(m0, size)) {
        T a[CP], d[CP];
        analysis_run_wrap<T, NU, CP>(xr, 1, m0, size, hr, gr, a, d);
#pragma unroll
        for (int p = 0; p < CP; ++p) yr[p] = a[p], yr[half + p] = d[p];
      } else if (PER || (m0 >= NU && m0 + CP - 1 < half - NU)) {
        T a[CP], d[CP];
        analysis_run<T, NU, CP>(xr + 2 * m0 - NU + 1, 1, hr, gr, a, d);
#pragma unroll
        for (int p = 0; p < CP; ++p) yr[p] = a[p], yr[half + p] = d[p];
      } else if (half >= CP) {
        T a[CP], d[CP];
        analysis_run_edge<T, NU, CP>(xr, 1, 0, size - 1, m0, half, hr, gr, tl.sLs, tl.sRs, a, d);
#pragma unroll
        for (int p = 0; p < CP; ++p) yr[p] = a[p], yr[half + p] = d[p];
      } else {
        auto X = [&](int n) { return xr[n]; };
        for (int p = 0; p < CP && m0 + p < half; ++p) {
          yr[p] = analysis_at<T, NU>(m0 + p, half, tl.hs, tl.gs, tl.sLs, tl.sRs, X);
          yr[half + p] = analysis_at<T, NU>(half + m0 + p, half, tl.hs, tl.gs, tl.sLs, tl.sRs, X);
        }
      }
    }
    __syncthreads();
    // columns: work item = (column, run of CP outputs)
    for (int item = int(threadIdx.x); item < size * runs; item += 1024) {
      const int c = item % size, m0 = (item / size) * CP;
      if (PER && half < CP) {
        T a[1], d[1];
        analysis_run_wrap<T, NU, 1>(tmp + c, P, m0, size, hr, gr, a, d);
        blk[m0 * P + c] = a[0], blk[(half + m0) * P + c] = d[0];
      } else if (PER && wraps(m0, size)) {
        T a[CP], d[CP];
        analysis_run_wrap<T, NU, CP>(tmp + c, P, m0, size, hr, gr, a, d);
#pragma unroll
        for (int p = 0; p < CP; ++p) blk[(m0 + p) * P + c] = a[p], blk[(half + m0 + p) * P + c] = d[p];
      } else if (PER || (m0 >= NU && m0 + CP - 1 < half - NU)) {
        T a[CP], d[CP];
        analysis_run<T, NU, CP>(tmp + (2 * m0 - NU + 1) * P + c, P, hr, gr, a, d);
#pragma unroll
        for (int p = 0; p < CP; ++p) blk[(m0 + p) * P + c] = a[p], blk[(half + m0 + p) * P + c] = d[p];
      } else if (half >= CP) {
        T a[CP], d[CP];
        analysis_run_edge<T, NU, CP>(tmp + c, P, 0, size - 1, m0, half, hr, gr, tl.sLs, tl.sRs, a, d);
#pragma unroll
        for (int p = 0; p < CP; ++p) blk[(m0 + p) * P + c] = a[p], blk[(half + m0 + p) * P + c] = d[p];
      } else {
        auto X = [&](int n) { return tmp[n * P + c]; };
        for (int p = 0; p < CP && m0 + p < half; ++p) {
          blk[(m0 + p) * P + c] = analysis_at<T, NU>(m0 + p, half, tl.hs, tl.gs, tl.sLs, tl.sRs, X);
          blk[(half + m0 + p) * P + c] = analysis_at<T, NU>(half + m0 + p, half, tl.hs, tl.gs, tl.sLs, tl.sRs, X);
        }
      }
    }
    __syncthreads();
  }
  for (int i = wave; i < S; i += 16)
    for (int c = lane; c < S; c += 64) x[int64_t(i) * ld_x + c] = blk[i * P + c];
}

// log2 of the largest block the one-workgroup kernel handles, for a j-level
// transform.  With nu <= 4 the levels up to a 64 x 64 output cost less in one
// workgroup than as a launch each (db4, 512^2: 78 -> 73 us per FP32 pair,
// 95 -> 89 us per FP64 pair), and an FP32 transform of at most 128 x 128 runs
// whole in one launch; the 128 x 128 level of a larger array is faster as a
// tile launch.  With nu > 4 the boundary rows fill most of the small levels
// and every level with a 16 x 16 or larger output runs as a tile launch.  The
// kernel's loads take blocks of at most 128 columns, and its LDS (two
// padded blocks) holds 128 x 128 in FP32, 64 x 64 in FP64.
template <typename T, int NU>
constexpr int coarse_limit(int j) {
  if (NU > 4) return 3;
  return sizeof(T) == 4 && j <= 7 ? 7 : 6;
}

// Largest input window (rows of one half) over the tiles of a level, from
// the same range functions the kernels use.
template <int NU, bool PER>
int max_synth_window(int half, int ts) {
  int w = 0;
  for (int n0 = 0; n0 < 2 * half; n0 += ts) {
    int lo, hi;
    if (PER)
      synth_input_range_per<NU>(n0, n0 + ts, lo, hi);
    else
      synth_input_range<NU>(n0, n0 + ts, half, lo, hi);
    w = hi - lo + 1 > w ? hi - lo + 1 : w;
  }
  return w;
}
template <int NU, bool PER>
int max_analysis_window(int half, int th) {
  int w = 0;
  for (int m0 = 0; m0 < half; m0 += th) {
    int lo, hi;
    if (PER)
      analysis_input_range_per<NU>(m0, m0 + th, lo, hi);
    else
      analysis_input_range<NU>(m0, m0 + th, half, lo, hi);
    w = hi - lo + 1 > w ? hi - lo + 1 : w;
  }
  return w;
}

// Tile shape (outputs per side) and run length per level, from per-level
// timings of every candidate: large tiles with long register runs where a
// level has enough tiles to fill the chip; on the small, latency-bound levels
// 16-point synthesis and 8-point analysis tiles, with single-output runs where
// those are faster.  A tile is at least nu wide: the window ranges assume
// that the outputs which read one end's boundary block lie in the tiles that
// reach that end.
struct TileShape {
  int t, p;
};
template <typename T>
constexpr TileShape synth_shape(int size) {
  if (sizeof(T) == 4 && size >= 2048) return {64, 8};
  if (size >= (sizeof(T) == 4 ? 512 : 1024)) return {32, 2};
  return {16, size == 32 ? 1 : 2};
}
template <typename T>
constexpr TileShape analysis_shape(int half, int nu) {
  TileShape s{8, 1};
  if (sizeof(T) == 4 && half >= 1024)
    s = {32, 8};
  else if (half >= 512)
    s = {16, 2};
  else if (sizeof(T) == 4 && half == 256)
    s = {8, 2};
  return s.t < nu ? TileShape{16, 2} : s;
}

template <typename T, int NU, bool PER, int TS, int P>
hipError_t launch_synth_direct(const T* ll, const T* det, T* dst, int64_t M, int k, int trans, const Tables<T>& t,
                               hipStream_t st) {
  const int half = 1 << k, size = 2 * half;
  if (size % TS || TS < NU) return hipErrorInvalidValue;
  const int nc = max_synth_window<NU, PER>(half, TS);
  const size_t smem = size_t(TS) * (2 * nc + 1) * sizeof(T);
  const int ntile = size / TS;
  hipLaunchKernelGGL((k_synth2d_direct<T, NU, TS, P, PER>), dim3(unsigned(ntile * ntile)), dim3(256), smem, st, ll,
                     det, M, dst, M, k, trans, t);
  return hipGetLastError();
}

template <typename T, int NU, bool PER, int TH, int P>
hipError_t launch_analysis_direct(const T* src, int trans, T* dst, T* x, int64_t M, int k, const Tables<T>& t,
                                  hipStream_t st) {
  const int half = 1 << k;
  if (half % TH || TH < NU) return hipErrorInvalidValue;
  const int nq = max_analysis_window<NU, PER>(half, TH);
  const size_t smem = size_t(2 * TH) * (nq + 1) * sizeof(T);
  const int ntile = half / TH;
  hipLaunchKernelGGL((k_analysis2d_direct<T, NU, TH, P, PER>), dim3(unsigned(ntile * ntile)), dim3(256), smem, st,
                     src, M, trans, dst, M, x, M, k, t);
  return hipGetLastError();
}

template <typename T, int NU, bool PER, int TH, int P>
hipError_t launch_analysis(const T* src, int trans, T* dst, T* x, int64_t M, int k, const Tables<T>& t,
                           hipStream_t st) {
  const int half = 1 << k;
  if (half % TH || TH < NU) return hipErrorInvalidValue;
  const int nr = max_analysis_window<NU, PER>(half, TH);
  if (nr > analysis_window_max<NU, TH>()) return hipErrorInvalidValue;  // the kernel's load window
  const size_t smem = (size_t(nr) * (nr + 1) + size_t(nr) * (2 * TH + 1)) * sizeof(T);
  const int ntile = half / TH;
  hipLaunchKernelGGL((k_analysis2d_tile<T, NU, TH, P, PER>), dim3(unsigned(ntile * ntile)), dim3(256), smem, st, src,
                     M, trans, dst, M, x, M, k, t);
  return hipGetLastError();
}

// No wavelet level (j0 == j): the coefficients are the scaling coefficients
// themselves; `out` = `in` transposed (the layout the line passes use).
template <typename T, int NU>
hipError_t copy_transposed(const T* in, T* out, int64_t M, int j, const Tables<T>& t, hipStream_t st) {
  if (M >= 32) return transpose<T>(in, out, M, st);
  const size_t smem = 2 * size_t(M) * (M + 1) * sizeof(T);
  hipLaunchKernelGGL((k_synth2d_coarse<T, NU, false>), dim3(1), dim3(1024), smem, st, in, M, out, M, j, j, 1, t);
  return hipGetLastError();
}

// PER: the periodic extension (indices modulo each level's size, no
// boundary functions) in the same kernels.
template <typename T, int NU, bool PER>
hipError_t idwt2d_impl(const T* x, T* outT, T* s0, T* s1, int64_t M, int j0, int j, const Tables<T>& t,
                       hipStream_t st) {
  if (j0 == j) return copy_transposed<T, NU>(x, outT, M, j, t, st);
  // Coarse levels in one workgroup, unless the coarsest block is already too
  // large for LDS (then the first tiled level reads LL_{j0} from x).
  const bool coarse = j0 < coarse_limit<T, NU>(j);
  const int kc = coarse ? (j < coarse_limit<T, NU>(j) ? j : coarse_limit<T, NU>(j)) : j0;
  const bool last = kc == j;
  hipError_t e = hipSuccess;
  if (coarse) {
    const int S = 1 << kc;
    const size_t smem_c = 2 * size_t(S) * (S + 1) * sizeof(T);
    T* prev = last ? outT : s0;
    hipLaunchKernelGGL((k_synth2d_coarse<T, NU, PER>), dim3(1), dim3(1024), smem_c, st, x, M, prev, M, j0, kc,
                       last ? 1 : 0, t);
    e = hipGetLastError();
    if (e != hipSuccess || last) return e;
  }
  const T* ll = coarse ? s0 : x;
  for (int k = kc; k < j; ++k) {
    const bool fin = k == j - 1;
    T* dst = fin ? outT : (ll == s0 ? s1 : s0);
    const TileShape sh = synth_shape<T>(2 << k);
    if (sh.t == 64)
      e = launch_synth_direct<T, NU, PER, 64, 8>(ll, x, dst, M, k, fin ? 1 : 0, t, st);
    else if (sh.t == 32)
      e = launch_synth_direct<T, NU, PER, 32, 2>(ll, x, dst, M, k, fin ? 1 : 0, t, st);
    else if (sh.p == 1)
      e = launch_synth_direct<T, NU, PER, 16, 1>(ll, x, dst, M, k, fin ? 1 : 0, t, st);
    else
      e = launch_synth_direct<T, NU, PER, 16, 2>(ll, x, dst, M, k, fin ? 1 : 0, t, st);
    if (e != hipSuccess) return e;
    ll = dst;
  }
  return hipSuccess;
}

template <typename T, int NU, bool PER>
hipError_t dwt2d_impl(const T* inT, T* x, T* s0, T* s1, int64_t M, int j0, int j, const Tables<T>& t,
                      hipStream_t st) {
  if (j0 == j) return copy_transposed<T, NU>(inT, x, M, j, t, st);
  const bool coarse = j0 < coarse_limit<T, NU>(j);
  const int kc = coarse ? (j < coarse_limit<T, NU>(j) ? j : coarse_limit<T, NU>(j)) : j0;
  const int S = 1 << kc;
  hipError_t e = hipSuccess;
  const T* src = inT;
  int trans = 1;
  for (int k = j - 1; k >= kc; --k) {
    // without a coarse stage the last tiled level writes LL_{j0} into x itself
    T* dst = (!coarse && k == kc) ? x : ((src == s0) ? s1 : s0);
    const TileShape sh = analysis_shape<T>(1 << k, NU);
    if (sh.t == 32)
      e = launch_analysis_direct<T, NU, PER, 32, 8>(src, trans, dst, x, M, k, t, st);
    else if (sh.t == 16)
      e = launch_analysis<T, NU, PER, 16, 2>(src, trans, dst, x, M, k, t, st);
    else if (sh.p == 1)
      e = launch_analysis<T, NU, PER, 8, 1>(src, trans, dst, x, M, k, t, st);
    else
      e = launch_analysis<T, NU, PER, 8, 2>(src, trans, dst, x, M, k, t, st);
    if (e != hipSuccess) return e;
    src = dst;
    trans = 0;
  }
  if (!coarse) return hipSuccess;
  const size_t smem_c = 2 * size_t(S) * (S + 1) * sizeof(T);
  hipLaunchKernelGGL((k_analysis2d_coarse<T, NU, PER>), dim3(1), dim3(1024), smem_c, st, src, M, trans, x, M, j0, kc,
                     t);
  return hipGetLastError();
}

// Raise the dynamic-LDS limit of the kernels that need more than 64 KB (once
// per plan, outside any stream work).
template <typename T, int NU, bool PER>
hipError_t prepare_impl() {
  // 160 KB per workgroup, less the static table each kernel keeps in LDS
  const int lim = 160 * 1024 - int(tab_lds_size<NU>() * sizeof(T));
  const void* kernels[] = {
      (const void*)k_synth2d_coarse<T, NU, PER>,         (const void*)k_analysis2d_coarse<T, NU, PER>,
      (const void*)k_analysis2d_tile<T, NU, 16, 2, PER>, (const void*)k_analysis2d_tile<T, NU, 8, 2, PER>,
      (const void*)k_analysis2d_tile<T, NU, 8, 1, PER>,  (const void*)k_synth2d_direct<T, NU, 64, 8, PER>,
      (const void*)k_synth2d_direct<T, NU, 32, 2, PER>,  (const void*)k_synth2d_direct<T, NU, 16, 2, PER>,
      (const void*)k_synth2d_direct<T, NU, 16, 1, PER>,  (const void*)k_analysis2d_direct<T, NU, 32, 8, PER>,
  };
  for (const void* f : kernels) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

#define WH2WAV_DWT_NUS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

}  // namespace

template <typename T>
hipError_t prepare_dwt2d(int nu) {
#define X(V) \
  if (nu == V) { \
    const hipError_t e = prepare_impl<T, V, false>(); \
    return e == hipSuccess ? prepare_impl<T, V, true>() : e; \
  }
  WH2WAV_DWT_NUS(X)
#undef X
  return hipErrorInvalidValue;
}
template hipError_t prepare_dwt2d<float>(int);
template hipError_t prepare_dwt2d<double>(int);

template <typename T>
hipError_t idwt2d(const T* x, T* outT, T* s0, T* s1, int64_t M, int j0, int j, const Tables<T>& t,
                  hipStream_t st) {
#define X(V) \
  if (t.nu == V) \
    return t.per ? idwt2d_impl<T, V, true>(x, outT, s0, s1, M, j0, j, t, st) \
                 : idwt2d_impl<T, V, false>(x, outT, s0, s1, M, j0, j, t, st);
  WH2WAV_DWT_NUS(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dwt2d(const T* inT, T* x, T* s0, T* s1, int64_t M, int j0, int j, const Tables<T>& t,
                 hipStream_t st) {
#define X(V) \
  if (t.nu == V) \
    return t.per ? dwt2d_impl<T, V, true>(inT, x, s0, s1, M, j0, j, t, st) \
                 : dwt2d_impl<T, V, false>(inT, x, s0, s1, M, j0, j, t, st);
  WH2WAV_DWT_NUS(X)
#undef X
  return hipErrorInvalidValue;
}

template hipError_t idwt2d<float>(const float*, float*, float*, float*, int64_t, int, int, const Tables<float>&,
                                  hipStream_t);
template hipError_t idwt2d<double>(const double*, double*, double*, double*, int64_t, int, int,
                                   const Tables<double>&, hipStream_t);
template hipError_t dwt2d<float>(const float*, float*, float*, float*, int64_t, int, int, const Tables<float>&,
                                 hipStream_t);
template hipError_t dwt2d<double>(const double*, double*, double*, double*, int64_t, int, int,
                                  const Tables<double>&, hipStream_t);

}  // namespace wh2wav_fast
