// Wave-level line kernels for the 2D operator on gfx950.
//
// A line of M = 64 R values lives in one wavefront, R consecutive values per
// lane ("layout A": element p = lane * R + r).  Every stage of one line is
// computed inside that wave:
//   * table product (operators D_l of Sec. 4.1 and the boundary terms of
//     Prop. 4.2): a (2nu-1)-tap correlation whose halo comes from the two
//     neighbouring lanes, with the taps held as wave-uniform values;
//   * natural-order Walsh-Hadamard transform: radix-R butterflies in
//     registers, then six butterfly stages across lanes (DPP quad
//     permutations for lane distance 1 and 2, ds_swizzle for 4..16,
//     ds_bpermute for 32);
//   * sequency order and the odd-phase mirror are index maps
//     (k = bitrev(gray(b)) xor (s & 1)), applied in the gather / scatter.
// Row passes run one workgroup per row of the N x M intermediate, one wave
// per phase s (the 1D operator on lines of up to 2048 values is the same
// kernel on its single row); the forward one gathers its samples from half a
// line of LDS at a time.  Column passes read or write the intermediate in
// 16-column (8 for the adjoint) tiles through an LDS staging area so that
// every global access is a contiguous segment; the forward one runs two
// phases per workgroup, the adjoint fetches the next phase's rows while the
// current one computes.
#include <algorithm>

#include "dwt_lines.h"
#include "fast2d.h"
#include "wave_ops.h"

namespace wh2wav_fast {
namespace {

using namespace wave;

// Halo: window w[0 .. R+2H) with w[H + r] = x[r]; the H values on each side
// come from the neighbouring lanes (from several lanes when H > R), zero
// beyond the ends of the line.  Position p of the line is register p % R of
// lane p / R.  ZERO = false: x is already zero at its first and last H
// positions, which is what the lane exchange wraps around to beyond the ends.
template <typename T, int R, int H, bool ZERO = true>
__device__ __forceinline__ void make_window(const T (&x)[R], T (&w)[R + 2 * H], int lane) {
#pragma unroll
  for (int r = 0; r < R; ++r) w[H + r] = x[r];
#pragma unroll
  for (int e = 0; e < H; ++e) {
    const int dl = 1 + e / R;  // lane distance of position lane R - 1 - e (left) / lane R + R + e (right)
    const T a = shfl_from(x[R - 1 - e % R], (lane - dl) & 63);
    const T b = shfl_from(x[e % R], (lane + dl) & 63);
    w[H - 1 - e] = ZERO && lane < dl ? T(0) : a;
    w[H + R + e] = ZERO && lane + dl > 63 ? T(0) : b;
  }
}

// v[r] = sum_l x[p - l] T_l  (p = lane R + r, l in [-nu+1, nu-1], tap[l + nu - 1] = T_l).
// x is zero at its first and last nu positions (the boundary coefficients
// enter through the bands), so the halo needs no zeroing at the line ends.
template <typename T, int R, int NU>
__device__ __forceinline__ void table_product(const T (&x)[R], T (&v)[R], const T (&tap)[2 * NU - 1], int lane) {
  constexpr int H = NU - 1;
  T w[R + 2 * H];
  make_window<T, R, H, false>(x, w, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T acc = 0;
#pragma unroll
    for (int li = 0; li < 2 * H + 1; ++li) acc = fma(w[2 * H + r - li], tap[li], acc);
    v[r] = acc;
  }
}

// acc[r] += sum_l T_l x[p + l]  (transpose of table_product on interior positions)
template <typename T, int R, int NU>
__device__ __forceinline__ void table_product_t(const T (&x)[R], T (&acc)[R], const T (&tap)[2 * NU - 1],
                                                int lane) {
  constexpr int H = NU - 1;
  T w[R + 2 * H];
  // no zeroing at the line ends: the outputs at the first and last nu
  // positions, the only ones that read beyond the ends, are replaced by the
  // boundary-column products (place_edges)
  make_window<T, R, H, false>(x, w, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T a = acc[r];
#pragma unroll
    for (int li = 0; li < 2 * H + 1; ++li) a = fma(w[r + li], tap[li], a);
    acc[r] = a;
  }
}

// Forward line: xi (layout A, all M values, boundary values included) -> the
// natural-order transform of phase s, in place in v.
template <typename T, int R, int NU>
__device__ __forceinline__ void line_forward(const T (&xi)[R], T (&v)[R], int s, const Tables<T>& t, int lane) {
  constexpr int B = 2 * NU - 1;
  const int Q = t.Q;
  T x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = xi[r];
  // Periodic extension: no boundary functions; the lane exchange of the
  // table product wraps around the line, which is the periodised product.
  // Otherwise the boundary values are zeroed (the bands below add them).
  const bool bd = !t.per;
  // e[m]: the boundary value that this lane's band row multiplies -- position
  // m (register m % R of lane m / R) in the left band lanes 0..B-1, position
  // M-1-m (register R-1-m % R of lane 63 - m / R) in the right band lanes
  // 64-B..63.  With R >= NU both sit in lanes 0 and 63: one select and one
  // lane exchange each.
  T e[NU];
#pragma unroll
  for (int m = 0; m < NU; ++m) {
    if constexpr (R >= NU) {
      const T w = lane == 63 ? xi[R - 1 - m] : xi[m];
      e[m] = shfl_from(w, lane < B ? 0 : 63);
    } else {
      const T a = read_lane(xi[m % R], m / R), b = read_lane(xi[R - 1 - m % R], 63 - m / R);
      e[m] = lane < B ? a : b;
    }
    // per-element selects (conditional stores would let the compiler merge
    // them into one dynamically indexed store and move x to scratch)
    x[m % R] = bd && lane == m / R ? T(0) : x[m % R];
    x[R - 1 - m % R] = bd && lane == 63 - m / R ? T(0) : x[R - 1 - m % R];
  }
  T tap[2 * NU - 1];
#pragma unroll
  for (int li = 0; li < 2 * NU - 1; ++li) tap[li] = t.tabT[li * Q + s];
  table_product<T, R, NU>(x, v, tap, lane);
  if (bd) {
    // boundary bands (Prop. 4.2): positions p < B and p >= M - B
    // lanes 0..B-1: left band row p = lane; lanes 64-B..63: right band row
    // lane - (64 - B).  Loads are unconditional (clamped row) so they overlap.
    T bv = T(0);
    {
      const bool left = lane < B, right = lane >= 64 - B;
      const int p = left ? lane : (right ? lane - (64 - B) : 0);
      const T* band = (left ? t.bandLf : t.bandRf) + (s * B + p) * NU;  // this row's nu values
#pragma unroll
      for (int m = 0; m < NU; ++m) bv = fma(e[m], band[m], bv);
      bv = left || right ? bv : T(0);
    }
    if constexpr (R >= B) {
      static_assert(R + 2 * B <= 64, "the other lanes must read zero lanes B .. B + R - 1");
      // the bands sit in lanes 0 and 63.  Register k of lane 0 takes lane k
      // (left band row k for k < B, a zero lane beyond), of lane 63 lane
      // 64 - R + k (right band row k - (R - B) for k >= R - B, a zero lane
      // below), of every other lane the zero lane B + k: one lane exchange
      // and one add per register that a band reaches.
      const int base = lane == 0 ? 0 : (lane == 63 ? 64 - R : B);
#pragma unroll
      for (int k = 0; k < R; ++k)
        if (k < B || k >= R - B) v[k] += shfl_from(bv, base + k);
    } else {
#pragma unroll
      for (int e = 0; e < B; ++e) {
        const T a = read_lane(bv, e), b = read_lane(bv, 64 - B + e);
        constexpr int M = 64 * R;
        const int pr = M - B + e;  // right band position
        v[e % R] += lane == e / R ? a : T(0);
        v[pr % R] += lane == pr / R ? b : T(0);
      }
    }
  }
  fwht_wave<T, R>(v, lane);
}

// Adjoint line for one phase: v holds the natural-order values of phase s
// (layout A); adds the transposed table product to acc (interior positions)
// and the boundary-column products to eacc (lanes 0..2nu-1: left m = lane,
// right position M-1-(lane-nu)).
template <typename T, int R, int NU>
__device__ __forceinline__ void line_adjoint(T (&v)[R], T (&acc)[R], T& eacc, int s, const Tables<T>& t, int lane) {
  constexpr int B = 2 * NU - 1;
  const int Q = t.Q;
  fwht_wave<T, R>(v, lane);
  T tap[2 * NU - 1];
#pragma unroll
  for (int li = 0; li < 2 * NU - 1; ++li) tap[li] = t.tabT[li * Q + s];
  table_product_t<T, R, NU>(v, acc, tap, lane);
  if (t.per) return;  // periodic: the wrapped correlation is the whole adjoint
  // lanes 0..nu-1: left boundary column m = lane, against positions 0..B-1;
  // lanes nu..2nu-1: right column lane - nu, against positions M-B..M-1
  // (unconditional loads, clamped column)
  T rl[B], rr[B];
#pragma unroll
  for (int e = 0; e < B; ++e) {
    constexpr int M = 64 * R;
    const int pr = M - B + e;
    rl[e] = read_lane(v[e % R], e / R);
    rr[e] = read_lane(v[pr % R], pr / R);
  }
  const bool left = lane < NU;
  const int m = left ? lane : (lane < 2 * NU ? lane - NU : 0);
  const T* band = (left ? t.bandLa : t.bandRa) + (s * NU + m) * B;  // this column's B values
  T el = T(0);
#pragma unroll
  for (int p = 0; p < B; ++p) el = fma(band[p], left ? rl[p] : rr[p], el);
  eacc += lane < 2 * NU ? el : T(0);
}

// Boundary positions of acc take their values from eacc (not for the periodic
// extension, whose wrapped correlation already covers every position).
template <typename T, int R, int NU>
__device__ __forceinline__ void place_edges(T (&acc)[R], T eacc, int lane, int per) {
  if (per) return;
#pragma unroll
  for (int m = 0; m < NU; ++m) {
    if constexpr (R >= NU) {
      // lane 0 takes column m from lane m, lane 63 column nu + m: one exchange
      const T a = shfl_from(eacc, lane == 63 ? NU + m : m);
      acc[m] = lane == 0 ? a : acc[m];
      acc[R - 1 - m] = lane == 63 ? a : acc[R - 1 - m];
    } else {
      const T a = read_lane(eacc, m), b = read_lane(eacc, NU + m);
      acc[m % R] = lane == m / R ? a : acc[m % R];
      acc[R - 1 - m % R] = lane == 63 - m / R ? b : acc[R - 1 - m % R];
    }
  }
}

// One line of M = 64 R values in LDS, without padding: the values of lane l
// occupy [l R, (l + 1) R), in chunks of CW = min(R, 4) values; chunk c is
// stored at chunk slot c ^ (l & SWZ), so that the vector accesses of
// consecutive lanes fall on different banks.
template <int R>
struct LineBuf {
  static constexpr int CW = R < 4 ? R : 4, NCH = R / CW, SWZ = (NCH < 8 ? NCH : 8) - 1;
  // address of line position k
  __device__ static __forceinline__ int addr(int k) {
    const int l = k / R, r = k % R;
    return l * R + (((r / CW) ^ (l & SWZ)) * CW) + r % CW;
  }
  template <typename T>
  __device__ static __forceinline__ void store(T* buf, int lane, const T (&v)[R]) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      T* p = buf + lane * R + ((c ^ (lane & SWZ)) * CW);
      T w[CW];
#pragma unroll
      for (int u = 0; u < CW; ++u) w[u] = v[c * CW + u];
      store_line<T, CW>(p, w);
    }
  }
  template <typename T>
  __device__ static __forceinline__ void load(const T* buf, int lane, T (&v)[R]) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const T* p = buf + lane * R + ((c ^ (lane & SWZ)) * CW);
      T w[CW];
      load_line<T, CW>(p, w);
#pragma unroll
      for (int u = 0; u < CW; ++u) v[c * CW + u] = w[u];
    }
  }
};

// ------------------------------------------------------------- row passes
// The gather of one phase line s of Omega row n1: the samples are
// y[o .. o + cnt), in sequency order, and pos holds each one's natural
// position (coalesced reads and writes).  prepare() loads the first 256
// positions, so that their latency overlaps the line transform; run() puts
// the line into LDS in two halves (lanes 0..31 hold the positions below M/2),
// each followed by the reads of the samples it holds: half a line of LDS per
// wave, so that more workgroups fit on a CU.
template <typename T, int LOGM>
struct PhaseGather {
  static constexpr int M = 1 << LOGM, R = M / 64, HM = M / 2;
  using LB = LineBuf<R>;
  const uint16_t* ps = nullptr;
  T* ys = nullptr;
  int cnt = 0;
  int kk[4], ka[4];  // positions of samples t0 + lane + 64 u (-1 beyond); their address within a half
  __device__ __forceinline__ void positions(int t0, int lane) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tt = t0 + lane + 64 * u;
      const int pv = int(ps[tt < cnt ? tt : cnt - 1]);  // cnt > 0 here
      kk[u] = tt < cnt ? pv : -1;
      ka[u] = LB::addr(pv & (HM - 1));
    }
  }
  __device__ __forceinline__ void prepare(const Omega& om, T* y, int64_t n1, int s, int Q, int lane) {
    int64_t o = 0;
    if (!om.full) {
      o = om.seg_ptr[n1 * Q + s];
      cnt = int(om.seg_ptr[n1 * Q + s + 1] - o);
    }
    ps = om.pos + o;
    ys = y + o;
    if (cnt > 0) positions(0, lane);
  }
  __device__ __forceinline__ void run(const T (&v)[R], T* buf, const Omega& om, T* y, int64_t n1, int s, int Q,
                                      int lane) {
    const int64_t N = int64_t(M) * Q;
    for (int h = 0; h < 2; ++h) {
      if ((lane >> 5) == h) LB::store(buf, lane & 31, v);
      wave_sync();
      if (om.full) {
        T* yrow = y + n1 * N + int64_t(s) * M;
        for (int b = lane; b < M; b += 64) {
          const int k = int(natural_of(uint32_t(b), uint32_t(s), LOGM));
          if ((k >> (LOGM - 1)) == h) yrow[b] = buf[LB::addr(k - h * HM)];
        }
      } else {
        for (int t0 = 0; t0 < cnt; t0 += 256) {
          if (t0 > 0 || (h == 1 && cnt > 256)) positions(t0, lane);  // more than 256 samples: reload
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (kk[u] >= 0 && (kk[u] >> (LOGM - 1)) == h) ys[t0 + lane + 64 * u] = buf[ka[u]];
        }
      }
      wave_sync();
    }
  }
};

// The scatter of phase line s of Omega row n1 into a line of LDS (zero where
// Omega has no sample), then the line into v (layout A).
template <typename T, int LOGM>
__device__ __forceinline__ void scatter_phase(const T* __restrict__ y, const Omega& om, int64_t n1, int s, int Q,
                                              T* buf, T (&v)[1 << (LOGM - 6)], int lane) {
  constexpr int M = 1 << LOGM, R = M / 64;
  using LB = LineBuf<R>;
  const int64_t N = int64_t(M) * Q;
  if (om.full) {
    const T* yrow = y + n1 * N + int64_t(s) * M;
    constexpr int NB = M / 64;
    T rv[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) rv[i] = yrow[lane + 64 * i];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const uint32_t k = natural_of(uint32_t(lane + 64 * i), uint32_t(s), LOGM);
      buf[LB::addr(int(k))] = rv[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = T(0);
    LB::store(buf, lane, v);
    const int64_t o = om.seg_ptr[n1 * Q + s];
    const int cnt = int(om.seg_ptr[n1 * Q + s + 1] - o);
    const uint16_t* __restrict__ ps = om.pos + o;
    const T* __restrict__ ys = y + o;
    wave_sync();  // zero fill of buf before the scatter
    // coalesced reads of this phase line's samples and their positions
    for (int t0 = 0; t0 < cnt; t0 += 256) {
      int kk[4];
      T rv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int tt = t0 + lane + 64 * u;
        const int pv = int(ps[tt < cnt ? tt : cnt - 1]);  // cnt > 0 inside the loop
        kk[u] = tt < cnt ? pv : -1;
        const T yv = ys[tt < cnt ? tt : cnt - 1];
        rv[u] = tt < cnt ? yv : T(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (kk[u] >= 0) buf[LB::addr(kk[u])] = rv[u];
    }
  }
  wave_sync();
  LB::load(buf, lane, v);
  wave_sync();
}

template <typename T, int LOGM, int NU>
__global__ void __launch_bounds__(1024) k_rowpass_fwd(const T* __restrict__ Z, T* __restrict__ y, Tables<T> t,
                                                     Omega om) {
  constexpr int M = 1 << LOGM, LOG_R = LOGM - 6, R = 1 << LOG_R;
  constexpr int HM = M / 2;  // LDS per wave: half a line
  extern __shared__ unsigned char smem_raw[];
  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int Q = t.Q;
  T* buf = reinterpret_cast<T*>(smem_raw) + wave * HM;
  const int64_t r = blockIdx.x;
  T xi[R];
  load_line<T, R>(Z + r * M + lane * R, xi);
  const uint32_t s1 = uint32_t(r >> LOGM), k1 = uint32_t(r & (M - 1));
  const int64_t n1 = int64_t(s1) * M + sequency_of(k1, s1, LOGM);
  // one wave per phase: the workgroup has Q waves
  PhaseGather<T, LOGM> g;
  g.prepare(om, y, n1, wave, Q, lane);
  T v[R];
  line_forward<T, R, NU>(xi, v, wave, t, lane);
  g.run(v, buf, om, y, n1, wave, Q, lane);
}

template <typename T, int LOGM, int NU>
__global__ void __launch_bounds__(1024) k_rowpass_adj(const T* __restrict__ y, T* __restrict__ Zt, Tables<T> t,
                                                     Omega om) {
  constexpr int M = 1 << LOGM, LOG_R = LOGM - 6, R = 1 << LOG_R;
  constexpr int BUF = M;
  using LB = LineBuf<R>;
  extern __shared__ unsigned char smem_raw[];
  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int nw = int(blockDim.x) >> 6;
  const int Q = t.Q;
  T* bufs = reinterpret_cast<T*>(smem_raw);
  T* buf = bufs + wave * BUF;
  const int64_t r = blockIdx.x;
  const uint32_t s1 = uint32_t(r >> LOGM), k1 = uint32_t(r & (M - 1));
  const int64_t n1 = int64_t(s1) * M + sequency_of(k1, s1, LOGM);
  T acc[R];
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = T(0);
  T eacc = T(0);
  {  // one wave per phase: the workgroup has Q waves
    T v[R];
    scatter_phase<T, LOGM>(y, om, n1, wave, Q, buf, v, lane);
    line_adjoint<T, R, NU>(v, acc, eacc, wave, t, lane);
  }
  place_edges<T, R, NU>(acc, eacc, lane, t.per);
  // cross-wave sum (waves that had no phase contribute zeros), a chunk of CW
  // consecutive positions (contiguous in every wave's buffer) per thread
  LB::store(buf, lane, acc);
  __syncthreads();
  constexpr int CW = LB::CW;
  for (int c = int(threadIdx.x); c < M / CW; c += int(blockDim.x)) {
    const int a = LB::addr(c * CW);
    T sum[CW], part[CW];
    load_line<T, CW>(bufs + a, sum);
    for (int w = 1; w < nw; ++w) {
      load_line<T, CW>(bufs + w * BUF + a, part);
#pragma unroll
      for (int u = 0; u < CW; ++u) sum[u] += part[u];
    }
    store_line<T, CW>(Zt + r * M + c * CW, sum);
  }
}

// ------------------------------------------------- one-dimensional lines
// The 1D operator on lines of M = 2^LOGM <= 2048 values in one launch per
// direction: the wavelet levels on the line in LDS (all of them, one
// workgroup of 1024 threads), and the row-pass line transform of each phase
// in its own wave with the gather (forward), or the scatter, the transposed
// line transform, the cross-wave sum and the analysis levels (adjoint).

// LDS of the fused kernels, in elements (besides the static table copy).
// forward: the final line, then two lines for the wavelet levels (their
// input and scratch), which the phase waves then reuse for the gather (half a
// line each); adjoint: a line per phase wave, at least three lines for the
// levels.
template <int LOGM>
constexpr int line1d_fwd_lds(int Q) {
  return (1 << LOGM) + ((Q << LOGM) / 2 > (2 << LOGM) ? (Q << LOGM) / 2 : (2 << LOGM));
}
template <int LOGM>
constexpr int line1d_adj_lds(int Q) {
  return (Q > 3 ? Q : 3) << LOGM;
}

template <typename T, int LOGM, int NU>
__global__ void __launch_bounds__(1024) k_line1d_fwd(const T* __restrict__ x, T* __restrict__ y, int j0, Tables<T> t,
                                                    Omega om) {
  constexpr int M = 1 << LOGM, R = M / 64, HM = M / 2;
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[lines::tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const lines::TileLds<T> tl = lines::load_tables<T, NU>(t, tab_lds, hr, gr);
  const int tid = int(threadIdx.x), lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Q = t.Q;
  T* a = reinterpret_cast<T*>(smem_raw);  // the line; then a half line per phase wave from a + M
  T* b = a + M;                            // the coefficients, then scratch of the levels
  PhaseGather<T, LOGM> g;
  if (wave < Q) g.prepare(om, y, 0, wave, Q, lane);
  for (int i = tid; i < M; i += int(blockDim.x)) b[i] = x[i];
  __syncthreads();
  lines::synth_levels_lds3<T, NU>(b, a, b + M, j0, LOGM, tl, hr, gr);
  if (wave >= Q) return;
  T xi[R];
  load_line<T, R>(a + lane * R, xi);
  T v[R];
  line_forward<T, R, NU>(xi, v, wave, t, lane);
  g.run(v, b + wave * HM, om, y, 0, wave, Q, lane);
}

template <typename T, int LOGM, int NU>
__global__ void __launch_bounds__(1024) k_line1d_adj(const T* __restrict__ y, T* __restrict__ x, int j0, Tables<T> t,
                                                    Omega om) {
  constexpr int M = 1 << LOGM, R = M / 64;
  using LB = LineBuf<R>;
  constexpr int CW = LB::CW;
  extern __shared__ unsigned char smem_raw[];
  __shared__ T tab_lds[lines::tab_lds_size<NU>()];
  T hr[2 * NU], gr[2 * NU];
  const lines::TileLds<T> tl = lines::load_tables<T, NU>(t, tab_lds, hr, gr);
  const int tid = int(threadIdx.x), lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Q = t.Q;
  T* bufs = reinterpret_cast<T*>(smem_raw);  // a line per phase wave; then the line and scratch
  if (wave < Q) {
    T* buf = bufs + wave * M;
    T v[R], acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = T(0);
    T eacc = T(0);
    scatter_phase<T, LOGM>(y, om, 0, wave, Q, buf, v, lane);
    line_adjoint<T, R, NU>(v, acc, eacc, wave, t, lane);
    place_edges<T, R, NU>(acc, eacc, lane, t.per);
    LB::store(buf, lane, acc);
  }
  __syncthreads();
  // cross-wave sum into registers (a chunk of CW positions per thread), then
  // the line in natural order into the first M elements
  T sum[CW];
  const int c = tid;
  if (c < M / CW) {
    const int ad = LB::addr(c * CW);
    T part[CW];
    load_line<T, CW>(bufs + ad, sum);
    for (int w = 1; w < Q; ++w) {
      load_line<T, CW>(bufs + w * M + ad, part);
#pragma unroll
      for (int u = 0; u < CW; ++u) sum[u] += part[u];
    }
  }
  __syncthreads();
  if (c < M / CW) store_line<T, CW>(bufs + c * CW, sum);
  __syncthreads();
  lines::analysis_levels_lds3<T, NU>(bufs, bufs + 2 * M, bufs + M, j0, LOGM, tl, hr, gr);
  for (int i = tid; i < M; i += int(blockDim.x)) x[i] = bufs[2 * M + i];
}

// ---------------------------------------------------------- column passes
// Forward: block = 16 waves = 16 rows of xi^T (columns c0..c0+15 of xi), a
// group of consecutive phases (the grid holds M/16 tiles x the number of
// groups); the stores of one phase drain while the next one computes.  Blocks
// that share a tile are placed on the same XCD (the dispatcher deals
// consecutive block ids round-robin over the 8 XCDs).
template <typename T>
constexpr int colpass_fwd_maxph() {
  return sizeof(T) == 4 ? 2 : 1;  // FP64 keeps no second line in registers
}
template <typename T, int LOGM, int NU>
__global__ void __launch_bounds__(1024) k_colpass_fwd(const T* __restrict__ xiT, T* __restrict__ Z, Tables<T> t) {
  constexpr int M = 1 << LOGM, LOG_R = LOGM - 6, R = 1 << LOG_R;
  constexpr int TILE = 16, SP = 64 * 4 + 4;  // staging stride per wave (padded)
  static_assert(R == 2 || R % 4 == 0, "column pass staging needs R = 2 or a multiple of 4");
  extern __shared__ unsigned char smem_raw[];
  T* stage = reinterpret_cast<T*>(smem_raw);
  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int Q = t.Q;
  const int nblk = int(gridDim.x), bid = int(blockIdx.x);
  const int per = nblk / 8;
  const int idx = (nblk % 8 == 0) ? (bid % 8) * per + bid / 8 : bid;
  const int ngrp = nblk / (M / TILE), ph = Q / ngrp;
  const int tile = idx / ngrp, s0 = (idx % ngrp) * ph;
  const int c = tile * TILE + wave;
  T xi[R];
  load_line<T, R>(xiT + int64_t(c) * M + lane * R, xi);
  const int tid = int(threadIdx.x);
  for (int i = 0; i < colpass_fwd_maxph<T>(); ++i) {
  if (i >= ph) break;
  const int s = s0 + i;
  T v[R];
  line_forward<T, R, NU>(xi, v, s, t, lane);
  if constexpr (R == 2) {
    // one round: the wave's 128 values, then 128 output rows x 8 column pairs
    constexpr int SP2 = 2 * 64 + 4;
    store_line<T, R>(stage + wave * SP2 + lane * 2, v);
    __syncthreads();
    const int k = tid >> 3, cp = tid & 7;
    T o0 = stage[(2 * cp) * SP2 + k], o1 = stage[(2 * cp + 1) * SP2 + k];
    pin(o0), pin(o1);
    T* dst = Z + (int64_t(s) * M + k) * M + tile * TILE + 2 * cp;
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float2*>(dst) = make_float2(o0, o1);
    } else {
      *reinterpret_cast<double2*>(dst) = make_double2(o0, o1);
    }
    __syncthreads();  // stage reused by the next phase
    continue;
  }
  const int e = tid >> 2, qg = tid & 3;            // 256 output rows x 4 column groups
  const int le = e >> 2, te = e & 3;
#pragma unroll
  for (int i = 0; i < R / 4; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u) stage[wave * SP + lane * 4 + u] = v[4 * i + u];
    __syncthreads();
    const int k = le * R + 4 * i + te;
    T o[4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) o[cc] = stage[(4 * qg + cc) * SP + le * 4 + te];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) pin(o[cc]);
    T* dst = Z + (int64_t(s) * M + k) * M + tile * TILE + 4 * qg;
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4*>(dst) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
      reinterpret_cast<double2*>(dst)[0] = make_double2(o[0], o[1]);
      reinterpret_cast<double2*>(dst)[1] = make_double2(o[2], o[3]);
    }
    __syncthreads();
  }
  }
}

// Adjoint: block = columns c0..c0+7 of the intermediate x NG phase groups
// (8 NG waves); group g takes phases g, g + NG, ...  Every group runs the
// same number of phases, so the block-wide barriers line up; the groups'
// partial sums are added through LDS at the end.  With one group, the rows
// of the group's next phase are fetched into registers while the current
// phase computes (two groups have no registers to spare for that).
template <typename T, int LOGM, int NU, int NG>
__global__ void __launch_bounds__(512 * NG) k_colpass_adj(const T* __restrict__ Zt, T* __restrict__ xiT, Tables<T> t) {
  constexpr int M = 1 << LOGM, LOG_R = LOGM - 6, R = 1 << LOG_R;
  constexpr int TILE = 8, SP = 64 * 4 + 4;
  static_assert(R == 2 || R % 4 == 0, "column pass staging needs R = 2 or a multiple of 4");
  extern __shared__ unsigned char smem_raw[];
  const int lane = lane_id();
  const int wave_all = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int g = wave_all >> 3, wave = wave_all & 7;  // 512 threads per phase group
  T* stage = reinterpret_cast<T*>(smem_raw) + g * TILE * SP;
  const int Q = t.Q;
  const int nblk = int(gridDim.x), bid = int(blockIdx.x);
  const int per = nblk / 8;
  const int tile = (nblk % 8 == 0) ? (bid % 8) * per + bid / 8 : bid;
  const int c = tile * TILE + wave;
  const int tid = int(threadIdx.x) & 511;
  const int e = tid >> 1, half = tid & 1;          // 256 input rows x 2 halves of 4 columns
  const int le = e >> 2, te = e & 3;
  T acc[R];
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = T(0);
  T eacc = T(0);
  // phase s of the tile, R/4 float4 rows per thread (the layout the exchange
  // rounds take apart); the next phase is fetched while this one computes
  T o[R / 4 > 0 ? R / 4 : 1][4];
  auto fetch = [&](int s) {
#pragma unroll
    for (int i = 0; i < R / 4; ++i) {
      const int k = le * R + 4 * i + te;
      const T* src = Zt + (int64_t(s) * M + k) * M + tile * TILE + 4 * half;
      if constexpr (sizeof(T) == 4) {
        const float4 f = *reinterpret_cast<const float4*>(src);
        o[i][0] = f.x, o[i][1] = f.y, o[i][2] = f.z, o[i][3] = f.w;
      } else {
        const double2 f0 = reinterpret_cast<const double2*>(src)[0], f1 = reinterpret_cast<const double2*>(src)[1];
        o[i][0] = f0.x, o[i][1] = f0.y, o[i][2] = f1.x, o[i][3] = f1.y;
      }
    }
  };
  if constexpr (R >= 4 && NG == 1) fetch(g);
  for (int s = g; s < Q; s += NG) {
    T v[R];
    if constexpr (R == 2) {
      // one round: 128 input rows x 4 column pairs
      constexpr int SP2 = 2 * 64 + 4;
      const int k = tid >> 2, cp = tid & 3;
      const T* src = Zt + (int64_t(s) * M + k) * M + tile * TILE + 2 * cp;
      T o0, o1;
      if constexpr (sizeof(T) == 4) {
        const float2 f = *reinterpret_cast<const float2*>(src);
        o0 = f.x, o1 = f.y;
      } else {
        const double2 f = *reinterpret_cast<const double2*>(src);
        o0 = f.x, o1 = f.y;
      }
      stage[(2 * cp) * SP2 + k] = o0;
      stage[(2 * cp + 1) * SP2 + k] = o1;
      __syncthreads();
      load_line<T, R>(stage + wave * SP2 + lane * 2, v);
#pragma unroll
      for (int u = 0; u < R; ++u) pin(v[u]);
      __syncthreads();
      line_adjoint<T, R, NU>(v, acc, eacc, s, t, lane);
      continue;
    }
    if constexpr (NG > 1) fetch(s);
#pragma unroll
    for (int i = 0; i < R / 4; ++i) {
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) stage[(4 * half + cc) * SP + le * 4 + te] = o[i][cc];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) v[4 * i + u] = stage[wave * SP + lane * 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) pin(v[4 * i + u]);
      __syncthreads();
    }
    if (NG == 1 && s + NG < Q) fetch(s + NG);
    line_adjoint<T, R, NU>(v, acc, eacc, s, t, lane);
  }
  place_edges<T, R, NU>(acc, eacc, lane, t.per);
  if constexpr (NG > 1) {
    static_assert(NG == 2, "two phase groups at most");
    // group 1 hands its partial sums to group 0, a few registers per round,
    // through its own staging area
    constexpr int RC = R < 4 ? R : 4;
#pragma unroll
    for (int i = 0; i < R / RC; ++i) {
      if (g == 1) {
#pragma unroll
        for (int u = 0; u < RC; ++u) stage[wave * SP + lane * RC + u] = acc[RC * i + u];
      }
      __syncthreads();
      if (g == 0) {
        const T* other = stage + TILE * SP;
#pragma unroll
        for (int u = 0; u < RC; ++u) acc[RC * i + u] += other[wave * SP + lane * RC + u], pin(acc[RC * i + u]);
      }
      __syncthreads();
    }
  }
  if (g == 0) store_line<T, R>(xiT + int64_t(c) * M + lane * R, acc);
}

// ------------------------------------------------------------ transpose
template <typename T>
__global__ void __launch_bounds__(256) k_transpose(const T* __restrict__ in, T* __restrict__ out, int64_t n) {
  __shared__ T tile[32][33];
  const int64_t bx = int64_t(blockIdx.x) * 32, by = int64_t(blockIdx.y) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) tile[j][tx] = in[(by + j) * n + bx + tx];
  __syncthreads();
  for (int j = ty; j < 32; j += 8) out[(bx + j) * n + by + tx] = tile[tx][j];
}

// ------------------------------------------------------------- dispatch
template <typename T, int LOGM, int NU>
hipError_t launch_rowpass_fwd(const T* Z, T* y, const Tables<T>& t, const Omega& om, int64_t rows, hipStream_t st) {
  constexpr int M = 1 << LOGM;
  const int nw = t.Q;  // one wave per phase, half a line of LDS each
  const size_t smem = size_t(nw) * (M / 2) * sizeof(T);
  hipLaunchKernelGGL((k_rowpass_fwd<T, LOGM, NU>), dim3(unsigned(rows)), dim3(64 * nw), smem, st, Z, y, t, om);
  return hipGetLastError();
}
template <typename T, int LOGM, int NU>
hipError_t launch_rowpass_adj(const T* y, T* Zt, const Tables<T>& t, const Omega& om, int64_t rows, hipStream_t st) {
  constexpr int M = 1 << LOGM;
  const int nw = t.Q;  // one wave per phase
  const size_t smem = size_t(nw) * M * sizeof(T);
  hipLaunchKernelGGL((k_rowpass_adj<T, LOGM, NU>), dim3(unsigned(rows)), dim3(64 * nw), smem, st, y, Zt, t, om);
  return hipGetLastError();
}
template <typename T, int LOGM, int NU>
hipError_t launch_colpass_fwd(const T* xiT, T* Z, const Tables<T>& t, hipStream_t st) {
  constexpr int M = 1 << LOGM;
  const size_t smem = size_t(16) * (64 * 4 + 4) * sizeof(T);
  // two phases per block where that still leaves a block per CU
  const int ph = colpass_fwd_maxph<T>() >= 2 && (M / 16) * t.Q / 2 >= 256 ? 2 : 1;
  hipLaunchKernelGGL((k_colpass_fwd<T, LOGM, NU>), dim3(unsigned((M / 16) * (t.Q / ph))), dim3(1024), smem, st, xiT,
                     Z, t);
  return hipGetLastError();
}
// Phase groups of the adjoint column pass: two (1024 threads) on FP32 lines
// up to 1024 values, where the grid of M/8 blocks is small and the line fits
// the 128 registers of a 1024-thread block; otherwise one, with the
// next-phase prefetch (Q >= 2 always).
template <typename T, int LOGM, int NU>
constexpr int colpass_adj_groups() {
  return sizeof(T) == 4 && LOGM <= 10 ? 2 : 1;
}
template <typename T, int LOGM, int NU>
hipError_t launch_colpass_adj(const T* Zt, T* xiT, const Tables<T>& t, hipStream_t st) {
  constexpr int M = 1 << LOGM, NG = colpass_adj_groups<T, LOGM, NU>();
  const size_t smem = size_t(NG) * 8 * (64 * 4 + 4) * sizeof(T);
  hipLaunchKernelGGL((k_colpass_adj<T, LOGM, NU, NG>), dim3(unsigned(M / 8)), dim3(512 * NG), smem, st, Zt, xiT, t);
  return hipGetLastError();
}

template <typename T, int LOGM, int NU>
hipError_t launch_line1d_fwd(const T* x, T* y, int j0, const Tables<T>& t, const Omega& om, hipStream_t st) {
  const size_t smem = size_t(line1d_fwd_lds<LOGM>(t.Q)) * sizeof(T);
  hipLaunchKernelGGL((k_line1d_fwd<T, LOGM, NU>), dim3(1), dim3(1024), smem, st, x, y, j0, t, om);
  return hipGetLastError();
}
template <typename T, int LOGM, int NU>
hipError_t launch_line1d_adj(const T* y, T* x, int j0, const Tables<T>& t, const Omega& om, hipStream_t st) {
  const size_t smem = size_t(line1d_adj_lds<LOGM>(t.Q)) * sizeof(T);
  hipLaunchKernelGGL((k_line1d_adj<T, LOGM, NU>), dim3(1), dim3(1024), smem, st, y, x, j0, t, om);
  return hipGetLastError();
}

// Supported (log2 M, nu).  Lines of M = 128 .. 2048 values (R = 2 .. 32 per
// lane); boundary values and the table-product halo may span several lanes.
// (log2 M, nu) of the wave kernels.  nu = 9, 10 stop at M = 1024: the band
// exchange of the forward line needs R + 2 (2 nu - 1) <= 64 (R = M / 64).
#define WH2WAV_FAST_CASES(X)                                                       \
  X(7, 2) X(7, 3) X(7, 4) X(7, 5) X(7, 6) X(7, 7) X(7, 8) X(7, 9) X(7, 10)         \
  X(8, 2) X(8, 3) X(8, 4) X(8, 5) X(8, 6) X(8, 7) X(8, 8) X(8, 9) X(8, 10)         \
  X(9, 2) X(9, 3) X(9, 4) X(9, 5) X(9, 6) X(9, 7) X(9, 8) X(9, 9) X(9, 10)         \
  X(10, 2) X(10, 3) X(10, 4) X(10, 5) X(10, 6) X(10, 7) X(10, 8) X(10, 9) X(10, 10) \
  X(11, 2) X(11, 3) X(11, 4) X(11, 5) X(11, 6) X(11, 7) X(11, 8)

}  // namespace

bool supported(int elem_bytes, int logm, int nu, int q) {
  // row passes: one wave (and one LDS line buffer) per phase
  const long long phases = 1LL << q, m = 1LL << logm;
  if (q > 4 || phases * m * elem_bytes > 160 * 1024) return false;
#define X(L, V) if (logm == L && nu == V) return true;
  WH2WAV_FAST_CASES(X)
#undef X
  return false;
}

bool line1d_fused(int elem_bytes, int logm, int nu, int q) {
  if (!supported(elem_bytes, logm, nu, q) || logm > 11) return false;
  const int Q = 1 << q, M = 1 << logm;
  const long long tab = (4LL * nu + 2LL * (3 * nu - 1) * 2 * nu) * elem_bytes;
  const long long fwd = (M + std::max((Q * M) / 2, 2 * M)) * 1LL * elem_bytes, adj = 1LL * std::max(Q, 3) * M * elem_bytes;
  return std::max(fwd, adj) + tab <= 160 * 1024;
}

template <typename T>
hipError_t line1d_fwd_fused(const T* x, T* y, int j0, int logm, const Tables<T>& t, const Omega& om,
                            hipStream_t st) {
#define X(L, V) if (logm == L && t.nu == V) return launch_line1d_fwd<T, L, V>(x, y, j0, t, om, st);
  WH2WAV_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t line1d_adj_fused(const T* y, T* x, int j0, int logm, const Tables<T>& t, const Omega& om,
                            hipStream_t st) {
#define X(L, V) if (logm == L && t.nu == V) return launch_line1d_adj<T, L, V>(y, x, j0, t, om, st);
  WH2WAV_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t rowpass_fwd(const T* Z, T* y, int logm, const Tables<T>& t, const Omega& om, int64_t rows,
                       hipStream_t st) {
#define X(L, V) if (logm == L && t.nu == V) return launch_rowpass_fwd<T, L, V>(Z, y, t, om, rows, st);
  WH2WAV_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t rowpass_adj(const T* y, T* Zt, int logm, const Tables<T>& t, const Omega& om, int64_t rows,
                       hipStream_t st) {
#define X(L, V) if (logm == L && t.nu == V) return launch_rowpass_adj<T, L, V>(y, Zt, t, om, rows, st);
  WH2WAV_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t colpass_fwd(const T* xiT, T* Z, int logm, const Tables<T>& t, hipStream_t st) {
#define X(L, V) if (logm == L && t.nu == V) return launch_colpass_fwd<T, L, V>(xiT, Z, t, st);
  WH2WAV_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t colpass_adj(const T* Zt, T* xiT, int logm, const Tables<T>& t, hipStream_t st) {
#define X(L, V) if (logm == L && t.nu == V) return launch_colpass_adj<T, L, V>(Zt, xiT, t, st);
  WH2WAV_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}
template <typename T, int LOGM, int NU>
hipError_t prepare_lines_impl() {
  const int lim = 160 * 1024;
  hipError_t e = hipFuncSetAttribute((const void*)k_rowpass_fwd<T, LOGM, NU>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_rowpass_adj<T, LOGM, NU>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_colpass_fwd<T, LOGM, NU>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_colpass_adj<T, LOGM, NU, colpass_adj_groups<T, LOGM, NU>()>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  const int tab = lines::tab_lds_size<NU>() * int(sizeof(T));  // the static table copy of the fused 1D kernels
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_line1d_fwd<T, LOGM, NU>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim - tab);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_line1d_adj<T, LOGM, NU>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim - tab);
  return e;
}

template <typename T>
hipError_t prepare_lines(int logm, int nu) {
#define X(L, V) if (logm == L && nu == V) return prepare_lines_impl<T, L, V>();
  WH2WAV_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}
template hipError_t prepare_lines<float>(int, int);
template hipError_t prepare_lines<double>(int, int);

template <typename T>
hipError_t transpose(const T* in, T* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_transpose<T>, dim3(unsigned(n / 32), unsigned(n / 32)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

template hipError_t rowpass_fwd<float>(const float*, float*, int, const Tables<float>&, const Omega&, int64_t,
                                       hipStream_t);
template hipError_t rowpass_fwd<double>(const double*, double*, int, const Tables<double>&, const Omega&, int64_t,
                                        hipStream_t);
template hipError_t rowpass_adj<float>(const float*, float*, int, const Tables<float>&, const Omega&, int64_t,
                                       hipStream_t);
template hipError_t rowpass_adj<double>(const double*, double*, int, const Tables<double>&, const Omega&, int64_t,
                                        hipStream_t);
template hipError_t colpass_fwd<float>(const float*, float*, int, const Tables<float>&, hipStream_t);
template hipError_t colpass_fwd<double>(const double*, double*, int, const Tables<double>&, hipStream_t);
template hipError_t colpass_adj<float>(const float*, float*, int, const Tables<float>&, hipStream_t);
template hipError_t colpass_adj<double>(const double*, double*, int, const Tables<double>&, hipStream_t);
template hipError_t line1d_fwd_fused<float>(const float*, float*, int, int, const Tables<float>&, const Omega&,
                                            hipStream_t);
template hipError_t line1d_fwd_fused<double>(const double*, double*, int, int, const Tables<double>&, const Omega&,
                                             hipStream_t);
template hipError_t line1d_adj_fused<float>(const float*, float*, int, int, const Tables<float>&, const Omega&,
                                            hipStream_t);
template hipError_t line1d_adj_fused<double>(const double*, double*, int, int, const Tables<double>&, const Omega&,
                                             hipStream_t);
template hipError_t transpose<float>(const float*, float*, int64_t, hipStream_t);
template hipError_t transpose<double>(const double*, double*, int64_t, hipStream_t);

}  // namespace wh2wav_fast
