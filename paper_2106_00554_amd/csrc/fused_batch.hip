// Fused launches of the small instances of a batch (the scheme is described
// in fused_batch.h).
//
// Stages of one instance (d = 1 or 2, M = 2^j per axis, the isotropic layout):
//   forward  copy-in (x -> A and B), then per level k = J0 .. j-1 and axis one
//            synthesis level on the block [0, 2^{k+1})^d (A and B in turn),
//            then G along axis 0 into Z (2D) and G along the last axis with
//            the gather onto Omega (Sec. 5: alpha = G xi G^T);
//   adjoint  G^T along the last axis with the scatter, G^T along axis 0 (2D),
//            then the analysis levels in reverse order; the last axis of each
//            level also writes its block to x, so that every element of x
//            ends with its final value.
// A stage writes only inside its block, and both buffers start as copies of
// x, so outside the block each buffer holds the coefficients a later level
// reads.
#include "fused_batch.h"

#include <algorithm>
#include <string>

#include "generic_lines.h"

namespace wh2wav_fused {
namespace {

using namespace wh2wav_generic;

enum StageKind { kCopyIn = 0, kLevel = 1, kFwdLines = 2, kAdjLines = 3, kCopyOut = 4 };
enum BufId { kIn = 0, kOut = 1, kBufA = 2, kBufB = 3, kBufZ = 4 };

template <typename T>
struct Inst {
  Tables<T> t;
  OmegaDev om;
  int dim, j;
  int64_t M;
  int64_t ws_off;  // bytes from the batch workspace to the instance's A | B | Z
};

struct Stage {
  int inst, kind;
  int k, axis, analysis, out_too;  // wavelet level
  int src, dst;                    // BufId
  int j, gather;                   // line pass
  LineMap im, omap;
  RowMap rm;
  int64_t tiles, item0;
};

// Level and copy stages: elements per work item (4 per thread).
constexpr int kTileElems = 4 * kThreads;

template <typename T>
__device__ __forceinline__ T* buffer(const Inst<T>& I, int id, char* ws, void* const* io, int slot) {
  T* base = reinterpret_cast<T*>(ws + I.ws_off);
  const int64_t x = I.dim == 2 ? I.M * I.M : I.M;
  switch (id) {
    case kIn: return static_cast<T*>(io[2 * slot]);
    case kOut: return static_cast<T*>(io[2 * slot + 1]);
    case kBufA: return base;
    case kBufB: return base + x;
    default: return base + 2 * x;
  }
}

// One round: the items [item0, item0 + nitems) of the stages
// [stage0, stage0 + nstages), a grid-stride loop of whole workgroups.  NU: the
// wavelet order of every instance when they share one (the line code then
// unrolls its taps), 0 for a mix.
template <typename T, int NU>
__global__ void __launch_bounds__(kThreads) k_round(const Inst<T>* __restrict__ insts,
                                                    const Stage* __restrict__ stages, int stage0, int nstages,
                                                    int64_t item0, int64_t nitems, char* ws, void* const* io) {
  extern __shared__ unsigned char smem_raw[];
  const int tid = int(threadIdx.x);
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t item = item0 + it;
    int lo = stage0, hi = stage0 + nstages - 1;  // the last stage whose first item is <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (stages[mid].item0 <= item) lo = mid;
      else hi = mid - 1;
    }
    const Stage S = stages[lo];
    const Inst<T> I = insts[S.inst];
    const int64_t tile = item - S.item0;
    const T* src = buffer<T>(I, S.src, ws, io, S.inst);
    T* dst = buffer<T>(I, S.dst, ws, io, S.inst);
    const int64_t M = I.M, xlen = I.dim == 2 ? M * M : M;
    if (S.kind == kCopyIn || S.kind == kCopyOut) {
      for (int64_t e = tile * kTileElems + tid; e < (tile + 1) * kTileElems && e < xlen; e += kThreads) {
        const T v = src[e];
        dst[e] = v;
        if (S.kind == kCopyIn) buffer<T>(I, kBufB, ws, io, S.inst)[e] = v;
      }
    } else if (S.kind == kLevel) {
      const int64_t size = int64_t(2) << S.k, belems = I.dim == 2 ? size * size : size;
      for (int64_t e = tile * kTileElems + tid; e < (tile + 1) * kTileElems && e < belems; e += kThreads) {
        int64_t pos = e, n = e, base = 0, es = 1;
        if (I.dim == 2) {
          const int64_t r = e / size, c = e % size;
          pos = r * M + c;
          if (S.axis == 0) n = r, base = c, es = M;
          else n = c, base = r * M, es = 1;
        }
        const T* line = src + base;
        T v;
        if (S.analysis)
          v = I.t.per ? analysis_value_per<T>(line, es, n, S.k, I.t) : analysis_value<T>(line, es, n, S.k, I.t);
        else
          v = I.t.per ? synth_value_per<T>(line, es, n, S.k, I.t) : synth_value<T>(line, es, n, S.k, I.t);
        dst[pos] = v;
        if (S.out_too) buffer<T>(I, kOut, ws, io, S.inst)[pos] = v;
      }
    } else if (S.kind == kFwdLines) {
      fwd_line<T, NU>(src, S.im, dst, S.omap, S.j, S.gather, S.rm, I.t, I.om, tile, smem_raw, int(threadIdx.x),
                      int(blockDim.x));
    } else {
      adj_line<T, NU>(src, S.im, dst, S.omap, S.j, S.gather, S.rm, I.t, I.om, tile, smem_raw, int(threadIdx.x),
                      int(blockDim.x));
    }
    __syncthreads();  // the next item reuses the LDS
  }
}

#define WH2WAV_ROUND_NUS(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)
template <typename T>
const void* round_kernel(int nu) {
#define X(V) \
  if (nu == V) return reinterpret_cast<const void*>(k_round<T, V>);
  WH2WAV_ROUND_NUS(X)
#undef X
  return nullptr;
}

LineMap lines_at(int64_t ls, int64_t es) { return LineMap{int64_t(1) << 62, 0, ls, es}; }

int herr(hipError_t e, const char* what) {
  return wh2wav::set_error(WH2WAV_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Stage chain of one instance (index `slot` in the program).
std::vector<Stage> chain(const wh2wav::PlanView& v, int slot, int dir) {
  std::vector<Stage> out;
  auto base = [&](int kind) {
    Stage s{};
    s.inst = slot, s.kind = kind;
    s.im = lines_at(0, 1), s.omap = lines_at(0, 1), s.rm = RowMap{0, 0, 0};
    return s;
  };
  const int64_t M = v.M, N = v.N, xlen = v.dim == 2 ? M * M : M;
  const int64_t copy_tiles = (xlen + kTileElems - 1) / kTileElems;
  auto level = [&](int k, int axis, int analysis, int src, int dst, int out_too) {
    Stage s = base(kLevel);
    const int64_t size = int64_t(2) << k, belems = v.dim == 2 ? size * size : size;
    s.k = k, s.axis = axis, s.analysis = analysis, s.src = src, s.dst = dst, s.out_too = out_too;
    s.tiles = (belems + kTileElems - 1) / kTileElems;
    return s;
  };
  auto lines = [&](int kind, int src, int dst, LineMap im, LineMap om, int gather, RowMap rm, int64_t n) {
    Stage s = base(kind);
    s.src = src, s.dst = dst, s.im = im, s.omap = om, s.gather = gather, s.rm = rm, s.j = v.j, s.tiles = n;
    return s;
  };
  if (dir == 0) {
    Stage c = base(kCopyIn);
    c.src = kIn, c.dst = kBufA, c.tiles = copy_tiles;
    out.push_back(c);
    int cur = kBufA;
    for (int k = v.j0; k < v.j; ++k)
      for (int a = 0; a < v.dim; ++a) {
        const int nxt = cur == kBufA ? kBufB : kBufA;
        out.push_back(level(k, a, 0, cur, nxt, 0));
        cur = nxt;
      }
    if (v.dim == 2) {
      out.push_back(lines(kFwdLines, cur, kBufZ, lines_at(1, M), lines_at(1, M), 0, RowMap{0, 0, 0}, M));
      out.push_back(lines(kFwdLines, kBufZ, kOut, lines_at(M, 1), lines_at(0, 0), 1, RowMap{1, v.j, 0}, N));
    } else {
      out.push_back(lines(kFwdLines, cur, kOut, lines_at(0, 1), lines_at(0, 0), 1, RowMap{0, 0, 0}, 1));
    }
  } else {
    if (v.dim == 2) {
      out.push_back(lines(kAdjLines, kIn, kBufZ, lines_at(0, 0), lines_at(M, 1), 1, RowMap{1, v.j, 0}, N));
      out.push_back(lines(kAdjLines, kBufZ, kBufA, lines_at(1, M), lines_at(1, M), 0, RowMap{0, 0, 0}, M));
    } else {
      out.push_back(lines(kAdjLines, kIn, kBufA, lines_at(0, 0), lines_at(0, 1), 1, RowMap{0, 0, 0}, 1));
    }
    int cur = kBufA;
    if (v.j0 == v.j) {
      Stage c = base(kCopyOut);
      c.src = kBufA, c.dst = kOut, c.tiles = copy_tiles;
      out.push_back(c);
    }
    for (int k = v.j - 1; k >= v.j0; --k)
      for (int a = v.dim - 1; a >= 0; --a) {
        const int nxt = cur == kBufA ? kBufB : kBufA;
        out.push_back(level(k, a, 1, cur, nxt, a == 0 ? 1 : 0));
        cur = nxt;
      }
  }
  return out;
}

template <typename T>
int upload(const std::vector<wh2wav::PlanView>& views, const std::vector<size_t>& ws_off,
           const std::vector<Stage>& stages, Program* P) {
  std::vector<Inst<T>> insts;
  for (int i : P->members) {
    const auto& v = views[i];
    Inst<T> I{};
    I.t.h = static_cast<const T*>(v.h), I.t.g = static_cast<const T*>(v.g);
    I.t.tabT = static_cast<const T*>(v.tabT), I.t.bandL = static_cast<const T*>(v.bandL);
    I.t.bandR = static_cast<const T*>(v.bandR), I.t.synL = static_cast<const T*>(v.synL);
    I.t.synR = static_cast<const T*>(v.synR);
    I.t.nu = v.nu, I.t.q = v.q, I.t.Q = v.Q, I.t.per = v.per;
    I.om.mask = v.mask, I.om.row_ptr = v.row_ptr, I.om.wpr = v.wpr, I.om.full = v.full_omega;
    I.dim = v.dim, I.j = v.j, I.M = v.M, I.ws_off = int64_t(ws_off[i]);
    insts.push_back(I);
  }
  hipError_t e = hipMalloc(&P->d_inst, sizeof(Inst<T>) * insts.size());
  if (e == hipSuccess) e = hipMemcpy(P->d_inst, insts.data(), sizeof(Inst<T>) * insts.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&P->d_stage, sizeof(Stage) * stages.size());
  if (e == hipSuccess)
    e = hipMemcpy(P->d_stage, stages.data(), sizeof(Stage) * stages.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return herr(e, "fused program upload");
  e = hipFuncSetAttribute(round_kernel<T>(P->nu), hipFuncAttributeMaxDynamicSharedMemorySize, int(P->smem));
  if (e != hipSuccess) return herr(e, "fused kernel setup");
  return WH2WAV_OK;
}

}  // namespace

bool eligible(const wh2wav::PlanView& v) {
  if (v.nd || v.tensor || v.m == 0) return false;
  return (v.dim == 1 && v.M <= 1024) || (v.dim == 2 && v.M <= 512);
}

int build(const std::vector<wh2wav::PlanView>& views, const std::vector<size_t>& ws_off,
          const std::vector<int>& members, int dtype, int dir, Program* P) {
  P->dtype = dtype, P->dir = dir, P->members = members, P->ninst = int(members.size());
  // the chains, then the stages numbered round by round
  std::vector<std::vector<Stage>> chains;
  size_t longest = 0;
  int64_t Mmax = 1, wpr_max = 0;
  bool sparse = false;
  P->nu = members.empty() ? 0 : views[members[0]].nu;  // the shared wavelet order, or 0
  for (int slot = 0; slot < P->ninst; ++slot) {
    const auto& v = views[members[slot]];
    chains.push_back(chain(v, slot, dir));
    longest = std::max(longest, chains.back().size());
    Mmax = std::max(Mmax, v.M);
    wpr_max = std::max(wpr_max, v.wpr);
    if (v.nu != P->nu) P->nu = 0;
    sparse = sparse || !v.full_omega;
  }
  const size_t elem = dtype == WH2WAV_F64 ? 8 : 4;
  P->smem = 2 * size_t(Mmax) * elem + (sparse ? sizeof(int) * (2 * size_t(wpr_max) + kThreads) : 0);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return herr(e, "device query");
  std::vector<Stage> stages;
  int64_t item = 0;
  for (size_t r = 0; r < longest; ++r) {
    Round rd{int(stages.size()), 0, item, 0, 0};
    for (int slot = 0; slot < P->ninst; ++slot) {
      if (r >= chains[slot].size()) continue;
      Stage s = chains[slot][r];
      s.item0 = item;
      item += s.tiles;
      stages.push_back(s);
      ++rd.nstages;
    }
    rd.nitems = item - rd.item0;
    // a few items per workgroup at most, and no more workgroups than the
    // machine holds at eight per CU
    rd.grid = int(std::min<int64_t>(rd.nitems, int64_t(cus) * 8));
    P->rounds.push_back(rd);
  }
  return dtype == WH2WAV_F64 ? upload<double>(views, ws_off, stages, P) : upload<float>(views, ws_off, stages, P);
}

int launch(const Program& P, void* ws, void* const* io_dev, hipStream_t st) {
  const void* kernel = P.dtype == WH2WAV_F64 ? round_kernel<double>(P.nu) : round_kernel<float>(P.nu);
  if (!kernel) return wh2wav::set_error(WH2WAV_EINTERNAL, "no fused kernel for this wavelet order");
  const void* insts = P.d_inst;
  const Stage* stages = static_cast<const Stage*>(P.d_stage);
  char* wsc = static_cast<char*>(ws);
  for (const Round& rd : P.rounds) {
    int stage0 = rd.stage0, nstages = rd.nstages;
    int64_t item0 = rd.item0, nitems = rd.nitems;
    void* const* io = io_dev;
    void* args[] = {&insts, &stages, &stage0, &nstages, &item0, &nitems, &wsc, &io};
    hipError_t e = hipLaunchKernel(kernel, dim3(unsigned(rd.grid)), dim3(kThreads), args, P.smem, st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return herr(e, "fused round");
  }
  return WH2WAV_OK;
}

void release(Program* P) {
  if (P->d_inst) (void)hipFree(P->d_inst);
  if (P->d_stage) (void)hipFree(P->d_stage);
  P->d_inst = P->d_stage = nullptr;
}

}  // namespace wh2wav_fused
