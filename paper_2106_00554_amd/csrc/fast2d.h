// Wave-level line kernels for the 2D operator (internal interface between the
// C-ABI file and the kernel file).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wh2wav_fast {

template <typename T>
struct Tables {
  const T* h;      // 2nu taps, index c + nu - 1
  const T* g;      // 2nu taps
  const T* tabT;   // (2nu-1) * Q, index (l + nu - 1) * Q + s
  const T* bandL;  // (2nu-1) * nu * Q, index (p * nu + m) * Q + s
  const T* bandR;  // (2nu-1) * nu * Q
  // the same bands, laid out so that the values one lane reads are
  // contiguous (compile-time offsets from one address):
  const T* bandLf;  // forward: index (s * (2nu-1) + p) * nu + m
  const T* bandRf;
  const T* bandLa;  // adjoint: index (s * nu + m) * (2nu-1) + p
  const T* bandRa;
  const T* synL;   // (3nu-1) * 2nu
  const T* synR;   // (3nu-1) * 2nu
  int nu, q, Q;
  int per;         // periodic extension (Sec. 3.2): no boundary functions, lines wrap around
};

struct Omega {
  const uint16_t* pos;     // natural position of every sample in its phase line (m entries)
  const int64_t* seg_ptr;  // N Q + 1 offsets into y, one per (row, phase)
  int full;                // every sample taken: y is the whole N x N array
};

// True when the wave kernels cover (element size, log2 M, nu, q).
bool supported(int elem_bytes, int logm, int nu, int q);

// Forward row pass: rows r of Z (N x M, natural row order) -> y (gather on Omega).
template <typename T>
hipError_t rowpass_fwd(const T* Z, T* y, int logm, const Tables<T>& t, const Omega& om, int64_t rows, hipStream_t st);
// Adjoint row pass: y (scatter from Omega) -> rows r of Zt (N x M).
template <typename T>
hipError_t rowpass_adj(const T* y, T* Zt, int logm, const Tables<T>& t, const Omega& om, int64_t rows, hipStream_t st);
// Forward column pass: rows of xi^T (M x M) -> Z (N x M), Z[s M + k, c] natural order.
template <typename T>
hipError_t colpass_fwd(const T* xiT, T* Z, int logm, const Tables<T>& t, hipStream_t st);
// Adjoint column pass: Zt (N x M) -> rows of xi'^T (M x M).
template <typename T>
hipError_t colpass_adj(const T* Zt, T* xiT, int logm, const Tables<T>& t, hipStream_t st);
// Multilevel 2D inverse DWT of the quadtree array x (M x M) into xi^T (outT);
// s0, s1 are M x M scratch arrays (row stride M).
template <typename T>
hipError_t idwt2d(const T* x, T* outT, T* s0, T* s1, int64_t M, int j0, int j, const Tables<T>& t, hipStream_t st);
// Its transpose: xi'^T (inT) -> quadtree x.
template <typename T>
hipError_t dwt2d(const T* inT, T* x, T* s0, T* s1, int64_t M, int j0, int j, const Tables<T>& t, hipStream_t st);
// The 1D operator on one line of M = 2^logm <= 2048 values in one launch per
// direction (wavelet levels in LDS fused with the line transform): whether
// (element size, log2 M, nu, q) fits, and the two directions (x, y device
// arrays of M and m values; J0 = j0).
bool line1d_fused(int elem_bytes, int logm, int nu, int q);
template <typename T>
hipError_t line1d_fwd_fused(const T* x, T* y, int j0, int logm, const Tables<T>& t, const Omega& om,
                            hipStream_t st);
template <typename T>
hipError_t line1d_adj_fused(const T* y, T* x, int j0, int logm, const Tables<T>& t, const Omega& om,
                            hipStream_t st);
// One-time setup (dynamic LDS limits) for the line kernels of (log2 M, nu).
template <typename T>
hipError_t prepare_lines(int logm, int nu);
// One-time setup (dynamic LDS limits) for the 2D wavelet kernels of order nu.
template <typename T>
hipError_t prepare_dwt2d(int nu);
// out = in^T for an n x n row-major block (n a multiple of 32).
template <typename T>
hipError_t transpose(const T* in, T* out, int64_t n, hipStream_t st);


// ------------------------------------------------ one-dimensional path
// True when the 1D kernels cover (element size, log2 M, nu, q).
bool supported1d(int elem_bytes, int logm, int nu, int q);
// Multilevel inverse DWT of x (M = 2^j values, C_{psi,j} order) into xi;
// s0 is an M-element scratch line.
template <typename T>
hipError_t idwt1d(const T* x, T* xi, T* s0, int j0, int j, const Tables<T>& t, hipStream_t st);
// Its transpose: xi (overwritten) -> x; s0 scratch.
template <typename T>
hipError_t dwt1d(T* xi, T* x, T* s0, int j0, int j, const Tables<T>& t, hipStream_t st);
// Table product, natural-order transform and gather (pos: flat natural index
// of every sample in L; full: every sample taken, m = N).  L: Q M scratch.
template <typename T>
hipError_t line1d_fwd(const T* xi, T* L, T* y, int j, const Tables<T>& t, const int32_t* pos, int64_t m, int full,
                      hipStream_t st);
// Its transpose: y -> xi.
template <typename T>
hipError_t line1d_adj(const T* y, T* L, T* xi, int j, const Tables<T>& t, const int32_t* pos, int64_t m, int full,
                      hipStream_t st);
// Every wavelet level of `lines` lines of 2^j values, one line per
// workgroup in LDS: synthesis j0 .. j-1, or with `analysis` its transpose.
// Line r starts at (r / inner) os + r % inner, its values es apart, in `in`
// and `out` alike (in == out allowed).  lines_levels_fit: whether a line of
// 2^j values of this element size fits.
bool lines_levels_fit(int elem_bytes, int j);
template <typename T>
hipError_t lines_levels(const T* in, T* out, int64_t lines, int64_t inner, int64_t os, int64_t es, int j0, int j,
                        int analysis, const Tables<T>& t, hipStream_t st);
// One-time setup (dynamic LDS limits) of the 1D wavelet kernels of order nu.
template <typename T>
hipError_t prepare_1d(int nu);

}  // namespace wh2wav_fast
