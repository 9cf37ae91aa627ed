// Host-side plan construction for the Walsh-to-boundary-wavelet operator.
//
// Everything here runs on the CPU in binary128 arithmetic and produces the
// small input-independent tables the GPU kernels consume:
//   * Daubechies filters h, g (Sec. 3.2, minimum phase, supp [-nu+1, nu]);
//   * the interior table T_l[s] = 2^{-j/2} (Walsh transform of phi(. + l) on
//     [0,1)) at s < 2^q, i.e. the coefficients of the operator D_l (Sec. 4.1),
//     which only needs s = floor(n / 2^j) < 2^q;
//   * the boundary tables of Prop. 4.2 for the vanishing-moment-preserving
//     ("bd") boundary functions, laid out as dense bands;
//   * the boundary blocks of the one-level synthesis matrix used by the
//     inverse DWT that maps C_{psi,j} to B_{phi,j} (Remark on compressive
//     sensing, Sec. 4);
//   * the sampling set Omega as a bitmask with per-row offsets.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wh2wav.h"

namespace wh2wav {

struct HostPlan {
  int dim = 1, j = 0, q = 1, j0 = 0, nu = 2, dtype = WH2WAV_F64;
  int family = WH2WAV_DB;
  bool per = false;          // periodic extension (Sec. 3.2): no boundary functions; bands and blocks are zero
  bool tensor = false;       // tensor-product basis (products of 1D basis functions), 2D and 3D
  int64_t M = 0, N = 0;      // per dimension: M = 2^j, N = 2^{j+q}
  int Q = 2;                 // 2^q phases
  // Three dimensions or unequal sides: the per-axis path.  Axis a has
  // M_a = 2^{ja[a]}, N_a = 2^{ja[a] + q} (entries at a >= dim are 1), and its
  // own interior and band tables (the 2^{-j_a/2} factor differs per axis).
  bool nd = false;
  int ja[3] = {0, 0, 0};
  int64_t Ma[3] = {1, 1, 1}, Na[3] = {1, 1, 1};
  std::vector<double> tabT_ax[3], tabBL_ax[3], tabBR_ax[3];

  std::vector<double> h, g;  // 2 nu taps each, index c + nu - 1 for c in [-nu+1, nu]
  // T[(l + nu - 1) * Q + s], l in [-nu+1, nu-1]
  std::vector<double> tabT;
  // Left band: rows p in [0, 2nu-2], cols m in [0, nu): BL[(p * nu + m) * Q + s]
  // Right band: rows p in [M-2nu+1, M-1] (stored p - (M-2nu+1)), cols m' in [0, nu)
  // for the function at position M-1-m': BR[(p * nu + m') * Q + s].
  std::vector<double> tabBL, tabBR;
  // One-level synthesis boundary blocks, level k -> k+1:
  // synL[n * 2nu + c], output rows n in [0, 3nu-2], input columns c < nu:
  //   scaling function c, c >= nu: wavelet c - nu (left boundary functions).
  // synR[n * 2nu + c], rows n in [2^{k+1}-3nu+1, 2^{k+1}-1] (stored relative),
  //   columns c < nu: scaling function at position 2^k-1-c, c >= nu: wavelet
  //   at position 2^k-1-(c-nu).
  std::vector<double> synL, synR;

  bool full_omega = true;
  int64_t m = 0;
  int64_t rows = 1;          // 1 (1D), N (2D) or N_1 ... N_{dim-1}: all but the last axis
  int64_t row_len = 0;       // samples per row: N (1D, 2D) or N_dim
  int64_t words_per_row = 0; // ceil(row_len / 32)
  std::vector<uint32_t> mask;        // rows * words_per_row
  std::vector<int64_t> row_ptr;      // rows + 1
  // 2D sample list for the line kernels (only when Omega is not full).  A
  // row n1 of the N x N Walsh array splits into Q phase lines n2 = s M + b;
  // seg_ptr[n1 * Q + s] is the offset in y of the first sample of that phase
  // line (N Q + 1 entries) and pos16[i] the natural-order position
  // k = bitrev(gray(b)) xor (s & 1) of sample i within its phase line.
  std::vector<uint16_t> pos16;
  std::vector<int64_t> seg_ptr;
  // 1D sample list (only when Omega is not full): pos32[i] = s M + k, the flat
  // natural-order index of sample n_i = s M + b, k = bitrev(gray(b)) xor (s & 1).
  std::vector<int32_t> pos32;
};

// Validates the descriptor and fills the plan.  Returns a WH2WAV_* status;
// on failure `err` holds a message.
int build_host_plan(const wh2wav_desc* d, HostPlan* out, std::string* err);

// Shape/table builders shared by the two entry points that need them
// (plan creation and host-table introspection).  They depend only on nu
// and q (and j for the 2^{-j/2} factor).
int build_tables(int family, int nu, int q, int j, HostPlan* out, std::string* err);

}  // namespace wh2wav
