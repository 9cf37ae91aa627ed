// Fused launches for the small operators of a batch (internal interface of
// batch.hip).
//
// Every instance the fused path takes is a chain of stages (copy-in, one
// wavelet level along one axis, a pass of line transforms, ...), each split
// into tiles of one workgroup's work: 1024 elements of a wavelet level, or
// one line.  Round r is stage r of every instance; one launch runs all the
// tiles of a round, whatever instance they belong to, so a batch of small
// operators costs one launch per round (about 2 + 2 (j - J0) + 2 in 2D)
// instead of its instances' launches one after another.  The kernel
// boundaries between rounds order the stages of each instance; no workgroup
// waits for another.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "abi_internal.h"

namespace wh2wav_fused {

// Instances the fused path can run: 1D lines of at most 1024 values and
// square 2D arrays of at most 512^2, isotropic basis (boundary-corrected or
// periodic), at least one sample.
bool eligible(const wh2wav::PlanView& v);

struct Round {
  int stage0, nstages;  // the round's stages in the stage table
  int64_t item0, nitems;
  int grid;             // workgroups of its launch (a grid-stride loop over the items)
};

// Device program of one direction for the eligible instances of one element
// type: instance and stage tables and the rounds.
struct Program {
  int dtype = 0, dir = 0;
  int ninst = 0;
  size_t smem = 0;          // dynamic LDS per workgroup
  int nu = 0;               // wavelet order shared by every instance, 0 for a mix
  void* d_inst = nullptr;   // Inst<T>[ninst]
  void* d_stage = nullptr;  // Stage[all rounds]
  std::vector<Round> rounds;
  std::vector<int> members;  // batch index of each program instance
};

// Builds the program of direction `dir` (0 forward, 1 adjoint) for the
// instances `members` of the batch (views[i], workspace offset ws_off[i] in
// bytes from the batch workspace), all of element type `dtype`.
int build(const std::vector<wh2wav::PlanView>& views, const std::vector<size_t>& ws_off,
          const std::vector<int>& members, int dtype, int dir, Program* out);

// Launches the rounds of the program on `st`, in order.  io_dev: device array
// of 2 pointers per program instance (input, output of the direction).
int launch(const Program& prog, void* ws, void* const* io_dev, hipStream_t st);

void release(Program* prog);

}  // namespace wh2wav_fused
