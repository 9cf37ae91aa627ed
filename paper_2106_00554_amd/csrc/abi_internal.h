// Internal helpers shared by the C-ABI translation units (not exported).
#pragma once

#include <cstdint>
#include <exception>
#include <new>
#include <string>

#include "../../include/wh2wav.h"

namespace wh2wav {

// Stores `msg` as the calling thread's last error and returns `code`.
int set_error(int code, const std::string& msg);

// The same, for use while handling an exception: never throws (on a failed
// copy of the message the last error is left empty).
int set_error_nothrow(int code, const char* msg) noexcept;

// Runs the body of an extern "C" entry point so that no C++ exception crosses
// the interface: std::bad_alloc becomes WH2WAV_ENOMEM, any other exception
// WH2WAV_EINTERNAL, each with a message in wh2wav_last_error().
template <typename F>
int guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return set_error_nothrow(WH2WAV_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error_nothrow(WH2WAV_EINTERNAL, e.what());
  } catch (...) {
    return set_error_nothrow(WH2WAV_EINTERNAL, "unexpected internal error");
  }
}

// Registry of live handles (plans and batches): calls with a handle that was
// never returned by a plan call, or was already destroyed, fail with
// WH2WAV_EINVAL instead of touching freed memory.
void handle_add(const void* h);
bool handle_remove(const void* h);
bool handle_live(const void* h);

struct PlanShape {
  int dim, j, q, nu, dtype;
  int64_t M, N, m;
  int64_t xlen, ntot;  // coefficients (M_1 ... M_dim) and Walsh samples (N_1 ... N_dim)
};
PlanShape plan_shape(wh2wav_plan_t p);

// What the fused batch launches need of a plan: its device tables and
// sample bitmask, and the shape flags that decide whether the kernel can run
// it (1D / square 2D, isotropic).
struct PlanView {
  const void *h, *g, *tabT, *bandL, *bandR, *synL, *synR;  // device, element type = dtype
  int nu, q, Q, per, dim, j, j0, tensor, nd, dtype, full_omega;
  int64_t M, N, m;
  const uint32_t* mask;
  const int64_t* row_ptr;
  int64_t wpr;
};
PlanView plan_view(wh2wav_plan_t p);

}  // namespace wh2wav
