// Internal helpers shared by the C-ABI translation units (not exported).
#pragma once

#include <cstdint>
#include <string>

#include "../../include/wh2wav.h"

namespace wh2wav {

// Stores `msg` as the calling thread's last error and returns `code`.
int set_error(int code, const std::string& msg);

struct PlanShape {
  int dim, j, q, nu, dtype;
  int64_t M, N, m;
};
PlanShape plan_shape(wh2wav_plan_t p);

}  // namespace wh2wav
