// selector.h -- learned plan selector (host side).
#pragma once

#include <stdint.h>

#include <string>

#include "offt_internal.h"

namespace offt {

// Ranks the candidate plans of a grid with the learned time model and returns
// the predicted-fastest one.  Fails (non-zero, reason in *why) when the weights
// are missing or unreadable or no candidate is feasible; the caller then falls
// back to exhaustive timing.
int learned_choice(int dtype, const int64_t dims[3], int64_t batch, const char* weights_path,
                   PlanChoice* c, std::string* why);

}  // namespace offt
