// selector.h -- learned plan selector (host side): plan features, weights
// file, host inference.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "offt_internal.h"

namespace offt {

// Feature vector of (grid, plan): log2 of the axis lengths, batch and total
// points, precision, one-hot axis order, and per axis (a, b, c): strided
// flag, stage count, counts of radix-16/8/4/2/3/5 stages, log2 tile width,
// log2 threads per line, position in the pass order, count of radix-32
// stages, log2 of the parts its LDS exchanges run in, XCD-contiguous tile
// order.
constexpr int kAxisFeatures = 15;
constexpr int kFeatureDim = 12 + 3 * kAxisFeatures;
void plan_features(int dtype, const int64_t dims[3], int64_t batch, const PlanChoice& c, float* out);

// Ranks the candidate plans of a grid with the learned time model and returns
// the predicted-fastest one.  Fails (non-zero, reason in *why) when the weights
// are missing or unreadable or do not match the feature layout; the caller
// then falls back to exhaustive timing.
int learned_choice(int dtype, const int64_t dims[3], int64_t batch, const char* weights_path,
                   PlanChoice* c, std::string* why);

}  // namespace offt
