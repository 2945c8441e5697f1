// Shapes of the sample-count predictor network (mlp.hip) shared with learned.hip.
#pragma once

#include "qfs_internal.h"

namespace qfs {

constexpr int kMlpF = 64, kMlpH = 128, kMlpO = 2;
// One FP32 parameter vector: W1 [H][F], b1 [H], W2 [H][H], b2 [H], W3 [O][H], b3 [O].
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpH * kMlpF;
constexpr int kMlpW2 = kMlpB1 + kMlpH;
constexpr int kMlpB2 = kMlpW2 + kMlpH * kMlpH;
constexpr int kMlpW3 = kMlpB2 + kMlpH;
constexpr int kMlpB3 = kMlpW3 + kMlpO * kMlpH;
constexpr int kMlpNP = kMlpB3 + kMlpO;
constexpr char kMlpMagic[8] = {'Q', 'F', 'S', 'M', 'L', 'P', '1', '\0'};

// Forward pass of the loaded network on B feature rows (device [B][64]) into device
// [B][2]; synchronises the stream. QFS_EINVAL when no weights are loaded.
int mlp_predict(int B, const float *features_dev, float *out_dev, hipStream_t s);

}  // namespace qfs
