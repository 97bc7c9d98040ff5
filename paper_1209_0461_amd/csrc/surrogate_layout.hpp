// Layout of the surrogate network's FP32 weight blob (see include/pm_nu.h).
#pragma once

namespace pmnu {
constexpr int kSurIn = 11;        // inputs: ln k, ln a, M_nu, 8 history ratios
constexpr int kSurHistory = 8;    // stored nodes used as inputs
constexpr int kOffW1 = 0;                         // [11][128]
constexpr int kOffB1 = kOffW1 + kSurIn * 128;     // [128]
constexpr int kOffW2 = kOffB1 + 128;              // [128][128]
constexpr int kOffB2 = kOffW2 + 128 * 128;
constexpr int kOffW3 = kOffB2 + 128;              // [128][128]
constexpr int kOffB3 = kOffW3 + 128 * 128;
constexpr int kOffW4 = kOffB3 + 128;              // [128]
constexpr int kOffB4 = kOffW4 + 128;
constexpr int kSurParams = kOffB4 + 1;            // 34689
constexpr int kOffMu = kSurParams;                // feature mean [11]
constexpr int kOffSigma = kOffMu + kSurIn;        // feature scale [11]
constexpr int kOffMin = kOffSigma + kSurIn;       // feature minimum [11]
constexpr int kOffMax = kOffMin + kSurIn;         // feature maximum [11]
constexpr int kOffYMu = kOffMax + kSurIn;         // target mean
constexpr int kOffYSigma = kOffYMu + 1;           // target scale
constexpr int kSurBlob = kOffYSigma + 1;          // 34735
static_assert(kSurParams == 34689, "parameter count");
}  // namespace pmnu
