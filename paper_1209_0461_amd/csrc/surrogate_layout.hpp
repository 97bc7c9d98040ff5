// Layout of the surrogate network's FP32 weight blob (see include/pm_nu.h) and the
// definition of its inputs.
//
// Inputs of (box, bin), with n stored nodes a_0 < ... < a_{n-1} before the current a_now,
// A(u) the stored P_M^{1/2}(k_b) linear in u = ln a between stored nodes (as the history
// integral reads it) and P = P_cdm^{1/2}(k_b, a_now):
//   0  ln k_b          1  ln a_now        2  M_nu [eV]
//   3  ln a_now - ln a_{n-1} (how far the current step is from the last stored node)
//   4  P_nu^{1/2}(k_b, a_{n-1}) / P (the neutrino amplitude the first iteration puts into
//      the current node, eq. (P-final) and Sec. 4.3 (iii))
//   5  ln(a_now / a_0) (how far back the history and its initial-condition term lie)
//   6  ln(k_b (s(a_now) - s(a_{n-1})) T_nu0 / m_nu): the free-streaming kernel's argument
//      across the last interval, eq. (P-final)
//   7 + m  A(ln a_{n-1} - lag_m) / P,  m = 0..8, lags in ln a below
// defined when the stored history reaches the last lag below the last stored node. The
// lags are in ln a rather than in stored nodes, so that the inputs mean the same for any
// spacing of the stored nodes. The network is trained on, and used for, inputs with
// input 6 at most kSurXLastMax: beyond it the kernel oscillates across the last interval
// (its argument is more than e^1.5 = 4.5 radians there) and the integral is left exact.
#pragma once

namespace pmnu {
constexpr int kSurIn = 16;        // inputs
constexpr int kSurLags = 9;       // history samples among them
constexpr double kSurLag[kSurLags] = {0.0, 0.05, 0.1, 0.2, 0.35, 0.55, 0.8, 1.2, 2.1};
constexpr double kSurXLastMax = 1.5;
constexpr int kOffW1 = 0;                         // [16][128]
constexpr int kOffB1 = kOffW1 + kSurIn * 128;     // [128]
constexpr int kOffW2 = kOffB1 + 128;              // [128][128]
constexpr int kOffB2 = kOffW2 + 128 * 128;
constexpr int kOffW3 = kOffB2 + 128;              // [128][128]
constexpr int kOffB3 = kOffW3 + 128 * 128;
constexpr int kOffW4 = kOffB3 + 128;              // [128]
constexpr int kOffB4 = kOffW4 + 128;
constexpr int kSurParams = kOffB4 + 1;            // 35329
constexpr int kOffMu = kSurParams;                // feature mean [16]
constexpr int kOffSigma = kOffMu + kSurIn;        // feature scale [16]
constexpr int kOffMin = kOffSigma + kSurIn;       // feature minimum [16]
constexpr int kOffMax = kOffMin + kSurIn;         // feature maximum [16]
constexpr int kOffYMu = kOffMax + kSurIn;         // target mean
constexpr int kOffYSigma = kOffYMu + 1;           // target scale
constexpr int kSurBlob = kOffYSigma + 1;          // 35395
static_assert(kSurParams == 35329, "parameter count");
}  // namespace pmnu
