// Constants shared by the host code and the kernels (no HIP dependency, so that the
// host-only arithmetic can be built and checked on a CPU).
#pragma once

namespace pmnu {

constexpr double kC_KMS = 299792.458;
constexpr double kH0 = 100.0 / kC_KMS;                 // h/Mpc, c = 1
constexpr double kTnu0 = 1.95 * 8.617333262e-5;         // eV (1.95 K)
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxSpecies = 4;                          // neutrino species with their own masses

}  // namespace pmnu
