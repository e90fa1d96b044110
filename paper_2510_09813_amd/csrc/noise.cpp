// Shot-to-shot parameter noise (Sec. III.A models open-system effects either by the Lindblad
// equation or by varying the Hamiltonian's parameters from shot to shot; this is the
// second).  Ensemble member s draws standard normal variates and perturbs
//   the drive amplitude by one factor for all atoms:  Omega_i(t) -> (1 + s_Omega g_0) Omega_i(t),
//   each atom's detuning by a constant offset:        delta_i(t) -> delta_i(t) + s_delta g_{1+i},
//   each atom's position on each axis:                r_i,a -> r_i,a + s_r g_{1+N+3i+a}.
// Variate c = s (4N + 1) + j is a Box-Muller transform (Box & Muller 1958) of outputs 2c and
// 2c + 1 of SplitMix64 (Steele, Lea & Flood 2014) seeded with the noise seed; the generator
// is counter based (output k is the finaliser of seed + (k + 1) * gamma), so each member is
// drawn independently of the others and of the order in which members are formed.
#include <cmath>
#include <cstdint>

#include "engine.h"

namespace rsv {

namespace {

uint64_t splitmix64_out(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr double kTwoPi = 6.283185307179586476925286766559;

}  // namespace

double noise_gaussian(uint64_t seed, uint64_t c) {
  const double u1 = (double)((splitmix64_out(seed, 2 * c) >> 11) + 1) * 0x1.0p-53;  // (0, 1]
  const double u2 = (double)(splitmix64_out(seed, 2 * c + 1) >> 11) * 0x1.0p-53;    // [0, 1)
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(kTwoPi * u2);
}

void noise_member(const rsv_noise& nz, uint64_t seed, int n, int64_t s, const double* xyz,
                  double* factor, double* offsets, double* xyz_out) {
  const uint64_t per = 4 * (uint64_t)n + 1, c0 = (uint64_t)s * per;
  *factor = 1.0 + nz.omega_rel_sigma * noise_gaussian(seed, c0);
  for (int i = 0; i < n; ++i) offsets[i] = nz.delta_sigma * noise_gaussian(seed, c0 + 1 + i);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a)
      xyz_out[3 * i + a] =
          xyz[3 * i + a] + nz.position_sigma_um * noise_gaussian(seed, c0 + 1 + n + 3 * i + a);
}

}  // namespace rsv
