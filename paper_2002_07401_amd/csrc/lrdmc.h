// Lattice-regularised diffusion Monte Carlo on the JAGP guiding function
// (Lattice regularized Monte Carlo section): device-side declarations.
#pragma once

#include "internal.h"

namespace qmc {

constexpr int kHops = 6;                 // +x, -x, +y, -y, +z, -z per electron
constexpr double kTfCoef = 0.8853;       // Thomas-Fermi length 0.8853 Z^{-1/3} bohr

// Per-walker terms (the order of qmc_lrdmc_term in qmc.h).
enum {
  kLrEloc = 0, kLrEkin = 1, kLrLapA = 2, kLrVaShift = 3, kLrVsf = 4, kLrEscape = 5,
  kLrHfnDiag = 6, kLrTerms = 7
};

struct LrdmcParams {
  double a;          // hop length (near nuclei with a double grid)
  double a_val;      // hop length in the valence region (> 0: double grid)
  double tf_scale;   // double grid: a within tf_scale Thomas-Fermi lengths of a nucleus
  double gamma;      // fixed-node spin-flip parameter
};

// Walker-owned LRDMC state (allocated with the walker set).
struct LrdmcDev {
  double* ratio;     // [Wk][N][6]  Psi(x')/Psi(x) of the lattice hops
  double* ah;        // [Wk][N]     hop length of each electron
  double* terms;     // [Wk][kLrTerms]
  double* ekin;      // [Wk] kinetic energy of the last evaluation
  double* eloc;      // [Wk] local energy of the last evaluation
};

hipError_t launch_lrdmc_hops(const SysDev& s, const WalkDev& w, const LrdmcDev& l, const LrdmcParams& p,
                             hipStream_t st);
hipError_t launch_lrdmc_advance(const SysDev& s, const WalkDev& w, const LrdmcDev& l, const LrdmcParams& p,
                                const double* xi, double* weight, double* tau_left, double* r_next,
                                int32_t* hop, hipStream_t st);

}  // namespace qmc
