// Species and mechanism tables handed to the reacting-flow kernels by value.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dg.h"

namespace dg {

constexpr int kMaxSpecies = 8;
constexpr int kMaxReactions = 8;
constexpr double kRu = 8.314462618;  // J / (mol K)
constexpr double kTmin = 100.0, kTmax = 6000.0;
constexpr double kTdefault = 1000.0;  // plain (cold) Newton start
constexpr int kLearnedMaxIter = 8;     // steps from the learned guess before the plain restart

struct ThermoTable {
  int ns;
  double R[kMaxSpecies];          // R_k = R_u / W_k
  double W[kMaxSpecies];
  double h[kMaxSpecies][6];       // h_k/R_k = T (h0 + T (h1 + ...)) + h5: (a1, a2/2, a3/3, a4/4, a5/5, a6)
  double cp[kMaxSpecies][5];      // cp_k/R_k coefficients (a1 .. a5)
};

struct MechTable {
  int ns, nr;
  double invW[kMaxSpecies];
  double A[kMaxReactions];
  double EaR[kMaxReactions];      // Ea_j / R_u
  int nu_r[kMaxReactions][kMaxSpecies];
  double Wnet[kMaxSpecies][kMaxReactions];  // W_k (nu''_kj - nu'_kj)
};

// Species sources of one node from its molar concentrations C_k = rho Y_k / W_k
// and 1 / T: k_j = A_j exp(-Ea_j / (R_u T)), r_j = k_j prod_k C_k^{nu'_kj},
// omega_k = sum_j W_k (nu''_kj - nu'_kj) r_j.
__device__ inline void node_sources(const MechTable& mk, const double* C, double iT, double* omega) {
  double r[kMaxReactions];
  for (int j = 0; j < mk.nr; ++j) {
    double rj = mk.A[j] * exp(-mk.EaR[j] * iT);
    for (int k = 0; k < mk.ns; ++k)
      for (int m = 0; m < mk.nu_r[j][k]; ++m) rj *= C[k];
    r[j] = rj;
  }
  for (int k = 0; k < mk.ns; ++k) {
    double w = 0.0;
    for (int j = 0; j < mk.nr; ++j) w += mk.Wnet[k][j] * r[j];
    omega[k] = w;
  }
}

dg_status launch_temperature(const ThermoTable& th, int64_t n, const double* q, const double* Tguess,
                             double Tdefault, double* Tout, int32_t* iters, double tol, int max_iter, hipStream_t s);
dg_status launch_sources(const MechTable& mk, int64_t n, const double* q, const double* T, double* omega,
                         hipStream_t s);

}  // namespace dg
