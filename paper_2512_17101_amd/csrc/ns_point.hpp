// Pointwise FP64 pieces of the reacting Navier-Stokes right-hand side with
// BR1 viscous terms: primitives, mixture properties, total (inviscid minus
// viscous) fluxes and the face jump.
//
// State (rho, rho u, rho v, rho w, E, rho Y_1 .. rho Y_7); temperature T from
// the Newton solve; primitives for the gradients v = (u, v, w, T, Y_1 .. Y_7);
// lifted gradients sig[3 c + d] = d v_c / d x_d.
//   p = rho R_mix T, R_mix = sum Y_k R_k, cp = sum Y_k cp_k(T),
//   c = sqrt(cp / (cp - R_mix) p / rho),
//   tau_id = mu (du_i/dx_d + du_d/dx_i) - 2/3 mu (div u) delta_id,
//   kappa = mu cp / Pr, rho D = mu / Sc, J_k = -rho D grad Y_k,
//   F_d = F^inv_d - F^v_d with
//   F^inv_d = (rho u_d, rho u_i u_d + p delta_id, (E + p) u_d, rho Y_k u_d),
//   F^v_d   = (0, tau_id, u_i tau_id + kappa dT/dx_d - sum_k h_k J_k,d, -J_k,d).
#pragma once
#include "euler_point.hpp"
#include "thermo.hpp"

namespace dg {

constexpr int kNsSpecies = 7;
constexpr int kNsFields = 5 + kNsSpecies;  // conserved fields
constexpr int kNsPrims = 4 + kNsSpecies;   // gradient primitives (u, v, w, T, Y)

struct Transport {
  double mu, Pr, Sc;
};

// cp, R_mix and species enthalpies h_k [J/kg] at T for mass fractions Y.
__device__ inline void mixture(const ThermoTable& th, double T, const double Y[kNsSpecies], double& cp, double& Rm,
                               double h[kNsSpecies]) {
  cp = 0.0;
  Rm = 0.0;
#pragma unroll
  for (int k = 0; k < kNsSpecies; ++k) {
    const double Rk = th.R[k];
    const double cpR = th.cp[k][0] + T * (th.cp[k][1] + T * (th.cp[k][2] + T * (th.cp[k][3] + T * th.cp[k][4])));
    const double hR = T * (th.h[k][0] + T * (th.h[k][1] + T * (th.h[k][2] + T * (th.h[k][3] + T * th.h[k][4])))) +
                      th.h[k][5];
    cp += Y[k] * Rk * cpR;
    Rm += Y[k] * Rk;
    h[k] = Rk * hR;
  }
}

// Primitives (u, v, w, T, Y_1 .. Y_7) of a node.
__device__ inline void ns_primitives(const double q[kNsFields], double T, double v[kNsPrims]) {
  const double ir = recip(q[0]);
  v[0] = q[1] * ir;
  v[1] = q[2] * ir;
  v[2] = q[3] * ir;
  v[3] = T;
#pragma unroll
  for (int k = 0; k < kNsSpecies; ++k) v[4 + k] = q[5 + k] * ir;
}

// Node quantities the fluxes need, formed once per node.
struct NsNode {
  double ir, u[3], p, c, cp, div;
  double h[kNsSpecies];
};

__device__ inline void ns_node(const ThermoTable& th, const double q[kNsFields], double T,
                               const double sig[3 * kNsPrims], NsNode& nd) {
  nd.ir = recip(q[0]);
  nd.u[0] = q[1] * nd.ir;
  nd.u[1] = q[2] * nd.ir;
  nd.u[2] = q[3] * nd.ir;
  double Y[kNsSpecies];
#pragma unroll
  for (int k = 0; k < kNsSpecies; ++k) Y[k] = q[5 + k] * nd.ir;
  double Rm;
  mixture(th, T, Y, nd.cp, Rm, nd.h);
  nd.p = q[0] * Rm * T;
  nd.c = sqrt_pos(nd.cp * recip(nd.cp - Rm) * nd.p * nd.ir);
  nd.div = sig[0] + sig[4] + sig[8];
}

// Total flux of one node along the vector n (a scaled normal or a metric
// row grad a): Fn = sum_d n_d (F^inv_d - F^v_d) for every field; returns
// U_n = n . u.
__device__ inline double ns_flux_along(const Transport& tr, const NsNode& nd, const double q[kNsFields],
                                       const double sig[3 * kNsPrims], const double n[3], double Fn[kNsFields]) {
  const double Un = n[0] * nd.u[0] + n[1] * nd.u[1] + n[2] * nd.u[2];
  // (tau n)_i = mu (grad u_i . n + d(u . n)/dx_i) - 2/3 mu (div u) n_i
  double taun[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double gin = sig[3 * i] * n[0] + sig[3 * i + 1] * n[1] + sig[3 * i + 2] * n[2];
    const double gni = sig[i] * n[0] + sig[3 + i] * n[1] + sig[6 + i] * n[2];
    taun[i] = tr.mu * (gin + gni) - (2.0 / 3.0) * tr.mu * nd.div * n[i];
  }
  const double kappa = tr.mu * nd.cp / tr.Pr;
  const double rhoD = tr.mu / tr.Sc;
  const double dTn = sig[9] * n[0] + sig[10] * n[1] + sig[11] * n[2];
  double hJ = 0.0;  // sum_k h_k grad Y_k . n
  Fn[0] = q[0] * Un;
#pragma unroll
  for (int i = 0; i < 3; ++i) Fn[1 + i] = q[1 + i] * Un + nd.p * n[i] - taun[i];
#pragma unroll
  for (int k = 0; k < kNsSpecies; ++k) {
    const double gYn = sig[3 * (4 + k)] * n[0] + sig[3 * (4 + k) + 1] * n[1] + sig[3 * (4 + k) + 2] * n[2];
    hJ += nd.h[k] * gYn;
    Fn[5 + k] = q[5 + k] * Un - rhoD * gYn;
  }
  Fn[4] = (q[4] + nd.p) * Un - (nd.u[0] * taun[0] + nd.u[1] * taun[1] + nd.u[2] * taun[2] + kappa * dTn + rhoD * hJ);
  return Un;
}

}  // namespace dg
