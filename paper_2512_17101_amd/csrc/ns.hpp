// Arguments and launchers of the reacting Navier-Stokes kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "thermo.hpp"

namespace dg {

struct NsArgs {
  const double* q;      // [12][E][Np] stage input
  const double* T;      // [E][Np] temperatures of q
  double* sigma;        // [E][Np][33] lifted gradients, entry 3 c + d = d v_c / d x_d
  double* rhs;          // [12][E][Np] (unfused)
  const double* res_in; // fused stage: res <- a res_in + dt rhs (res skipped when null)
  double* res;          //              qout <- q + b res
  double* qout;         // (res_in, res and qout may share a buffer: entry-wise)
  const double* geo;    // [9][Epad]
  const int2* conn;     // [4][Epad]
  const double* opT;    // [3 Np + 4 Nfp][Np]: D_a[i][j] at row a Np + j, LIFT[i][m] at row 3 Np + m
  const int* fmask;     // [4 Nfp]
  const uint8_t* nbtab; // [4][24][Nfp]
  int64_t E, Epad;
  double mu, Pr, Sc;
  double a, b, dt;
  int with_sources;
  ThermoTable th;
  MechTable mk;
};

dg_status launch_ns_gradients(int p, const NsArgs& A, hipStream_t s);
dg_status launch_ns_rhs(int p, const NsArgs& A, bool fused, hipStream_t s);

}  // namespace dg
