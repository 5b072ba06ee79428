// Reacting-flow pointwise kernels, FP64: temperature from internal energy by
// Newton's method, and irreversible Arrhenius species sources.
//
// Species k: R_k = R_u / W_k, cp_k/R_k = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4,
// h_k/R_k = a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a5 T^5/5 + a6,
// e_k = h_k - R_k T.  For one node with mass fractions Y the mixture
//   e(T)  = sum_k Y_k R_k (h_k/R_k - T)   and   cv(T) = sum_k Y_k R_k (cp_k/R_k - 1)
// are polynomials in T whose coefficients are formed once per node, so each
// Newton step T <- T - (e(T) - e) / cv(T) is two Horner evaluations.
// Iterates are clamped to [100, 6000] K; the step count is returned, or -1
// when |T_{n+1} - T_n| < tol is not reached within max_iter steps (a step cut
// by the clamp never counts as converged).  A point without a root to find
// (non-finite iterate) ends at once with -1 and a non-finite T.  Failures
// raise the device's no-convergence / non-finite flags.
//
// Sources: C_k = rho Y_k / W_k, k_j = A_j exp(-Ea_j / (R_u T)),
// r_j = k_j prod_k C_k^{nu'_kj}, omega_k = W_k sum_j (nu''_kj - nu'_kj) r_j.
#include "internal.hpp"
#include "thermo.hpp"

namespace dg {
namespace {

__global__ __launch_bounds__(256) void temperature_kernel(ThermoTable th, int64_t n, const double* __restrict__ q,
                                                          const double* __restrict__ Tguess, double Tdefault,
                                                          double* __restrict__ Tout, int32_t* __restrict__ iters,
                                                          double tol, int max_iter, unsigned* flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  bool noconv = false, bad = false;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double rho = q[i];
    const double ir = 1.0 / rho;
    const double mx = q[n + i], my = q[2 * n + i], mz = q[3 * n + i];
    const double e = q[4 * n + i] * ir - 0.5 * (mx * mx + my * my + mz * mz) * ir * ir;
    double Bh[6] = {0, 0, 0, 0, 0, 0};  // sum_k Y_k R_k (a1, a2/2, a3/3, a4/4, a5/5, a6)
    double Bc[5] = {0, 0, 0, 0, 0};     // sum_k Y_k R_k (a1 .. a5)
    double cR = 0.0;                    // sum_k Y_k R_k
    for (int k = 0; k < th.ns; ++k) {
      const double c = q[(5 + k) * n + i] * ir * th.R[k];
      cR += c;
#pragma unroll
      for (int m = 0; m < 6; ++m) Bh[m] += c * th.h[k][m];
#pragma unroll
      for (int m = 0; m < 5; ++m) Bc[m] += c * th.cp[k][m];
    }
    double T = Tguess ? Tguess[i] : Tdefault;
    int32_t it = -1;
    for (int s = 1; s <= max_iter; ++s) {
      const double eT = T * (Bh[0] + T * (Bh[1] + T * (Bh[2] + T * (Bh[3] + T * Bh[4])))) + Bh[5] - cR * T;
      const double cv = Bc[0] + T * (Bc[1] + T * (Bc[2] + T * (Bc[3] + T * Bc[4]))) - cR;
      const double Tu = T - (eT - e) / cv;
      if (nonfinite(Tu)) {  // non-finite state or guess: no root to find
        T = Tu;
        bad = true;
        break;
      }
      const double Tn = fmin(fmax(Tu, kTmin), kTmax);
      // a step that had to be clamped is not convergence: a root outside
      // [Tmin, Tmax] would otherwise be reported as the clamp bound
      const bool done = fabs(Tn - T) < tol && Tn == Tu;
      T = Tn;
      if (done) { it = s; break; }
    }
    noconv |= it < 0;
    Tout[i] = T;
    iters[i] = it;
  }
  raise_flag(flags, noconv, kFlagNoConv);
  raise_flag(flags, bad, kFlagNonFinite);
}

__global__ __launch_bounds__(256) void sources_kernel(MechTable mk, int64_t n, const double* __restrict__ q,
                                                      const double* __restrict__ T, double* __restrict__ omega) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    double C[kMaxSpecies], w[kMaxSpecies];
    // all loads of the node issued together (slots past ns are not used)
#pragma unroll
    for (int k = 0; k < kMaxSpecies; ++k) C[k] = q[(5 + (k < mk.ns ? k : mk.ns - 1)) * n + i] * mk.invW[k];
    node_sources(mk, C, 1.0 / T[i], w);
    for (int k = 0; k < mk.ns; ++k) omega[k * n + i] = w[k];
  }
}

int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 256 * 64) b = 256 * 64;
  return static_cast<int>(b < 1 ? 1 : b);
}

}  // namespace

dg_status launch_temperature(const ThermoTable& th, int64_t n, const double* q, const double* Tguess, double Tdefault,
                             double* Tout, int32_t* iters, double tol, int max_iter, hipStream_t s) {
  temperature_kernel<<<grid_for(n), 256, 0, s>>>(th, n, q, Tguess, Tdefault, Tout, iters, tol, max_iter,
                                                  device_flags());
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_sources(const MechTable& mk, int64_t n, const double* q, const double* T, double* omega,
                         hipStream_t s) {
  sources_kernel<<<grid_for(n), 256, 0, s>>>(mk, n, q, T, omega);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
