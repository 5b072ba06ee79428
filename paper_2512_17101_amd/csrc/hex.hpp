// Tensor-product hexahedra on a periodic rectilinear grid: host mesh record
// and the kernel launcher.
#pragma once
#include "internal.hpp"

namespace dg {

constexpr int kHexMaxOrder = 4;

struct HexMesh {
  int device = 0;
  int p = 0, N1 = 0, Np = 0;
  int nx = 0, ny = 0, nz = 0;
  int64_t E = 0;
  std::vector<double> gx, gy, gz;  // grid lines, n + 1 per axis
  std::vector<double> x1;          // [N1] LGL points
  std::vector<double> D1;          // [N1][N1] D1[i][j] = l_j'(x_i)
  std::vector<double> lift;        // [N1][2] columns M1^-1 e_0, M1^-1 e_p
  // device
  double* d_ih = nullptr;  // [nx + ny + nz]: 2 / h of each cell, x cells then y then z
  double* d_op = nullptr;  // [N1 N1 | 2 N1]: D1 row-major, then lift row-major
  // overintegrated form: nq Gauss points per direction and the tables
  // [B (nq x N1) | S (N1 x nq) | P (N1 x nq) | lift (N1 x 2)], row-major
  int nq = 0;
  std::vector<double> oi;
  double* d_oi = nullptr;
  // shock capturing: [Vinv (N1 x N1) | w1 (N1)], the inverse of the 1-D
  // orthonormal Legendre Vandermonde and the 1-D weights int l_i
  double* d_sh = nullptr;
};

// 1-D tables of order p (1..kHexMaxOrder): LGL points, D1, lift columns,
// formed in binary128 and rounded once.  False for other orders.
bool build_hex_1d(int p, std::vector<double>& x, std::vector<double>& D1, std::vector<double>& lift);

// Overintegration tables of order p with nq = ceil(3 (p + 1) / 2) Gauss
// points: points xq, weights wq and [B | S | P | lift] as in HexMesh::oi,
// formed in binary128 at the rounded points and weights and rounded once.
int hex_oi_points(int p);
bool build_hex_oi(int p, std::vector<double>& xq, std::vector<double>& wq, std::vector<double>& tables);

// Overintegrated RHS (weak form, fluxes at the Gauss points), optionally
// through the fused stage update as below.
dg_status launch_rhs_hex_oi(const HexMesh& m, double gamma, const double* q, double* rhs, const double* res_in,
                            double* res, double* q_out, double a, double b, double dt, bool fused_lsrk,
                            hipStream_t s);

// Shock-capturing tables of order p: the inverse orthonormal Legendre
// Vandermonde on the LGL points (row-major) and the weights int l_i.
bool build_hex_shock_tables(int p, std::vector<double>& tables);
// Indicator s (may be null), viscosity eps (required: the RHS reads it)
// per element and the viscous fluxes G [3][5][E][Np] of q, stored only in
// elements with eps > 0.
dg_status launch_hex_av_flux(const HexMesh& m, const dg_av_params& av, double gamma, const double* q, double* G,
                             double* s_out, double* eps_out, hipStream_t s);
// Positivity limiter of q in place.
dg_status launch_hex_limit(const HexMesh& m, const dg_av_params& av, double gamma, double* q, hipStream_t s);
// Euler RHS plus the divergence of the viscous fluxes G (BR1 central flux;
// G is read only in elements with eps > 0, elsewhere it is zero), optionally
// through the fused stage update.
dg_status launch_rhs_hex_av(const HexMesh& m, double gamma, const double* q, const double* G, const double* eps,
                            double* rhs, const double* res_in, double* res, double* q_out, double a, double b,
                            double dt, bool fused_lsrk, hipStream_t s);

// RHS of q on the hex mesh; with fused_lsrk the result goes through the
// stage update (res <- a res_in + dt rhs; q_out <- q + b res, res skipped
// when null; res_in, res and q_out may share a buffer, as the stage reads
// every entry before the same thread writes it) instead of rhs.
dg_status launch_rhs_hex(const HexMesh& m, double gamma, const double* q, double* rhs, const double* res_in,
                         double* res, double* q_out, double a, double b, double dt, bool fused_lsrk, hipStream_t s);

}  // namespace dg
