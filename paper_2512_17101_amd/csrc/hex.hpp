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

// Tiles of the p = 1 kernels: a 256-thread block owns a box of TX x TY x TZ
// cells of 8 nodes (one thread per node), so most face neighbours are in the
// block; NSX / NSY / NSZ count the box's face nodes normal to x / y / z,
// boundary planes included.
constexpr int kTileX1 = 4, kTileY1 = 4, kTileZ1 = 2;

template <int P, int TX, int TY, int TZ>
struct HexTileCfg {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1 * N1;
  static constexpr int NFP = N1 * N1;
  static constexpr int NC = TX * TY * TZ;  // cells of the tile
  static constexpr int NT = NC * NP;       // threads owning a node
  static constexpr int NSX = (TX + 1) * TY * TZ * NFP;
  static constexpr int NSY = TX * (TY + 1) * TZ * NFP;
  static constexpr int NSZ = TX * TY * (TZ + 1) * NFP;
  static constexpr int NS = NSX + NSY + NSZ;  // face nodes of the tile
  static constexpr int KF = (NS + 255) / 256;
  static_assert(NT <= 256, "one thread per node");
};

// wraps a cell coordinate into [0, n) (it lies in [-n, 2 n + T))
__device__ inline int wrap_cell(int c, int n) {
  c = c < 0 ? c + n : c;
  while (c >= n) c -= n;
  return c;
}

// Face node s of a tile whose first cell is (X0, Y0, Z0): the faces normal
// to x come first (planes k = 0..TX, then y, then z, then the face node m),
// and L, R are the cells before and after the face along its direction d.
// For each side: whether the side is a cell of the tile inside the grid
// (`in`; never when `real` is false, i.e. for a clamped duplicate slot),
// its tile-local cell, its global element (periodic wrap; 0 when the
// transverse cells are outside the grid, in which case no valid cell
// touches this face) and the global index of its node on the face
// (position P of L along d, 0 of R).
struct TileFaceNode {
  int d, m;
  bool in[2];
  int cell[2], ge[2], gi[2];
};

template <int P, int TX, int TY, int TZ>
__device__ inline TileFaceNode tile_face_node(int s, bool real, int X0, int Y0, int Z0, int nx, int ny, int nz) {
  using C = HexTileCfg<P, TX, TY, TZ>;
  constexpr int N1 = C::N1, NFP = C::NFP;
  TileFaceNode o;
  int r;
  if (s < C::NSX) {
    o.d = 0; r = s;
  } else if (s < C::NSX + C::NSY) {
    o.d = 1; r = s - C::NSX;
  } else {
    o.d = 2; r = s - C::NSX - C::NSY;
  }
  const int d = o.d;
  o.m = r % NFP;
  r /= NFP;
  const int Td = d == 0 ? TX : d == 1 ? TY : TZ;
  const int T1 = d == 0 ? TY : TX;  // first transverse extent (y for x faces, else x)
  const int k = r % (Td + 1);
  r /= Td + 1;
  const int t1 = r % T1, t2 = r / T1;
  const int n_d = d == 0 ? nx : d == 1 ? ny : nz;
  const int O_d = d == 0 ? X0 : d == 1 ? Y0 : Z0;
  const bool trans_ok = d == 0 ? (Y0 + t1 < ny && Z0 + t2 < nz)
                               : d == 1 ? (X0 + t1 < nx && Z0 + t2 < nz) : (X0 + t1 < nx && Y0 + t2 < ny);
  const int uu = o.m % N1, vv = o.m / N1;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int kd = k - 1 + side;
    const int cx = d == 0 ? kd : t1, cy = d == 0 ? t1 : (d == 1 ? kd : t2), cz = d == 2 ? kd : t2;
    o.in[side] = real && trans_ok && kd >= 0 && kd < Td && O_d + kd < n_d;
    o.cell[side] = cx + TX * (cy + TY * cz);
    const int pd = side ? 0 : P;
    const int nn = d == 0 ? pd + N1 * (uu + N1 * vv) : d == 1 ? uu + N1 * (pd + N1 * vv) : uu + N1 * (vv + N1 * pd);
    int g3[3] = {X0 + cx, Y0 + cy, Z0 + cz};
    g3[d] = wrap_cell(O_d + kd, n_d);
    o.ge[side] = trans_ok ? g3[0] + nx * (g3[1] + ny * g3[2]) : 0;
    o.gi[side] = o.ge[side] * C::NP + nn;
  }
  return o;
}

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
