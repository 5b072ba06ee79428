// Reference tetrahedron tables for the nodal DG basis, host side.
//
// Node set: warp & blend (Warburton 2006): an equidistant lattice whose edge
// points are moved to the Legendre-Gauss-Lobatto positions, the in-face and
// interior points following through blended edge warps; the index of each
// lattice point is kept.  Operators are basis-independent (nodal Lagrange
// basis l_j): Dr[i][j] = d l_j/dr (x_i), M[i][j] = int_T l_i l_j,
// E[i][(f,m)] = int_{face f} l_i l_{Fmask[f][m]} (face parametrised by two
// reference coordinates, area 2) and LIFT = M^{-1} E.  They are computed here
// in the Bernstein basis of degree p, whose element and face integrals have
// closed forms (the Dirichlet integral of barycentric monomials).
#include "refelem.hpp"

#include <algorithm>
#include <cmath>

namespace dg {

const int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};

namespace {

// Warburton's optimised blend parameter (orders 1..3 need none).
double blend_alpha(int p) { return p == 4 ? 0.1002 : 0.0; }

// Legendre-Gauss-Lobatto points of order p <= 4, ascending (closed forms).
void lgl_points(int p, double* x) {
  x[0] = -1.0;
  x[p] = 1.0;
  if (p == 2) x[1] = 0.0;
  if (p == 3) { x[1] = -1.0 / std::sqrt(5.0); x[2] = -x[1]; }
  if (p == 4) { x[1] = -std::sqrt(3.0 / 7.0); x[2] = 0.0; x[3] = -x[1]; }
}

// Edge warp divided by the bubble 1 - x^2: the degree-p interpolant, on
// equidistant points, of (LGL point - equidistant point), over (1 - x^2).
// The blend factors that multiply it vanish at the end points, where it is
// returned as zero.
double scaled_warp(int p, double x) {
  if (std::fabs(x) >= 1.0 - 1e-10) return 0.0;
  double lgl[kMaxOrder + 1];
  lgl_points(p, lgl);
  double w = 0.0;
  for (int i = 0; i <= p; ++i) {
    const double xi = -1.0 + 2.0 * i / p;
    double li = 1.0;
    for (int j = 0; j <= p; ++j) {
      if (j == i) continue;
      const double xj = -1.0 + 2.0 * j / p;
      li *= (x - xj) / (xi - xj);
    }
    w += (lgl[i] - xi) * li;
  }
  return w / (1.0 - x * x);
}

struct V3 { double x, y, z; };
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
double norm(V3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }

// Gauss-Jordan inverse with partial pivoting (n <= 35).
bool invert(std::vector<double>& A, int n) {
  std::vector<double> inv(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) < 1e-300) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) { std::swap(A[c * n + k], A[piv * n + k]); std::swap(inv[c * n + k], inv[piv * n + k]); }
    const double d = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] *= d; inv[c * n + k] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
    }
  }
  A.swap(inv);
  return true;
}

// C = A (n x k) * B (k x m)
std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n, int k, int m) {
  std::vector<double> C(static_cast<size_t>(n) * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      const double a = A[i * k + l];
      for (int j = 0; j < m; ++j) C[i * m + j] += a * B[l * m + j];
    }
  return C;
}

double fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

}  // namespace

bool build_ref_elem(int p, RefElem& out) {
  if (p < 1 || p > kMaxOrder) return false;
  const int Np = nodes_of(p), Nfp = face_nodes_of(p);
  out.p = p; out.Np = Np; out.Nfp = Nfp;
  out.lattice.assign(Np * 4, 0);
  out.rst.assign(Np * 3, 0.0);

  // equilateral tetrahedron carrying the warp & blend construction
  const V3 V[4] = {{-1.0, -1.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                   {1.0, -1.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                   {0.0, 2.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                   {0.0, 0.0, 3.0 / std::sqrt(6.0)}};
  const double alpha = blend_alpha(p);
  const double tol = 1e-10;
  int idx = 0;
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= p - n; ++m)
      for (int q = 0; q <= p - n - m; ++q, ++idx) {
        const int lab[4] = {p - n - m - q, q, m, n};
        double lam[4];
        for (int a = 0; a < 4; ++a) { out.lattice[idx * 4 + a] = lab[a]; lam[a] = static_cast<double>(lab[a]) / p; }
        V3 X{0, 0, 0};
        for (int a = 0; a < 4; ++a) X = X + lam[a] * V[a];
        V3 shift{0, 0, 0};
        bool on_edge = false;
        V3 edge_shift{0, 0, 0};
        for (int opp = 0; opp < 4; ++opp) {
          int fv[3], c = 0;
          for (int a = 0; a < 4; ++a) if (a != opp) fv[c++] = a;
          const double La = lam[opp];
          const double L[3] = {lam[fv[0]], lam[fv[1]], lam[fv[2]]};
          V3 s{0, 0, 0};
          for (int k = 0; k < 3; ++k) {
            const int a = (k + 1) % 3, b = (k + 2) % 3;  // edge a -> b, opposite vertex k
            const double warp = 4.0 * scaled_warp(p, L[b] - L[a]) * L[a] * L[b] * (1.0 + (alpha * L[k]) * (alpha * L[k]));
            const V3 d = V[fv[b]] - V[fv[a]];
            s = s + (warp / norm(d)) * d;
          }
          double blend = L[0] * L[1] * L[2];
          const double denom = (L[0] + 0.5 * La) * (L[1] + 0.5 * La) * (L[2] + 0.5 * La);
          if (denom > tol) blend = (1.0 + (alpha * La) * (alpha * La)) * blend / denom;
          shift = shift + blend * s;
          const int inside = (L[0] > tol) + (L[1] > tol) + (L[2] > tol);
          if (La < tol && inside < 3) { on_edge = true; edge_shift = s; }
        }
        X = X + (on_edge ? edge_shift : shift);
        // X - V1 = sum_d (1 + rst_d)/2 (V_{d+1} - V1): solve the 3x3 system
        const V3 a1 = 0.5 * (V[1] - V[0]), a2 = 0.5 * (V[2] - V[0]), a3 = 0.5 * (V[3] - V[0]);
        const V3 b = X - V[0];
        const double det = a1.x * (a2.y * a3.z - a2.z * a3.y) - a2.x * (a1.y * a3.z - a1.z * a3.y) + a3.x * (a1.y * a2.z - a1.z * a2.y);
        const double c1 = (b.x * (a2.y * a3.z - a2.z * a3.y) - a2.x * (b.y * a3.z - b.z * a3.y) + a3.x * (b.y * a2.z - b.z * a2.y)) / det;
        const double c2 = (a1.x * (b.y * a3.z - b.z * a3.y) - b.x * (a1.y * a3.z - a1.z * a3.y) + a3.x * (a1.y * b.z - a1.z * b.y)) / det;
        const double c3 = (a1.x * (a2.y * b.z - a2.z * b.y) - a2.x * (a1.y * b.z - a1.z * b.y) + b.x * (a1.y * a2.z - a1.z * a2.y)) / det;
        out.rst[idx * 3 + 0] = c1 - 1.0;
        out.rst[idx * 3 + 1] = c2 - 1.0;
        out.rst[idx * 3 + 2] = c3 - 1.0;
      }

  // face masks
  out.Fmask.assign(4 * Nfp, 0);
  for (int f = 0; f < 4; ++f) {
    int c = 0;
    for (int i = 0; i < Np; ++i) {
      const double r = out.rst[i * 3], s = out.rst[i * 3 + 1], t = out.rst[i * 3 + 2];
      const double d = f == 0 ? 1 + t : f == 1 ? 1 + s : f == 2 ? 1 + r + s + t : 1 + r;
      if (std::fabs(d) < tol) { if (c >= Nfp) return false; out.Fmask[f * Nfp + c++] = i; }
    }
    if (c != Nfp) return false;
  }

  // Bernstein basis B_a = p!/(a!) prod lam^a, multi-indices = lattice labels
  auto bary = [&](int i, double* lam) {
    const double r = out.rst[i * 3], s = out.rst[i * 3 + 1], t = out.rst[i * 3 + 2];
    lam[0] = -0.5 * (1 + r + s + t); lam[1] = 0.5 * (1 + r); lam[2] = 0.5 * (1 + s); lam[3] = 0.5 * (1 + t);
  };
  auto bern = [&](const int* a, const double* lam, int deg) {
    double v = fact(deg);
    for (int k = 0; k < 4; ++k) v *= std::pow(lam[k], a[k]) / fact(a[k]);
    return v;
  };
  // d lambda_k / d(r,s,t)
  const double dl[3][4] = {{-0.5, 0.5, 0, 0}, {-0.5, 0, 0.5, 0}, {-0.5, 0, 0, 0.5}};
  std::vector<double> Vm(Np * Np), Vd[3];
  for (int d = 0; d < 3; ++d) Vd[d].assign(Np * Np, 0.0);
  for (int i = 0; i < Np; ++i) {
    double lam[4];
    bary(i, lam);
    for (int j = 0; j < Np; ++j) {
      const int* a = &out.lattice[j * 4];
      Vm[i * Np + j] = bern(a, lam, p);
      for (int k = 0; k < 4; ++k) {
        if (a[k] == 0) continue;
        int am[4] = {a[0], a[1], a[2], a[3]};
        am[k] -= 1;
        const double dB = p * bern(am, lam, p - 1);  // dB_a/dlam_k
        for (int d = 0; d < 3; ++d) Vd[d][i * Np + j] += dB * dl[d][k];
      }
    }
  }
  std::vector<double> Vinv = Vm;
  if (!invert(Vinv, Np)) return false;
  out.Dr = matmul(Vd[0], Vinv, Np, Np, Np);
  out.Ds = matmul(Vd[1], Vinv, Np, Np, Np);
  out.Dt = matmul(Vd[2], Vinv, Np, Np, Np);

  // Bernstein Gram matrices: element (|T| = 4/3) and faces (parametric area 2)
  std::vector<double> MB(Np * Np), EB[4];
  for (int f = 0; f < 4; ++f) EB[f].assign(Np * Np, 0.0);
  const double pf2 = fact(p) * fact(p);
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      const int* a = &out.lattice[i * 4];
      const int* b = &out.lattice[j * 4];
      double num = pf2;
      for (int k = 0; k < 4; ++k) num *= fact(a[k] + b[k]) / (fact(a[k]) * fact(b[k]));
      MB[i * Np + j] = num * fact(3) * (4.0 / 3.0) / fact(2 * p + 3);
      for (int f = 0; f < 4; ++f) {
        const int opp = 6 - kFaceVerts[f][0] - kFaceVerts[f][1] - kFaceVerts[f][2];
        if (a[opp] != 0 || b[opp] != 0) continue;
        EB[f][i * Np + j] = num * fact(2) * 2.0 / fact(2 * p + 2);
      }
    }
  // nodal matrices: N = Vinv^T G Vinv
  std::vector<double> VinvT(Np * Np);
  for (int i = 0; i < Np; ++i) for (int j = 0; j < Np; ++j) VinvT[i * Np + j] = Vinv[j * Np + i];
  std::vector<double> M = matmul(matmul(VinvT, MB, Np, Np, Np), Vinv, Np, Np, Np);
  std::vector<double> Minv = M;
  if (!invert(Minv, Np)) return false;
  std::vector<double> E(Np * 4 * Nfp, 0.0);
  for (int f = 0; f < 4; ++f) {
    std::vector<double> Ef = matmul(matmul(VinvT, EB[f], Np, Np, Np), Vinv, Np, Np, Np);
    for (int i = 0; i < Np; ++i)
      for (int m = 0; m < Nfp; ++m) E[i * 4 * Nfp + f * Nfp + m] = Ef[i * Np + out.Fmask[f * Nfp + m]];
  }
  out.LIFT = matmul(Minv, E, Np, Np, 4 * Nfp);
  return true;
}

}  // namespace dg
