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

// Every quantity below is formed in IEEE binary128 (113-bit significand) and
// rounded to FP64 once: the nodes, and then the operators at those FP64
// nodes.  The Vandermonde solves lose a few hundred units in the last place
// of FP64 at p = 4 (the error grows with the basis' condition number), far
// below binary128's resolution, so the stored tables are the correctly
// rounded exact values except where an entry lies within ~1e-30 of a
// rounding midpoint.
using qd = __float128;

qd qabs(qd a) { return a < 0 ? -a : a; }

// square root by Newton's method from the FP64 root (53 -> 106 -> 212 bits)
qd qsqrt(qd a) {
  if (a <= 0) return 0;
  qd x = std::sqrt(static_cast<double>(a));
  for (int k = 0; k < 2; ++k) x = 0.5 * (x + a / x);
  return x;
}

qd qpow(qd x, int n) { qd v = 1; for (int k = 0; k < n; ++k) v *= x; return v; }

// Warburton's optimised blend parameter (orders 1..3 need none); the
// tabulated decimal value 0.1002, rounded in binary128
qd blend_alpha(int p) { return p == 4 ? qd(1002) / qd(10000) : qd(0); }

// Legendre-Gauss-Lobatto points of order p <= 4, ascending (closed forms).
void lgl_points(int p, qd* x) {
  x[0] = -1;
  x[p] = 1;
  if (p == 2) x[1] = 0;
  if (p == 3) { x[1] = -1 / qsqrt(5); x[2] = -x[1]; }
  if (p == 4) { x[1] = -qsqrt(qd(3) / qd(7)); x[2] = 0; x[3] = -x[1]; }
}

// Edge warp divided by the bubble 1 - x^2: the degree-p interpolant, on
// equidistant points, of (LGL point - equidistant point), over (1 - x^2).
// The blend factors that multiply it vanish at the end points, where it is
// returned as zero.
qd scaled_warp(int p, qd x) {
  if (qabs(x) >= 1 - qd(1e-10)) return 0;
  qd lgl[kMaxOrder + 1];
  lgl_points(p, lgl);
  qd w = 0;
  for (int i = 0; i <= p; ++i) {
    const qd xi = -1 + qd(2 * i) / p;
    qd li = 1;
    for (int j = 0; j <= p; ++j) {
      if (j == i) continue;
      const qd xj = -1 + qd(2 * j) / p;
      li *= (x - xj) / (xi - xj);
    }
    w += (lgl[i] - xi) * li;
  }
  return w / (1 - x * x);
}

struct V3 { qd x, y, z; };
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator*(qd s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
qd norm(V3 a) { return qsqrt(a.x * a.x + a.y * a.y + a.z * a.z); }

using QMat = std::vector<qd>;

// Gauss-Jordan inverse with partial pivoting (n <= 35).
bool invert(QMat& A, int n) {
  QMat inv(static_cast<size_t>(n) * n, 0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (qabs(A[r * n + c]) > qabs(A[piv * n + c])) piv = r;
    if (qabs(A[piv * n + c]) < qd(1e-300)) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) { std::swap(A[c * n + k], A[piv * n + k]); std::swap(inv[c * n + k], inv[piv * n + k]); }
    const qd d = 1 / A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] *= d; inv[c * n + k] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const qd f = A[r * n + c];
      if (f == 0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
    }
  }
  A.swap(inv);
  return true;
}

// C = A (n x k) * B (k x m)
QMat matmul(const QMat& A, const QMat& B, int n, int k, int m) {
  QMat C(static_cast<size_t>(n) * m, 0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      const qd a = A[i * k + l];
      for (int j = 0; j < m; ++j) C[i * m + j] += a * B[l * m + j];
    }
  return C;
}

std::vector<double> to_double(const QMat& A) {
  std::vector<double> out(A.size());
  for (size_t i = 0; i < A.size(); ++i) out[i] = static_cast<double>(A[i]);
  return out;
}

qd fact(int n) { qd f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

}  // namespace

bool build_ref_elem(int p, RefElem& out) {
  if (p < 1 || p > kMaxOrder) return false;
  const int Np = nodes_of(p), Nfp = face_nodes_of(p);
  out.p = p; out.Np = Np; out.Nfp = Nfp;
  out.lattice.assign(Np * 4, 0);
  out.rst.assign(Np * 3, 0.0);

  // equilateral tetrahedron carrying the warp & blend construction
  const qd s3 = qsqrt(3), s6 = qsqrt(6);
  const V3 V[4] = {{-1, -1 / s3, -1 / s6}, {1, -1 / s3, -1 / s6}, {0, 2 / s3, -1 / s6}, {0, 0, 3 / s6}};
  const qd alpha = blend_alpha(p);
  const qd tol = qd(1e-10);
  int idx = 0;
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= p - n; ++m)
      for (int q = 0; q <= p - n - m; ++q, ++idx) {
        const int lab[4] = {p - n - m - q, q, m, n};
        qd lam[4];
        for (int a = 0; a < 4; ++a) { out.lattice[idx * 4 + a] = lab[a]; lam[a] = qd(lab[a]) / p; }
        V3 X{0, 0, 0};
        for (int a = 0; a < 4; ++a) X = X + lam[a] * V[a];
        V3 shift{0, 0, 0};
        bool on_edge = false;
        V3 edge_shift{0, 0, 0};
        for (int opp = 0; opp < 4; ++opp) {
          int fv[3], c = 0;
          for (int a = 0; a < 4; ++a) if (a != opp) fv[c++] = a;
          const qd La = lam[opp];
          const qd L[3] = {lam[fv[0]], lam[fv[1]], lam[fv[2]]};
          V3 s{0, 0, 0};
          for (int k = 0; k < 3; ++k) {
            const int a = (k + 1) % 3, b = (k + 2) % 3;  // edge a -> b, opposite vertex k
            const qd warp = 4 * scaled_warp(p, L[b] - L[a]) * L[a] * L[b] * (1 + (alpha * L[k]) * (alpha * L[k]));
            const V3 d = V[fv[b]] - V[fv[a]];
            s = s + (warp / norm(d)) * d;
          }
          qd blend = L[0] * L[1] * L[2];
          const qd denom = (L[0] + La / 2) * (L[1] + La / 2) * (L[2] + La / 2);
          if (denom > tol) blend = (1 + (alpha * La) * (alpha * La)) * blend / denom;
          shift = shift + blend * s;
          const int inside = (L[0] > tol) + (L[1] > tol) + (L[2] > tol);
          if (La < tol && inside < 3) { on_edge = true; edge_shift = s; }
        }
        X = X + (on_edge ? edge_shift : shift);
        // X - V1 = sum_d (1 + rst_d)/2 (V_{d+1} - V1): solve the 3x3 system
        const V3 a1 = qd(0.5) * (V[1] - V[0]), a2 = qd(0.5) * (V[2] - V[0]), a3 = qd(0.5) * (V[3] - V[0]);
        const V3 b = X - V[0];
        const qd det = a1.x * (a2.y * a3.z - a2.z * a3.y) - a2.x * (a1.y * a3.z - a1.z * a3.y) + a3.x * (a1.y * a2.z - a1.z * a2.y);
        const qd c1 = (b.x * (a2.y * a3.z - a2.z * a3.y) - a2.x * (b.y * a3.z - b.z * a3.y) + a3.x * (b.y * a2.z - b.z * a2.y)) / det;
        const qd c2 = (a1.x * (b.y * a3.z - b.z * a3.y) - b.x * (a1.y * a3.z - a1.z * a3.y) + a3.x * (a1.y * b.z - a1.z * b.y)) / det;
        const qd c3 = (a1.x * (a2.y * b.z - a2.z * b.y) - a2.x * (a1.y * b.z - a1.z * b.y) + b.x * (a1.y * a2.z - a1.z * a2.y)) / det;
        out.rst[idx * 3 + 0] = static_cast<double>(c1 - 1);
        out.rst[idx * 3 + 1] = static_cast<double>(c2 - 1);
        out.rst[idx * 3 + 2] = static_cast<double>(c3 - 1);
      }

  // face masks
  out.Fmask.assign(4 * Nfp, 0);
  for (int f = 0; f < 4; ++f) {
    int c = 0;
    for (int i = 0; i < Np; ++i) {
      const double r = out.rst[i * 3], s = out.rst[i * 3 + 1], t = out.rst[i * 3 + 2];
      const double d = f == 0 ? 1 + t : f == 1 ? 1 + s : f == 2 ? 1 + r + s + t : 1 + r;
      if (std::fabs(d) < 1e-10) { if (c >= Nfp) return false; out.Fmask[f * Nfp + c++] = i; }
    }
    if (c != Nfp) return false;
  }

  // Operators at the FP64 nodes.  Bernstein basis B_a = p!/(a!) prod lam^a,
  // multi-indices = lattice labels.
  auto bary = [&](int i, qd* lam) {
    const qd r = out.rst[i * 3], s = out.rst[i * 3 + 1], t = out.rst[i * 3 + 2];
    lam[0] = -(1 + r + s + t) / 2; lam[1] = (1 + r) / 2; lam[2] = (1 + s) / 2; lam[3] = (1 + t) / 2;
  };
  auto bern = [&](const int* a, const qd* lam, int deg) {
    qd v = fact(deg);
    for (int k = 0; k < 4; ++k) v *= qpow(lam[k], a[k]) / fact(a[k]);
    return v;
  };
  // d lambda_k / d(r,s,t)
  const qd h = qd(1) / 2;
  const qd dl[3][4] = {{-h, h, 0, 0}, {-h, 0, h, 0}, {-h, 0, 0, h}};
  QMat Vm(Np * Np), Vd[3];
  for (int d = 0; d < 3; ++d) Vd[d].assign(Np * Np, 0);
  for (int i = 0; i < Np; ++i) {
    qd lam[4];
    bary(i, lam);
    for (int j = 0; j < Np; ++j) {
      const int* a = &out.lattice[j * 4];
      Vm[i * Np + j] = bern(a, lam, p);
      for (int k = 0; k < 4; ++k) {
        if (a[k] == 0) continue;
        int am[4] = {a[0], a[1], a[2], a[3]};
        am[k] -= 1;
        const qd dB = p * bern(am, lam, p - 1);  // dB_a/dlam_k
        for (int d = 0; d < 3; ++d) Vd[d][i * Np + j] += dB * dl[d][k];
      }
    }
  }
  QMat Vinv = Vm;
  if (!invert(Vinv, Np)) return false;
  out.Dr = to_double(matmul(Vd[0], Vinv, Np, Np, Np));
  out.Ds = to_double(matmul(Vd[1], Vinv, Np, Np, Np));
  out.Dt = to_double(matmul(Vd[2], Vinv, Np, Np, Np));

  // Bernstein Gram matrices: element (|T| = 4/3) and faces (parametric area 2)
  QMat MB(Np * Np), EB[4];
  for (int f = 0; f < 4; ++f) EB[f].assign(Np * Np, 0);
  const qd pf2 = fact(p) * fact(p);
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      const int* a = &out.lattice[i * 4];
      const int* b = &out.lattice[j * 4];
      qd num = pf2;
      for (int k = 0; k < 4; ++k) num *= fact(a[k] + b[k]) / (fact(a[k]) * fact(b[k]));
      MB[i * Np + j] = num * fact(3) * (qd(4) / 3) / fact(2 * p + 3);
      for (int f = 0; f < 4; ++f) {
        const int opp = 6 - kFaceVerts[f][0] - kFaceVerts[f][1] - kFaceVerts[f][2];
        if (a[opp] != 0 || b[opp] != 0) continue;
        EB[f][i * Np + j] = num * fact(2) * 2 / fact(2 * p + 2);
      }
    }
  // nodal matrices: N = Vinv^T G Vinv
  QMat VinvT(Np * Np);
  for (int i = 0; i < Np; ++i) for (int j = 0; j < Np; ++j) VinvT[i * Np + j] = Vinv[j * Np + i];
  QMat M = matmul(matmul(VinvT, MB, Np, Np, Np), Vinv, Np, Np, Np);
  QMat Minv = M;
  if (!invert(Minv, Np)) return false;
  QMat E(Np * 4 * Nfp, 0);
  for (int f = 0; f < 4; ++f) {
    QMat Ef = matmul(matmul(VinvT, EB[f], Np, Np, Np), Vinv, Np, Np, Np);
    for (int i = 0; i < Np; ++i)
      for (int m = 0; m < Nfp; ++m) E[i * 4 * Nfp + f * Nfp + m] = Ef[i * Np + out.Fmask[f * Nfp + m]];
  }
  out.LIFT = to_double(matmul(Minv, E, Np, Np, 4 * Nfp));
  return true;
}

}  // namespace dg
