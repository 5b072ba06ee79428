// C ABI of the tensor-product hexahedron path: 1-D reference tables, the
// periodic rectilinear mesh, right-hand side and LSRK step.
//
// Reference element: the tensor product of the p + 1 Legendre-Gauss-Lobatto
// points (closed forms for p <= 4), node (a, b, c) at index
// a + (p + 1)(b + (p + 1) c).  The 1-D tables are the Lagrange derivative
// matrix D1[i][j] = l_j'(x_i) and the lift columns M1^{-1} e_0, M1^{-1} e_p of
// the exact 1-D mass matrix M1[i][j] = int_{-1}^{1} l_i l_j; they are formed
// at the rounded FP64 points in IEEE binary128 and rounded once (the mass
// matrix from the monomial Vandermonde V and the monomial Gram matrix H:
// M1^{-1} = V H^{-1} V^T).
#include <cmath>
#include <cstring>
#include <string>

#include "hex.hpp"

namespace dg {

namespace {

using qd = __float128;

qd qsqrt(qd a) {
  if (a <= 0) return 0;
  qd x = std::sqrt(static_cast<double>(a));
  for (int k = 0; k < 2; ++k) x = 0.5 * (x + a / x);
  return x;
}

qd qabs(qd a) { return a < 0 ? -a : a; }

// Gauss-Jordan inverse with partial pivoting of a small matrix.
bool qinvert(std::vector<qd>& A, int n) {
  std::vector<qd> inv(static_cast<size_t>(n) * n, 0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (qabs(A[r * n + c]) > qabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0) return false;
    for (int k = 0; k < n; ++k) { std::swap(A[c * n + k], A[piv * n + k]); std::swap(inv[c * n + k], inv[piv * n + k]); }
    const qd d = 1 / A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] *= d; inv[c * n + k] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c || A[r * n + c] == 0) continue;
      const qd f = A[r * n + c];
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
    }
  }
  A.swap(inv);
  return true;
}

// M1^{-1} of the Lagrange basis on the points x (exact 1-D mass matrix
// int_{-1}^{1} l_i l_j): V H^{-1} V^T with V[i][k] = x_i^k and
// H[k][l] = int x^(k + l).
bool exact_inverse_mass(const std::vector<qd>& x, std::vector<qd>& Minv) {
  const int n = static_cast<int>(x.size());
  std::vector<qd> V(n * n), H(n * n);
  for (int i = 0; i < n; ++i) {
    qd pw = 1;
    for (int k = 0; k < n; ++k) { V[i * n + k] = pw; pw *= x[i]; }
  }
  for (int k = 0; k < n; ++k)
    for (int l = 0; l < n; ++l) H[k * n + l] = (k + l) % 2 ? qd(0) : qd(2) / (k + l + 1);
  if (!qinvert(H, n)) return false;
  Minv.assign(n * n, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      qd s = 0;
      for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l) s += V[i * n + k] * H[k * n + l] * V[j * n + l];
      Minv[i * n + j] = s;
    }
  return true;
}

}  // namespace

bool build_hex_1d(int p, std::vector<double>& x, std::vector<double>& D1, std::vector<double>& lift) {
  if (p < 1 || p > kHexMaxOrder) return false;
  const int n = p + 1;
  // LGL points (closed forms), rounded to FP64
  qd xq[kHexMaxOrder + 1];
  xq[0] = -1;
  xq[p] = 1;
  if (p == 2) xq[1] = 0;
  if (p == 3) { xq[1] = -1 / qsqrt(5); xq[2] = -xq[1]; }
  if (p == 4) { xq[1] = -qsqrt(qd(3) / 7); xq[2] = 0; xq[3] = -xq[1]; }
  x.resize(n);
  for (int i = 0; i < n; ++i) { x[i] = static_cast<double>(xq[i]); xq[i] = x[i]; }
  // derivative matrix from the barycentric weights w_j = 1 / prod_{m != j} (x_j - x_m)
  qd w[kHexMaxOrder + 1];
  for (int j = 0; j < n; ++j) {
    qd pr = 1;
    for (int m = 0; m < n; ++m) if (m != j) pr *= xq[j] - xq[m];
    w[j] = 1 / pr;
  }
  std::vector<qd> D(n * n, 0);
  for (int i = 0; i < n; ++i) {
    qd diag = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      D[i * n + j] = (w[j] / w[i]) / (xq[i] - xq[j]);
      diag += 1 / (xq[i] - xq[j]);
    }
    D[i * n + i] = diag;
  }
  // lift columns: M1^{-1} e_k = V H^{-1} V^T e_k, V[i][k] = x_i^k, H[k][l] = int x^(k + l)
  std::vector<qd> V(n * n), H(n * n);
  for (int i = 0; i < n; ++i) {
    qd pw = 1;
    for (int k = 0; k < n; ++k) { V[i * n + k] = pw; pw *= xq[i]; }
  }
  for (int k = 0; k < n; ++k)
    for (int l = 0; l < n; ++l) H[k * n + l] = (k + l) % 2 ? qd(0) : qd(2) / (k + l + 1);
  if (!qinvert(H, n)) return false;
  D1.resize(n * n);
  for (int i = 0; i < n * n; ++i) D1[i] = static_cast<double>(D[i]);
  lift.assign(n * 2, 0.0);
  for (int side = 0; side < 2; ++side) {
    const int row = side == 0 ? 0 : p;  // V^T e_row = (x_row^k)_k
    std::vector<qd> y(n, 0);
    for (int k = 0; k < n; ++k)
      for (int l = 0; l < n; ++l) y[k] += H[k * n + l] * V[row * n + l];
    for (int i = 0; i < n; ++i) {
      qd s = 0;
      for (int k = 0; k < n; ++k) s += V[i * n + k] * y[k];
      lift[i * 2 + side] = static_cast<double>(s);
    }
  }
  return true;
}

bool build_hex_oi(int p, std::vector<double>& xqd, std::vector<double>& wqd, std::vector<double>& tables) {
  if (p < 1 || p > kHexMaxOrder) return false;
  const int n = p + 1, nq = hex_oi_points(p);
  std::vector<double> xg, D1, lift;
  if (!build_hex_1d(p, xg, D1, lift)) return false;
  // Gauss-Legendre points: Newton on P_nq from the Chebyshev-like guesses,
  // in FP64 and then in binary128; weights 2 / ((1 - x^2) P'(x)^2)
  auto legendre = [&](qd x, qd& Pn, qd& dPn) {
    qd P0 = 1, P1 = x, d0 = 0, d1 = 1;
    for (int k = 1; k < nq; ++k) {
      const qd P2 = ((2 * k + 1) * x * P1 - k * P0) / (k + 1);
      const qd d2 = ((2 * k + 1) * (P1 + x * d1) - k * d0) / (k + 1);
      P0 = P1; P1 = P2; d0 = d1; d1 = d2;
    }
    Pn = P1;
    dPn = d1;
  };
  // the rule is symmetric: the negative half by Newton, the rest mirrored,
  // the middle point of an odd rule exactly 0
  std::vector<qd> xq(nq), wq(nq);
  xqd.assign(nq, 0.0);
  wqd.assign(nq, 0.0);
  for (int i = 0; i < (nq + 1) / 2; ++i) {
    qd x = 0;
    if (2 * i + 1 != nq) {
      x = -std::cos(3.14159265358979323846 * (i + 0.75) / (nq + 0.5));
      for (int it = 0; it < 12; ++it) {
        qd Pn, dPn;
        legendre(x, Pn, dPn);
        x -= Pn / dPn;
      }
    }
    qd Pn, dPn;
    legendre(x, Pn, dPn);
    xqd[i] = static_cast<double>(x);
    if (2 * i + 1 != nq) xqd[nq - 1 - i] = -xqd[i];
    wqd[i] = wqd[nq - 1 - i] = static_cast<double>(2 / ((1 - x * x) * dPn * dPn));
  }
  for (int i = 0; i < nq; ++i) {
    xq[i] = xqd[i];
    wq[i] = wqd[i];
  }
  // Lagrange basis on the FP64 LGL points, at the FP64 Gauss points
  std::vector<qd> x(n);
  for (int j = 0; j < n; ++j) x[j] = xg[j];
  std::vector<qd> B(nq * n), Bd(nq * n);
  for (int k = 0; k < nq; ++k)
    for (int j = 0; j < n; ++j) {
      qd l = 1, dl = 0;
      for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        const qd f = (xq[k] - x[m]) / (x[j] - x[m]);
        dl = dl * f + l / (x[j] - x[m]);
        l *= f;
      }
      B[k * n + j] = l;
      Bd[k * n + j] = dl;
    }
  // S = M1^{-1} B'^T W, P = M1^{-1} B^T W with the exact mass matrix
  // (M1^{-1} = V H^{-1} V^T, monomial Vandermonde V and Gram matrix H)
  std::vector<qd> M;
  if (!exact_inverse_mass(x, M)) return false;
  tables.assign(3 * nq * n + 2 * n, 0.0);
  for (int k = 0; k < nq; ++k)
    for (int j = 0; j < n; ++j) tables[k * n + j] = static_cast<double>(B[k * n + j]);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < nq; ++k) {
      qd s = 0, pp = 0;
      for (int j = 0; j < n; ++j) {
        s += M[i * n + j] * Bd[k * n + j] * wq[k];
        pp += M[i * n + j] * B[k * n + j] * wq[k];
      }
      tables[nq * n + i * nq + k] = static_cast<double>(s);
      tables[2 * nq * n + i * nq + k] = static_cast<double>(pp);
    }
  for (int i = 0; i < 2 * n; ++i) tables[3 * nq * n + i] = lift[i];
  return true;
}

bool build_hex_shock_tables(int p, std::vector<double>& tables) {
  if (p < 1 || p > kHexMaxOrder) return false;
  const int n = p + 1;
  std::vector<double> xg, D1, lift;
  if (!build_hex_1d(p, xg, D1, lift)) return false;
  // orthonormal Legendre Vandermonde Vm[i][k] = sqrt((2k + 1)/2) P_k(x_i) and
  // the monomial one (for the weights int l_i = sum_k (V^{-1})[k][i] int x^k)
  std::vector<qd> Vm(n * n), V(n * n);
  for (int i = 0; i < n; ++i) {
    const qd x = xg[i];
    qd P0 = 1, P1 = x, pw = 1;
    for (int k = 0; k < n; ++k) {
      const qd Pk = k == 0 ? P0 : P1;
      Vm[i * n + k] = Pk * qsqrt(qd(2 * k + 1) / 2);
      if (k >= 1) {
        const qd P2 = ((2 * k + 1) * x * P1 - k * P0) / (k + 1);
        P0 = P1;
        P1 = P2;
      }
      V[i * n + k] = pw;
      pw *= x;
    }
  }
  if (!qinvert(Vm, n) || !qinvert(V, n)) return false;
  tables.assign(n * n + n, 0.0);
  for (int i = 0; i < n * n; ++i) tables[i] = static_cast<double>(Vm[i]);
  for (int i = 0; i < n; ++i) {
    qd w = 0;
    for (int k = 0; k < n; k += 2) w += V[k * n + i] * qd(2) / (k + 1);
    tables[n * n + i] = static_cast<double>(w);
  }
  return true;
}

}  // namespace dg

using namespace dg;

namespace {

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

dg_status check_euler_params(const char* who, const dg_params* prm) {
  if (!prm) return fail(DG_ERR_ARG, std::string(who) + ": params is NULL");
  if (prm->model != 0) return fail(DG_ERR_UNSUPPORTED, std::string(who) + ": hexahedra run the Euler model (0) only");
  if (!(prm->gamma > 1.0) || !std::isfinite(prm->gamma)) return fail(DG_ERR_ARG, std::string(who) + ": gamma must be > 1");
  return DG_OK;
}

}  // namespace

extern "C" dg_status dg_hex_reference_operators(int order, double* x, double* D1, double* lift) {
  std::vector<double> xs, Ds, ls;
  if (!build_hex_1d(order, xs, Ds, ls)) return fail(DG_ERR_ARG, "dg_hex_reference_operators: order must be in 1..4");
  if (x) std::memcpy(x, xs.data(), xs.size() * sizeof(double));
  if (D1) std::memcpy(D1, Ds.data(), Ds.size() * sizeof(double));
  if (lift) std::memcpy(lift, ls.data(), ls.size() * sizeof(double));
  return DG_OK;
}

extern "C" dg_status dg_hex_mesh_create(int order, int nx, int ny, int nz, const double* gx, const double* gy,
                                        const double* gz, int device, dg_hex_mesh* out) {
  if (!out) return fail(DG_ERR_ARG, "dg_hex_mesh_create: out is NULL");
  *out = nullptr;
  if (order < 1 || order > kHexMaxOrder) return fail(DG_ERR_ARG, "dg_hex_mesh_create: order must be in 1..4");
  if (nx < 1 || ny < 1 || nz < 1) return fail(DG_ERR_ARG, "dg_hex_mesh_create: cell counts must be >= 1");
  const int64_t E = static_cast<int64_t>(nx) * ny * nz;
  const int64_t N1 = order + 1;
  if (E * N1 * N1 * N1 > 0x7fffffff) return fail(DG_ERR_ARG, "dg_hex_mesh_create: more than 2^31 - 1 nodes");
  if (!gx || !gy || !gz) return fail(DG_ERR_ARG, "dg_hex_mesh_create: null grid-line array");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(DG_ERR_ARG, "dg_hex_mesh_create: invalid device");
  HexMesh* m = new (std::nothrow) HexMesh();
  if (!m) return fail(DG_ERR_ALLOC, "dg_hex_mesh_create: host allocation failed");
  auto cleanup = [&](dg_status s) { dg_hex_mesh_destroy(reinterpret_cast<dg_hex_mesh>(m)); return s; };
  m->device = device;
  m->p = order;
  m->N1 = order + 1;
  m->Np = m->N1 * m->N1 * m->N1;
  m->nx = nx; m->ny = ny; m->nz = nz;
  m->E = E;
  m->gx.assign(gx, gx + nx + 1);
  m->gy.assign(gy, gy + ny + 1);
  m->gz.assign(gz, gz + nz + 1);
  std::vector<double> ih;
  ih.reserve(nx + ny + nz);
  for (const std::vector<double>* g : {&m->gx, &m->gy, &m->gz})
    for (size_t i = 0; i + 1 < g->size(); ++i) {
      const double h = (*g)[i + 1] - (*g)[i];
      if (!(h > 0.0) || !std::isfinite(h))
        return cleanup(fail(DG_ERR_MESH, "dg_hex_mesh_create: grid lines must increase strictly"));
      ih.push_back(2.0 / h);
    }
  if (!build_hex_1d(order, m->x1, m->D1, m->lift))
    return cleanup(fail(DG_ERR_ARG, "dg_hex_mesh_create: reference tables failed"));
  std::vector<double> op(m->D1);
  op.insert(op.end(), m->lift.begin(), m->lift.end());
  {
    std::vector<double> xq, wq;
    if (!build_hex_oi(order, xq, wq, m->oi))
      return cleanup(fail(DG_ERR_ARG, "dg_hex_mesh_create: overintegration tables failed"));
    m->nq = hex_oi_points(order);
  }
  std::vector<double> sh;
  if (!build_hex_shock_tables(order, sh))
    return cleanup(fail(DG_ERR_ARG, "dg_hex_mesh_create: shock-capturing tables failed"));
  DeviceGuard g(device);
  if (!g.ok) return cleanup(fail(DG_ERR_HIP, "dg_hex_mesh_create: hipSetDevice failed"));
  auto up = [&](double** dst, const std::vector<double>& src) -> dg_status {
    if (hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(double)) != hipSuccess)
      return fail(DG_ERR_ALLOC, "dg_hex_mesh_create: hipMalloc failed");
    if (hipMemcpy(*dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return fail(DG_ERR_HIP, "dg_hex_mesh_create: hipMemcpy failed");
    return DG_OK;
  };
  dg_status st = up(&m->d_ih, ih);
  if (st == DG_OK) st = up(&m->d_op, op);
  if (st == DG_OK) st = up(&m->d_oi, m->oi);
  if (st == DG_OK) st = up(&m->d_sh, sh);
  if (st != DG_OK) return cleanup(st);
  *out = reinterpret_cast<dg_hex_mesh>(m);
  return DG_OK;
}

extern "C" dg_status dg_hex_mesh_destroy(dg_hex_mesh h) {
  if (!h) return DG_OK;
  HexMesh* m = reinterpret_cast<HexMesh*>(h);
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(m->device);
  hipFree(m->d_ih);
  hipFree(m->d_op);
  hipFree(m->d_oi);
  hipFree(m->d_sh);
  hipSetDevice(prev);
  delete m;
  return DG_OK;
}

extern "C" dg_status dg_hex_mesh_info(dg_hex_mesh h, int64_t* n_elem, int* np) {
  if (!h) return fail(DG_ERR_ARG, "dg_hex_mesh_info: null mesh");
  const HexMesh* m = reinterpret_cast<const HexMesh*>(h);
  if (n_elem) *n_elem = m->E;
  if (np) *np = m->Np;
  return DG_OK;
}

extern "C" dg_status dg_hex_mesh_nodes(dg_hex_mesh h, double* xyz) {
  if (!h || !xyz) return fail(DG_ERR_ARG, "dg_hex_mesh_nodes: null argument");
  const HexMesh* m = reinterpret_cast<const HexMesh*>(h);
  const int N1 = m->N1;
  for (int k = 0; k < m->nz; ++k)
    for (int j = 0; j < m->ny; ++j)
      for (int i = 0; i < m->nx; ++i) {
        const int64_t e = i + static_cast<int64_t>(m->nx) * (j + static_cast<int64_t>(m->ny) * k);
        const double hx = m->gx[i + 1] - m->gx[i], hy = m->gy[j + 1] - m->gy[j], hz = m->gz[k + 1] - m->gz[k];
        for (int c = 0; c < N1; ++c)
          for (int b = 0; b < N1; ++b)
            for (int a = 0; a < N1; ++a) {
              double* X = xyz + (e * m->Np + a + N1 * (b + N1 * c)) * 3;
              X[0] = m->gx[i] + 0.5 * (1.0 + m->x1[a]) * hx;
              X[1] = m->gy[j] + 0.5 * (1.0 + m->x1[b]) * hy;
              X[2] = m->gz[k] + 0.5 * (1.0 + m->x1[c]) * hz;
            }
      }
  return DG_OK;
}

namespace {

dg_status hex_rhs_form(dg_hex_mesh h, const dg_params* prm, const double* q, double* rhs, hipStream_t stream, bool oi) {
  const char* who = oi ? "dg_hex_rhs_oi" : "dg_hex_rhs";
  if (!h) return fail(DG_ERR_ARG, std::string(who) + ": null mesh");
  dg_status st = check_euler_params(who, prm);
  if (st != DG_OK) return st;
  if (!q || !rhs || !aligned8(q) || !aligned8(rhs))
    return fail(DG_ERR_ARG, std::string(who) + ": null or misaligned state pointer");
  const HexMesh& m = *reinterpret_cast<const HexMesh*>(h);
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  if (rhs < q + n && q < rhs + n) return fail(DG_ERR_ARG, std::string(who) + ": q and rhs overlap");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, std::string(who) + ": hipSetDevice failed");
  return oi ? launch_rhs_hex_oi(m, prm->gamma, q, rhs, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, false, stream)
            : launch_rhs_hex(m, prm->gamma, q, rhs, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, false, stream);
}

dg_status hex_step_form(dg_hex_mesh h, const dg_params* prm, double* q, double* work, double dt, hipStream_t stream,
                        bool oi) {
  const char* who = oi ? "dg_hex_rk_step_oi" : "dg_hex_rk_step";
  if (!h) return fail(DG_ERR_ARG, std::string(who) + ": null mesh");
  dg_status st = check_euler_params(who, prm);
  if (st != DG_OK) return st;
  if (!std::isfinite(dt)) return fail(DG_ERR_ARG, std::string(who) + ": dt must be finite");
  if (!q || !work || !aligned8(q) || !aligned8(work)) return fail(DG_ERR_ARG, std::string(who) + ": null or misaligned pointer");
  const HexMesh& m = *reinterpret_cast<const HexMesh*>(h);
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  if (work < q + n && q < work + 2 * n) return fail(DG_ERR_ARG, std::string(who) + ": work overlaps q");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, std::string(who) + ": hipSetDevice failed");
  // fused stages write another buffer than they read (neighbouring
  // elements still read the stage input); q and the two halves of work
  // rotate so that the fifth stage writes q
  for (int s = 0; s < 5; ++s) {
    const LsrkBuffers B = lsrk_buffers(s, q, work, work + n);
    st = oi ? launch_rhs_hex_oi(m, prm->gamma, B.q_in, nullptr, B.res_in, B.res_out, B.q_out, kLsrkA[s], kLsrkB[s],
                                dt, true, stream)
            : launch_rhs_hex(m, prm->gamma, B.q_in, nullptr, B.res_in, B.res_out, B.q_out, kLsrkA[s], kLsrkB[s], dt,
                             true, stream);
    if (st != DG_OK) return st;
  }
  return DG_OK;
}

}  // namespace

extern "C" dg_status dg_hex_rhs(dg_hex_mesh h, const dg_params* prm, const double* q, double* rhs, hipStream_t stream) {
  return hex_rhs_form(h, prm, q, rhs, stream, false);
}

extern "C" dg_status dg_hex_rhs_oi(dg_hex_mesh h, const dg_params* prm, const double* q, double* rhs,
                                   hipStream_t stream) {
  return hex_rhs_form(h, prm, q, rhs, stream, true);
}

extern "C" dg_status dg_hex_rk_step_oi(dg_hex_mesh h, const dg_params* prm, double* q, double* work, double t,
                                       double dt, hipStream_t stream) {
  (void)t;
  return hex_step_form(h, prm, q, work, dt, stream, true);
}

extern "C" dg_status dg_hex_oi_operators(int order, int* nq, double* xq, double* wq, double* tables) {
  std::vector<double> x, w, tab;
  if (!build_hex_oi(order, x, w, tab)) return fail(DG_ERR_ARG, "dg_hex_oi_operators: order must be in 1..4");
  if (nq) *nq = static_cast<int>(x.size());
  if (xq) std::memcpy(xq, x.data(), x.size() * sizeof(double));
  if (wq) std::memcpy(wq, w.data(), w.size() * sizeof(double));
  if (tables) std::memcpy(tables, tab.data(), tab.size() * sizeof(double));
  return DG_OK;
}

extern "C" dg_status dg_hex_rk_step(dg_hex_mesh h, const dg_params* prm, double* q, double* work, double t, double dt,
                                    hipStream_t stream) {
  (void)t;
  return hex_step_form(h, prm, q, work, dt, stream, false);
}

namespace {

dg_status check_av(const char* who, const dg_av_params* av) {
  if (!av) return fail(DG_ERR_ARG, std::string(who) + ": av params is NULL");
  if (!std::isfinite(av->s0) || !(av->kappa > 0.0) || !std::isfinite(av->kappa) || !(av->c_eps >= 0.0) ||
      !std::isfinite(av->c_eps) || !(av->delta > 0.0) || !std::isfinite(av->delta))
    return fail(DG_ERR_ARG, std::string(who) + ": need finite s0, kappa > 0, c_eps >= 0, delta > 0");
  return DG_OK;
}

}  // namespace

extern "C" dg_status dg_hex_av_viscosity(dg_hex_mesh h, const dg_params* prm, const dg_av_params* av, const double* q,
                                         double* s_out, double* eps_out, double* G_out, hipStream_t stream) {
  if (!h) return fail(DG_ERR_ARG, "dg_hex_av_viscosity: null mesh");
  dg_status st = check_euler_params("dg_hex_av_viscosity", prm);
  if (st == DG_OK) st = check_av("dg_hex_av_viscosity", av);
  if (st != DG_OK) return st;
  if (!q || !G_out || !eps_out || !aligned8(q) || !aligned8(G_out) || !aligned8(eps_out) || (s_out && !aligned8(s_out)))
    return fail(DG_ERR_ARG, "dg_hex_av_viscosity: null or misaligned pointer");
  const HexMesh& m = *reinterpret_cast<const HexMesh*>(h);
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_hex_av_viscosity: hipSetDevice failed");
  return launch_hex_av_flux(m, *av, prm->gamma, q, G_out, s_out, eps_out, stream);
}

extern "C" dg_status dg_hex_av_rhs(dg_hex_mesh h, const dg_params* prm, const dg_av_params* av, const double* q,
                                   double* rhs, double* work, hipStream_t stream) {
  if (!h) return fail(DG_ERR_ARG, "dg_hex_av_rhs: null mesh");
  dg_status st = check_euler_params("dg_hex_av_rhs", prm);
  if (st == DG_OK) st = check_av("dg_hex_av_rhs", av);
  if (st != DG_OK) return st;
  if (!q || !rhs || !work || !aligned8(q) || !aligned8(rhs) || !aligned8(work))
    return fail(DG_ERR_ARG, "dg_hex_av_rhs: null or misaligned pointer");
  const HexMesh& m = *reinterpret_cast<const HexMesh*>(h);
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  const size_t nw = 3 * n + 2 * static_cast<size_t>(m.E);
  if ((rhs < q + n && q < rhs + n) || (work < q + n && q < work + nw) || (work < rhs + n && rhs < work + nw))
    return fail(DG_ERR_ARG, "dg_hex_av_rhs: q, rhs and work must not overlap");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_hex_av_rhs: hipSetDevice failed");
  double* G = work;
  st = launch_hex_av_flux(m, *av, prm->gamma, q, G, work + 3 * n, work + 3 * n + m.E, stream);
  if (st != DG_OK) return st;
  return launch_rhs_hex_av(m, prm->gamma, q, G, work + 3 * n + m.E, rhs, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, false, stream);
}

extern "C" dg_status dg_hex_limit(dg_hex_mesh h, const dg_params* prm, const dg_av_params* av, double* q,
                                  hipStream_t stream) {
  if (!h) return fail(DG_ERR_ARG, "dg_hex_limit: null mesh");
  dg_status st = check_euler_params("dg_hex_limit", prm);
  if (st == DG_OK) st = check_av("dg_hex_limit", av);
  if (st != DG_OK) return st;
  if (!q || !aligned8(q)) return fail(DG_ERR_ARG, "dg_hex_limit: null or misaligned q");
  const HexMesh& m = *reinterpret_cast<const HexMesh*>(h);
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_hex_limit: hipSetDevice failed");
  return launch_hex_limit(m, *av, prm->gamma, q, stream);
}

extern "C" dg_status dg_hex_shock_rk_step(dg_hex_mesh h, const dg_params* prm, const dg_av_params* av, double* q,
                                          double* work, double t, double dt, hipStream_t stream) {
  (void)t;
  if (!h) return fail(DG_ERR_ARG, "dg_hex_shock_rk_step: null mesh");
  dg_status st = check_euler_params("dg_hex_shock_rk_step", prm);
  if (st == DG_OK) st = check_av("dg_hex_shock_rk_step", av);
  if (st != DG_OK) return st;
  if (!std::isfinite(dt)) return fail(DG_ERR_ARG, "dg_hex_shock_rk_step: dt must be finite");
  if (!q || !work || !aligned8(q) || !aligned8(work))
    return fail(DG_ERR_ARG, "dg_hex_shock_rk_step: null or misaligned pointer");
  const HexMesh& m = *reinterpret_cast<const HexMesh*>(h);
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  const size_t nw = 5 * n + 2 * static_cast<size_t>(m.E);
  if (work < q + n && q < work + nw) return fail(DG_ERR_ARG, "dg_hex_shock_rk_step: work overlaps q");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_hex_shock_rk_step: hipSetDevice failed");
  // work = [two state buffers | G (3 n) | s (E) | eps (E)]; each stage: the
  // viscous fluxes of its input, the fused RHS + stage update into another
  // buffer (rotating as in the plain step), the limiter on that new state
  double* G = work + 2 * n;
  for (int s = 0; s < 5; ++s) {
    const LsrkBuffers B = lsrk_buffers(s, q, work, work + n);
    st = launch_hex_av_flux(m, *av, prm->gamma, B.q_in, G, work + 5 * n, work + 5 * n + m.E, stream);
    if (st == DG_OK)
      st = launch_rhs_hex_av(m, prm->gamma, B.q_in, G, work + 5 * n + m.E, nullptr, B.res_in, B.res_out, B.q_out,
                             kLsrkA[s], kLsrkB[s], dt, true, stream);
    if (st == DG_OK) st = launch_hex_limit(m, *av, prm->gamma, B.q_out, stream);
    if (st != DG_OK) return st;
  }
  return DG_OK;
}
