// Mesh handle construction: affine geometric factors, face connectivity with
// vertex permutations, neighbour-node tables, and device upload.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace dg {

OpLayout op_layout(int p) {
  OpLayout L{};
  L.p = p;
  L.Np = nodes_of(p);
  L.Nfp = face_nodes_of(p);
  L.NPP = (L.Np + 3) / 4 * 4;
  L.NB16 = L.Np / 16;
  L.NB4 = (L.Np - 16 * L.NB16 + 3) / 4;
  L.KV = L.NPP / 4;
  L.KL = L.Nfp;
  L.KS = 3 * L.KV + L.KL;
  L.NRB = L.NB16 + L.NB4;
  return L;
}

namespace {

// the six permutations of (0, 1, 2) in lexicographic order
const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Neighbour-node table: for own face f, neighbour face fp and permutation pi
// (own face vertex i is neighbour face vertex pi[i]), the neighbour volume node
// matching own face node m.  Matching uses the integer lattice labels, which
// the symmetric warp & blend map carries to coincident physical points.
bool build_nbtab(const RefElem& R, std::vector<uint8_t>& tab) {
  const int Nfp = R.Nfp;
  tab.assign(4 * 24 * Nfp, 0);
  for (int f = 0; f < 4; ++f)
    for (int fp = 0; fp < 4; ++fp)
      for (int pi = 0; pi < 6; ++pi)
        for (int m = 0; m < Nfp; ++m) {
          const int j = R.Fmask[f * Nfp + m];
          int want[3];
          for (int i = 0; i < 3; ++i) want[kPerm[pi][i]] = R.lattice[j * 4 + kFaceVerts[f][i]];
          int found = -1;
          for (int mp = 0; mp < Nfp; ++mp) {
            const int jp = R.Fmask[fp * Nfp + mp];
            bool ok = true;
            for (int k = 0; k < 3; ++k) ok = ok && R.lattice[jp * 4 + kFaceVerts[fp][k]] == want[k];
            if (ok) { found = jp; break; }
          }
          if (found < 0) return false;
          tab[(f * 24 + fp * 6 + pi) * Nfp + m] = static_cast<uint8_t>(found);
        }
  return true;
}

// The FP64 contraction table [-Dr | -Ds | -Dt | LIFT / 2] in the kernel's
// MFMA operand order (the face kernels contract twice the jump).
void build_op64(const RefElem& R, const OpLayout& L, std::vector<double>& A) {
  const int Np = R.Np, Nfp = R.Nfp;
  const int K = 3 * L.NPP + 4 * Nfp;
  std::vector<double> Op(static_cast<size_t>(Np) * K, 0.0);
  const std::vector<double>* D[3] = {&R.Dr, &R.Ds, &R.Dt};
  for (int i = 0; i < Np; ++i) {
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < Np; ++j) Op[i * K + a * L.NPP + j] = -(*D[a])[i * Np + j];
    for (int c = 0; c < 4 * Nfp; ++c) Op[i * K + 3 * L.NPP + c] = 0.5 * R.LIFT[i * 4 * Nfp + c];
  }
  A.assign(static_cast<size_t>(L.KS) * L.NRB * 64, 0.0);
  for (int ks = 0; ks < L.KS; ++ks)
    for (int rb = 0; rb < L.NRB; ++rb)
      for (int l = 0; l < 64; ++l) {
        const int k = 4 * ks + l / 16;
        const int row = rb < L.NB16 ? 16 * rb + l % 16 : 16 * L.NB16 + 4 * (rb - L.NB16) + l % 4;
        A[(static_cast<size_t>(ks) * L.NRB + rb) * 64 + l] = row < Np ? Op[row * K + k] : 0.0;
      }
}

// round-to-nearest-even FP32 -> BF16 bit pattern (finite inputs)
uint16_t bf16_bits(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t b = static_cast<uint32_t>(h) << 16;
  float x;
  std::memcpy(&x, &b, 4);
  return x;
}

// Op[i][col] of [-Dr | -Ds | -Dt | LIFT / 2] with each D block padded to NPP
// columns (the face kernels contract twice the Lax-Friedrichs jump)
double op_entry(const RefElem& R, int NPP, int i, int col) {
  if (i >= R.Np) return 0.0;
  if (col < 3 * NPP) {
    const int a = col / NPP, j = col % NPP;
    if (j >= R.Np) return 0.0;
    const std::vector<double>& D = a == 0 ? R.Dr : a == 1 ? R.Ds : R.Dt;
    return -D[i * R.Np + j];
  }
  return 0.5 * R.LIFT[i * 4 * R.Nfp + (col - 3 * NPP)];
}

void build_lowp_tables(const RefElem& R, std::vector<float>& op32, std::vector<uint16_t>& opbf) {
  const LowpLayout L = lowp_layout(R.p);
  op32.assign(static_cast<size_t>(L.KS32) * L.NR * 64, 0.f);
  for (int ks = 0; ks < L.KS32; ++ks)
    for (int rb = 0; rb < L.NR; ++rb)
      for (int l = 0; l < 64; ++l) {
        const int row = L.REM4 && rb == L.NR - 1 ? 16 * rb + l % 4 : 16 * rb + l % 16;
        op32[(static_cast<size_t>(ks) * L.NR + rb) * 64 + l] =
            static_cast<float>(op_entry(R, L.NPP, row, 4 * ks + l / 16));
      }
  opbf.assign(static_cast<size_t>(L.VKS + L.FKS) * L.NR * 2 * 64 * 8, 0);
  for (int k = 0; k < L.VKS + L.FKS; ++k)
    for (int rb = 0; rb < L.NR; ++rb)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          const int i = 16 * rb + l % 16, g = l / 16;
          int col = -1;
          if (k < L.VKS) {
            const int t = 8 * k + e;
            if (t < 3 * L.KV) col = (t % 3) * L.NPP + 4 * (t / 3) + g;
          } else {
            const int t = 8 * (k - L.VKS) + e;
            if (t < L.KL) col = 3 * L.NPP + 4 * t + g;
          }
          const float x = static_cast<float>(col < 0 ? 0.0 : op_entry(R, L.NPP, i, col));
          const uint16_t hi = bf16_bits(x);
          const uint16_t lo = bf16_bits(x - bf16_value(hi));
          const size_t base = ((static_cast<size_t>(k) * L.NR + rb) * 2) * 64 * 8;
          opbf[base + (0 * 64 + l) * 8 + e] = hi;
          opbf[base + (1 * 64 + l) * 8 + e] = lo;
        }
}

struct FaceRec {
  int64_t a, b, c;  // sorted vertex ids
  int64_t id;       // 4 * element + face
};

}  // namespace

}  // namespace dg

using namespace dg;

extern "C" dg_status dg_mesh_create(int order, int64_t n_elem, const double* elem_xyz, const int64_t* elem_vid,
                                    int device, dg_mesh* out) {
  if (!out) return fail(DG_ERR_ARG, "dg_mesh_create: out is NULL");
  *out = nullptr;
  if (order < 1 || order > kMaxOrder) return fail(DG_ERR_ARG, "dg_mesh_create: order must be in 1..4");
  if (n_elem < 1 || n_elem > (int64_t(1) << 27)) return fail(DG_ERR_ARG, "dg_mesh_create: n_elem out of range");
  if (!elem_xyz || !elem_vid) return fail(DG_ERR_ARG, "dg_mesh_create: null input array");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(DG_ERR_ARG, "dg_mesh_create: invalid device");

  Mesh* m = new (std::nothrow) Mesh();
  if (!m) return fail(DG_ERR_ALLOC, "dg_mesh_create: host allocation failed");
  auto cleanup = [&](dg_status s) { dg_mesh_destroy(reinterpret_cast<dg_mesh>(m)); return s; };
  m->device = device;
  m->p = order;
  if (!build_ref_elem(order, m->ref)) return cleanup(fail(DG_ERR_ARG, "dg_mesh_create: reference element failed"));
  m->Np = m->ref.Np;
  m->Nfp = m->ref.Nfp;
  m->E = n_elem;
  m->Epad = (n_elem + 15) / 16 * 16;
  m->lay = op_layout(order);
  const int64_t E = n_elem, Ep = m->Epad;
  m->elem_xyz.assign(elem_xyz, elem_xyz + E * 12);

  // geometric factors: columns x_r, x_s, x_t of the affine map; the rows of
  // the inverse are grad r = (x_s x x_t)/J, grad s = (x_t x x_r)/J, grad t = (x_r x x_s)/J
  std::vector<double> geo(9 * Ep, 0.0);
  for (int64_t e = 0; e < Ep; ++e) {
    const int64_t k = e < E ? e : E - 1;
    const double* X = elem_xyz + k * 12;
    double c[3][3];
    for (int d = 0; d < 3; ++d) {
      c[0][d] = 0.5 * (X[3 + d] - X[d]);
      c[1][d] = 0.5 * (X[6 + d] - X[d]);
      c[2][d] = 0.5 * (X[9 + d] - X[d]);
    }
    auto cross = [](const double* u, const double* v, double* w) {
      w[0] = u[1] * v[2] - u[2] * v[1];
      w[1] = u[2] * v[0] - u[0] * v[2];
      w[2] = u[0] * v[1] - u[1] * v[0];
    };
    double gr[3], gs[3], gt[3];
    cross(c[1], c[2], gr);
    cross(c[2], c[0], gs);
    cross(c[0], c[1], gt);
    const double J = c[0][0] * gr[0] + c[0][1] * gr[1] + c[0][2] * gr[2];
    if (!(J > 0.0) || !std::isfinite(J))
      return cleanup(fail(DG_ERR_MESH, "dg_mesh_create: element " + std::to_string(k) + " has non-positive Jacobian"));
    for (int d = 0; d < 3; ++d) {
      geo[(0 + d) * Ep + e] = gr[d] / J;
      geo[(3 + d) * Ep + e] = gs[d] / J;
      geo[(6 + d) * Ep + e] = gt[d] / J;
    }
  }

  // face matching on sorted global-vertex-id triples
  std::vector<FaceRec> faces(E * 4);
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 4; ++f) {
      int64_t v[3] = {elem_vid[e * 4 + kFaceVerts[f][0]], elem_vid[e * 4 + kFaceVerts[f][1]],
                      elem_vid[e * 4 + kFaceVerts[f][2]]};
      std::sort(v, v + 3);
      if (v[0] == v[1] || v[1] == v[2])
        return cleanup(fail(DG_ERR_MESH, "dg_mesh_create: degenerate face (repeated vertex id)"));
      faces[e * 4 + f] = {v[0], v[1], v[2], e * 4 + f};
    }
  std::sort(faces.begin(), faces.end(), [](const FaceRec& x, const FaceRec& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.c != y.c) return x.c < y.c;
    return x.id < y.id;
  });
  m->conn_host.assign(4 * Ep * 2, 0);
  for (int64_t i = 0; i < E * 4; i += 2) {
    const FaceRec& x = faces[i];
    if (i + 1 >= E * 4) return cleanup(fail(DG_ERR_MESH, "dg_mesh_create: unmatched face"));
    const FaceRec& y = faces[i + 1];
    if (x.a != y.a || x.b != y.b || x.c != y.c)
      return cleanup(fail(DG_ERR_MESH, "dg_mesh_create: unmatched face"));
    if (i + 2 < E * 4 && faces[i + 2].a == x.a && faces[i + 2].b == x.b && faces[i + 2].c == x.c)
      return cleanup(fail(DG_ERR_MESH, "dg_mesh_create: face shared by more than two elements"));
    for (int side = 0; side < 2; ++side) {
      const FaceRec& own = side ? y : x;
      const FaceRec& nb = side ? x : y;
      const int64_t e = own.id / 4, en = nb.id / 4;
      const int f = static_cast<int>(own.id % 4), fn = static_cast<int>(nb.id % 4);
      int pim[3];
      for (int a = 0; a < 3; ++a) {
        const int64_t g = elem_vid[e * 4 + kFaceVerts[f][a]];
        pim[a] = -1;
        for (int b = 0; b < 3; ++b)
          if (elem_vid[en * 4 + kFaceVerts[fn][b]] == g) pim[a] = b;
      }
      int code = -1;
      for (int k = 0; k < 6; ++k)
        if (kPerm[k][0] == pim[0] && kPerm[k][1] == pim[1] && kPerm[k][2] == pim[2]) code = k;
      if (code < 0) return cleanup(fail(DG_ERR_MESH, "dg_mesh_create: inconsistent face vertices"));
      m->conn_host[(f * Ep + e) * 2 + 0] = static_cast<int32_t>(en);
      m->conn_host[(f * Ep + e) * 2 + 1] = fn * 6 + code;
    }
  }
  // padded tail: point at the last element's own data
  for (int f = 0; f < 4; ++f)
    for (int64_t e = E; e < Ep; ++e) {
      m->conn_host[(f * Ep + e) * 2 + 0] = m->conn_host[(f * Ep + E - 1) * 2 + 0];
      m->conn_host[(f * Ep + e) * 2 + 1] = m->conn_host[(f * Ep + E - 1) * 2 + 1];
    }
  if (!build_nbtab(m->ref, m->nbtab)) return cleanup(fail(DG_ERR_MESH, "dg_mesh_create: face-node table failed"));
  std::vector<double> op64;
  build_op64(m->ref, m->lay, op64);
  // plain FP64 operator, row k of [D_r | D_s | D_t | LIFT] transposed:
  // opT[k][i] = Op[i][k] (consecutive rows i of one column are contiguous)
  const int Np = m->Np, KO = 3 * Np + 4 * m->Nfp;
  std::vector<double> opT(static_cast<size_t>(KO) * Np);
  for (int i = 0; i < Np; ++i) {
    for (int j = 0; j < Np; ++j) {
      opT[static_cast<size_t>(j) * Np + i] = m->ref.Dr[i * Np + j];
      opT[static_cast<size_t>(Np + j) * Np + i] = m->ref.Ds[i * Np + j];
      opT[static_cast<size_t>(2 * Np + j) * Np + i] = m->ref.Dt[i * Np + j];
    }
    for (int k = 0; k < 4 * m->Nfp; ++k) opT[static_cast<size_t>(3 * Np + k) * Np + i] = m->ref.LIFT[i * 4 * m->Nfp + k];
  }
  std::vector<float> op32;
  std::vector<uint16_t> opbf;
  build_lowp_tables(m->ref, op32, opbf);

  int prev = 0;
  hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return cleanup(fail(DG_ERR_HIP, "dg_mesh_create: hipSetDevice failed"));
  auto up = [&](void** dst, const void* src, size_t bytes) -> dg_status {
    if (hipMalloc(dst, bytes) != hipSuccess) return fail(DG_ERR_ALLOC, "dg_mesh_create: hipMalloc failed");
    if (hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
      return fail(DG_ERR_HIP, "dg_mesh_create: hipMemcpy failed");
    return DG_OK;
  };
  dg_status st = up(reinterpret_cast<void**>(&m->d_geo), geo.data(), geo.size() * sizeof(double));
  if (st == DG_OK) st = up(reinterpret_cast<void**>(&m->d_conn), m->conn_host.data(), m->conn_host.size() * sizeof(int32_t));
  if (st == DG_OK) st = up(reinterpret_cast<void**>(&m->d_op64), op64.data(), op64.size() * sizeof(double));
  if (st == DG_OK) st = up(reinterpret_cast<void**>(&m->d_opT), opT.data(), opT.size() * sizeof(double));
  if (st == DG_OK) st = up(reinterpret_cast<void**>(&m->d_op32), op32.data(), op32.size() * sizeof(float));
  if (st == DG_OK) st = up(reinterpret_cast<void**>(&m->d_opbf), opbf.data(), opbf.size() * sizeof(uint16_t));
  if (st == DG_OK) st = up(reinterpret_cast<void**>(&m->d_fmask), m->ref.Fmask.data(), m->ref.Fmask.size() * sizeof(int));
  if (st == DG_OK) st = up(reinterpret_cast<void**>(&m->d_nbtab), m->nbtab.data(), m->nbtab.size());
  hipSetDevice(prev);
  if (st != DG_OK) return cleanup(st);
  *out = reinterpret_cast<dg_mesh>(m);
  return DG_OK;
}

extern "C" dg_status dg_mesh_destroy(dg_mesh h) {
  if (!h) return DG_OK;
  Mesh* m = reinterpret_cast<Mesh*>(h);
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(m->device);
  hipFree(m->d_geo);
  hipFree(m->d_conn);
  hipFree(m->d_op64);
  hipFree(m->d_opT);
  hipFree(m->d_op32);
  hipFree(m->d_opbf);
  hipFree(m->d_fmask);
  hipFree(m->d_nbtab);
  hipSetDevice(prev);
  delete m;
  return DG_OK;
}

extern "C" dg_status dg_mesh_info(dg_mesh h, int64_t* n_elem, int* np, int* nfp) {
  if (!h) return fail(DG_ERR_ARG, "dg_mesh_info: null mesh");
  const Mesh* m = reinterpret_cast<const Mesh*>(h);
  if (n_elem) *n_elem = m->E;
  if (np) *np = m->Np;
  if (nfp) *nfp = m->Nfp;
  return DG_OK;
}

extern "C" dg_status dg_mesh_nodes(dg_mesh h, double* xyz) {
  if (!h || !xyz) return fail(DG_ERR_ARG, "dg_mesh_nodes: null argument");
  const Mesh* m = reinterpret_cast<const Mesh*>(h);
  for (int64_t e = 0; e < m->E; ++e) {
    const double* X = &m->elem_xyz[e * 12];
    for (int i = 0; i < m->Np; ++i) {
      const double r = m->ref.rst[i * 3], s = m->ref.rst[i * 3 + 1], t = m->ref.rst[i * 3 + 2];
      const double w[4] = {-0.5 * (1 + r + s + t), 0.5 * (1 + r), 0.5 * (1 + s), 0.5 * (1 + t)};
      for (int d = 0; d < 3; ++d)
        xyz[(e * m->Np + i) * 3 + d] = w[0] * X[d] + w[1] * X[3 + d] + w[2] * X[6 + d] + w[3] * X[9 + d];
    }
  }
  return DG_OK;
}

extern "C" dg_status dg_mesh_face_map(dg_mesh h, int64_t* nbr_elem, int32_t* nbr_node) {
  if (!h || !nbr_elem || !nbr_node) return fail(DG_ERR_ARG, "dg_mesh_face_map: null argument");
  const Mesh* m = reinterpret_cast<const Mesh*>(h);
  const int Nfp = m->Nfp;
  for (int64_t e = 0; e < m->E; ++e)
    for (int f = 0; f < 4; ++f) {
      const int32_t en = m->conn_host[(f * m->Epad + e) * 2 + 0];
      const int32_t code = m->conn_host[(f * m->Epad + e) * 2 + 1];
      for (int k = 0; k < Nfp; ++k) {
        nbr_elem[e * 4 * Nfp + f * Nfp + k] = en;
        nbr_node[e * 4 * Nfp + f * Nfp + k] = m->nbtab[(f * 24 + code) * Nfp + k];
      }
    }
  return DG_OK;
}
