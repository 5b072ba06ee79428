// Reference tetrahedron of the nodal DG basis (host side): node set, nodal
// differentiation matrices, lift matrix, face masks and lattice labels.
#pragma once
#include <cstdint>
#include <vector>

namespace dg {

constexpr int kMaxOrder = 4;

inline int nodes_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
inline int face_nodes_of(int p) { return (p + 1) * (p + 2) / 2; }

// local vertices of each face (f0: t=-1, f1: s=-1, f2: r+s+t=-1, f3: r=-1)
extern const int kFaceVerts[4][3];

struct RefElem {
  int p = 0, Np = 0, Nfp = 0;
  std::vector<double> rst;        // [Np][3]
  std::vector<double> Dr, Ds, Dt; // [Np][Np] row-major
  std::vector<double> LIFT;       // [Np][4*Nfp]
  std::vector<int> Fmask;         // [4][Nfp]
  std::vector<int> lattice;       // [Np][4] integer barycentric labels (sum p)
};

// Builds the reference element of order p (1..4).  Returns false for other p.
bool build_ref_elem(int p, RefElem& out);

}  // namespace dg
