// Device-side descriptors of a batch of meshes and the launchers of the
// batched stage and copy kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dg.h"

namespace dg {

// One mesh of a batch: its bound state buffers and geometry.
struct BatchMesh {
  double* q;          // [5][E][Np] state (stage input on even stages)
  double* tmp;        // [5][E][Np] second state buffer
  double* res;        // [5][E][Np] Runge-Kutta residual
  const double* geo;  // [9][Epad] metric terms
  const int2* conn;   // [4][Epad] neighbour element, 6 nbr_face + perm
  int64_t E, Epad;
  int p, pad;
};

// One work item: a 16-element tile of a mesh.
struct BatchItem {
  int mesh;
  int tile;
};

// Face tables of every order present in the batch, staged in LDS by each
// block of the mixed-order kernel (nb bytes at nb_off[p], fm ints at
// fm_off[p]); the operator tables op[p] are read from memory.  The
// per-order kernels stage their own order's tables and one state tile per
// wave in static LDS.
struct BatchTables {
  const uint32_t* op[5];
  const uint8_t* nb[5];
  const int* fm[5];
  int nb_bytes[5], fm_n[5];
  int nb_off[5], fm_off[5];  // byte offsets into LDS
  int lds_bytes;
};

struct BatchLaunch {
  const BatchMesh* meshes;
  const BatchItem* items;
  int64_t n_items;
  // items [p_begin[p], p_end[p]) of the list have order p (the list of the
  // per-order launches is grouped by order)
  int64_t p_begin[5], p_end[5];
  const double* dt;  // [n meshes]
  double gamma;
  unsigned* flags;   // device failure flags (non-finite state)
  BatchTables tabs;
  int waves_per_block, blocks, xcd_chunks;
};

// Stage s of the LSRK scheme over every item (one persistent launch of the
// mixed-order kernel): reads q (odd == 0) or tmp (odd == 1), writes the
// other, res <- a res + dt rhs.
dg_status launch_batch_stage(dg_precision prec, const BatchLaunch& L, double a, double b, int odd, hipStream_t s);
// The same stage over the items of order p only, with the kernel specialised
// for that order (one wave per item).
dg_status launch_batch_order_stage(dg_precision prec, const BatchLaunch& L, int p, double a, double b, int odd,
                                   hipStream_t s);
// q <- tmp for the elements of items [begin, end).
dg_status launch_batch_copy(const BatchLaunch& L, int64_t begin, int64_t end, hipStream_t s);
// Largest resident blocks per CU of the stage kernel for a launch shape.
int batch_stage_occupancy(dg_precision prec, int waves_per_block, int lds_bytes);
// Allows the stage kernels their dynamic LDS size (once per device and size).
dg_status batch_prepare(dg_precision prec, int waves_per_block, int lds_bytes);

}  // namespace dg
