// kernels.h -- launch interface between the C ABI runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "rlbm_defs.h"

namespace rlbm {

enum Op : int { OP_STEP = 0, OP_MOMENTS = 1, OP_INIT = 2 };

// Device pointers of the macroscopic output fields (NULL = skip).
struct FieldPtrs {
  double *n, *eps, *T, *U;
  int any;
};

// Launch variants of the step kernel: block shape bx x by x bz (2D lattices
// fold bz into by), occupancy target (minimum waves per SIMD the compiler must
// allow, 0 = its choice) and tile order (0 = as dealt, 1 = a contiguous band of
// tiles per XCD, 2 = (y, z) patches per XCD in 3D, a band in 2D).  lds: the 2D
// product rules stage their upstream windows in LDS (64 x 4 band tiles); lattices
// the staged kernel does not cover take the register kernel of the same shape.
struct Variant {
  int bx, by, bz, occ, xcd, lds;
};
constexpr int kNumVariants = 13;
constexpr Variant kVariants[kNumVariants] = {
    {64, 4, 1, 0, 0, 0}, {64, 4, 1, 0, 1, 0}, {64, 4, 1, 2, 0, 0}, {64, 4, 1, 2, 2, 0}, {64, 2, 1, 0, 1, 0},
    {64, 1, 1, 0, 1, 0}, {128, 2, 1, 0, 1, 0}, {256, 1, 1, 0, 1, 0}, {64, 1, 1, 2, 2, 0}, {64, 2, 2, 2, 2, 0},
    {64, 4, 1, 4, 1, 0}, {64, 4, 1, 0, 2, 0}, {64, 4, 1, 0, 1, 1}};

struct LaunchArgs {
  int op = 0;
  int variant = 1;
  int stencil = 0, order = 0, storage = 0;
  int nx = 0, ny = 0, nz = 1;
  const Tables *tb = nullptr;      // device pointer
  const void *fin = nullptr;
  void *fout = nullptr;
  const void *tau_field = nullptr;
  FieldPtrs fields = {nullptr, nullptr, nullptr, nullptr, 0};
  const double *n0 = nullptr, *T0 = nullptr, *u0 = nullptr, *noise = nullptr;
  double amp = 0.0;
  int *err = nullptr;               // device error flag
  int ext = 0;                      // the lattice has an external force or no-slip walls
  int nt = 0;                       // step kernels store the populations non-temporally
  int lds_ok = 0;                   // the LDS-staged 2D product kernel covers this lattice
  hipStream_t stream = 0;
};

hipError_t launch(const LaunchArgs &a);

enum AdjOp : int { ADJ_STEP = 0, ADJ_MOMENTS = 1, ADJ_INIT = 2 };

struct AdjointArgs {
  int op = 0;
  int stencil = 0, order = 0, storage = 0;
  int nx = 0, ny = 0, nz = 1;
  const Tables *tb = nullptr;
  const void *state = nullptr;      // B_{t-1} (step) or B_T (moments)
  const void *lam_in = nullptr;     // lam_{t+1} (step) or lam_1 (init)
  void *lam_out = nullptr;
  const void *tau_field = nullptr;
  double *dtau = nullptr;
  FieldPtrs grads = {nullptr, nullptr, nullptr, nullptr, 0};
  const double *n0 = nullptr, *T0 = nullptr, *u0 = nullptr, *noise = nullptr;
  double amp = 0.0;
  double *du0 = nullptr, *dn0 = nullptr, *dT0 = nullptr;
  int *err = nullptr;
  hipStream_t stream = 0;
};

// reverse-mode kernels (2D product rules, periodic boundaries)
hipError_t launch_adjoint(const AdjointArgs &a);

// Batched step: tile shapes (0: 64 x 4, 1: 64 x 2, 2: 128 x 2 sites; 3: 256 consecutive sites of
// a lattice, its rows joined end to end, so that no lane idles past a row's end) and grid sizes
constexpr int kBatchTiles[4][2] = {{64, 4}, {64, 2}, {128, 2}, {256, 1}};
constexpr int kBatchLinearTile = 3;
struct BatchArgs {
  int stencil = 0, order = 0, storage = 0;
  int tile = 0;                  // index into kBatchTiles
  int blocks = 0;                // persistent grid size (multiple of 8)
  const Tables *tabs = nullptr;  // [nlat] device
  const int64_t *elem_off = nullptr;
  const int2 *tiles = nullptr;   // [ntiles] (lattice, tile index)
  int ntiles = 0;
  const void *fin = nullptr;
  void *fout = nullptr;
  int *err = nullptr;
  hipStream_t stream = 0;
  int ext = 0;                   // some member has an external force or no-slip walls
  int nt = 0;                    // non-temporal population stores
};
hipError_t launch_batch(const BatchArgs &a);

}  // namespace rlbm
