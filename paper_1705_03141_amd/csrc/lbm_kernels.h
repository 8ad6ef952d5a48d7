// lbm_kernels.h -- launch-side view of the kernels (argument blocks and launchers).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_cell.h"
#include "lbm_device.h"

namespace lbm {

// Thread layout of the step kernel: one thread per cell of a TX x TY tile; the first
// 2(TX+2) + 2TY threads also pull one cell of the ring around the tile.
template <int TX, int TY>
struct StepTile {
  static constexpr int kThreads = TX * TY;
  static constexpr int kRing = 2 * (TX + 2) + 2 * TY;
  static constexpr int SX = TX + 4, SY = TY + 4, kStaged = SX * SY;  // scalars, 2-cell halo
  static constexpr int DX = TX + 2, DY = TY + 2, kDense = DX * DY;   // densities, 1-cell ring
  static constexpr int kStagePerThread = (kStaged + kThreads - 1) / kThreads;
  static_assert(kThreads % 64 == 0, "tile must be whole waves");
  static_assert(kRing <= kThreads, "ring larger than the tile");
};

struct StepArgs {
  const void* g_in;      // populations written by the previous step (storage type)
  const float* sc_in;    // scalars written by the previous step
  void* g_out;
  float* sc_out;
  const float* init;     // init mode: rho_r, rho_b, ux, uy, uz planes of ncells floats
  const float* outlet;   // outlet record of the current time (outflow face only)
  long long step;
  int init_mode;
  int zchunk, tiles_x, tiles_y, nchunks;
  int tile_set;          // a TileSet value
  int tx_lo, tx_hi, ty_lo, ty_hi;  // the interior rectangle of tiles [tx_lo, tx_hi) x [ty_lo, ty_hi)
  int* unstable;         // set to 1 by a cell whose density is NaN, infinite or <= 0
  int skip_unstable;     // 1: workgroups of a flagged lattice return at once (batches)
  Geo geo;
  PullConst pc;
  CollideParams cp;
  GroupRates rates;
};

// The tiles one launch of the step kernel covers.  With lateral walls the tiles whose cells
// and ring cells are all off the walls (the interior rectangle) take the plain pull.  The
// frame around it is split by the walls its tiles touch: left and right of the rectangle (in
// its rows) the tiles touch only x walls, -x on the left and +x on the right; below and above
// it (in its columns) only y walls; the corner blocks touch both axes.  The edges are one set
// per axis (kEdgeX, kEdgeY) or one per wall (kEdgeXLo ... kEdgeYHi); each set takes the
// instance that reflects at its walls only.
enum TileSet {
  kAllTiles = 0,
  kInteriorTiles = 1,
  kEdgeX = 2,
  kEdgeY = 3,
  kEdgeXLo = 4,
  kEdgeXHi = 5,
  kEdgeYLo = 6,
  kEdgeYHi = 7,
  kCorners = 8
};

// The tile sets a step of a lattice with lateral walls launches, by storage code (0 FP32, 1
// FP16, 2 BF16): with FP16 storage one set per wall along the edges, because its instances
// that reflect at both walls of an axis spill registers (measured on the jet between walls:
// 4.82 against 5.99 ms per step); with the others one per axis, where the extra launches of
// the per-wall split cost more than it saves.  Returns the count written to sets.
inline int wall_tile_sets(int storage, int* sets) {
  int n = 0;
  sets[n++] = kInteriorTiles;
  if (storage == 1) {
    sets[n++] = kEdgeXLo;
    sets[n++] = kEdgeXHi;
    sets[n++] = kEdgeYLo;
    sets[n++] = kEdgeYHi;
  } else {
    sets[n++] = kEdgeX;
    sets[n++] = kEdgeY;
  }
  sets[n++] = kCorners;
  return n;
}

// Reflection mode of the step kernel instance for a tile set: the walls it reflects at, in
// the bits of wall_flags (1: -x, 2: +x, 4: -y, 8: +y).
__host__ __device__ inline int lat_mode_of(int tile_set, bool walls) {
  if (!walls || tile_set == kInteriorTiles) return 0;
  switch (tile_set) {
    case kEdgeX: return 3;
    case kEdgeY: return 12;
    case kEdgeXLo: return 1;
    case kEdgeXHi: return 2;
    case kEdgeYLo: return 4;
    case kEdgeYHi: return 8;
    default: return 15;
  }
}

__host__ __device__ inline int tiles_in_set(const StepArgs& a) {
  const int w_in = a.tx_hi - a.tx_lo, h_in = a.ty_hi - a.ty_lo;
  const int x_hi = a.tiles_x - a.tx_hi, y_hi = a.tiles_y - a.ty_hi;
  switch (a.tile_set) {
    case kInteriorTiles: return w_in * h_in;
    case kEdgeX: return (a.tx_lo + x_hi) * h_in;
    case kEdgeY: return w_in * (a.ty_lo + y_hi);
    case kEdgeXLo: return a.tx_lo * h_in;
    case kEdgeXHi: return x_hi * h_in;
    case kEdgeYLo: return w_in * a.ty_lo;
    case kEdgeYHi: return w_in * y_hi;
    case kCorners: return (a.tx_lo + x_hi) * (a.ty_lo + y_hi);
    default: return a.tiles_x * a.tiles_y;
  }
}

// Tile (txi, tyi) of the t-th tile of the launch's set (row by row within the set).
__host__ __device__ inline void tile_of(const StepArgs& a, int t, int& txi, int& tyi) {
  const int w_in = a.tx_hi - a.tx_lo, x_hi = a.tiles_x - a.tx_hi, side = a.tx_lo + x_hi;
  // the k-th column left or right of the rectangle, and the r-th row below or above it
  auto side_col = [&](int k) { return k < a.tx_lo ? k : a.tx_hi + (k - a.tx_lo); };
  auto out_row = [&](int r) { return r < a.ty_lo ? r : a.ty_hi + (r - a.ty_lo); };
  switch (a.tile_set) {
    case kInteriorTiles:
      tyi = a.ty_lo + t / w_in;
      txi = a.tx_lo + t % w_in;
      return;
    case kEdgeX:
      tyi = a.ty_lo + t / side;
      txi = side_col(t % side);
      return;
    case kEdgeY:
      tyi = out_row(t / w_in);
      txi = a.tx_lo + t % w_in;
      return;
    case kEdgeXLo:
      tyi = a.ty_lo + t / a.tx_lo;
      txi = t % a.tx_lo;
      return;
    case kEdgeXHi:
      tyi = a.ty_lo + t / x_hi;
      txi = a.tx_hi + t % x_hi;
      return;
    case kEdgeYLo:
      tyi = t / w_in;
      txi = a.tx_lo + t % w_in;
      return;
    case kEdgeYHi:
      tyi = a.ty_hi + t / w_in;
      txi = a.tx_lo + t % w_in;
      return;
    case kCorners:
      tyi = out_row(t / side);
      txi = side_col(t % side);
      return;
    default:
      tyi = t / a.tiles_x;
      txi = t - tyi * a.tiles_x;
  }
}

// Arguments of the outlet and read-back kernels.
struct AuxArgs {
  const void* g_in;
  const float* sc_in;
  const float* init;
  const float* outlet_in;  // outlet record of the previous time
  float* outlet_out;       // outlet record of the current time
  long long step;
  int init_mode;
  Geo geo;
  PullConst pc;
  CollideParams cp;
};

struct DiagQuery {
  double xc, yc, zc, r_in, r_out;
};

// Typed launchers, instantiated once per storage type (lbm_storage_*.hip).
template <typename T>
hipError_t launch_step_T(const StepArgs& a, int tx, int ty, hipStream_t s);
template <typename T>
hipError_t launch_inflow_T(const StepArgs& a, hipStream_t s);
template <typename T>
hipError_t launch_batch_T(const StepArgs* cases, const int* first, int ncases, int nblocks, bool init, int tx, int ty,
                          int lat, hipStream_t s);
template <typename T>
int step_resident_blocks_T(int tx, int ty, int device);
template <typename T>
hipError_t launch_outlet_T(const AuxArgs& a, hipStream_t s);
template <typename T>
hipError_t launch_batch_outlet_T(const AuxArgs* cases, const int* first, int ncases, int nblocks, long long step,
                                 hipStream_t s);
template <typename T>
hipError_t launch_batch_inflow_T(const StepArgs* cases, const int* first, int ncases, int nblocks, long long step,
                                 hipStream_t s);
template <typename T>
hipError_t launch_fields_T(const AuxArgs& a, int x0, int y0, int z0, int wx, int wy, int wz, double* out, hipStream_t s);
template <typename T>
hipError_t launch_populations_T(const AuxArgs& a, double* out, hipStream_t s);
template <typename T>
hipError_t launch_coarse_T(const AuxArgs& a, int f, float inv_u, float* out, int ph, int pw, hipStream_t s);
template <typename T>
hipError_t launch_diag_T(const AuxArgs& a, const DiagQuery& q, double* part, long long nblocks, double* out,
                         hipStream_t s);

// Dispatch on the storage code of lbm_params (0 FP32, 1 FP16, 2 BF16).
bool step_tiling_supported(int tx, int ty);
hipError_t launch_step(int storage, const StepArgs& a, int tx, int ty, hipStream_t s);
// One step of several lattices in one launch: cases (device array of ncases argument blocks,
// all with the same storage, tile shape and lateral rule: lat = free-slip x or y walls),
// first (device, ncases + 1 block offsets, each a multiple of 8), nblocks = first[ncases].
hipError_t launch_batch(int storage, const StepArgs* cases, const int* first, int ncases, int nblocks, bool init,
                        int tx, int ty, int lat, hipStream_t s);
// Inflow sites of plane z = 0 written into the step's output state (after launch_step).
hipError_t launch_inflow(int storage, const StepArgs& a, hipStream_t s);
// Workgroups of the step kernel that fit on the device at once (0 if unknown).
int step_resident_blocks(int storage, int tx, int ty, int device);
hipError_t launch_outlet(int storage, const AuxArgs& a, hipStream_t s);
// The outlet records, and the inflow planes, of several lattices of one storage type at one
// step in one launch: cases (device array of ncases argument blocks of the step's parity),
// first (device, ncases + 1 block offsets of 256-thread blocks over each plane),
// nblocks = first[ncases].
hipError_t launch_batch_outlet(int storage, const AuxArgs* cases, const int* first, int ncases, int nblocks,
                               long long step, hipStream_t s);
hipError_t launch_batch_inflow(int storage, const StepArgs* cases, const int* first, int ncases, int nblocks,
                               long long step, hipStream_t s);
hipError_t launch_fields(int storage, const AuxArgs& a, int x0, int y0, int z0, int wx, int wy, int wz, double* out,
                         hipStream_t s);
hipError_t launch_populations(int storage, const AuxArgs& a, double* out, hipStream_t s);
hipError_t launch_coarse(int storage, const AuxArgs& a, int f, float inv_u, float* out, int ph, int pw, hipStream_t s);
hipError_t launch_diag(int storage, const AuxArgs& a, const DiagQuery& q, double* part, long long nblocks,
                       double* out, hipStream_t s);

}  // namespace lbm
