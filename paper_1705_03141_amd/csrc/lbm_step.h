// lbm_step.h -- the fused step kernel: streaming (as a pull), colour densities, isotropic
// gradient, MRT collision with enhanced equilibrium, forcing and perturbation, and the
// recolouring scalars, one pass over HBM per time step (Sec. II).
//
// Work decomposition.  A workgroup of TX*TY threads owns a TX x TY column of cells and marches
// through a chunk of z planes; every thread owns one cell of the column.  The colour gradient
// of a cell needs the densities of time t of its 26 neighbours, so the 2(TX+2)+2TY cells of
// the ring around the column are pulled as well (densities only), each by one of the first
// threads.  Per plane counter p the workgroup
//   1. issues the loads of the scalars (e, psi, w) of source plane p+3 with a 2-cell halo and
//      the 27 population loads of the cells of plane p+1 (and of its ring cells),
//   2. completes the pull of plane p+1, consuming the population loads in the order they
//      were issued, and writes rho_r/rho, rho_b/rho and rho of its cells and ring into an
//      LDS ring of 4 planes (the pull reads the staged scalars of planes p..p+2, stored in
//      earlier passes),
//   3. writes the scalars of plane p+3, decoded into (e, a, b, w), into an LDS ring of 4
//      planes; barrier (the only one per plane),
//   4. collides plane p with the gradient taken from the density ring, and stores 27
//      deviations + 5 scalars per cell.
// The deviations of plane p+1 stay in registers until step 4 of the next plane.  Steps 1-3
// run at a raised wave priority (s_setprio), step 4 at the normal one.
//
// Blocks are numbered so that the blocks the hardware sends to one XCD (block ids congruent
// modulo 8) cover consecutive tiles and z chunks: neighbouring tiles then share one L2 and
// halo rows are fetched from HBM once.
#pragma once

#include <type_traits>

#include "lbm_kernels_impl.h"

namespace lbm {

// ---------------------------------------------------------------- buffer access
// The population and scalar planes are read and written with raw buffer instructions: the
// plane's base is a workgroup-uniform descriptor, the population index j enters as the scalar
// offset j * plane * sizeof(T), and only the cell's column offset is a per-lane register.
// This keeps per-lane 64-bit address arithmetic (and its registers) out of the plane loop.
using rsrc_t = __amdgpu_buffer_rsrc_t;

// Raw buffer descriptor over [base, base + bytes); the last word is the GFX9 default format.
__device__ __forceinline__ rsrc_t buffer_of(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
struct Word;
template <>
struct Word<float> {
  using W = unsigned;
  static __device__ __forceinline__ W load(rsrc_t r, unsigned vo, int so) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, so, 0);
  }
  static __device__ __forceinline__ void store(W v, rsrc_t r, unsigned vo, int so) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)vo, so, 0);
  }
  static __device__ __forceinline__ float dec(W v) { return __uint_as_float(v); }
  static __device__ __forceinline__ W enc(float f) { return __float_as_uint(f); }
  static constexpr float kPullScale = 1.0f;
  static __device__ __forceinline__ float dec_scaled(W v) { return dec(v); }
  static constexpr int kOutShift = 0;
  static __device__ __forceinline__ W enc_scaled(float f) { return enc(f); }
};
template <>
struct Word<_Float16> {
  using W = unsigned short;
  static __device__ __forceinline__ W load(rsrc_t r, unsigned vo, int so) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, so, 0);
  }
  static __device__ __forceinline__ void store(W v, rsrc_t r, unsigned vo, int so) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)vo, so, 0);
  }
  static __device__ __forceinline__ float dec(W v) { return Codec<_Float16>::dec(__builtin_bit_cast(_Float16, v)); }
  static __device__ __forceinline__ W enc(float f) { return __builtin_bit_cast(W, Codec<_Float16>::enc(f)); }
  // The pull works on deviations times the storage scale: the stored half then enters an FMA
  // as it is (converted inside the instruction).  Every scaled product and sum is the
  // unscaled one times a power of two wherever the unscaled one is a normal number; only
  // products below about 1e-38 (of a vanishing minority fraction) round differently.
  static constexpr float kPullScale = Codec<_Float16>::kScale;
  static __device__ __forceinline__ float dec_scaled(W v) { return (float)__builtin_bit_cast(_Float16, v); }
  static constexpr int kOutShift = 10;  // log2 of the storage scale
  static __device__ __forceinline__ W enc_scaled(float f) { return __builtin_bit_cast(W, (_Float16)f); }
};
template <>
struct Word<bf16> {
  using W = unsigned short;
  static __device__ __forceinline__ W load(rsrc_t r, unsigned vo, int so) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, so, 0);
  }
  static __device__ __forceinline__ void store(W v, rsrc_t r, unsigned vo, int so) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)vo, so, 0);
  }
  static __device__ __forceinline__ float dec(W v) { return Codec<bf16>::dec(bf16{v}); }
  static __device__ __forceinline__ W enc(float f) { return Codec<bf16>::enc(f).bits; }
  static constexpr float kPullScale = 1.0f;
  static __device__ __forceinline__ float dec_scaled(W v) { return dec(v); }
  static constexpr int kOutShift = 0;
  static __device__ __forceinline__ W enc_scaled(float f) { return enc(f); }
};

__device__ __forceinline__ float load_f32(rsrc_t r, unsigned vo, int so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, so, 0));
}
__device__ __forceinline__ void store_f32(float v, rsrc_t r, unsigned vo, int so) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, so, 0);
}

// Offsets, in bytes, of the 3 x 3 neighbourhood of column (x, y) within one population plane.
template <typename T>
__device__ __forceinline__ void column_offsets(const Geo& G, int x, int y, unsigned (&o)[3][3]) {
  const int xs[3] = {x == 0 ? G.nx - 1 : x - 1, x, x == G.nx - 1 ? 0 : x + 1};
  const int ys[3] = {y == 0 ? G.ny - 1 : y - 1, y, y == G.ny - 1 ? 0 : y + 1};
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) o[b][a] = (unsigned)((ys[b] * G.nx + xs[a]) * (int)sizeof(T));
}

// Bit of wall_flags for the wall a source offset D along AXIS (0: x, 1: y) crosses.
template <int AXIS, int D>
constexpr int wall_bit() {
  return (AXIS == 0 ? 0 : 2) + (D < 0 ? 0 : 1);
}

// Lateral reflection of a source offset at a cell with wall flags wf (wall_flags): true where
// the source (dx, dy) lies beyond a free-slip wall in x (AXIS 0) or y (AXIS 1).  LAT is the
// instance's reflection mode, the walls it reflects at in the bits of wall_flags; a wall it
// leaves out never reflects.
template <int AXIS, int D, int LAT>
__device__ __forceinline__ bool reflects(int wf) {
  if constexpr (D == 0 || ((LAT >> wall_bit<AXIS, D>()) & 1) == 0) return false;
  else return (wf >> wall_bit<AXIS, D>()) & 1;
}

// Whether a pull direction with source offset (DX, DY) can reflect at a lateral wall in
// reflection mode LAT.
template <int LAT, int DX, int DY>
constexpr bool lat_dir() {
  return (DX != 0 && ((LAT >> wall_bit<0, DX>()) & 1)) || (DY != 0 && ((LAT >> wall_bit<1, DY>()) & 1));
}

// Issue the 27 population loads of a pull in mode MODE.  slab[k] covers the 27 population
// planes of source plane z - 1 + k; the raw word of direction i is left in ld[i].  With
// lateral walls (LAT != 0) a source beyond a wall is the boundary cell and the mirrored
// population (reading R9), chosen per lane: its population plane then enters the per-lane
// offset.
template <typename T, int MODE, int LAT>
__device__ __forceinline__ void issue_pull(const rsrc_t (&slab)[3], int plane_bytes, const unsigned (&o)[3][3], int wf,
                                           typename Word<T>::W (&ld)[Q]) {
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr Src s = resolve<i, MODE>();
    if constexpr (!lat_dir<LAT, s.dx, s.dy>()) {
      ld[i] = Word<T>::load(slab[s.dz + 1], o[s.dy + 1][s.dx + 1], s.j * plane_bytes);
    } else {
      const bool rx = reflects<0, s.dx, LAT>(wf), ry = reflects<1, s.dy, LAT>(wf);
      constexpr int jx = mirror_x(s.j), jy = mirror_y(s.j), jxy = mirror_x(mirror_y(s.j));
      const unsigned col = rx ? (ry ? o[1][1] : o[s.dy + 1][1]) : (ry ? o[1][s.dx + 1] : o[s.dy + 1][s.dx + 1]);
      const int j = rx ? (ry ? jxy : jx) : (ry ? jy : s.j);
      ld[i] = Word<T>::load(slab[s.dz + 1], col + (unsigned)(j * plane_bytes), 0);
    }
  });
}

// Single operations the compiler may not fuse with their neighbours into an FMA.
__device__ __forceinline__ float add_nc(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}
__device__ __forceinline__ float sub_nc(float a, float b) {
#pragma clang fp contract(off)
  return a - b;
}
__device__ __forceinline__ float mul_nc(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ float div_nc(float a, float b) {
#pragma clang fp contract(off)
  return a / b;
}

template <typename T, int MODE, bool WANT_DF, int SX, int LAT>
__device__ __forceinline__ void finish_pull(const typename Word<T>::W (&ld)[Q], const float4* const (&S)[3], const float2* const (&W)[3],
                                            int idx0, int wf, const PullConst& C, float& rho, float& rho_r, float& rho_b,
                                            float& e_new, float (&df)[Q], float& shift_out, float& drho_out) {
  const float4 me = S[1][idx0 + SX + 1];
  const float e_self = me.x, a_self = me.y, b_self = me.z;
  const bool track_red = a_self <= b_self;  // the reader's minority colour
  const float t_self = track_red ? a_self : b_self;
  const float rho_old = rho_of(C, e_self, a_self, b_self);
  const float E_self = add_nc(C.E0, e_self);
  const float sgn = track_red ? 1.0f : -1.0f;  // recolouring adds to red, removes from blue
  // the sums run on deviations times SC (the storage scale of FP16 storage, else 1); SC is a
  // power of two, so the scaled products and sums are exact scalings of the unscaled ones
  constexpr float SC = Word<T>::kPullScale;
  const float qE[4] = {0.0f, mul_nc(q_of(1) * SC, E_self), mul_nc(q_of(7) * SC, E_self), mul_nc(q_of(19) * SC, E_self)};
  const float sq[4] = {0.0f, sgn * (qc_of(1) * SC), sgn * (qc_of(7) * SC), sgn * (qc_of(19) * SC)};
  // Every operation below is spelled out (fmaf or an *_nc operation) so that the compiler
  // cannot contract it differently in the cell and ring instances of this function: a cell's
  // densities are then bitwise the same whichever workgroup pulls it, and results do not
  // depend on the tiling.
  float d_rho = Word<T>::dec_scaled(ld[0]);
  float d_t = mul_nc(t_self, d_rho);
  if constexpr (WANT_DF) df[0] = d_rho;
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr Src s = resolve<i, MODE>();
    constexpr int off = (s.dy + 1) * SX + s.dx + 1;
    constexpr int sh = shell_of(i);
    constexpr bool self_src = s.dx == 0 && s.dy == 0 && s.dz == 0;  // bounce-back
    constexpr bool lat = lat_dir<LAT, s.dx, s.dy>();
    // lateral wall: the source is the boundary cell along a reflected axis, and the velocity
    // component normal to that wall is reversed
    bool rx = false, ry = false;
    int offl = off;
    if constexpr (lat) {
      rx = reflects<0, s.dx, LAT>(wf);
      ry = reflects<1, s.dy, LAT>(wf);
      offl = ((ry ? 0 : s.dy) + 1) * SX + (rx ? 0 : s.dx) + 1;
    }
    const float4 src = S[s.dz + 1][idx0 + offl];
    const float2 w = W[s.dz + 1][idx0 + offl];
    // c_j . w of the source from its non-zero components (a sum started at 0.0f would cost
    // one more add: 0 + x is not folded because of the sign of zero)
    const bool px = (s.ccx > 0) != rx, py = (s.ccy > 0) != ry;
    const float wy = py ? w.x : -w.x, wz = s.ccz > 0 ? w.y : -w.y;
    float cw = s.ccx != 0 ? (px ? src.w : -src.w) : (s.ccy != 0 ? wy : wz);
    if constexpr (s.ccx != 0 && s.ccy != 0) cw = add_nc(cw, wy);
    if constexpr ((s.ccx != 0 || s.ccy != 0) && s.ccz != 0) cw = add_nc(cw, wz);
    float d, inc;
    if constexpr (self_src) {
      d = Word<T>::dec_scaled(ld[i]);
      inc = fmaf(sq[sh], cw, mul_nc(t_self, d));
    } else {
      d = fmaf(q_of(i) * SC, sub_nc(src.x, e_self), Word<T>::dec_scaled(ld[i]));
      const float t = track_red ? src.y : src.z;
      inc = fmaf(sq[sh], cw, fmaf(qE[sh], sub_nc(t, t_self), mul_nc(t, d)));
    }
    d_rho = add_nc(d_rho, d);
    d_t = add_nc(d_t, inc);
    if constexpr (WANT_DF) df[i] = d;
  });
  if constexpr (SC != 1.0f) {
    d_rho = mul_nc(d_rho, 1.0f / SC);
    d_t = mul_nc(d_t, 1.0f / SC);
    if constexpr (WANT_DF)
#pragma unroll
      for (int i = 0; i < Q; ++i) df[i] = mul_nc(df[i], 1.0f / SC);
  }
  rho = add_nc(rho_old, d_rho);
  const float rho_t = fmaf(t_self, rho_old, d_t), rho_o = sub_nc(rho, rho_t);
  rho_r = track_red ? rho_t : rho_o;
  rho_b = track_red ? rho_o : rho_t;
  const float d_rhor = track_red ? d_t : sub_nc(d_rho, d_t);
  const float shift = fmaf(C.dalpha, d_rhor, -mul_nc(1.0f - C.alpha_b, d_rho));  // E(t-1) - E(t)
  e_new = sub_nc(e_self, shift);
  shift_out = shift;
  drho_out = d_rho;
}

// Call f(std::integral_constant<int, MODE>) for the (workgroup-uniform) pull mode.
template <typename F>
__device__ __forceinline__ void with_mode(int mode, F&& f) {
  switch (mode) {
    case kLoBB: f(std::integral_constant<int, kLoBB>{}); break;
    case kLoFS: f(std::integral_constant<int, kLoFS>{}); break;
    case kHiBB: f(std::integral_constant<int, kHiBB>{}); break;
    case kHiFS: f(std::integral_constant<int, kHiFS>{}); break;
    default: f(std::integral_constant<int, kBulk>{}); break;
  }
}

// Position of ring cell r (0 <= r < 2(TX+2)+2TY) relative to the column origin.
template <int TX, int TY>
__device__ __forceinline__ void ring_cell(int r, int& x, int& y) {
  if (r < TX + 2) {
    x = r - 1;
    y = -1;
  } else if (r < 2 * (TX + 2)) {
    x = r - (TX + 2) - 1;
    y = TY;
  } else if (r < 2 * (TX + 2) + TY) {
    x = -1;
    y = r - 2 * (TX + 2);
  } else {
    x = TX;
    y = r - 2 * (TX + 2) - TY;
  }
}

// Pre-collision state of one plane's cell, carried from its pull to its collision.
struct PlaneState {
  float df[Q];
  float rho, rho_r, rho_b, e, shift, drho;
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < Q; ++i) df[i] = 0.0f;
    rho = 1.0f;
    rho_r = 0.0f;
    rho_b = 1.0f;
    e = shift = drho = 0.0f;
  }
};

template <typename T, int TX, int TY, bool INIT, int LAT>
#ifndef LBM_STEP_WAVES_PER_EU
#define LBM_STEP_WAVES_PER_EU 2
#endif
__device__ __forceinline__ void step_body(const StepArgs& A, int L, const int nb) {
  using Tile = StepTile<TX, TY>;
  constexpr int NT = Tile::kThreads, NR = Tile::kRing, SX = Tile::SX, NS = Tile::kStaged, DX = Tile::DX,
                ND = Tile::kDense, KS = Tile::kStagePerThread;
  // Four slots each, so that one barrier per plane suffices: the scalars of plane p+3 are
  // staged while planes p..p+2 are read (their slot held p-1, last read before the previous
  // barrier), and the densities of plane p+1 are written while planes p-1..p+1 are read by
  // the collision (their slot held p-3, last read two barriers earlier).
  __shared__ float4 sS[4][NS];  // staged scalars (e, a, b, w_x) of source planes
  __shared__ float2 sW[4][NS];  // (w_y, w_z)
  // Density ring of time t with a 1-cell ring, 4 slots: per cell the pairs (rho_r/rho, rho)
  // (sel 0) and (rho_b/rho, rho) (sel 1), so that a reader takes its minority colour's fraction
  // and rho with one 8-byte read.  The two pairs lie in separate arrays of 4 slots each, where
  // a wave's reads of neighbouring cells fall on distinct banks; with FP16 storage they are
  // interleaved per cell, because the separate form makes that instance spill (measured on
  // the jet: +1.3 % FP32, +7.6 % with lateral walls, -6 % FP16 for the separate form).
  constexpr bool kSplitRing = !std::is_same<T, _Float16>::value;
  __shared__ float2 sDf[8 * ND];
  // index of pair sel of cell d in slot s
  auto dat = [](int s, int sel, int d) { return kSplitRing ? (sel * 4 + s) * ND + d : s * 2 * ND + 2 * d + sel; };
  auto slot4 = [](int q) { return q & 3; };
  // Issue order of a pass's loads (measured): with FP32 populations the staged scalars go
  // first, with 16-bit populations after the population loads.  Their LDS write waits until
  // the pull is complete, so that the pull consumes each population load as soon as it and
  // the older loads have arrived, rather than after all of them.  The instances that spill
  // (the corner instance, and with FP16 storage every reflecting one) keep the scalars first
  // and their LDS write before the pull, so that the staged values are not live across it
  // (FP16 jet between walls: 4.47 against 4.81 ms per step).
  constexpr bool kHalfWall = std::is_same<T, _Float16>::value && LAT != 0;
  constexpr bool kStoreLate = LAT != 15 && !kHalfWall;
  constexpr bool kStageFirst = LAT == 15 || sizeof(T) == 4 || kHalfWall;

  const Geo& G = A.geo;
  const bool zper = G.face_lo == FACE_PERIODIC;
  const bool outflow = G.face_hi == FACE_OUTFLOW;
  const int plane = G.plane;
  const char* gin = static_cast<const char*>(A.g_in);
  char* gout = static_cast<char*>(A.g_out);
  const int pb = plane * (int)sizeof(T);                    // bytes of one population plane
  const unsigned slab_bytes = (unsigned)(Q * pb);           // 27 population planes of one z
  const unsigned sc_bytes = (unsigned)(5 * plane * 4);      // 5 scalar planes of one z

  // block L of nb -> (z chunk, tile); XCD x receives blocks x, x + 8, ...: give it a
  // contiguous range (nb and the first block of the range are multiples of 8 when remapped)
  if ((nb & 7) == 0) L = (L & 7) * (nb >> 3) + (L >> 3);
  const int ntiles = tiles_in_set(A);
  const int chunk = L / ntiles, tile = L - chunk * ntiles;
  if (chunk >= A.nchunks) return;  // padding block of a batch (the whole block leaves)
  // a lattice of a batch that went unstable is not stepped further (the flag is read once per
  // workgroup, before any barrier; the whole workgroup leaves)
  if (A.skip_unstable && __hip_atomic_load(A.unstable, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  int txi, tyi;
  tile_of(A, tile, txi, tyi);
  const int x0 = txi * TX, y0 = tyi * TY;
  const int z0 = chunk * A.zchunk, z1 = min(z0 + A.zchunk, G.nz);

  // own cell
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const int gx = wrap(x0 + lx, G.nx), gy = wrap(y0 + ly, G.ny);
  const bool live = (x0 + lx < G.nx) && (y0 + ly < G.ny);
  const int col = gy * G.nx + gx;
  const int sI = (ly + 2) * SX + lx + 2, dI = (ly + 1) * DX + lx + 1;
  // ring cell
  const bool ringer = tid < NR;
  int rx = 0, ry = 0;
  if (ringer) ring_cell<TX, TY>(tid, rx, ry);
  const int rgx = wrap(x0 + rx, G.nx), rgy = wrap(y0 + ry, G.ny);
  const int rcol = rgy * G.nx + rgx;
  const int sR = (ry + 2) * SX + rx + 2, dR = (ry + 1) * DX + rx + 1;
  // lateral wall flags of the own and the ring cell (0 without lateral walls)
  // (only the walls of the instance's mode: the tiles it serves touch no others)
  constexpr int kWallMask = LAT;
  const int wfI = LAT ? wall_flags(G, gx, gy) & kWallMask : 0, wfR = LAT ? wall_flags(G, rgx, rgy) & kWallMask : 0;
  // staged cells
  unsigned stOff[KS];  // byte offsets in a scalar plane
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int idx = min(tid + k * NT, NS - 1);
    const int sx = idx % SX, sy = idx / SX;
    stOff[k] = (unsigned)((wrap(y0 + sy - 2, G.ny) * G.nx + wrap(x0 + sx - 2, G.nx)) * 4);
  }
  const unsigned colT = (unsigned)(col * (int)sizeof(T)), col4 = (unsigned)(col * 4);

  auto zsrc = [&](int q) { return zper ? wrap(q, G.nz) : min(max(q, 0), G.nz - 1); };
  auto needs_pull = [&](int q) { return zper || (q >= 0 && q < G.nz); };

  float st[KS][5];
  auto stage_load = [&](int q) {
    const rsrc_t r = buffer_of(A.sc_in + (size_t)zsrc(q) * 5 * (size_t)plane, sc_bytes);
#pragma unroll
    for (int k = 0; k < KS; ++k)
      if (k < KS - 1 || tid + k * NT < NS)
#pragma unroll
        for (int c = 0; c < 5; ++c) st[k][c] = load_f32(r, stOff[k], c * plane * 4);
  };
  auto stage_store = [&](int q) {
    const int s = slot4(q);
#pragma unroll
    for (int k = 0; k < KS; ++k)
      if (k < KS - 1 || tid + k * NT < NS) {
        const float psi = st[k][1];
        sS[s][tid + k * NT] = make_float4(st[k][0], psi_a(psi), psi_b(psi), st[k][2]);
        sW[s][tid + k * NT] = make_float2(st[k][3], st[k][4]);
      }
  };

  PlaneState bufA, bufB;
  bufA.clear();
  bufB.clear();
  bool bad = false;  // a collided cell had a NaN, infinite or non-positive density

  if constexpr (!INIT) {
    stage_load(z0 - 2);
    stage_store(z0 - 2);
    stage_load(z0 - 1);
    stage_store(z0 - 1);
    stage_load(z0);
    stage_store(z0);
  }
  __syncthreads();

  // one pass: pull plane p+1 into nxt, collide plane p from cur
  auto pass = [&](const int p, PlaneState& cur, PlaneState& nxt) {
    const int q = p + 1;  // the plane pulled in this pass
    const bool pull_q = needs_pull(q);
    const int zq = zper ? wrap(q, G.nz) : q;
    const bool outlet_q = outflow && zq == G.nz - 1;
    const bool loads_q = !INIT && pull_q && !outlet_q;
    const int mode = plane_mode(G, zq);

    // Steps 1-3 end at the workgroup's barrier, and the waves of the other workgroup on the
    // same SIMD are usually colliding meanwhile: the pull takes the higher issue priority so
    // that its loads go out, and the barrier is reached, sooner.
    __builtin_amdgcn_s_setprio(1);
    // 1. the loads of the scalars of plane p+3 and of the populations of plane p+1
    if constexpr (!INIT && kStageFirst) stage_load(p + 3);
    __builtin_amdgcn_sched_barrier(0);
    typename Word<T>::W ldI[Q], ldR[Q];
    if (loads_q) {
      const rsrc_t slab[3] = {buffer_of(gin + (size_t)zsrc(q - 1) * slab_bytes, slab_bytes),
                              buffer_of(gin + (size_t)zq * slab_bytes, slab_bytes),
                              buffer_of(gin + (size_t)zsrc(q + 1) * slab_bytes, slab_bytes)};
      // neighbour offsets, recomputed per plane (cheaper than 18 registers across the loop)
      int ax = gx, ay = gy, arx = rgx, ary = rgy;
      asm volatile("" : "+v"(ax), "+v"(ay), "+v"(arx), "+v"(ary));
      unsigned oI[3][3], oR[3][3];
      column_offsets<T>(G, ax, ay, oI);
      column_offsets<T>(G, arx, ary, oR);
      with_mode(mode, [&](auto M) {
        if (ringer) issue_pull<T, decltype(M)::value, LAT>(slab, pb, oR, wfR, ldR);
        issue_pull<T, decltype(M)::value, LAT>(slab, pb, oI, wfI, ldI);
      });
    }
    if constexpr (!INIT && !kStageFirst) stage_load(p + 3);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (!INIT && !kStoreLate) stage_store(p + 3);

    // 2. complete the pull of plane q: own cell (with deviations) and ring cell (densities).
    // The LDS bases are made opaque per pass so that the compiler does not hoist one address
    // per neighbour out of the plane loop.
    int bI = sI - SX - 1, bR = sR - SX - 1;
    asm volatile("" : "+v"(bI), "+v"(bR));
    if (!pull_q) nxt.clear();
    if (pull_q) {
      const int s = slot4(q);
      const float4* S[3] = {sS[slot4(q - 1)], sS[s], sS[slot4(q + 1)]};
      const float2* W[3] = {sW[slot4(q - 1)], sW[s], sW[slot4(q + 1)]};
      // the ring first: its loads are the older ones and its registers are freed sooner
      if (ringer) {
        float r_rho, r_r, r_b, r_e, r_sh, r_dr, r_df[Q];
        if constexpr (INIT) {
          init_cell<false>(A.init, A.pc, G.n, (long long)zq * plane + rcol, r_rho, r_r, r_b, r_e, r_df);
        } else if (outlet_q) {
          outlet_cell<false>(A.outlet, A.pc, plane, rcol, r_rho, r_r, r_b, r_e, r_df);
        } else {
          with_mode(mode, [&](auto M) {
            finish_pull<T, decltype(M)::value, false, SX, LAT>(ldR, S, W, bR, wfR, A.pc, r_rho, r_r, r_b, r_e, r_df,
                                                               r_sh, r_dr);
          });
        }
        if (is_inflow(G, rgx, rgy, zq)) {
          r_rho = G.rho_r0;
          r_r = G.rho_r0;
          r_b = 0.0f;
        }
        const float r_inv = rcp(r_rho);
        sDf[dat(s, 0, dR)] = make_float2(r_r * r_inv, r_rho);
        sDf[dat(s, 1, dR)] = make_float2(r_b * r_inv, r_rho);
      }
      if constexpr (INIT) {
        init_cell<true>(A.init, A.pc, G.n, (long long)zq * plane + col, nxt.rho, nxt.rho_r, nxt.rho_b, nxt.e, nxt.df);
        nxt.shift = nxt.drho = 0.0f;
      } else if (outlet_q) {
        outlet_cell<true>(A.outlet, A.pc, plane, col, nxt.rho, nxt.rho_r, nxt.rho_b, nxt.e, nxt.df);
        nxt.shift = nxt.drho = 0.0f;
      } else {
        with_mode(mode, [&](auto M) {
          finish_pull<T, decltype(M)::value, true, SX, LAT>(ldI, S, W, bI, wfI, A.pc, nxt.rho, nxt.rho_r, nxt.rho_b,
                                                            nxt.e, nxt.df, nxt.shift, nxt.drho);
        });
      }
      if (is_inflow(G, gx, gy, zq)) {  // R10: inflow sites are pure red at rho_r0
        nxt.rho = G.rho_r0;
        nxt.rho_r = G.rho_r0;
        nxt.rho_b = 0.0f;
      }
      const float inv = rcp(nxt.rho);
      sDf[dat(s, 0, dI)] = make_float2(nxt.rho_r * inv, nxt.rho);
      sDf[dat(s, 1, dI)] = make_float2(nxt.rho_b * inv, nxt.rho);
    }
    // 3. the staged scalars to LDS, after the pull: planes p..p+2, which the pull reads, were
    // stored in earlier passes, and the slot written here held plane p-1, last read before the
    // previous barrier
    if constexpr (!INIT && kStoreLate) stage_store(p + 3);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();

    // 4. collide plane p
    if (p >= z0 && live) {
      const rsrc_t gslab = buffer_of(gout + (size_t)p * slab_bytes, slab_bytes);
      const rsrc_t sslab = buffer_of(A.sc_out + (size_t)p * 5 * (size_t)plane, sc_bytes);
      // (inflow sites are collided like any cell here; inflow_kernel overwrites them)
      {
        const int sm = (!zper && p == 0) ? slot4(p) : slot4(p - 1);
        const int sp = (!zper && p == G.nz - 1) ? slot4(p) : slot4(p + 1);
        const int s0 = slot4(p);
        // grad phi from the cell's minority colour fraction t (phi = 2a - 1 = 1 - 2b): near a
        // pure phase phi = -1 + 2a carries only the absolute precision of 1 in FP32, while a
        // itself keeps its relative precision, so the direction of grad phi stays defined
        // wherever the fields define it.
        const bool red_minor = cur.rho_r <= cur.rho_b;
        float gp[3], gr[3];
        {
          float vp[3][3][3], vr[3][3][3];
          int b0 = dI - DX - 1;
          asm volatile("" : "+v"(b0));
          // (a, rho) or (b, rho) of each neighbour, by the cell's minority colour
          const float2* D2 = sDf + dat(0, red_minor ? 0 : 1, 0);
          constexpr int kCellStride = kSplitRing ? 1 : 2, kSlotStride = kSplitRing ? ND : 2 * ND;
          const int slots[3] = {sm, s0, sp};
          // beyond a lateral wall the stencil sees the boundary cell (reading R9)
          const int xo[3] = {(wfI & 1) ? 1 : 0, 1, (wfI & 2) ? 1 : 2};
          const int yo[3] = {(wfI & 4) ? DX : 0, DX, (wfI & 8) ? DX : 2 * DX};
#pragma unroll
          for (int dz = 0; dz < 3; ++dz) {
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
              for (int dx = 0; dx < 3; ++dx) {
                const float2 v = D2[slots[dz] * kSlotStride + kCellStride * (b0 + yo[dy] + xo[dx])];
                vp[dz][dy][dx] = v.x;
                vr[dz][dy][dx] = v.y;
              }
            __builtin_amdgcn_sched_barrier(0);  // one plane of reads at a time
          }
          gradient27(vp, gp);
          gradient27(vr, gr);
          const float two = red_minor ? 2.0f : -2.0f;
          gp[0] *= two;
          gp[1] *= two;
          gp[2] *= two;
        }
        // instability: a NaN anywhere in the pulled populations reaches rho (noted here, stored
        // once when the workgroup leaves)
        bad |= !(cur.rho > 0.0f && cur.rho < 3.0e38f);
        CellOut o;
        collide_cell<Word<T>::kOutShift>(A.cp, A.rates, cur.df, cur.shift, cur.drho, cur.rho, cur.rho_r, cur.rho_b, gp,
                                         gr, o);
#pragma unroll
        for (int i = 0; i < Q; ++i) Word<T>::store(Word<T>::enc_scaled(o.g[i]), gslab, colT, i * pb);
        store_f32(cur.e, sslab, col4, 0);
        store_f32(psi_encode(cur.rho_r, cur.rho_b, cur.rho), sslab, col4, plane * 4);
        store_f32(o.wx, sslab, col4, 2 * plane * 4);
        store_f32(o.wy, sslab, col4, 3 * plane * 4);
        store_f32(o.wz, sslab, col4, 4 * plane * 4);
      }
    }
  };

  // unrolled by two so that the two plane states swap roles instead of being copied
  for (int p = z0 - 2; p < z1; p += 2) {
    pass(p, bufA, bufB);
    if (p + 1 < z1) pass(p + 1, bufB, bufA);
  }
  if (bad) *A.unstable = 1;
}

template <typename T, int TX, int TY, bool INIT, int LAT>
__global__ void __launch_bounds__(TX * TY, LBM_STEP_WAVES_PER_EU) step_kernel(const StepArgs A) {
  step_body<T, TX, TY, INIT, LAT>(A, (int)blockIdx.x, (int)gridDim.x);
}

// Many lattices in one launch: case c owns blocks [first[c], first[c+1]) of the grid, each
// range padded to a multiple of 8 blocks so that the XCD-aware numbering holds per case.
template <typename T, int TX, int TY, bool INIT, int LAT>
__global__ void __launch_bounds__(TX * TY, LBM_STEP_WAVES_PER_EU)
    batch_step_kernel(const StepArgs* __restrict__ cases, const int* __restrict__ first, int ncases) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = ncases;  // first[lo] <= b < first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  step_body<T, TX, TY, INIT, LAT>(cases[lo], b - first[lo], first[lo + 1] - first[lo]);
}

// Inflow sites (R10) after a step: each emits the red equilibrium at rho_r0 and u_in(1 + eps xi)
// e_z with Phi = 0 and no blue; the step kernel collided them like any cell.
template <typename T>
__device__ __forceinline__ void inflow_body(const StepArgs& A, const int col, const long long step) {
  const Geo& G = A.geo;
  if (col >= G.plane) return;
  const int x = col % G.nx, y = col / G.nx;
  if (!is_inflow(G, x, y, 0)) return;
  const int pb = G.plane * (int)sizeof(T);
  const rsrc_t gslab = buffer_of(A.g_out, (unsigned)(Q * pb));
  const rsrc_t sslab = buffer_of(A.sc_out, (unsigned)(5 * G.plane * 4));
  const unsigned colT = (unsigned)(col * (int)sizeof(T)), col4 = (unsigned)(col * 4);
  const float u = inflow_speed(G, (long long)col, step);
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    Word<T>::store(Word<T>::enc(eq_dev<i>(G.rho_r0, 0.0f, 0.0f, u)), gslab, colT, i * pb);
  });
  store_f32(0.0f, sslab, col4, 0);                // rho_r0 (1 - alpha_r) = E0 exactly
  store_f32(-0.0f, sslab, col4, G.plane * 4);     // pure red
  store_f32(0.0f, sslab, col4, 2 * G.plane * 4);
  store_f32(0.0f, sslab, col4, 3 * G.plane * 4);
  store_f32(0.0f, sslab, col4, 4 * G.plane * 4);
}

template <typename T>
__global__ void __launch_bounds__(256) inflow_kernel(const StepArgs A) {
  inflow_body<T>(A, (int)(blockIdx.x * blockDim.x + threadIdx.x), A.step);
}

// The inflow planes of many lattices in one launch (case c owns blocks [first[c],
// first[c+1]); every case of a batch is at the same step, which is passed in).
template <typename T>
__global__ void __launch_bounds__(256)
    batch_inflow_kernel(const StepArgs* __restrict__ cases, const int* __restrict__ first, int ncases, long long step) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = ncases;  // first[lo] <= b < first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  inflow_body<T>(cases[lo], (b - first[lo]) * 256 + (int)threadIdx.x, step);
}

// ================================================================== launchers
template <typename T, int TX, int TY, int LAT>
hipError_t launch_step_lat(const StepArgs& a, hipStream_t s) {
  const long long blocks = (long long)tiles_in_set(a) * a.nchunks;
  if (blocks == 0) return hipSuccess;
  if (a.init_mode)
    hipLaunchKernelGGL((step_kernel<T, TX, TY, true, LAT>), dim3((unsigned)blocks), dim3(TX * TY), 0, s, a);
  else
    hipLaunchKernelGGL((step_kernel<T, TX, TY, false, LAT>), dim3((unsigned)blocks), dim3(TX * TY), 0, s, a);
  return hipGetLastError();
}

// Whether storage type T takes one step-kernel instance per lateral wall along the frame's
// edges (FP16 storage) rather than one per axis (wall_tile_sets on the host side).
template <typename T>
constexpr bool kWallPerSide = std::is_same<T, _Float16>::value;

// The step kernel with lateral free-slip walls comes in instances that reflect at the walls
// of one axis or one wall (the frame's edges, by storage) or at all four (its corners);
// lattices with periodic sides, and the interior tiles of a lattice with walls, keep the
// plain pull.  Only the modes of T's tile sets are instantiated.
template <typename T, int TX, int TY>
hipError_t launch_step_tile(const StepArgs& a, hipStream_t s) {
  const int mode = lat_mode_of(a.tile_set, a.geo.wall_x || a.geo.wall_y);
  if (mode == 0) return launch_step_lat<T, TX, TY, 0>(a, s);
  if (mode == 15) return launch_step_lat<T, TX, TY, 15>(a, s);
  if constexpr (kWallPerSide<T>) {
    switch (mode) {
      case 1: return launch_step_lat<T, TX, TY, 1>(a, s);
      case 2: return launch_step_lat<T, TX, TY, 2>(a, s);
      case 4: return launch_step_lat<T, TX, TY, 4>(a, s);
      case 8: return launch_step_lat<T, TX, TY, 8>(a, s);
    }
  } else {
    switch (mode) {
      case 3: return launch_step_lat<T, TX, TY, 3>(a, s);
      case 12: return launch_step_lat<T, TX, TY, 12>(a, s);
    }
  }
  return hipErrorInvalidValue;
}

template <typename T, int TX, int TY, int LAT>
hipError_t launch_batch_lat(const StepArgs* cases, const int* first, int ncases, int nblocks, bool init,
                            hipStream_t s) {
  if (init)
    hipLaunchKernelGGL((batch_step_kernel<T, TX, TY, true, LAT>), dim3((unsigned)nblocks), dim3(TX * TY), 0, s, cases,
                       first, ncases);
  else
    hipLaunchKernelGGL((batch_step_kernel<T, TX, TY, false, LAT>), dim3((unsigned)nblocks), dim3(TX * TY), 0, s, cases,
                       first, ncases);
  return hipGetLastError();
}

template <typename T, int TX, int TY>
hipError_t launch_batch_tile(const StepArgs* cases, const int* first, int ncases, int nblocks, bool init, int lat,
                             hipStream_t s) {
  if (lat == 0) return launch_batch_lat<T, TX, TY, 0>(cases, first, ncases, nblocks, init, s);
  if (lat == 15) return launch_batch_lat<T, TX, TY, 15>(cases, first, ncases, nblocks, init, s);
  if constexpr (kWallPerSide<T>) {
    switch (lat) {
      case 1: return launch_batch_lat<T, TX, TY, 1>(cases, first, ncases, nblocks, init, s);
      case 2: return launch_batch_lat<T, TX, TY, 2>(cases, first, ncases, nblocks, init, s);
      case 4: return launch_batch_lat<T, TX, TY, 4>(cases, first, ncases, nblocks, init, s);
      case 8: return launch_batch_lat<T, TX, TY, 8>(cases, first, ncases, nblocks, init, s);
    }
  } else {
    switch (lat) {
      case 3: return launch_batch_lat<T, TX, TY, 3>(cases, first, ncases, nblocks, init, s);
      case 12: return launch_batch_lat<T, TX, TY, 12>(cases, first, ncases, nblocks, init, s);
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_batch_T(const StepArgs* cases, const int* first, int ncases, int nblocks, bool init, int tx, int ty,
                          int lat, hipStream_t s) {
  if (tx == 32 && ty == 4) return launch_batch_tile<T, 32, 4>(cases, first, ncases, nblocks, init, lat, s);
  if (tx == 32 && ty == 8) return launch_batch_tile<T, 32, 8>(cases, first, ncases, nblocks, init, lat, s);
  if (tx == 64 && ty == 4) return launch_batch_tile<T, 64, 4>(cases, first, ncases, nblocks, init, lat, s);
  if (tx == 64 && ty == 8) return launch_batch_tile<T, 64, 8>(cases, first, ncases, nblocks, init, lat, s);
  if (tx == 32 && ty == 16) return launch_batch_tile<T, 32, 16>(cases, first, ncases, nblocks, init, lat, s);
  return hipErrorInvalidValue;
}

template <typename T, int TX, int TY>
int resident_tile(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)step_kernel<T, TX, TY, false, false>, TX * TY, 0) !=
      hipSuccess)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return per_cu * cus;
}

template <typename T>
hipError_t launch_step_T(const StepArgs& a, int tx, int ty, hipStream_t s) {
  if (tx == 32 && ty == 4) return launch_step_tile<T, 32, 4>(a, s);
  if (tx == 32 && ty == 8) return launch_step_tile<T, 32, 8>(a, s);
  if (tx == 64 && ty == 4) return launch_step_tile<T, 64, 4>(a, s);
  if (tx == 64 && ty == 8) return launch_step_tile<T, 64, 8>(a, s);
  if (tx == 32 && ty == 16) return launch_step_tile<T, 32, 16>(a, s);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_inflow_T(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(inflow_kernel<T>, dim3((unsigned)((a.geo.plane + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_inflow_T(const StepArgs* cases, const int* first, int ncases, int nblocks, long long step,
                                 hipStream_t s) {
  hipLaunchKernelGGL(batch_inflow_kernel<T>, dim3((unsigned)nblocks), dim3(256), 0, s, cases, first, ncases, step);
  return hipGetLastError();
}

template <typename T>
int step_resident_blocks_T(int tx, int ty, int device) {
  if (tx == 32 && ty == 4) return resident_tile<T, 32, 4>(device);
  if (tx == 32 && ty == 8) return resident_tile<T, 32, 8>(device);
  if (tx == 64 && ty == 4) return resident_tile<T, 64, 4>(device);
  if (tx == 64 && ty == 8) return resident_tile<T, 64, 8>(device);
  if (tx == 32 && ty == 16) return resident_tile<T, 32, 16>(device);
  return 0;
}

#define LBM_INSTANTIATE_STEP(T)                                                 \
  template hipError_t launch_step_T<T>(const StepArgs&, int, int, hipStream_t); \
  template hipError_t launch_batch_T<T>(const StepArgs*, const int*, int, int, bool, int, int, int, hipStream_t); \
  template hipError_t launch_inflow_T<T>(const StepArgs&, hipStream_t);                                         \
  template hipError_t launch_batch_inflow_T<T>(const StepArgs*, const int*, int, int, long long, hipStream_t);          \
  template int step_resident_blocks_T<T>(int, int, int);

}  // namespace lbm
