// lbm_device.h -- device-side data layout, storage codecs, boundary resolution and the
// population "pull" shared by the step kernel and the read-back kernels.
//
// State layout in HBM: structure of arrays grouped by z plane ("z-slabs"), so that every
// population a cell pulls lies in one of three slabs addressed by a 32-bit offset:
//   g [(z 27 + i) nx ny + y nx + x]  i = 0..26  post-collision deviation
//                                    f''_i - rho varphi_i(alpha_bar) of the emitting cell (type T)
//   sc[(z 5 + k) nx ny + y nx + x]   k = 0..4   e, psi, w_x, w_y, w_z of that cell
//                                               (FP32), w = beta (rho_r rho_b/rho)(1 - alpha_bar) n
// e = E - E0 with E = rho (1 - alpha_bar) = sum_k rho_k (1 - alpha_k) = 19 p / 9 (Eq. (press))
// and E0 = rho_b0 (1 - alpha_b) = rho_r0 (1 - alpha_r): the pressure is nearly uniform across
// both phases, so e is small and FP32 keeps it to ~1e-10; rho = (E0 + e)/(1 - alpha_bar(a)).
// psi carries the colour fraction of the minority colour at full relative precision:
// psi = a = rho_r/rho when a <= 1/2, psi = -(1 - a) = -rho_b/rho otherwise (sign bit set,
// also for -0), so a few 1e-10 of blue in the red phase survive as they do in FP64.
// A reader at y pulls population i from its source x = y - c_i and rebuilds
//   f_i   = g_i(x) + q_i E(x)          E = rho (1 - alpha_bar) = rho (1 - alpha_b) - rho_r (alpha_r - alpha_b)
//   f^r_i = a(x) f_i + (q_i/|c_i|) c_i . w(x)    (recolouring, Sec. II),   f^b_i = f_i - f^r_i,
// which is exactly the two-colour streaming of Eq. (LBE) written with 32 values per cell
// instead of 54.  The rest population (i = 0) is f_0 = g_0(y) + rho(y) alpha_bar(y).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "lbm_cell.h"

namespace lbm {

enum { FACE_PERIODIC = 0, FACE_BOUNCEBACK = 1, FACE_FREESLIP = 2, FACE_OUTFLOW = 3 };

// ---------------------------------------------------------------- storage codecs
struct bf16 {
  uint16_t bits;
};

template <typename T>
struct Codec;
template <>
struct Codec<float> {
  static __device__ __forceinline__ float dec(float v) { return v; }
  static __device__ __forceinline__ float enc(float v) { return v; }
};
// FP16 deviations are stored scaled by 2^10 so that small deviations stay normal numbers.
template <>
struct Codec<_Float16> {
  static constexpr float kScale = 1024.0f;
  static __device__ __forceinline__ float dec(_Float16 v) { return (float)v * (1.0f / kScale); }
  static __device__ __forceinline__ _Float16 enc(float v) { return (_Float16)(v * kScale); }
};
// BF16 (round to nearest even from FP32).
template <>
struct Codec<bf16> {
  static __device__ __forceinline__ float dec(bf16 v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
  static __device__ __forceinline__ bf16 enc(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    bf16 r;
    r.bits = (uint16_t)(u >> 16);
    return r;
  }
};

// ---------------------------------------------------------------- geometry
struct Geo {
  int nx, ny, nz;
  int plane;                 // nx ny
  long long n;               // nx ny nz
  int face_lo, face_hi;      // rules of the -z and +z faces
  int wall_x, wall_y;        // 1: free-slip walls on both faces of that axis, 0: periodic
  int inflow;                // inflow disk on z = 0
  float xc, yc, r2;          // disk centre and squared radius
  float rho_r0;              // density emitted by the inflow
  float u_in, noise;         // inflow speed and relative noise amplitude
  unsigned long long seed;   // noise seed
};

__device__ __forceinline__ int wrap(int v, int n) {
  v = v % n;
  return v < 0 ? v + n : v;
}

__device__ __forceinline__ bool is_inflow(const Geo& G, int x, int y, int z) {
  if (!G.inflow || z != 0) return false;
  const float dx = (float)x - G.xc, dy = (float)y - G.yc;
  return dx * dx + dy * dy < G.r2;
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator: uniform on [-1, 1).
__device__ __forceinline__ double splitmix64_uniform(unsigned long long seed, unsigned long long counter) {
  unsigned long long z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Inflow speed of site `cell` at step `step`: u0 (1 + eps xi).
__device__ __forceinline__ float inflow_speed(const Geo& G, long long cell, long long step) {
  if (G.noise == 0.0f) return G.u_in;
  const double xi = splitmix64_uniform(G.seed, (unsigned long long)step * (unsigned long long)G.n + (unsigned long long)cell);
  return (float)((double)G.u_in * (1.0 + (double)G.noise * xi));
}

// Deviation of a colour equilibrium at rest-density rho_k: rho_k w_i [3 c.u + 9/2 (c.u)^2 - 3/2 u^2].
template <int I>
__device__ __forceinline__ float cdot(float ux, float uy, float uz) {
  float r = 0.0f;
  if constexpr (CX[I] != 0) r += (float)CX[I] * ux;
  if constexpr (CY[I] != 0) r += (float)CY[I] * uy;
  if constexpr (CZ[I] != 0) r += (float)CZ[I] * uz;
  return r;
}

template <int I>
__device__ __forceinline__ float eq_dev(float rho_k, float ux, float uy, float uz) {
  const float cu = cdot<I>(ux, uy, uz);
  const float uu = ux * ux + uy * uy + uz * uz;
  return rho_k * w_of(I) * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
}

// ---------------------------------------------------------------- boundary resolution
// Where population I arriving at a cell comes from: the source offset (dx, dy, dz) relative
// to the reader, the population index J at the source, and the velocity of J (for the
// recolouring dot product).  x and y wrap.  MODE selects the z rule of the reader's plane:
// bulk planes stream straight; the first plane of a bounce-back or free-slip -z face and the
// last plane of such a +z face redirect the populations that would come from outside (R8,
// R9).  The outlet plane of an outflow face is never resolved this way.
enum { kBulk = 0, kLoBB = 1, kLoFS = 2, kHiBB = 3, kHiFS = 4 };

struct Src {
  int dx, dy, dz;
  int j;
  int ccx, ccy, ccz;
};

template <int I, int MODE>
__host__ __device__ constexpr Src resolve() {
  Src s{-CX[I], -CY[I], -CZ[I], I, CX[I], CY[I], CZ[I]};
  const bool from_below = CZ[I] == 1 && (MODE == kLoBB || MODE == kLoFS);
  const bool from_above = CZ[I] == -1 && (MODE == kHiBB || MODE == kHiFS);
  if (from_below || from_above) {
    if (MODE == kLoFS || MODE == kHiFS) {  // specular: keep the tangential shift
      s.dz = 0;
      s.j = mirror_z(I);
      s.ccz = -CZ[I];
    } else {  // half-way bounce-back: the reader's own opposite population
      s.dx = s.dy = s.dz = 0;
      s.j = opposite(I);
      s.ccx = -CX[I];
      s.ccy = -CY[I];
      s.ccz = -CZ[I];
    }
  }
  return s;
}

// The source of population I at a cell (x, y) of a plane in pull mode MODE, with the lateral
// walls of G (reading R9 on the x and y faces): where the source would lie beyond a free-slip
// wall, the population comes from the boundary cell itself along that axis, with the normal
// component of its velocity reversed (the tangential shift is kept).  A bounce-back of the z
// rule takes precedence, as its source is the cell itself.
struct RSrc {
  int dx, dy, dz, j, ccx, ccy, ccz;
};

template <int I, int MODE>
__device__ __forceinline__ RSrc resolve_at(const Geo& G, int x, int y) {
  constexpr Src s = resolve<I, MODE>();
  RSrc r{s.dx, s.dy, s.dz, s.j, s.ccx, s.ccy, s.ccz};
  if constexpr (s.dx != 0 || s.dy != 0) {
    const bool rx = G.wall_x && ((s.dx == -1 && x == 0) || (s.dx == 1 && x == G.nx - 1));
    const bool ry = G.wall_y && ((s.dy == -1 && y == 0) || (s.dy == 1 && y == G.ny - 1));
    constexpr int jx = mirror_x(s.j), jy = mirror_y(s.j), jxy = mirror_x(mirror_y(s.j));
    if (rx) {
      r.dx = 0;
      r.ccx = -s.ccx;
    }
    if (ry) {
      r.dy = 0;
      r.ccy = -s.ccy;
    }
    r.j = rx ? (ry ? jxy : jx) : (ry ? jy : s.j);
  }
  return r;
}

// Lateral wall flags of a cell: bit 0 at a -x wall, 1 at a +x wall, 2 at a -y wall, 3 at a
// +y wall.
__device__ __forceinline__ int wall_flags(const Geo& G, int x, int y) {
  return (G.wall_x && x == 0 ? 1 : 0) | (G.wall_x && x == G.nx - 1 ? 2 : 0) | (G.wall_y && y == 0 ? 4 : 0) |
         (G.wall_y && y == G.ny - 1 ? 8 : 0);
}

// Pull mode of plane z.
__host__ __device__ inline int plane_mode(const Geo& G, int z) {
  if (z == 0 && G.face_lo == FACE_BOUNCEBACK) return kLoBB;
  if (z == 0 && G.face_lo == FACE_FREESLIP) return kLoFS;
  if (z == G.nz - 1 && (G.face_hi == FACE_BOUNCEBACK || G.face_hi == FACE_OUTFLOW)) return kHiBB;
  if (z == G.nz - 1 && G.face_hi == FACE_FREESLIP) return kHiFS;
  return kBulk;
}

// Outlet plane record: 27 red and 27 blue deviations f^k_i - rho_k varphi_i(alpha_k),
// then e and a of the outlet cell; 56 planes of nx*ny floats.
constexpr int kOutletPlanes = 56;

// Per-run constants for the pull (the differences are formed in FP64, then rounded).
struct PullConst {
  float alpha_r, alpha_b, dalpha;  // dalpha = alpha_r - alpha_b
  float E0;                        // rho_b0 (1 - alpha_b)
  float one_m_ab, one_m_ar;        // 1 - alpha_b, 1 - alpha_r = (1 - alpha_b)/gamma
};

// Colour fractions (a, b) = (rho_r/rho, rho_b/rho) of a stored psi.
__host__ __device__ __forceinline__ bool psi_red_major(float psi) { return std::signbit(psi); }
__host__ __device__ __forceinline__ float psi_a(float psi) { return psi_red_major(psi) ? 1.0f + psi : psi; }
__host__ __device__ __forceinline__ float psi_b(float psi) { return psi_red_major(psi) ? -psi : 1.0f - psi; }
__host__ __device__ __forceinline__ float psi_encode(float rho_r, float rho_b, float rho) {
  return rho_r <= rho_b ? rho_r / rho : -(rho_b / rho);
}

// Density of a cell from its stored (e, a, b): rho = E/(1 - alpha_bar), E = E0 + e.
__host__ __device__ __forceinline__ float rho_of(const PullConst& C, float e, float a, float b) {
  return (C.E0 + e) * rcp(one_minus_abar(a, b, C.dalpha, C.one_m_ab, C.one_m_ar));
}
__host__ __device__ __forceinline__ float rho_of_psi(const PullConst& C, float e, float psi) {
  return rho_of(C, e, psi_a(psi), psi_b(psi));
}

}  // namespace lbm
