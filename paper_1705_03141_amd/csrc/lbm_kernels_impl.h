// lbm_kernels_impl.h -- device building blocks of the D3Q27 colour-fluid step (pull of one
// cell, isotropic gradient, initial and outlet states) and the small kernels around the step:
// convective outlet, read-back of fields and populations, FP64 diagnostics.  The fused step
// kernel itself is in lbm_step.h.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_device.h"
#include "lbm_kernels.h"

namespace lbm {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

__device__ __forceinline__ int slot3(int q) { return ((q % 3) + 3) % 3; }

// Neighbourhood addressing of a cell: source z planes (wrapped when z is periodic, clamped
// otherwise; clamped entries are never read), row offsets y nx and columns x, all wrapped in
// x and y.
struct Nbr {
  int zs[3];
  int row[3];
  int xs[3];
  int x, y;
  // entries at a run-time offset d in {-1, 0, 1} (selects, not indexed loads)
  __device__ __forceinline__ int z_at(int d) const { return d < 0 ? zs[0] : (d > 0 ? zs[2] : zs[1]); }
  __device__ __forceinline__ int row_at(int d) const { return d < 0 ? row[0] : (d > 0 ? row[2] : row[1]); }
  __device__ __forceinline__ int x_at(int d) const { return d < 0 ? xs[0] : (d > 0 ? xs[2] : xs[1]); }
};

__device__ __forceinline__ Nbr neighbours(const Geo& G, int x, int y, int z) {
  Nbr b;
  const bool per = G.face_lo == FACE_PERIODIC;
  b.zs[0] = z == 0 ? (per ? G.nz - 1 : 0) : z - 1;
  b.zs[1] = z;
  b.zs[2] = z == G.nz - 1 ? (per ? 0 : G.nz - 1) : z + 1;
  b.row[0] = (y == 0 ? G.ny - 1 : y - 1) * G.nx;
  b.row[1] = y * G.nx;
  b.row[2] = (y == G.ny - 1 ? 0 : y + 1) * G.nx;
  b.xs[0] = x == 0 ? G.nx - 1 : x - 1;
  b.xs[1] = x;
  b.xs[2] = x == G.nx - 1 ? 0 : x + 1;
  b.x = x;
  b.y = y;
  return b;
}

// Population J of the cell at reader + (dx, dy, dz).
template <typename T>
__device__ __forceinline__ float load_pop(const Geo& G, const T* __restrict__ g, const Nbr& b, int j, int dx, int dy,
                                          int dz) {
  const T* slab = g + (size_t)(b.z_at(dz) * Q + j) * (size_t)G.plane;
  return Codec<T>::dec(slab[b.row_at(dy) + b.x_at(dx)]);
}

// Pull of one cell in a plane of pull mode MODE.  Scalars of the source cells come from
// `acc`:  acc.self_e(), acc.self_psi()  e and psi of the reader at t-1;
//         acc.e/psi/w(dx, dy, dz)        e, psi, w of the cell at reader + (dx, dy, dz).
// Returns rho, rho_r, rho_b and e of time t; with WANT_DF also the deviations in the reader's
// form d_i = g_i(src) + q_i (e(src) - e(self)) (from the rest equilibrium of the previous
// state) with shift = E(t-1) - E(t) and drho = sum_i d_i that move them to the present one
// (collide_cell takes them so; to_deviation() applies them).  Everything is formed from
// increments so that no O(1) quantity is subtracted from another, and the colour that is the
// reader's minority is accumulated from its own fractions.
template <typename T, bool WANT_DF, int MODE, typename Acc>
__device__ __forceinline__ void pull_cell(const Geo& G, const PullConst& C, const T* __restrict__ g, const Nbr& b,
                                          const Acc& acc, float& rho, float& rho_r, float& rho_b, float& e_new,
                                          float (&df)[Q], float& shift_out, float& drho_out) {
  const float e_self = acc.self_e(), psi_self = acc.self_psi();
  const bool track_red = !psi_red_major(psi_self);  // the reader's minority colour
  const float a_self = psi_a(psi_self);
  const float t_self = track_red ? psi_self : -psi_self;  // fraction of the tracked colour
  const float rho_old = rho_of_psi(C, e_self, psi_self);
  const float E_self = C.E0 + e_self;
  const float sgn = track_red ? 1.0f : -1.0f;  // recolouring adds to red, removes from blue
  // rest population: its source is the reader itself
  float d_rho = load_pop<T>(G, g, b, 0, 0, 0, 0);
  float d_t = t_self * d_rho;
  if constexpr (WANT_DF) df[0] = d_rho;
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr Src s0 = resolve<i, MODE>();
    const RSrc s = resolve_at<i, MODE>(G, b.x, b.y);
    const float gv = load_pop<T>(G, g, b, s.j, s.dx, s.dy, s.dz);
    const float de = acc.e(s.dx, s.dy, s.dz) - e_self, psi = acc.psi(s.dx, s.dy, s.dz);
    const float t = track_red ? psi_a(psi) : psi_b(psi);
    float cw = 0.0f;  // c_j . w of the source, only the non-zero components
    if constexpr (s0.ccx != 0) cw += (float)s.ccx * acc.w(0, s.dx, s.dy, s.dz);
    if constexpr (s0.ccy != 0) cw += (float)s.ccy * acc.w(1, s.dx, s.dy, s.dz);
    if constexpr (s0.ccz != 0) cw += (float)s.ccz * acc.w(2, s.dx, s.dy, s.dz);
    const float d = gv + q_of(i) * de;
    d_rho += d;
    d_t += t * d + q_of(i) * E_self * (t - t_self) + sgn * qc_of(i) * cw;
    if constexpr (WANT_DF) df[i] = d;
    if constexpr (i % 9 == 0) __builtin_amdgcn_sched_barrier(0);  // bound the loads in flight
  });
  rho = rho_old + d_rho;
  const float rho_t = t_self * rho_old + d_t, rho_o = rho - rho_t;
  rho_r = track_red ? rho_t : rho_o;
  rho_b = track_red ? rho_o : rho_t;
  // E = (1 - alpha_b) rho - (alpha_r - alpha_b) rho_r is linear: its increment is exact
  const float d_rhor = track_red ? d_t : d_rho - d_t;
  const float shift = C.dalpha * d_rhor - (1.0f - C.alpha_b) * d_rho;  // E(t-1) - E(t)
  e_new = e_self - shift;
  shift_out = shift;
  drho_out = d_rho;
}

// Total deviations df_i = f_i - rho varphi_i(alpha_bar) from the reader's form.
__device__ __forceinline__ void to_deviation(float (&df)[Q], float shift) {
  float sum = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    df[i] += q_of(i) * shift;
    sum += df[i];
  }
  df[0] = -sum;  // sum_i df_i = 0 exactly
}

// Scalars straight from HBM (small kernels).
struct GlobalAcc {
  const float* sc;
  const Geo* G;
  const Nbr* b;
  __device__ __forceinline__ float val(int k, int dx, int dy, int dz) const {
    return sc[(size_t)(b->z_at(dz) * 5 + k) * (size_t)G->plane + b->row_at(dy) + b->x_at(dx)];
  }
  __device__ __forceinline__ float self_e() const { return val(0, 0, 0, 0); }
  __device__ __forceinline__ float self_psi() const { return val(1, 0, 0, 0); }
  __device__ __forceinline__ float e(int dx, int dy, int dz) const { return val(0, dx, dy, dz); }
  __device__ __forceinline__ float psi(int dx, int dy, int dz) const { return val(1, dx, dy, dz); }
  __device__ __forceinline__ float w(int k, int dx, int dy, int dz) const { return val(2 + k, dx, dy, dz); }
};

// Dispatch of the pull on the plane's mode (uniform across the workgroup).
template <typename T, bool WANT_DF, typename Acc>
__device__ __forceinline__ void pull_any(int mode, const Geo& G, const PullConst& C, const T* __restrict__ g,
                                         const Nbr& b, const Acc& acc, float& rho, float& rho_r, float& rho_b,
                                         float& e, float (&df)[Q], float& shift, float& drho) {
  switch (mode) {
    case kLoBB: pull_cell<T, WANT_DF, kLoBB>(G, C, g, b, acc, rho, rho_r, rho_b, e, df, shift, drho); break;
    case kLoFS: pull_cell<T, WANT_DF, kLoFS>(G, C, g, b, acc, rho, rho_r, rho_b, e, df, shift, drho); break;
    case kHiBB: pull_cell<T, WANT_DF, kHiBB>(G, C, g, b, acc, rho, rho_r, rho_b, e, df, shift, drho); break;
    case kHiFS: pull_cell<T, WANT_DF, kHiFS>(G, C, g, b, acc, rho, rho_r, rho_b, e, df, shift, drho); break;
    default: pull_cell<T, WANT_DF, kBulk>(G, C, g, b, acc, rho, rho_r, rho_b, e, df, shift, drho); break;
  }
}

// Isotropic gradient of Sec. II, 3 sum_i w_i chi(x + c_i) c_i, from a 3x3x3 neighbourhood
// v[dz+1][dy+1][dx+1]: weights 2/9, 1/18, 1/72 on the axis, edge and corner differences.
__device__ __forceinline__ void gradient27(const float (&v)[3][3][3], float (&gr)[3]) {
  const float c1 = 2.0f / 9.0f, c2 = 1.0f / 18.0f, c3 = 1.0f / 72.0f;
  float D[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) D[a][b] = v[a][b][2] - v[a][b][0];
  gr[0] = c1 * D[1][1] + c2 * (D[0][1] + D[2][1] + D[1][0] + D[1][2]) + c3 * (D[0][0] + D[0][2] + D[2][0] + D[2][2]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) D[a][b] = v[a][2][b] - v[a][0][b];
  gr[1] = c1 * D[1][1] + c2 * (D[0][1] + D[2][1] + D[1][0] + D[1][2]) + c3 * (D[0][0] + D[0][2] + D[2][0] + D[2][2]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) D[a][b] = v[2][a][b] - v[0][a][b];
  gr[2] = c1 * D[1][1] + c2 * (D[0][1] + D[2][1] + D[1][0] + D[1][2]) + c3 * (D[0][0] + D[0][2] + D[2][0] + D[2][2]);
}

// Initial state at a cell (reading R1): each colour at its equilibrium with Phi = 0, so the
// total deviation is rho w_i [3 c.u + 9/2 (c.u)^2 - 3/2 u^2].  The initial fields are held as
// (e, psi, ux, uy, uz), planes of ncells floats.
template <bool WANT_DF>
__device__ __forceinline__ void init_cell(const float* __restrict__ init, const PullConst& C, long long n,
                                          long long c, float& rho, float& rho_r, float& rho_b, float& e,
                                          float (&df)[Q]) {
  e = init[c];
  const float psi = init[n + c];
  rho = rho_of_psi(C, e, psi);
  rho_r = psi_a(psi) * rho;
  rho_b = psi_b(psi) * rho;
  if constexpr (WANT_DF) {
    const float ux = init[2 * n + c], uy = init[3 * n + c], uz = init[4 * n + c];
    const float r = rho;
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      df[i] = eq_dev<i>(r, ux, uy, uz);
    });
  }
}

// Outlet-plane record at a column: total deviations, e and the colour densities.
template <bool WANT_DF>
__device__ __forceinline__ void outlet_cell(const float* __restrict__ outlet, const PullConst& C, int plane, int col,
                                            float& rho, float& rho_r, float& rho_b, float& e, float (&df)[Q]) {
  // The record does not depend on the plane counter; without this the compiler hoists its
  // 54 loads out of the plane loop and keeps them live across the whole march.
  asm volatile("" : "+v"(col));
  e = outlet[54 * plane + col];
  const float psi = outlet[55 * plane + col];
  rho = rho_of_psi(C, e, psi);
  rho_r = psi_a(psi) * rho;
  rho_b = psi_b(psi) * rho;
  if constexpr (WANT_DF) {
#pragma unroll
    for (int i = 0; i < Q; ++i) df[i] = outlet[i * plane + col] + outlet[(Q + i) * plane + col];
  }
}

// ================================================================== outlet and read-back
// Per-colour pre-collision populations of a cell from the stored state (no LDS).
template <typename T>
__device__ __forceinline__ void pull_colours(const AuxArgs& A, int x, int y, int z, float (&fr)[Q], float (&fb)[Q]) {
  const Geo& G = A.geo;
  const Nbr b = neighbours(G, x, y, z);
  GlobalAcc acc{A.sc_in, &A.geo, &b};
  const T* g = static_cast<const T*>(A.g_in);
  const float e_self = acc.self_e(), psi_self = acc.self_psi();
  const float rho_self = rho_of_psi(A.pc, e_self, psi_self);
  auto one = [&](auto ic, auto mode) {
    constexpr int i = decltype(ic)::value;
    constexpr Src s0 = resolve<i, decltype(mode)::value>();
    const RSrc s = resolve_at<i, decltype(mode)::value>(G, x, y);
    const float gv = load_pop<T>(G, g, b, s.j, s.dx, s.dy, s.dz);
    if constexpr (i == 0) {
      const float f0 = gv + rho_self - (A.pc.E0 + e_self);  // g_0 + rho alpha_bar
      fr[0] = psi_a(psi_self) * f0;
      fb[0] = psi_b(psi_self) * f0;
    } else {
      const float fi = gv + q_of(i) * (A.pc.E0 + acc.e(s.dx, s.dy, s.dz));
      float cw = 0.0f;
      if constexpr (s0.ccx != 0) cw += (float)s.ccx * acc.w(0, s.dx, s.dy, s.dz);
      if constexpr (s0.ccy != 0) cw += (float)s.ccy * acc.w(1, s.dx, s.dy, s.dz);
      if constexpr (s0.ccz != 0) cw += (float)s.ccz * acc.w(2, s.dx, s.dy, s.dz);
      const float psi = acc.psi(s.dx, s.dy, s.dz);
      fr[i] = psi_a(psi) * fi + qc_of(i) * cw;
      fb[i] = psi_b(psi) * fi - qc_of(i) * cw;
    }
  };
  switch (plane_mode(G, z)) {
    case kLoBB: static_for<0, Q>([&](auto ic) { one(ic, std::integral_constant<int, kLoBB>{}); }); break;
    case kLoFS: static_for<0, Q>([&](auto ic) { one(ic, std::integral_constant<int, kLoFS>{}); }); break;
    case kHiBB: static_for<0, Q>([&](auto ic) { one(ic, std::integral_constant<int, kHiBB>{}); }); break;
    case kHiFS: static_for<0, Q>([&](auto ic) { one(ic, std::integral_constant<int, kHiFS>{}); }); break;
    default: static_for<0, Q>([&](auto ic) { one(ic, std::integral_constant<int, kBulk>{}); }); break;
  }
}

// Moments (increment form, as in the step) and per-colour populations of a bulk cell.
template <typename T>
__device__ __forceinline__ void pull_global(const AuxArgs& A, int x, int y, int z, float& rho, float& rho_r,
                                            float& rho_b, float& e, float (&df)[Q]) {
  const Nbr b = neighbours(A.geo, x, y, z);
  GlobalAcc acc{A.sc_in, &A.geo, &b};
  float shift, drho;
  pull_any<T, true>(plane_mode(A.geo, z), A.geo, A.pc, static_cast<const T*>(A.g_in), b, acc, rho, rho_r, rho_b, e,
                    df, shift, drho);
  to_deviation(df, shift);
}

__device__ __forceinline__ float varphi_of(int i, float alpha) { return i == 0 ? alpha : (1.0f - alpha) * q_of(i); }

// Convective outflow (R11): per column, the outlet plane's pre-collision state of time t is
// [state(t-1) + lambda f(N-1, t)] / (1 + lambda), colour by colour and population by
// population, lambda = max(0, u_z(N-1, t)).  Returned as deviations from each colour's
// rest equilibrium, dr_i = f^r_i - rho_r varphi_i(alpha_r) (likewise blue), and (e, psi).
template <typename T>
__device__ void outlet_state(const AuxArgs& A, int x, int y, float (&dr)[Q], float (&db)[Q], float& e_out,
                             float& psi_out) {
  const Geo& G = A.geo;
  const int plane = G.plane, col = y * G.nx + x;
  if (A.init_mode) {
    const long long c = (long long)(G.nz - 1) * plane + col;
    float rho, rho_r, rho_b, e, df[Q];
    init_cell<false>(A.init, A.pc, G.n, c, rho, rho_r, rho_b, e, df);
    const float ux = A.init[2 * G.n + c], uy = A.init[3 * G.n + c], uz = A.init[4 * G.n + c];
    const float r_ = rho_r, b_ = rho_b;
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      dr[i] = eq_dev<i>(r_, ux, uy, uz);
      db[i] = eq_dev<i>(b_, ux, uy, uz);
    });
    e_out = e;
    psi_out = A.init[G.n + c];
    return;
  }
  // the cell below the outlet at time t
  const int z = G.nz - 2;
  float rho, rho_r, rho_b, e_b, df[Q];
  pull_global<T>(A, x, y, z, rho, rho_r, rho_b, e_b, df);
  float fr[Q], fb[Q];
  pull_colours<T>(A, x, y, z, fr, fb);
  float jz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) jz += (float)CZ[i] * df[i];
  float Fz = 0.0f;
  if (A.cp.force) Fz = (rho - A.cp.rho_ref) * A.cp.gz;
  float lam = (jz + 0.5f * Fz) / rho;
  lam = lam > 0.0f ? lam : 0.0f;
  const float inv = 1.0f / (1.0f + lam);
  // the minority colour's deviations directly, the majority's as the rest of the total
  const bool red_minor = rho_r <= rho_b;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    float dri, dbi;
    if (red_minor) {
      dri = fr[i] - rho_r * varphi_of(i, A.pc.alpha_r);
      dbi = df[i] - dri;
    } else {
      dbi = fb[i] - rho_b * varphi_of(i, A.pc.alpha_b);
      dri = df[i] - dbi;
    }
    dr[i] = (A.outlet_in[i * plane + col] + lam * dri) * inv;
    db[i] = (A.outlet_in[(Q + i) * plane + col] + lam * dbi) * inv;
  }
  const float e_prev = A.outlet_in[54 * plane + col], psi_prev = A.outlet_in[55 * plane + col];
  const float rho_prev = rho_of_psi(A.pc, e_prev, psi_prev);
  const float rr = (psi_a(psi_prev) * rho_prev + lam * rho_r) * inv;
  const float rb = (psi_b(psi_prev) * rho_prev + lam * rho_b) * inv;
  e_out = (e_prev + lam * e_b) * inv;
  psi_out = psi_encode(rr, rb, rr + rb);
}

template <typename T>
__device__ __forceinline__ void outlet_body(const AuxArgs& A, const int col) {
  const Geo& G = A.geo;
  const int plane = G.plane;
  if (col >= plane) return;
  float dr[Q], db[Q], e, psi;
  outlet_state<T>(A, col % G.nx, col / G.nx, dr, db, e, psi);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    A.outlet_out[i * plane + col] = dr[i];
    A.outlet_out[(Q + i) * plane + col] = db[i];
  }
  A.outlet_out[54 * plane + col] = e;
  A.outlet_out[55 * plane + col] = psi;
}

template <typename T>
__global__ void __launch_bounds__(256) outlet_kernel(const AuxArgs A) {
  outlet_body<T>(A, (int)(blockIdx.x * blockDim.x + threadIdx.x));
}

// The outlets of many lattices in one launch: case c owns blocks [first[c], first[c+1]);
// every case of a batch is at the same step, which is passed in.
template <typename T>
__global__ void __launch_bounds__(256)
    batch_outlet_kernel(const AuxArgs* __restrict__ cases, const int* __restrict__ first, int ncases, long long step) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = ncases;  // first[lo] <= b < first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  AuxArgs A = cases[lo];
  A.step = step;
  A.init_mode = step == 0 ? 1 : 0;
  outlet_body<T>(A, (b - first[lo]) * 256 + (int)threadIdx.x);
}

// Densities, momentum sum_i f_i c_i and (optionally) per-colour pre-collision populations of
// one cell at the current time.
template <typename T>
__device__ void cell_state(const AuxArgs& A, int x, int y, int z, float& rho, float& rho_r, float& rho_b,
                           float (&j)[3], float (&fr)[Q], float (&fb)[Q], bool want_pops) {
  const Geo& G = A.geo;
  const long long c = (long long)z * G.plane + (long long)y * G.nx + x;
  const float ar = A.pc.alpha_r, ab = A.pc.alpha_b;
  if (is_inflow(G, x, y, z)) {
    const float u = inflow_speed(G, c, A.step);
    rho = rho_r = G.rho_r0;
    rho_b = 0.0f;
    j[0] = j[1] = 0.0f;
    j[2] = G.rho_r0 * u;  // read-back reports the set velocity (no F/2 shift)
    if (want_pops) {
      static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        fr[i] = G.rho_r0 * varphi_of(i, ar) + eq_dev<i>(G.rho_r0, 0.0f, 0.0f, u);
        fb[i] = 0.0f;
      });
    }
    return;
  }
  if (A.init_mode || (G.face_hi == FACE_OUTFLOW && z == G.nz - 1)) {
    float dr[Q], db[Q], e, psi;
    if (A.init_mode) {
      float df[Q];
      init_cell<false>(A.init, A.pc, G.n, c, rho, rho_r, rho_b, e, df);
      const float ux = A.init[2 * G.n + c], uy = A.init[3 * G.n + c], uz = A.init[4 * G.n + c];
      const float r_ = rho_r, b_ = rho_b;
      static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dr[i] = eq_dev<i>(r_, ux, uy, uz);
        db[i] = eq_dev<i>(b_, ux, uy, uz);
      });
    } else {
      outlet_state<T>(A, x, y, dr, db, e, psi);
      rho = rho_of_psi(A.pc, e, psi);
      rho_r = psi_a(psi) * rho;
      rho_b = psi_b(psi) * rho;
    }
    j[0] = j[1] = j[2] = 0.0f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float d = dr[i] + db[i];
      j[0] += (float)CX[i] * d;
      j[1] += (float)CY[i] * d;
      j[2] += (float)CZ[i] * d;
      if (want_pops) {
        fr[i] = dr[i] + rho_r * varphi_of(i, ar);
        fb[i] = db[i] + rho_b * varphi_of(i, ab);
      }
    }
    return;
  }
  // bulk cell: moments exactly as the step kernel forms them, populations rebuilt per colour
  float df[Q], e;
  pull_global<T>(A, x, y, z, rho, rho_r, rho_b, e, df);
  j[0] = j[1] = j[2] = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    j[0] += (float)CX[i] * df[i];
    j[1] += (float)CY[i] * df[i];
    j[2] += (float)CZ[i] * df[i];
  }
  if (want_pops) pull_colours<T>(A, x, y, z, fr, fb);
}

__device__ __forceinline__ void body_force(const AuxArgs& A, float rho, float (&F)[3]) {
  F[0] = F[1] = F[2] = 0.0f;
  if (A.cp.force) {
    const float dr = rho - A.cp.rho_ref;
    F[0] = dr * A.cp.gx;
    F[1] = dr * A.cp.gy;
    F[2] = dr * A.cp.gz;
  }
}

// Macroscopic fields of a box: out[field][cell of box] in FP64.
template <typename T>
__global__ void __launch_bounds__(256) fields_kernel(const AuxArgs A, int x0, int y0, int z0, int wx, int wy, int wz,
                                                     double* __restrict__ out) {
  const long long nb = (long long)wx * wy * wz;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  const int x = x0 + (int)(k % wx), y = y0 + (int)((k / wx) % wy), z = z0 + (int)(k / ((long long)wx * wy));
  float rho, rho_r, rho_b, j[3], fr[Q], fb[Q];
  cell_state<T>(A, x, y, z, rho, rho_r, rho_b, j, fr, fb, false);
  float F[3];
  body_force(A, rho, F);
  if (is_inflow(A.geo, x, y, z)) F[0] = F[1] = F[2] = 0.0f;
  const double r = rho, rr = rho_r, rb = rho_b;
  out[k] = rr;
  out[nb + k] = rb;
  out[2 * nb + k] = ((double)j[0] + 0.5 * F[0]) / r;
  out[3 * nb + k] = ((double)j[1] + 0.5 * F[1]) / r;
  out[4 * nb + k] = ((double)j[2] + 0.5 * F[2]) / r;
  out[5 * nb + k] = (rr - rb) / r;
  out[6 * nb + k] = rr * 9.0 * (1.0 - (double)A.pc.alpha_r) / 19.0 + rb * 9.0 * (1.0 - (double)A.pc.alpha_b) / 19.0;
}

// Coarse-grained state: (phi, ux/u_scale, uy/u_scale, uz/u_scale) averaged over f^3 blocks of
// cells, written as FP32 into out[cz][cy][cx][4] of a padded box of pd x ph x pw voxels.
template <typename T>
__global__ void __launch_bounds__(256) coarse_kernel(const AuxArgs A, int f, float inv_u, float* __restrict__ out,
                                                     int ph, int pw) {
  const Geo& G = A.geo;
  const int cx_n = G.nx / f, cy_n = G.ny / f, cz_n = G.nz / f;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)cx_n * cy_n * cz_n) return;
  const int cx = (int)(k % cx_n), cy = (int)((k / cx_n) % cy_n), cz = (int)(k / ((long long)cx_n * cy_n));
  float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int dz = 0; dz < f; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const int x = cx * f + dx, y = cy * f + dy, z = cz * f + dz;
        float rho, rho_r, rho_b, j[3], fr[Q], fb[Q];
        cell_state<T>(A, x, y, z, rho, rho_r, rho_b, j, fr, fb, false);
        float F[3];
        body_force(A, rho, F);
        if (is_inflow(G, x, y, z)) F[0] = F[1] = F[2] = 0.0f;
        const float inv = 1.0f / rho;
        s[0] += (rho_r - rho_b) * inv;
        s[1] += (j[0] + 0.5f * F[0]) * inv * inv_u;
        s[2] += (j[1] + 0.5f * F[1]) * inv * inv_u;
        s[3] += (j[2] + 0.5f * F[2]) * inv * inv_u;
      }
  const float w = 1.0f / (float)(f * f * f);
  float4* o = reinterpret_cast<float4*>(out) + ((long long)cz * ph + cy) * pw + cx;
  *o = make_float4(s[0] * w, s[1] * w, s[2] * w, s[3] * w);
}

template <typename T>
__global__ void __launch_bounds__(256) populations_kernel(const AuxArgs A, double* __restrict__ out) {
  const Geo& G = A.geo;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.n) return;
  const int x = (int)(c % G.nx), y = (int)((c / G.nx) % G.ny), z = (int)(c / G.plane);
  float rho, rho_r, rho_b, j[3], fr[Q], fb[Q];
  cell_state<T>(A, x, y, z, rho, rho_r, rho_b, j, fr, fb, true);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    out[(long long)i * G.n + c] = fr[i];
    out[(long long)(Q + i) * G.n + c] = fb[i];
  }
}

// Diagnostics: per-block FP64 partial sums, reduced in a fixed order by a second kernel.
//   part[b] = {mass_r, mass_b, p_in, n_in, p_out, n_out, bad cells, umax}
template <typename T>
__global__ void __launch_bounds__(256) diag_kernel(const AuxArgs A, DiagQuery Qy, double* __restrict__ part) {
  const Geo& G = A.geo;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (c < G.n) {
    const int x = (int)(c % G.nx), y = (int)((c / G.nx) % G.ny), z = (int)(c / G.plane);
    float rho, rho_r, rho_b, j[3], fr[Q], fb[Q];
    cell_state<T>(A, x, y, z, rho, rho_r, rho_b, j, fr, fb, false);
    const double rr = rho_r, rb = rho_b;
    float F[3];
    body_force(A, rho, F);
    if (is_inflow(G, x, y, z)) F[0] = F[1] = F[2] = 0.0f;
    const double ux = ((double)j[0] + 0.5 * F[0]) / rho, uy = ((double)j[1] + 0.5 * F[1]) / rho,
                 uz = ((double)j[2] + 0.5 * F[2]) / rho;
    const double p = rr * 9.0 * (1.0 - (double)A.pc.alpha_r) / 19.0 + rb * 9.0 * (1.0 - (double)A.pc.alpha_b) / 19.0;
    const double dx = x - Qy.xc, dy = y - Qy.yc, dz = z - Qy.zc;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const bool bad = !(rho > 0.0f) || isnan(rho_r) || isnan(rho_b) || isnan(j[0]) || isnan(j[1]) || isnan(j[2]);
    v[0] = rr;
    v[1] = rb;
    if (r <= Qy.r_in) {
      v[2] = p;
      v[3] = 1.0;
    }
    if (r >= Qy.r_out) {
      v[4] = p;
      v[5] = 1.0;
    }
    v[6] = bad ? 1.0 : 0.0;
    v[7] = bad ? 0.0 : sqrt(ux * ux + uy * uy + uz * uz);
  }
  // wave64 butterfly reduction, then across the 4 waves through LDS
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double o = __shfl_xor(v[k], off, 64);
      v[k] = (k == 7) ? fmax(v[k], o) : v[k] + o;
    }
  }
  __shared__ double red[4][8];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0)
    for (int k = 0; k < 8; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 8) {
    const int k = threadIdx.x;
    double s = red[0][k];
    for (int w = 1; w < 4; ++w) s = (k == 7) ? fmax(s, red[w][k]) : s + red[w][k];
    part[(long long)blockIdx.x * 8 + k] = s;
  }
}

static __global__ void __launch_bounds__(256) diag_finish_kernel(const double* __restrict__ part, long long nblocks,
                                                          double* __restrict__ out) {
  // fixed-order reduction: thread t sums blocks t, t+256, ...; then a tree over threads
  __shared__ double red[256][8];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long b = threadIdx.x; b < nblocks; b += 256)
    for (int k = 0; k < 8; ++k) v[k] = (k == 7) ? fmax(v[k], part[b * 8 + k]) : v[k] + part[b * 8 + k];
  for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = v[k];
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 8; ++k)
        red[threadIdx.x][k] = (k == 7) ? fmax(red[threadIdx.x][k], red[threadIdx.x + s][k])
                                       : red[threadIdx.x][k] + red[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x < 8) out[threadIdx.x] = red[0][threadIdx.x];
}

// ================================================================== launchers (per storage type)
template <typename T>
hipError_t launch_outlet_T(const AuxArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.geo.plane + 255) / 256);
  hipLaunchKernelGGL(outlet_kernel<T>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_outlet_T(const AuxArgs* cases, const int* first, int ncases, int nblocks, long long step,
                                 hipStream_t s) {
  hipLaunchKernelGGL(batch_outlet_kernel<T>, dim3((unsigned)nblocks), dim3(256), 0, s, cases, first, ncases, step);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fields_T(const AuxArgs& a, int x0, int y0, int z0, int wx, int wy, int wz, double* out,
                           hipStream_t s) {
  const long long nb = (long long)wx * wy * wz;
  hipLaunchKernelGGL(fields_kernel<T>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, a, x0, y0, z0, wx, wy, wz,
                     out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_T(const AuxArgs& a, int f, float inv_u, float* out, int ph, int pw, hipStream_t s) {
  const long long nb = (long long)(a.geo.nx / f) * (a.geo.ny / f) * (a.geo.nz / f);
  hipLaunchKernelGGL(coarse_kernel<T>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, a, f, inv_u, out, ph, pw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_populations_T(const AuxArgs& a, double* out, hipStream_t s) {
  hipLaunchKernelGGL(populations_kernel<T>, dim3((unsigned)((a.geo.n + 255) / 256)), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_diag_T(const AuxArgs& a, const DiagQuery& q, double* part, long long nblocks, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(diag_kernel<T>, dim3((unsigned)nblocks), dim3(256), 0, s, a, q, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(256), 0, s, part, nblocks, out);
  return hipGetLastError();
}

#define LBM_INSTANTIATE_STORAGE(T)                                                                                \
  template hipError_t launch_outlet_T<T>(const AuxArgs&, hipStream_t);                                            \
  template hipError_t launch_batch_outlet_T<T>(const AuxArgs*, const int*, int, int, long long, hipStream_t);                                            \
  template hipError_t launch_fields_T<T>(const AuxArgs&, int, int, int, int, int, int, double*, hipStream_t);    \
  template hipError_t launch_populations_T<T>(const AuxArgs&, double*, hipStream_t);                              \
  template hipError_t launch_coarse_T<T>(const AuxArgs&, int, float, float*, int, int, hipStream_t);             \
  template hipError_t launch_diag_T<T>(const AuxArgs&, const DiagQuery&, double*, long long, double*, hipStream_t);

}  // namespace lbm
