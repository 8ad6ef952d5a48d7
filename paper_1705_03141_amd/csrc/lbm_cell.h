// lbm_cell.h -- per-cell arithmetic of the D3Q27 colour-fluid step (Sec. II of Saito,
// Abe & Koyama 2017), written for the GPU and usable from host code for self-checks.
//
// Representation.  The collision works on deviations from the local rest equilibrium:
//   df_i = f_i - rho varphi_i(alpha_bar),  since  sum_k rho_k varphi_i(alpha_k) = rho varphi_i(alpha_bar)
// with alpha_bar = ((1+phi) alpha_r + (1-phi) alpha_b)/2 (Eq. (varphi_ik) is linear in alpha),
// so every quantity the transforms touch is O(u) and keeps FP32 precision.
//
// Moment transform.  The orthogonal moment matrix M of Eq. (momentSet) factors as
// M = P T: T is the tensor product of the 1-D map (f(-1), f(0), f(1)) ->
// (f(-1)+f(0)+f(1), f(1)-f(-1), f(-1)-2f(0)+f(1)), the orthogonal polynomials 1, c, 3c^2-2;
// P is sparse (43 non-zeros) and well conditioned.  Rows of M and of T are orthogonal, so
// M^-1 = M^T D^-1 = T^T P^T D^-1 with D_j the squared row norms of M.  A collision costs two
// ~110-flop separable passes plus ~150 flops for P, P^T and the relaxation instead of two
// dense 27x27 products.
//
// The equilibrium (Eqs. (EES), (Phi)), the forcing (Eq. (ketFd)) and the perturbation
// (Eq. (perturb), with the square on c_i . n) enter through their moments in the basis of
// Eq. (momentSet): short closed forms in (rho, u, grad rho, F, n).
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

constexpr int Q = 27;

// Lattice velocities of Eq. (velSet) in the paper's numbering (index 0 = paper's i = 1),
// the numbering fixed by rows 2-4 of the matrix in Appendix A.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};

__host__ __device__ constexpr int shell_of(int i) { return CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]; }

// Index of the velocity (cx, cy, cz).
__host__ __device__ constexpr int dir_of(int cx, int cy, int cz) {
  int r = 0;
  for (int i = 0; i < Q; ++i)
    if (CX[i] == cx && CY[i] == cy && CZ[i] == cz) r = i;
  return r;
}
__host__ __device__ constexpr int opposite(int i) { return dir_of(-CX[i], -CY[i], -CZ[i]); }
__host__ __device__ constexpr int mirror_x(int i) { return dir_of(-CX[i], CY[i], CZ[i]); }
__host__ __device__ constexpr int mirror_y(int i) { return dir_of(CX[i], -CY[i], CZ[i]); }
__host__ __device__ constexpr int mirror_z(int i) { return dir_of(CX[i], CY[i], -CZ[i]); }

// varphi_i(alpha) = (1 - alpha) q_i for i >= 1 (Eq. (varphi_ik)); q = 2/19, 1/38, 1/152 by shell.
__host__ __device__ constexpr float q_of(int i) {
  return shell_of(i) == 1 ? 2.0f / 19.0f : (shell_of(i) == 2 ? 1.0f / 38.0f : (shell_of(i) == 3 ? 1.0f / 152.0f : 0.0f));
}
// q_i / |c_i|: cos(theta_i) of the recolouring operator carries 1/|c_i|.
__host__ __device__ constexpr float qc_of(int i) {
  return shell_of(i) == 1 ? 2.0f / 19.0f
                          : (shell_of(i) == 2 ? 0.01860807318959f   /* 1/(38 sqrt 2)  */
                                              : (shell_of(i) == 3 ? 0.00379839255f /* 1/(152 sqrt 3) */ : 0.0f));
}
// Lattice weights w_i.
__host__ __device__ constexpr float w_of(int i) {
  return shell_of(i) == 0 ? 8.0f / 27.0f
                          : (shell_of(i) == 1 ? 2.0f / 27.0f : (shell_of(i) == 2 ? 1.0f / 54.0f : 1.0f / 216.0f));
}

// Reciprocal and reciprocal square root: the hardware's 1-ulp instructions on the GPU (the
// IEEE-rounded division costs about ten instructions), plain division on the host.
__host__ __device__ __forceinline__ float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ float rsq(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}

// 1 - alpha_bar of a cell with colour fractions (a, b), a + b = 1, from the minority one:
// (1 - alpha_b) - a dalpha where blue is the majority, (1 - alpha_r) + b dalpha where red is.
// The majority fraction is 1 minus a rounded number; near pure red its rounding would be
// amplified by 1/(1 - alpha_r) = gamma/(1 - alpha_b) (about 14 at gamma = 10).
__host__ __device__ __forceinline__ float one_minus_abar(float a, float b, float dalpha, float one_m_ab,
                                                         float one_m_ar) {
  return a <= b ? fmaf(-a, dalpha, one_m_ab) : fmaf(b, dalpha, one_m_ar);
}

// Per-run constants of the collision.
struct CollideParams {
  float alpha_r, alpha_b;  // alpha_b = 8/27; alpha_r = 1 - (1 - alpha_b)/gamma
  float dalpha, one_m_ab, one_m_ar;  // alpha_r - alpha_b, 1 - alpha_b, 1 - alpha_r (from FP64)
  float nu_r, nu_b;
  float A, beta;
  float gx, gy, gz, rho_ref;  // body force F = (rho - rho_ref) g when force != 0
  int force;
};

// One collided cell: stored deviations and the per-cell scalars readers need.
struct CellOut {
  float g[Q];        // df''_i = f''_i - rho varphi_i(alpha_bar)
  float rho;         // rho of the cell
  float a;           // rho_r / rho
  float wx, wy, wz;  // beta (rho_r rho_b / rho) (1 - alpha_bar) n
};

// ---------------------------------------------------------------- separable moment transform
// Tensor-product orthogonal moments Q_abc = sum_i f_i t_a(cx) t_b(cy) t_c(cz) with the 1-D
// polynomials t_0 = 1, t_1 = c, t_2 = 3c^2 - 2, which are orthogonal on c in {-1, 0, 1}.
// Unlike raw moments (1, c, c^2) this basis is well conditioned: the map to the moment set
// of Eq. (momentSet) has condition number 3, and most of its rows are single Q_abc.
// v[z][y][x] holds the value at velocity (x-1, y-1, z-1); in place it becomes Q[c][b][a].
__host__ __device__ inline void orth_forward(float (&v)[3][3][3]) {
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const float s = v[z][y][2] + v[z][y][0], d = v[z][y][2] - v[z][y][0], c0 = v[z][y][1];
      v[z][y][0] = s + c0;
      v[z][y][1] = d;
      v[z][y][2] = s - 2.0f * c0;
    }
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const float s = v[z][2][x] + v[z][0][x], d = v[z][2][x] - v[z][0][x], c0 = v[z][1][x];
      v[z][0][x] = s + c0;
      v[z][1][x] = d;
      v[z][2][x] = s - 2.0f * c0;
    }
#pragma unroll
  for (int y = 0; y < 3; ++y)
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const float s = v[2][y][x] + v[0][y][x], d = v[2][y][x] - v[0][y][x], c0 = v[1][y][x];
      v[0][y][x] = s + c0;
      v[1][y][x] = d;
      v[2][y][x] = s - 2.0f * c0;
    }
}

// Evaluation of sum_abc Y[c][b][a] t_a(cx) t_b(cy) t_c(cz) at the 27 velocities; in place,
// the value at velocity (x-1, y-1, z-1) lands in Y[z][y][x].
__host__ __device__ inline void orth_evaluate(float (&k)[3][3][3]) {
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const float k0 = k[z][y][0], k1 = k[z][y][1], k2 = k[z][y][2], t = k0 + k2;
      k[z][y][0] = t - k1;
      k[z][y][1] = k0 - 2.0f * k2;
      k[z][y][2] = t + k1;
    }
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const float k0 = k[z][0][x], k1 = k[z][1][x], k2 = k[z][2][x], t = k0 + k2;
      k[z][0][x] = t - k1;
      k[z][1][x] = k0 - 2.0f * k2;
      k[z][2][x] = t + k1;
    }
#pragma unroll
  for (int y = 0; y < 3; ++y)
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const float k0 = k[0][y][x], k1 = k[1][y][x], k2 = k[2][y][x], t = k0 + k2;
      k[0][y][x] = t - k1;
      k[1][y][x] = k0 - 2.0f * k2;
      k[2][y][x] = t + k1;
    }
}

// Moments m = P Q of Eq. (momentSet), 0-based rows, from the tensor moments Q[c][b][a].
#define LBM_Q(a, b, c) Qm[c][b][a]
__host__ __device__ inline void orth_to_moments(const float (&Qm)[3][3][3], float (&m)[Q]) {
  const float third = 1.0f / 3.0f;
  const float q200 = LBM_Q(2, 0, 0), q020 = LBM_Q(0, 2, 0), q002 = LBM_Q(0, 0, 2);
  const float q220 = LBM_Q(2, 2, 0), q202 = LBM_Q(2, 0, 2), q022 = LBM_Q(0, 2, 2);
  const float q120 = LBM_Q(1, 2, 0), q102 = LBM_Q(1, 0, 2), q210 = LBM_Q(2, 1, 0), q012 = LBM_Q(0, 1, 2);
  const float q201 = LBM_Q(2, 0, 1), q021 = LBM_Q(0, 2, 1);
  m[0] = LBM_Q(0, 0, 0);
  m[1] = LBM_Q(1, 0, 0);
  m[2] = LBM_Q(0, 1, 0);
  m[3] = LBM_Q(0, 0, 1);
  m[4] = (q200 + q020 + q002) * third;
  m[5] = (2.0f * q200 - q020 - q002) * third;
  m[6] = (q020 - q002) * third;
  m[7] = LBM_Q(1, 1, 0);
  m[8] = LBM_Q(0, 1, 1);
  m[9] = LBM_Q(1, 0, 1);
  m[10] = q120 + q102;
  m[11] = q210 + q012;
  m[12] = q201 + q021;
  m[13] = LBM_Q(1, 2, 2);
  m[14] = LBM_Q(2, 1, 2);
  m[15] = LBM_Q(2, 2, 1);
  m[16] = (q220 + q202 + q022) * third;
  m[17] = LBM_Q(2, 2, 2);
  m[18] = (q220 + q202 - 2.0f * q022) * third;
  m[19] = (q220 - q202) * third;
  m[20] = LBM_Q(1, 1, 2);
  m[21] = LBM_Q(2, 1, 1);
  m[22] = LBM_Q(1, 2, 1);
  m[23] = (q120 - q102) * third;
  m[24] = (q012 - q210) * third;
  m[25] = (q201 - q021) * third;
  m[26] = LBM_Q(1, 1, 1);
}

// Tensor coefficients Y = P^T y (transpose of orth_to_moments), into Qm[c][b][a].
__host__ __device__ inline void moments_to_orth(const float (&y)[Q], float (&Qm)[3][3][3]) {
  const float third = 1.0f / 3.0f;
  LBM_Q(0, 0, 0) = y[0];
  LBM_Q(1, 0, 0) = y[1];
  LBM_Q(0, 1, 0) = y[2];
  LBM_Q(0, 0, 1) = y[3];
  LBM_Q(2, 0, 0) = (y[4] + 2.0f * y[5]) * third;
  LBM_Q(0, 2, 0) = (y[4] - y[5] + y[6]) * third;
  LBM_Q(0, 0, 2) = (y[4] - y[5] - y[6]) * third;
  LBM_Q(1, 1, 0) = y[7];
  LBM_Q(0, 1, 1) = y[8];
  LBM_Q(1, 0, 1) = y[9];
  LBM_Q(1, 2, 0) = y[10] + y[23] * third;
  LBM_Q(1, 0, 2) = y[10] - y[23] * third;
  LBM_Q(2, 1, 0) = y[11] - y[24] * third;
  LBM_Q(0, 1, 2) = y[11] + y[24] * third;
  LBM_Q(2, 0, 1) = y[12] + y[25] * third;
  LBM_Q(0, 2, 1) = y[12] - y[25] * third;
  LBM_Q(1, 2, 2) = y[13];
  LBM_Q(2, 1, 2) = y[14];
  LBM_Q(2, 2, 1) = y[15];
  LBM_Q(2, 2, 0) = (y[16] + y[18] + y[19]) * third;
  LBM_Q(2, 0, 2) = (y[16] + y[18] - y[19]) * third;
  LBM_Q(0, 2, 2) = (y[16] - 2.0f * y[18]) * third;
  LBM_Q(2, 2, 2) = y[17];
  LBM_Q(1, 1, 2) = y[20];
  LBM_Q(2, 1, 1) = y[21];
  LBM_Q(1, 2, 1) = y[22];
  LBM_Q(1, 1, 1) = y[26];
}
#undef LBM_Q

// 1 / D_j, D_j = squared norm of row j of M.
__host__ __device__ constexpr float inv_norm(int j) {
  constexpr float D[Q] = {27, 18, 18, 18, 18, 36, 12, 12, 12, 12, 72, 72, 72, 72,
                          72, 72, 36, 216, 72, 24, 24, 24, 24, 8, 8, 8, 8};
  return 1.0f / D[j];
}

// The perturbation and the recolouring segregation need the interface normal, which exists
// wherever grad phi != 0 (Sec. II; where grad phi = 0 both are zero, reading R7).  At a point
// of exact symmetry the computed gradient is rounding noise whose direction the fields do not
// define.  grad phi comes from the cell's minority colour fraction t (phi = 2a - 1 = 1 - 2b),
// whose FP32 rounding is a few ulps of t, so the noise is ~1e-7 t: the normal is taken as
// defined where |grad phi| > 2 kNormalRel t, about 250 ulps of t above that noise, and where
// |grad phi|^2 is a normal FP32 number (the reciprocal square root is taken of it).  The
// cells this excludes besides the FP32 noise change the FP64 solution by less than 1e-12 on
// the parity problems (measured against the absolute 1e-12 cut-off of an FP64 evaluation).
constexpr float kNormalRel = 1.52587890625e-5f;  // 2^-16
constexpr float kGradPhi2Min = 1.17549435e-38f;  // 2^-126

// Relaxation rates of the moment groups of K (Sec. II): rows 1-4 are conserved (s1 = 0),
// rows 6-10 take the local s_nu; the others share one rate per group.
struct GroupRates {
  float s5, s11, s14, s17, s18, s19, s21, s24, s27;
};

// Collision, perturbation and the recolouring scalars of one cell.
//   d[i], shift, drho pre-collision deviations in the reader's form: the total deviation is
//                     df_i = d_i + q_i shift (i >= 1), df_0 = -sum_{i>=1} df_i, i.e. d is taken
//                     from the rest equilibrium of the previous state and shift, drho move it to
//                     the present one.  The shift is applied to the moments (rows 0, 4, 16, 17)
//                     instead of to each population, which keeps one rounding off every value.
//   rho, rho_r, rho_b densities of time t (rho_b passed separately: it may be far below the
//                     rounding of rho - rho_r)
//   gp, gr            grad phi and grad rho from the isotropic stencil
// Writes df''_i = f''_i - rho varphi_i(alpha_bar) and (rho, rho_r/rho, w) into out.
//
// In the orthogonal basis the operator of Eqs. (scoll), (ketF), (perturb) is
//   m*_j = m_j - s_j (m_j - meq_j) + (1 - s_j/2) mF_j + G mP_j,
// with meq = M (f_eq - rho varphi(alpha_bar)) from Eqs. (EES), (Phi), mF = M F' from
// Eq. (ketFd) and G mP = M Omega2 from Eq. (perturb), each a closed form of
// (rho, u, grad rho, F, n) obtained by applying the rows of Eq. (momentSet) to them.
template <int OUT_SHIFT = 0>
__host__ __device__ inline void collide_cell(const CollideParams& P, const GroupRates& S, const float (&df)[Q],
                                             float shift, float drho, float rho, float rho_r, float rho_b,
                                             const float (&gp)[3], const float (&gr)[3], CellOut& out) {
  float m[Q];
  {
    float R[3][3][3];
#pragma unroll
    for (int i = 0; i < Q; ++i) R[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = df[i];
    orth_forward(R);
    orth_to_moments(R, m);
  }
  // moments of (q_i shift, i >= 1; -(drho + shift), i = 0): isotropic rows only
  m[0] -= drho;
  m[4] += (27.0f / 19.0f) * shift + 2.0f * drho;
  m[16] += -(81.0f / 19.0f) * shift - 4.0f * drho;
  m[17] += (189.0f / 19.0f) * shift + 8.0f * drho;
  const float inv_rho = rcp(rho);
  const float a = rho_r * inv_rho;
  float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
  if (P.force) {
    const float dr = rho - P.rho_ref;
    Fx = dr * P.gx;
    Fy = dr * P.gy;
    Fz = dr * P.gz;
  }
  // Eq. (Momentum): rho u = sum_i f_i c_i + F/2 (the rest equilibrium carries no momentum).
  const float rux = m[1] + 0.5f * Fx, ruy = m[2] + 0.5f * Fy, ruz = m[3] + 0.5f * Fz;
  const float ux = rux * inv_rho, uy = ruy * inv_rho, uz = ruz * inv_rho;
  const float nu = P.nu_b + a * (P.nu_r - P.nu_b);  // (1 + phi)/2 = rho_r/rho
  const float snu = rcp(3.0f * nu + 0.5f);          // Eq. (shear)

  // Perturbation strength G = A |grad phi| and the interface normal n.
  const float g2 = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2];
  const float cut = (2.0f * kNormalRel) * (fminf(rho_r, rho_b) * inv_rho);
  float nx = 0.0f, ny = 0.0f, nz = 0.0f, G = 0.0f;
  if (g2 >= kGradPhi2Min && g2 > cut * cut) {
    const float inv = rsq(g2);
    nx = gp[0] * inv;
    ny = gp[1] * inv;
    nz = gp[2] * inv;
    G = P.A * g2 * inv;
  }

  // equilibrium moments (deviation part)
  const float ug = ux * gr[0] + uy * gr[1] + uz * gr[2];
  const float ruu = rux * ux + ruy * uy + ruz * uz;
  const float pxx = rux * ux + nu * 2.0f * ux * gr[0], pyy = ruy * uy + nu * 2.0f * uy * gr[1],
              pzz = ruz * uz + nu * 2.0f * uz * gr[2];
  const float eq4 = ruu + 5.0f * nu * ug;
  const float eq5 = 2.0f * pxx - pyy - pzz;
  const float eq6 = pyy - pzz;
  const float eq7 = rux * uy + nu * (ux * gr[1] + uy * gr[0]);
  const float eq8 = ruy * uz + nu * (uy * gr[2] + uz * gr[1]);
  const float eq9 = rux * uz + nu * (ux * gr[2] + uz * gr[0]);
  const float eq16 = -2.0f * ruu - 13.0f * nu * ug;
  const float eq17 = 3.0f * ruu + 27.0f * nu * ug;
  // forcing moments
  const float fxx = ux * Fx, fyy = uy * Fy, fzz = uz * Fz, uF = fxx + fyy + fzz;
  const float fo5 = 2.0f * (2.0f * fxx - fyy - fzz), fo6 = 2.0f * (fyy - fzz);
  const float fo7 = ux * Fy + uy * Fx, fo8 = uy * Fz + uz * Fy, fo9 = ux * Fz + uz * Fx;
  // perturbation moments, times G
  const float k9 = (2.0f / 9.0f) * G;
  const float pe5 = k9 * (3.0f * nx * nx - 1.0f), pe6 = k9 * (ny * ny - nz * nz);
  const float pe7 = k9 * nx * ny, pe8 = k9 * ny * nz, pe9 = k9 * nx * nz;

  float y[Q];
  // the outputs come out times 2^OUT_SHIFT (the storage scale of FP16), folded into 1/D_j
  constexpr float os = (float)(1 << OUT_SHIFT);
  // conserved: mass, momentum (+F)
  y[0] = m[0] * (inv_norm(0) * os);
  y[1] = (m[1] + Fx) * (inv_norm(1) * os);
  y[2] = (m[2] + Fy) * (inv_norm(2) * os);
  y[3] = (m[3] + Fz) * (inv_norm(3) * os);
#define LBM_RELAX(j, s, eq, fo, pe) y[j] = (m[j] - (s) * (m[j] - (eq)) + (1.0f - 0.5f * (s)) * (fo) + (pe)) * (inv_norm(j) * os)
  LBM_RELAX(4, S.s5, eq4, 2.0f * uF, -(4.0f / 9.0f) * G);
  LBM_RELAX(5, snu, eq5, fo5, pe5);
  LBM_RELAX(6, snu, eq6, fo6, pe6);
  LBM_RELAX(7, snu, eq7, fo7, pe7);
  LBM_RELAX(8, snu, eq8, fo8, pe8);
  LBM_RELAX(9, snu, eq9, fo9, pe9);
  LBM_RELAX(10, S.s11, -2.0f * rux, -2.0f * Fx, 0.0f);
  LBM_RELAX(11, S.s11, -2.0f * ruy, -2.0f * Fy, 0.0f);
  LBM_RELAX(12, S.s11, -2.0f * ruz, -2.0f * Fz, 0.0f);
  LBM_RELAX(13, S.s14, rux, Fx, 0.0f);
  LBM_RELAX(14, S.s14, ruy, Fy, 0.0f);
  LBM_RELAX(15, S.s14, ruz, Fz, 0.0f);
  LBM_RELAX(16, S.s17, eq16, -4.0f * uF, (14.0f / 9.0f) * G);
  LBM_RELAX(17, S.s18, eq17, 6.0f * uF, -4.0f * G);
  LBM_RELAX(18, S.s19, -eq5, -fo5, -pe5);
  LBM_RELAX(19, S.s19, -eq6, -fo6, -pe6);
  LBM_RELAX(20, S.s21, -eq7, -fo7, -pe7);
  LBM_RELAX(21, S.s21, -eq8, -fo8, -pe8);
  LBM_RELAX(22, S.s21, -eq9, -fo9, -pe9);
  LBM_RELAX(23, S.s24, 0.0f, 0.0f, 0.0f);
  LBM_RELAX(24, S.s24, 0.0f, 0.0f, 0.0f);
  LBM_RELAX(25, S.s24, 0.0f, 0.0f, 0.0f);
  LBM_RELAX(26, S.s27, 0.0f, 0.0f, 0.0f);
#undef LBM_RELAX

  float K[3][3][3];
  moments_to_orth(y, K);
  orth_evaluate(K);
#pragma unroll
  for (int i = 0; i < Q; ++i) out.g[i] = K[CZ[i] + 1][CY[i] + 1][CX[i] + 1];

  // Mass and momentum of the result are fixed by the conserved rows (m0, m1 + F): remove the
  // rounding the two transforms left in them.  Momentum is summed from differences of
  // opposite populations, which are exact for the nearly symmetric O(1e-3) deviations of an
  // interface; the defect goes to the axis pairs, the mass defect to the rest population.
  {
    float jx = 0.0f, jy = 0.0f, jz = 0.0f, mass = 0.0f;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const float d = out.g[i] - out.g[i + 1];  // populations i and i+1 are opposite
      if (CX[i] != 0) jx += (float)CX[i] * d;
      if (CY[i] != 0) jy += (float)CY[i] * d;
      if (CZ[i] != 0) jz += (float)CZ[i] * d;
    }
    const float hx = 0.5f * ((m[1] + Fx) * os - jx), hy = 0.5f * ((m[2] + Fy) * os - jy),
                hz = 0.5f * ((m[3] + Fz) * os - jz);
    out.g[1] += hx;
    out.g[2] -= hx;
    out.g[3] += hy;
    out.g[4] -= hy;
    out.g[5] += hz;
    out.g[6] -= hz;
#pragma unroll
    for (int i = 1; i < Q; ++i) mass += out.g[i];
    out.g[0] = m[0] * os - mass;
  }

  // Recolouring (Latva-Kokko & Rothman), carried to the readers as rho_r/rho and
  // w = beta (rho_r rho_b / rho) (1 - alpha_bar) n; f^r_i = (rho_r/rho) f''_i + (q_i/|c_i|) c_i . w.
  const float wmag = P.beta * rho_r * rho_b * inv_rho *
                     one_minus_abar(a, rho_b * inv_rho, P.dalpha, P.one_m_ab, P.one_m_ar);
  out.rho = rho;
  out.a = a;
  out.wx = wmag * nx;
  out.wy = wmag * ny;
  out.wz = wmag * nz;
}

}  // namespace lbm
