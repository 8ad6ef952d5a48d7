/*
 * lbm_oracle.c -- plain FP64 CPU reference ("the oracle") for the D3Q27 colour-fluid
 * lattice Boltzmann time step of Saito, Abe & Koyama, "Lattice Boltzmann modeling and
 * simulation of liquid jet breakup", Phys. Rev. E 96, 013317 (2017), arXiv:1705.03141.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this file's library.  It shares no code, header, table or helper
 * with the HIP implementation; the two meet only through seeded input fields.
 *
 * Everything is written the obvious way: the 27x27 moment matrix is evaluated from the
 * moment polynomials of Eq. (momentSet), its inverse is obtained by Gauss-Jordan
 * elimination, and the collision is four dense 27x27 matrix-vector products per cell.
 * Every per-cell operation follows the equation it cites, in the order of Sec. II:
 * single-phase MRT collision with enhanced equilibrium and forcing, then the perturbation
 * operator, then recolouring, then streaming.  OpenMP only splits the loop over cells.
 *
 * Readings of points the paper leaves open (numbered as in the design notes):
 *   R1  initial populations: per-colour equilibrium, Eq. (EES) with Phi = 0.
 *   R2  gradients use the densities of time t (post-streaming, pre-collision).
 *   R3  the collision acts on the total f_i = f^r_i + f^b_i with sum_k Phi^k = Phi(grad rho);
 *       the colours enter through rho_k, phi and grad phi only.
 *   R4  the forcing term |F> is added once, to the total.
 *   R5  the perturbation operator carries the square (c_i . grad phi)^2 / |grad phi|^2,
 *       without which it does not conserve mass.
 *   R6  A is a run constant, A_r = A_b = A.
 *   R7  cos(theta_1) = 0 for the rest velocity.  Both the perturbation and the recolouring
 *       segregation need the interface normal grad phi / |grad phi|, which exists wherever
 *       grad phi != 0; where grad phi = 0 both are zero (the perturbation is continuous
 *       there; the segregation term is 0/0).  At a symmetry point the exact gradient is 0
 *       but the FP64 one is rounding noise of ~1e-17 with an arbitrary direction, so the
 *       normal is taken as undefined where |grad phi| <= gphi_cut, set at the FP64 noise
 *       floor (1e-12 by the test wrapper); results do not change when it moves by 100x.
 *   R8  no-slip walls are half-way bounce-back, per colour; walls lie half a cell outside
 *       the first/last plane.  Gradient stencils see a ghost layer equal to the adjacent
 *       cell (zero normal gradient).
 *   R9  free-slip walls are half-way specular reflection, per colour; same ghost rule.
 *   R10 inflow sites (plane z = 0, inside the disk) are not collided; each step they emit
 *       the red equilibrium f^r(e)(rho_r0, u_in e_z, alpha_r) with Phi = 0 and no blue.
 *       Their densities are (rho_r0, 0) for the stencils of their neighbours.
 *   R11 convective outflow on the last z plane (Lou et al.): after streaming the whole
 *       plane is overwritten with [f(N,t) + lambda f(N-1,t+1)]/(1+lambda) per colour and
 *       direction, lambda = max(0, u_z(N-1, t+1)).  f(N,t) is the plane's pre-collision
 *       state of the previous step.
 *   R12 body force F = (rho - rho_ref) g (the printed RT form with g = (0,0,-g) is
 *       F = (rho - rho_bar)(0,0,+g)); the caller places the heavy fluid accordingly.
 *   R23 inflow velocity noise: u_in = u0 (1 + eps xi), xi uniform on [-1,1) from the
 *       SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014) evaluated as a
 *       counter-based hash of (seed, step * ncells + cell).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 27

enum { FACE_PERIODIC = 0, FACE_BOUNCEBACK = 1, FACE_FREESLIP = 2, FACE_OUTFLOW = 3 };

/* Lattice velocities of Eq. (velSet).  The numbering i = 1..27 of the paper is fixed by
 * rows 2-4 of the matrix printed in Appendix A (they list c_ix, c_iy, c_iz column by
 * column); index 0 here is the paper's i = 1. */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {0, 1, 1},   {0, -1, -1},
    {0, 1, -1},  {0, -1, 1},  {1, 0, 1},   {-1, 0, -1}, {-1, 0, 1},  {1, 0, -1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {-1, 1, 1},  {1, -1, -1},
    {1, -1, 1},  {-1, 1, -1}};

typedef struct {
  int nx, ny, nz;
  double rho_r0, rho_b0; /* reference densities of the two fluids, gamma = rho_r0/rho_b0 */
  double nu_r, nu_b;     /* kinematic viscosities */
  double A;              /* surface-tension parameter of Eq. (perturb) */
  double beta;           /* recolouring parameter */
  double s[Q];           /* relaxation rates; all zero selects Suga's set (Sec. II) */
  int face[6];           /* -x,+x,-y,+y,-z,+z: FACE_* */
  int force_model;       /* 0: none, 1: F = (rho - rho_ref) g */
  double g[3];
  double rho_ref;
  int inflow;            /* 1: inflow disk on the z = 0 plane */
  double xc, yc, diameter, u_in, noise_rel;
  unsigned long long seed;
  int gnx, gny, gnz;     /* dimensions of the whole domain the noise counter refers to */
  int ox, oy, oz;        /* origin of this lattice inside that domain */
  double gphi_cut;       /* R7: no normal where |grad phi| <= gphi_cut (FP64 noise floor) */
} oracle_params;

typedef struct {
  oracle_params p;
  long n;
  int dir_of[3][3][3];      /* velocity index of (cx,cy,cz) + 1 */
  double alpha_r, alpha_b;
  double M[Q][Q], Minv[Q][Q];
  double *f, *fpost, *fnew; /* [colour][i][cell] */
  double *rr, *rb;          /* per-cell densities of the current step */
  double *outlet;           /* [colour][i][nx*ny]: outlet plane, previous step */
  unsigned char *inflow;    /* per cell: 1 if an inflow site */
  long long step;
} oracle;

/* ---------------------------------------------------------------- lattice constants */

static int shell(int i) { return CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2]; }

/* Weights w_i (Sec. II, after Eq. (EES)). */
static double weight(int i) {
  static const double w[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
  return w[shell(i)];
}

/* varphi_i^k of Eq. (varphi_ik) for a colour with parameter alpha. */
static double varphi(int i, double alpha) {
  switch (shell(i)) {
    case 0: return alpha;
    case 1: return 2.0 * (1.0 - alpha) / 19.0;
    case 2: return (1.0 - alpha) / 38.0;
    default: return (1.0 - alpha) / 152.0;
  }
}

/* B_i of Eq. (B_i), c = 1. */
static double Bcoef(int i) {
  static const double b[4] = {-10.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
  return b[shell(i)];
}

/* Row j (0-based) of the moment set Eq. (momentSet) evaluated at velocity c. */
static double moment_poly(int j, const int *c) {
  const double x = c[0], y = c[1], z = c[2];
  const double x2 = x * x, y2 = y * y, z2 = z * z, c2 = x2 + y2 + z2;
  switch (j) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return -2.0 + c2;
    case 5: return 2.0 * x2 - (y2 + z2);
    case 6: return y2 - z2;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return -4.0 * x + 3.0 * (x * y2 + z2 * x);
    case 11: return -4.0 * y + 3.0 * (y * z2 + x2 * y);
    case 12: return -4.0 * z + 3.0 * (z * x2 + y2 * z);
    case 13: return 4.0 * x - 6.0 * (x * y2 + z2 * x) + 9.0 * (x * y2 * z2);
    case 14: return 4.0 * y - 6.0 * (y * z2 + x2 * y) + 9.0 * (x2 * y * z2);
    case 15: return 4.0 * z - 6.0 * (z * x2 + y2 * z) + 9.0 * (x2 * y2 * z);
    case 16: return 4.0 * (1.0 - c2) + 3.0 * (x2 * y2 + y2 * z2 + z2 * x2);
    case 17: return -8.0 + 12.0 * c2 - 18.0 * (x2 * y2 + y2 * z2 + z2 * x2) + 27.0 * (x2 * y2 * z2);
    case 18: return 2.0 * (z2 + y2) + 3.0 * (x2 * y2 + z2 * x2) - 4.0 * x2 - 6.0 * (y2 * z2);
    case 19: return 2.0 * (z2 - y2) + 3.0 * (x2 * y2 - z2 * x2);
    case 20: return -2.0 * x * y + 3.0 * (x * y * z2);
    case 21: return -2.0 * y * z + 3.0 * (x2 * y * z);
    case 22: return -2.0 * z * x + 3.0 * (x * y2 * z);
    case 23: return x * y2 - z2 * x;
    case 24: return y * z2 - x2 * y;
    case 25: return z * x2 - y2 * z;
    default: return x * y * z;
  }
}

static void build_moment_matrix(double M[Q][Q]) {
  for (int j = 0; j < Q; j++)
    for (int i = 0; i < Q; i++) M[j][i] = moment_poly(j, CV[i]);
}

/* Gauss-Jordan inversion with partial pivoting; returns 0 on success. */
static int invert(int n, const double *a, double *ainv) {
  double *w = (double *)malloc(sizeof(double) * n * 2 * n);
  if (!w) return -1;
  for (int r = 0; r < n; r++)
    for (int c = 0; c < 2 * n; c++) w[r * 2 * n + c] = c < n ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int col = 0; col < n; col++) {
    int piv = col;
    for (int r = col + 1; r < n; r++)
      if (fabs(w[r * 2 * n + col]) > fabs(w[piv * 2 * n + col])) piv = r;
    if (fabs(w[piv * 2 * n + col]) < 1e-300) { free(w); return -1; }
    if (piv != col)
      for (int c = 0; c < 2 * n; c++) {
        double t = w[col * 2 * n + c]; w[col * 2 * n + c] = w[piv * 2 * n + c]; w[piv * 2 * n + c] = t;
      }
    const double d = w[col * 2 * n + col];
    for (int c = 0; c < 2 * n; c++) w[col * 2 * n + c] /= d;
    for (int r = 0; r < n; r++) {
      if (r == col) continue;
      const double m = w[r * 2 * n + col];
      if (m != 0.0)
        for (int c = 0; c < 2 * n; c++) w[r * 2 * n + c] -= m * w[col * 2 * n + c];
    }
  }
  for (int r = 0; r < n; r++)
    for (int c = 0; c < n; c++) ainv[r * n + c] = w[r * 2 * n + n + c];
  free(w);
  return 0;
}

/* Diagonal of the relaxation matrix K (Sec. II): rates for the 27 moment rows.  Rows
 * 6-10 (1-based) carry the local shear rate s_nu = 1/(3 nu + 1/2) from Eq. (shear). */
static void relaxation_diag(const double *s_user, double snu, double K[Q]) {
  int user = 0;
  for (int j = 0; j < Q; j++) user |= (s_user[j] != 0.0);
  if (user) {
    for (int j = 0; j < Q; j++) K[j] = s_user[j];
  } else {
    const double s1 = 0.0, s5 = 1.5, s11 = 1.5, s14 = 1.83, s17 = 1.4, s18 = 1.61, s19 = 1.98,
                 s21 = 1.98, s24 = 1.74, s27 = 1.74;
    const double tab[Q] = {s1,  s1,  s1,  s1,  s5,  0,   0,   0,   0,   0,   s11, s11, s11, s14,
                           s14, s14, s17, s18, s19, s19, s21, s21, s21, s24, s24, s24, s27};
    for (int j = 0; j < Q; j++) K[j] = tab[j];
  }
  for (int j = 5; j <= 9; j++) K[j] = snu;
}

/* ---------------------------------------------------------------- per-cell operators */

/* Total enhanced equilibrium, Eq. (EES) summed over both colours:
 *   sum_k rho_k (varphi_i^k + w_i [3 c.u + 9/2 (c.u)^2 - 3/2 u^2]) + Phi_i,
 * with Phi_i of Eq. (Phi) built from G = (u (x) grad rho + (u (x) grad rho)^T)/48. */
void oracle_equilibrium(double rho_r, double rho_b, double alpha_r, double alpha_b, const double *u,
                        double nubar, const double *grad_rho, double *feq) {
  const double rho = rho_r + rho_b;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double G[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) G[a][b] = (u[a] * grad_rho[b] + u[b] * grad_rho[a]) / 48.0;
  const double udg = u[0] * grad_rho[0] + u[1] * grad_rho[1] + u[2] * grad_rho[2];
  for (int i = 0; i < Q; i++) {
    const double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double phi_i;
    if (i == 0) {
      phi_i = -3.0 * nubar * udg;
    } else {
      double gcc = 0.0;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) gcc += G[a][b] * CV[i][a] * CV[i][b];
      const double coef = shell(i) == 1 ? 16.0 : (shell(i) == 2 ? 4.0 : 1.0);
      phi_i = coef * nubar * gcc;
    }
    feq[i] = rho_r * varphi(i, alpha_r) + rho_b * varphi(i, alpha_b) +
             rho * weight(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu) + phi_i;
  }
}

/* One colour's equilibrium with Phi = 0 (used for initial states and inflow sites). */
void oracle_colour_equilibrium(double rho_k, double alpha_k, const double *u, double *feq) {
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; i++) {
    const double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    feq[i] = rho_k * (varphi(i, alpha_k) + weight(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
  }
}

/* |F'> of Eq. (ketFd): F'_i = w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F. */
void oracle_forcing_velocity_space(const double *u, const double *F, double *Fp) {
  for (int i = 0; i < Q; i++) {
    const double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double acc = 0.0;
    for (int a = 0; a < 3; a++) acc += (3.0 * (CV[i][a] - u[a]) + 9.0 * cu * CV[i][a]) * F[a];
    Fp[i] = weight(i) * acc;
  }
}

/* Eq. (scoll) on the total distribution, with |F> of Eq. (ketF):
 *   f' = f - M^-1 K M (f - f_eq) + M^-1 (I - K/2) M F'. */
static void mrt_collide(const double M[Q][Q], const double Minv[Q][Q], const double *K, const double *f,
                        const double *feq, const double *Fp, double *fout) {
  double m[Q], meq[Q], mF[Q], ms[Q];
  for (int j = 0; j < Q; j++) {
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < Q; i++) {
      a += M[j][i] * f[i];
      b += M[j][i] * feq[i];
      c += M[j][i] * Fp[i];
    }
    m[j] = a; meq[j] = b; mF[j] = c;
  }
  for (int j = 0; j < Q; j++) ms[j] = m[j] - K[j] * (m[j] - meq[j]) + (1.0 - 0.5 * K[j]) * mF[j];
  for (int i = 0; i < Q; i++) {
    double a = 0;
    for (int j = 0; j < Q; j++) a += Minv[i][j] * ms[j];
    fout[i] = a;
  }
}

/* Perturbation operator Eq. (perturb) summed over the two colours (A_r = A_b = A), with
 * the square of R5:  f_i += A |grad phi| [ w_i (c_i . grad phi)^2 / |grad phi|^2 - B_i ]. */
void oracle_perturbation(double A, double gphi_cut, const double *gphi, double *f) {
  const double g2 = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
  if (!(g2 > gphi_cut * gphi_cut)) return; /* R7: no normal */
  const double gn = sqrt(g2);
  for (int i = 0; i < Q; i++) {
    const double cg = CV[i][0] * gphi[0] + CV[i][1] * gphi[1] + CV[i][2] * gphi[2];
    f[i] += A * gn * (weight(i) * cg * cg / g2 - Bcoef(i));
  }
}

/* Recolouring operator (Sec. II, Latva-Kokko & Rothman):
 *   f^r_i = rho_r/rho f_i + beta rho_r rho_b/rho^2 cos(theta_i) f_i^(e)(rho, 0, alpha_bar)
 *   f^b_i = rho_b/rho f_i - beta rho_r rho_b/rho^2 cos(theta_i) f_i^(e)(rho, 0, alpha_bar)
 * with cos(theta_i) = c_i . grad phi / (|c_i| |grad phi|) and f^(e)(rho,0,a) = rho varphi_i(a). */
void oracle_recolour(double rho_r, double rho_b, double beta, double alpha_bar, double gphi_cut,
                     const double *gphi, const double *f, double *fr, double *fb) {
  const double rho = rho_r + rho_b;
  const double g2 = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
  const double gn = sqrt(g2);
  for (int i = 0; i < Q; i++) {
    double cosv = 0.0;
    if (i != 0 && g2 > gphi_cut * gphi_cut) { /* R7 */
      const double cg = CV[i][0] * gphi[0] + CV[i][1] * gphi[1] + CV[i][2] * gphi[2];
      cosv = cg / (sqrt((double)shell(i)) * gn);
    }
    const double seg = beta * rho_r * rho_b / (rho * rho) * cosv * rho * varphi(i, alpha_bar);
    fr[i] = rho_r / rho * f[i] + seg;
    fb[i] = rho_b / rho * f[i] - seg;
  }
}

/* ---------------------------------------------------------------- helpers */

static double splitmix64_uniform(unsigned long long seed, unsigned long long counter) {
  uint64_t z = (uint64_t)seed + ((uint64_t)counter + 1u) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

double oracle_noise(unsigned long long seed, unsigned long long counter) { return splitmix64_uniform(seed, counter); }

/* The surface-tension parameter of an interfacial tension sigma: Eq. (sigma), sigma = (4/9) A tau,
 * solved for A with tau = 3 nu + 1/2 the relaxation time of the fluid of viscosity nu (R6). */
double oracle_A_from_sigma(double sigma, double nu) { return 9.0 * sigma / (4.0 * (3.0 * nu + 0.5)); }

static inline long cidx(const oracle *o, int x, int y, int z) { return ((long)z * o->p.ny + y) * o->p.nx + x; }
static inline double *pop(double *base, const oracle *o, int k, int i) { return base + ((long)k * Q + i) * o->n; }

static void body_force(const oracle *o, double rho, double *F) {
  if (o->p.force_model == 1) {
    for (int a = 0; a < 3; a++) F[a] = (rho - o->p.rho_ref) * o->p.g[a];
  } else {
    F[0] = F[1] = F[2] = 0.0;
  }
}

/* Inflow speed of a site at a step: u0 (1 + eps xi), xi drawn from the counter
 * step * (cells of the whole domain) + (global index of the site). */
static double inflow_velocity(const oracle *o, long cell, long long step) {
  double xi = 0.0;
  if (o->p.noise_rel != 0.0) {
    const long x = cell % o->p.nx, y = (cell / o->p.nx) % o->p.ny, z = cell / ((long)o->p.nx * o->p.ny);
    const long gx = x + o->p.ox, gy = y + o->p.oy, gz = z + o->p.oz;
    const unsigned long long gn = (unsigned long long)o->p.gnx * o->p.gny * o->p.gnz;
    const unsigned long long gc = ((unsigned long long)gz * o->p.gny + gy) * o->p.gnx + gx;
    xi = splitmix64_uniform(o->p.seed, (unsigned long long)step * gn + gc);
  }
  return o->p.u_in * (1.0 + o->p.noise_rel * xi);
}

/* Value of a per-cell field at (x,y,z) + c seen by the gradient stencil: periodic faces
 * wrap; other faces repeat the boundary cell (R8, R9, R11). */
static double stencil_value(const oracle *o, const double *fld, int x, int y, int z) {
  const int n[3] = {o->p.nx, o->p.ny, o->p.nz};
  int q[3] = {x, y, z};
  for (int d = 0; d < 3; d++) {
    if (q[d] < 0) q[d] = o->p.face[2 * d] == FACE_PERIODIC ? q[d] + n[d] : 0;
    if (q[d] >= n[d]) q[d] = o->p.face[2 * d + 1] == FACE_PERIODIC ? q[d] - n[d] : n[d] - 1;
  }
  return fld[cidx(o, q[0], q[1], q[2])];
}

/* ---------------------------------------------------------------- public API */

int oracle_create(const oracle_params *p, oracle **out) {
  *out = NULL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 1;
  if (!(p->rho_r0 > 0 && p->rho_b0 > 0 && p->nu_r > 0 && p->nu_b > 0)) return 1;
  for (int d = 0; d < 3; d++)
    if ((p->face[2 * d] == FACE_PERIODIC) != (p->face[2 * d + 1] == FACE_PERIODIC)) return 1;
  oracle *o = (oracle *)calloc(1, sizeof(oracle));
  if (!o) return 2;
  o->p = *p;
  o->n = (long)p->nx * p->ny * p->nz;
  /* alpha_b = 8/27 (Sec. II), alpha_r from gamma = (1 - alpha_b)/(1 - alpha_r). */
  o->alpha_b = 8.0 / 27.0;
  o->alpha_r = 1.0 - (1.0 - o->alpha_b) * p->rho_b0 / p->rho_r0;
  if (o->alpha_r < 0.0 || o->alpha_r >= 1.0) { free(o); return 1; }
  if (o->p.gnx <= 0) { o->p.gnx = p->nx; o->p.gny = p->ny; o->p.gnz = p->nz; }
  for (int i = 0; i < Q; i++) o->dir_of[CV[i][0] + 1][CV[i][1] + 1][CV[i][2] + 1] = i;
  build_moment_matrix(o->M);
  if (invert(Q, &o->M[0][0], &o->Minv[0][0])) { free(o); return 3; }
  const size_t pb = sizeof(double) * 2 * Q * (size_t)o->n;
  o->f = (double *)calloc(1, pb);
  o->fpost = (double *)calloc(1, pb);
  o->fnew = (double *)calloc(1, pb);
  o->rr = (double *)calloc(o->n, sizeof(double));
  o->rb = (double *)calloc(o->n, sizeof(double));
  o->outlet = (double *)calloc((size_t)2 * Q * p->nx * p->ny, sizeof(double));
  o->inflow = (unsigned char *)calloc(o->n, 1);
  if (!o->f || !o->fpost || !o->fnew || !o->rr || !o->rb || !o->outlet || !o->inflow) return 2;
  if (p->inflow) {
    const double r2 = 0.25 * p->diameter * p->diameter;
    for (int y = 0; y < p->ny; y++)
      for (int x = 0; x < p->nx; x++) {
        const double dx = x - p->xc, dy = y - p->yc;
        if (dx * dx + dy * dy < r2) o->inflow[cidx(o, x, y, 0)] = 1;
      }
  }
  *out = o;
  return 0;
}

void oracle_destroy(oracle *o) {
  if (!o) return;
  free(o->f); free(o->fpost); free(o->fnew); free(o->rr); free(o->rb); free(o->outlet); free(o->inflow);
  free(o);
}

void oracle_get_matrices(const oracle *o, double *M, double *Minv) {
  memcpy(M, &o->M[0][0], sizeof(double) * Q * Q);
  memcpy(Minv, &o->Minv[0][0], sizeof(double) * Q * Q);
}

void oracle_get_lattice(int *c, double *w, double *B) {
  for (int i = 0; i < Q; i++) {
    for (int a = 0; a < 3; a++) c[3 * i + a] = CV[i][a];
    w[i] = weight(i);
    B[i] = Bcoef(i);
  }
}

void oracle_get_varphi(double alpha, double *out) {
  for (int i = 0; i < Q; i++) out[i] = varphi(i, alpha);
}

double oracle_alpha_r(const oracle *o) { return o->alpha_r; }

void oracle_relaxation_diag(const oracle *o, double snu, double *K) { relaxation_diag(o->p.s, snu, K); }

/* Initialise from per-cell densities and (optionally) velocity: R1. */
void oracle_init(oracle *o, const double *rho_r, const double *rho_b, const double *u) {
  double fe[Q];
  for (long c = 0; c < o->n; c++) {
    double uc[3] = {0, 0, 0};
    if (u) { uc[0] = u[c]; uc[1] = u[o->n + c]; uc[2] = u[2 * o->n + c]; }
    double rr = rho_r[c], rb = rho_b[c];
    if (o->inflow[c]) { rr = o->p.rho_r0; rb = 0.0; uc[0] = uc[1] = 0.0; uc[2] = inflow_velocity(o, c, 0); }
    oracle_colour_equilibrium(rr, o->alpha_r, uc, fe);
    for (int i = 0; i < Q; i++) pop(o->f, o, 0, i)[c] = fe[i];
    oracle_colour_equilibrium(rb, o->alpha_b, uc, fe);
    for (int i = 0; i < Q; i++) pop(o->f, o, 1, i)[c] = o->inflow[c] ? 0.0 : fe[i];
  }
  /* the outlet plane's "previous" state is its initial state */
  if (o->p.face[5] == FACE_OUTFLOW) {
    const long pl = (long)o->p.nx * o->p.ny;
    for (int k = 0; k < 2; k++)
      for (int i = 0; i < Q; i++)
        for (long c = 0; c < pl; c++) o->outlet[((long)k * Q + i) * pl + c] = pop(o->f, o, k, i)[(long)(o->p.nz - 1) * pl + c];
  }
  o->step = 0;
}

/* Collide one cell: pre-collision colour populations -> post-collision colour populations.
 * grad_phi / grad_rho come from the stencil; F is the body force at the cell. */
void oracle_collide_cell(const oracle *o, const double *fr_in, const double *fb_in, const double *grad_phi,
                         const double *grad_rho, const double *F, double *fr_out, double *fb_out) {
  double rr = 0, rb = 0, j[3] = {0, 0, 0}, f[Q];
  for (int i = 0; i < Q; i++) {
    rr += fr_in[i];
    rb += fb_in[i];
    f[i] = fr_in[i] + fb_in[i];
    for (int a = 0; a < 3; a++) j[a] += f[i] * CV[i][a];
  }
  const double rho = rr + rb;
  const double phi = (rr - rb) / rho;                                  /* Eq. (order) */
  double u[3];
  for (int a = 0; a < 3; a++) u[a] = (j[a] + 0.5 * F[a]) / rho;        /* Eq. (Momentum) */
  const double nubar = 0.5 * (1.0 + phi) * o->p.nu_r + 0.5 * (1.0 - phi) * o->p.nu_b;
  const double snu = 1.0 / (3.0 * nubar + 0.5);                        /* Eq. (shear) */
  const double abar = 0.5 * (1.0 + phi) * o->alpha_r + 0.5 * (1.0 - phi) * o->alpha_b;
  double K[Q], feq[Q], Fp[Q], fc[Q];
  relaxation_diag(o->p.s, snu, K);
  oracle_equilibrium(rr, rb, o->alpha_r, o->alpha_b, u, nubar, grad_rho, feq);
  oracle_forcing_velocity_space(u, F, Fp);
  mrt_collide(o->M, o->Minv, K, f, feq, Fp, fc);
  oracle_perturbation(o->p.A, o->p.gphi_cut, grad_phi, fc);
  oracle_recolour(rr, rb, o->p.beta, abar, o->p.gphi_cut, grad_phi, fc, fr_out, fb_out);
}

/* Source of the population arriving at (x,y,z) along direction i: returns the source
 * cell and direction, applying periodic wrap, specular reflection (free slip) or
 * half-way bounce-back at non-periodic faces. */
static void stream_source(const oracle *o, int x, int y, int z, int i, long *src_cell, int *src_dir) {
  const int n[3] = {o->p.nx, o->p.ny, o->p.nz};
  const int pos[3] = {x, y, z};
  int s[3], c[3];
  int bounce = 0;
  for (int d = 0; d < 3; d++) { c[d] = CV[i][d]; s[d] = pos[d] - c[d]; }
  for (int d = 0; d < 3; d++) {
    if (s[d] >= 0 && s[d] < n[d]) continue;
    const int face = s[d] < 0 ? o->p.face[2 * d] : o->p.face[2 * d + 1];
    if (face == FACE_PERIODIC) {
      s[d] = (s[d] + n[d]) % n[d];
    } else if (face == FACE_FREESLIP) {
      s[d] = pos[d];   /* no displacement along the normal ... */
      c[d] = -c[d];    /* ... and the normal component was reversed at the wall */
    } else {
      bounce = 1;      /* bounce-back; also used beyond the outlet, which is overwritten */
    }
  }
  if (bounce) {
    *src_cell = cidx(o, x, y, z);
    *src_dir = o->dir_of[1 - CV[i][0]][1 - CV[i][1]][1 - CV[i][2]];
    return;
  }
  /* after reflections the source may need a periodic wrap in another dimension */
  for (int d = 0; d < 3; d++) s[d] = (s[d] % n[d] + n[d]) % n[d];
  *src_cell = cidx(o, s[0], s[1], s[2]);
  *src_dir = o->dir_of[c[0] + 1][c[1] + 1][c[2] + 1];
}

void oracle_step(oracle *o, int nsteps) {
  const oracle_params *p = &o->p;
  const long n = o->n;
  const long plane = (long)p->nx * p->ny;
  for (int it = 0; it < nsteps; it++) {
    /* 1. densities of time t (R10 for inflow sites) */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) {
      double rr = 0, rb = 0;
      for (int i = 0; i < Q; i++) { rr += pop(o->f, o, 0, i)[c]; rb += pop(o->f, o, 1, i)[c]; }
      if (o->inflow[c]) { rr = p->rho_r0; rb = 0.0; }
      o->rr[c] = rr;
      o->rb[c] = rb;
    }
    /* 2. collision, perturbation and recolouring of every cell */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) {
      const int x = (int)(c % p->nx), y = (int)((c / p->nx) % p->ny), z = (int)(c / plane);
      double fr[Q], fb[Q], outr[Q], outb[Q];
      if (o->inflow[c]) {
        const double u[3] = {0.0, 0.0, inflow_velocity(o, c, o->step)};
        oracle_colour_equilibrium(p->rho_r0, o->alpha_r, u, outr);
        for (int i = 0; i < Q; i++) outb[i] = 0.0;
      } else {
        /* isotropic gradient: grad chi = 3 sum_i w_i chi(x + c_i) c_i */
        double gphi[3] = {0, 0, 0}, grho[3] = {0, 0, 0};
        for (int i = 1; i < Q; i++) {
          const double r1 = stencil_value(o, o->rr, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
          const double b1 = stencil_value(o, o->rb, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
          const double ph = (r1 - b1) / (r1 + b1), rh = r1 + b1;
          for (int a = 0; a < 3; a++) {
            gphi[a] += 3.0 * weight(i) * ph * CV[i][a];
            grho[a] += 3.0 * weight(i) * rh * CV[i][a];
          }
        }
        for (int i = 0; i < Q; i++) { fr[i] = pop(o->f, o, 0, i)[c]; fb[i] = pop(o->f, o, 1, i)[c]; }
        double F[3];
        body_force(o, o->rr[c] + o->rb[c], F);
        oracle_collide_cell(o, fr, fb, gphi, grho, F, outr, outb);
      }
      for (int i = 0; i < Q; i++) { pop(o->fpost, o, 0, i)[c] = outr[i]; pop(o->fpost, o, 1, i)[c] = outb[i]; }
    }
    /* 3. streaming, Eq. (LBE), with the face rules */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) {
      const int x = (int)(c % p->nx), y = (int)((c / p->nx) % p->ny), z = (int)(c / plane);
      for (int i = 0; i < Q; i++) {
        long sc; int sd;
        stream_source(o, x, y, z, i, &sc, &sd);
        pop(o->fnew, o, 0, i)[c] = pop(o->fpost, o, 0, sd)[sc];
        pop(o->fnew, o, 1, i)[c] = pop(o->fpost, o, 1, sd)[sc];
      }
    }
    /* 4. convective outflow on the last plane (R11) */
    if (p->face[5] == FACE_OUTFLOW && p->nz >= 2) {
      const long zo = (long)(p->nz - 1) * plane, zm = (long)(p->nz - 2) * plane;
      for (long q = 0; q < plane; q++) {
        double rho = 0, jz = 0;
        for (int k = 0; k < 2; k++)
          for (int i = 0; i < Q; i++) {
            const double v = pop(o->fnew, o, k, i)[zm + q];
            rho += v;
            jz += v * CV[i][2];
          }
        double F[3];
        body_force(o, rho, F);
        double lam = (jz + 0.5 * F[2]) / rho;
        if (lam < 0.0) lam = 0.0;
        for (int k = 0; k < 2; k++)
          for (int i = 0; i < Q; i++) {
            double *prev = &o->outlet[((long)k * Q + i) * plane + q];
            const double v = (*prev + lam * pop(o->fnew, o, k, i)[zm + q]) / (1.0 + lam);
            pop(o->fnew, o, k, i)[zo + q] = v;
            *prev = v;
          }
      }
    }
    /* 5. inflow sites hold the red equilibrium they emit at the next step (R10) */
    if (p->inflow) {
#pragma omp parallel for schedule(static)
      for (long c = 0; c < plane; c++) {
        if (!o->inflow[c]) continue;
        double fe[Q];
        const double u[3] = {0.0, 0.0, inflow_velocity(o, c, o->step + 1)};
        oracle_colour_equilibrium(p->rho_r0, o->alpha_r, u, fe);
        for (int i = 0; i < Q; i++) { pop(o->fnew, o, 0, i)[c] = fe[i]; pop(o->fnew, o, 1, i)[c] = 0.0; }
      }
    }
    double *t = o->f; o->f = o->fnew; o->fnew = t;
    o->step++;
  }
}

/* Macroscopic fields of time t (post-streaming, pre-collision): rho_r, rho_b and
 * u = (sum_i f_i c_i + F/2)/rho (Eq. (Momentum)); inflow sites report their set state. */
void oracle_fields(const oracle *o, double *rho_r, double *rho_b, double *u) {
  for (long c = 0; c < o->n; c++) {
    double rr = 0, rb = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; i++) {
      const double a = pop(o->f, o, 0, i)[c], b = pop(o->f, o, 1, i)[c];
      rr += a; rb += b;
      for (int d = 0; d < 3; d++) j[d] += (a + b) * CV[i][d];
    }
    double uc[3];
    if (o->inflow[c]) {
      rr = o->p.rho_r0; rb = 0.0;
      uc[0] = uc[1] = 0.0; uc[2] = inflow_velocity(o, c, o->step);
    } else {
      double F[3];
      body_force(o, rr + rb, F);
      for (int d = 0; d < 3; d++) uc[d] = (j[d] + 0.5 * F[d]) / (rr + rb);
    }
    rho_r[c] = rr; rho_b[c] = rb;
    if (u) for (int d = 0; d < 3; d++) u[(long)d * o->n + c] = uc[d];
  }
}

/* The isotropic gradient stencil of Sec. II applied to a per-cell field:
 * grad chi(x) = 3 sum_i w_i chi(x + c_i) c_i, with the face rules of stencil_value. */
void oracle_gradient(const oracle *o, const double *fld, double *out /* [3][cell] */) {
  const long plane = (long)o->p.nx * o->p.ny;
  for (long c = 0; c < o->n; c++) {
    const int x = (int)(c % o->p.nx), y = (int)((c / o->p.nx) % o->p.ny), z = (int)(c / plane);
    double g[3] = {0, 0, 0};
    for (int i = 1; i < Q; i++) {
      const double v = stencil_value(o, fld, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
      for (int a = 0; a < 3; a++) g[a] += 3.0 * weight(i) * v * CV[i][a];
    }
    for (int a = 0; a < 3; a++) out[(long)a * o->n + c] = g[a];
  }
}

/* Pre-collision colour populations [colour][i][cell]. */
void oracle_populations(const oracle *o, double *out) { memcpy(out, o->f, sizeof(double) * 2 * Q * (size_t)o->n); }
void oracle_set_populations(oracle *o, const double *in) { memcpy(o->f, in, sizeof(double) * 2 * Q * (size_t)o->n); }
long long oracle_step_count(const oracle *o) { return o->step; }
