// lbm_capi.hip -- host side of the C ABI declared in include/lbm.h: parameter checks,
// device buffers, the step loop and the read-back entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_cell.h"
#include "lbm_device.h"
#include "lbm_kernels.h"

using namespace lbm;

struct lbm_ctx {
  lbm_params p;
  hipStream_t stream = nullptr;
  Geo geo{};
  PullConst pc{};
  CollideParams cp{};
  GroupRates rates{};
  size_t elem = 4;          // bytes per stored population
  void* g[2] = {nullptr, nullptr};
  float* sc[2] = {nullptr, nullptr};
  float* outlet[2] = {nullptr, nullptr};
  float* init = nullptr;    // initial fields, needed until the first step
  double* dbuf = nullptr;   // read-back staging
  size_t dbuf_bytes = 0;
  double* diag_part = nullptr;
  double* diag_out = nullptr;
  int* unstable = nullptr;  // device flag the step kernel sets on a NaN / non-positive density
  int device = 0;           // the device current at lbm_create
  long long diag_blocks = 0;
  int cur = 0;              // index of the state holding the current time
  int out_cur = 0;          // index of the outlet record of the latest time
  long long step = 0;
  bool initialised = false;
  int tx = 0, ty = 0, zchunk = 0;  // 0: chosen at the first step (choose_tiling, auto_zchunk)
  int zchunk_set[kCorners + 1] = {};  // with lateral walls and an automatic zchunk: the z
                                      // chunk of each tile set's launch (0: zchunk)
  bool in_batch = false;           // advanced only by lbm_batch_step
  bool frozen = false;             // a batch case found unstable: no longer stepped
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  std::string err;
};

static std::string g_create_error;

static lbm_status fail(lbm_ctx* c, lbm_status st, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return st;
}

static lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* what) {
  return fail(c, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define LBM_HIP(ctx, call)                          \
  do {                                              \
    hipError_t e_ = (call);                         \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

static const double kAlphaB = 8.0 / 27.0;

// ---------------------------------------------------------------- no-allocation staging
// lbm_read_field_box_noalloc stages the FP64 fields of one z slice of the box in this
// file-scope array instead of a buffer the context allocates: 2^20 doubles (8 MiB) per
// device, held until the process ends.  The fields kernel writes 7 values per cell, so a slice
// holds at most kScratchDoubles / 7 cells.  Host code must not pass the array's name to a
// kernel: each device's address comes from hipGetSymbolAddress, taken once per device in
// lbm_create with that device current, and is used everywhere instead.  Every call on a
// device shares its array; calls that overlap on one device race.
constexpr size_t kScratchDoubles = size_t(1) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
static double* g_scratch_ptr[kScratchDevices] = {};
static std::mutex g_scratch_mu;

// Address of this device's scratch array (set up on the first call for the device; the
// device must be current).  nullptr if the lookup failed.
static double* scratch_on(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    double* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

// Validation of lbm_params; fills the derived constants.
static lbm_status check_params(const lbm_params* p, lbm_ctx* c, std::string& msg) {
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return msg = "lattice sizes must be >= 1", LBM_EINVAL;
  const long long plane = (long long)p->nx * p->ny;
  // the kernels address the 27 population planes of one z (4-byte words at most) with 32-bit
  // signed byte offsets
  if (plane * Q * 4 >= (1LL << 31)) return msg = "nx*ny too large: nx*ny*108 must stay below 2^31", LBM_EINVAL;
  if (!(p->rho_r0 > 0.0) || !(p->rho_b0 > 0.0)) return msg = "rho_r0 and rho_b0 must be > 0", LBM_EINVAL;
  const double alpha_r = 1.0 - (1.0 - kAlphaB) * p->rho_b0 / p->rho_r0;
  if (!(alpha_r >= 0.0 && alpha_r < 1.0))
    return msg = "density ratio gives alpha_r outside [0,1) (gamma must be >= 19/27)", LBM_EINVAL;
  if (!(p->nu_r > 0.0) || !(p->nu_b > 0.0)) return msg = "viscosities must be > 0", LBM_EINVAL;
  if (!(p->A >= 0.0)) return msg = "A must be >= 0", LBM_EINVAL;
  if (!(p->beta >= 0.0 && p->beta <= 1.0)) return msg = "beta must lie in [0, 1]", LBM_EINVAL;
  for (int d = 0; d < 2; ++d) {
    const int lo_d = p->face[2 * d], hi_d = p->face[2 * d + 1];
    if (lo_d != hi_d || (lo_d != LBM_PERIODIC && lo_d != LBM_FREESLIP))
      return msg = "x and y faces must be both periodic or both free-slip", LBM_EINVAL;
  }
  const int lo = p->face[4], hi = p->face[5];
  if (lo < 0 || lo > 2 || hi < 0 || hi > 3) return msg = "invalid z face rule", LBM_EINVAL;
  if ((lo == LBM_PERIODIC) != (hi == LBM_PERIODIC)) return msg = "periodic z faces must be paired", LBM_EINVAL;
  if (lo != LBM_PERIODIC && p->nz < 3) return msg = "nz must be >= 3 with walls in z", LBM_EINVAL;
  if (p->force != 0 && p->force != 1) return msg = "force must be 0 or 1", LBM_EINVAL;
  if (p->storage < LBM_F32 || p->storage > LBM_BF16) return msg = "invalid storage", LBM_EINVAL;
  // relaxation rates: all zero -> the set of Sec. II; otherwise the grouped structure of K
  bool user = false;
  for (int j = 0; j < Q; ++j) user |= (p->s[j] != 0.0);
  GroupRates r{1.5f, 1.5f, 1.83f, 1.4f, 1.61f, 1.98f, 1.98f, 1.74f, 1.74f};
  if (user) {
    for (int j = 0; j < 4; ++j)
      if (p->s[j] != 0.0) return msg = "s[0..3] (conserved moments) must be 0", LBM_EINVAL;
    const int groups[9][3] = {{4, 4, 4},    {10, 12, 12}, {13, 15, 15}, {16, 16, 16}, {17, 17, 17},
                              {18, 19, 19}, {20, 22, 22}, {23, 25, 25}, {26, 26, 26}};
    float* out[9] = {&r.s5, &r.s11, &r.s14, &r.s17, &r.s18, &r.s19, &r.s21, &r.s24, &r.s27};
    for (int gi = 0; gi < 9; ++gi) {
      const double v = p->s[groups[gi][0]];
      for (int j = groups[gi][0]; j <= groups[gi][1]; ++j)
        if (p->s[j] != v) return msg = "relaxation rates must be equal within each group of K", LBM_EINVAL;
      if (!(v > 0.0 && v < 2.0)) return msg = "relaxation rates must lie in (0, 2)", LBM_EINVAL;
      *out[gi] = (float)v;
    }
  }
  if (c) {
    c->rates = r;
    c->pc.alpha_r = (float)alpha_r;
    c->pc.alpha_b = (float)kAlphaB;
    c->pc.dalpha = (float)(alpha_r - kAlphaB);
    c->pc.E0 = (float)(p->rho_b0 * (1.0 - kAlphaB));
    c->pc.one_m_ab = (float)(1.0 - kAlphaB);
    c->pc.one_m_ar = (float)((1.0 - kAlphaB) * p->rho_b0 / p->rho_r0);
    c->cp.alpha_r = (float)alpha_r;
    c->cp.alpha_b = (float)kAlphaB;
    c->cp.dalpha = c->pc.dalpha;
    c->cp.one_m_ab = c->pc.one_m_ab;
    c->cp.one_m_ar = c->pc.one_m_ar;
    c->cp.nu_r = (float)p->nu_r;
    c->cp.nu_b = (float)p->nu_b;
    c->cp.A = (float)p->A;
    c->cp.beta = (float)p->beta;
    c->cp.force = p->force;
    c->cp.gx = (float)p->g[0];
    c->cp.gy = (float)p->g[1];
    c->cp.gz = (float)p->g[2];
    c->cp.rho_ref = (float)p->rho_ref;
    Geo& G = c->geo;
    G.nx = p->nx;
    G.ny = p->ny;
    G.nz = p->nz;
    G.plane = p->nx * p->ny;
    G.n = plane * p->nz;
    G.face_lo = lo;
    G.face_hi = hi;
    G.wall_x = p->face[0] == LBM_FREESLIP ? 1 : 0;
    G.wall_y = p->face[2] == LBM_FREESLIP ? 1 : 0;
    G.inflow = 0;
    c->elem = p->storage == LBM_F32 ? 4 : 2;
  }
  return LBM_OK;
}

extern "C" double lbm_sigma_from_A(double A, double nu) {
  if (!(nu > 0.0) || !(A >= 0.0)) return NAN;
  return 4.0 / 9.0 * A * (3.0 * nu + 0.5);
}

extern "C" double lbm_A_from_sigma(double sigma, double nu) {
  if (!(nu > 0.0) || !(sigma >= 0.0)) return NAN;
  return 9.0 * sigma / (4.0 * (3.0 * nu + 0.5));
}

extern "C" lbm_status lbm_create(const lbm_params* params, void* hip_stream, lbm_ctx** out) {
  if (!params || !out) return fail(nullptr, LBM_EINVAL, "null argument");
  *out = nullptr;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
  c->p = *params;
  std::string msg;
  lbm_status st = check_params(params, c, msg);
  if (st != LBM_OK) {
    delete c;
    return fail(nullptr, st, msg);
  }
  c->stream = static_cast<hipStream_t>(hip_stream);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete c;
    return fail(nullptr, LBM_EDEVICE, "no HIP device");
  }
  if (hipGetDevice(&c->device) != hipSuccess || !scratch_on(c->device)) {
    delete c;
    return fail(nullptr, LBM_EDEVICE, "no device address for the staging array");
  }
  const size_t n = (size_t)c->geo.n, plane = (size_t)c->geo.plane;
  bool ok = true;
  for (int k = 0; k < 2 && ok; ++k) {
    ok &= hipMalloc(&c->g[k], n * Q * c->elem) == hipSuccess;
    ok &= hipMalloc((void**)&c->sc[k], n * 5 * sizeof(float)) == hipSuccess;
    if (c->geo.face_hi == FACE_OUTFLOW)
      ok &= hipMalloc((void**)&c->outlet[k], plane * kOutletPlanes * sizeof(float)) == hipSuccess;
  }
  c->diag_blocks = (long long)((n + 255) / 256);
  ok = ok && hipMalloc((void**)&c->diag_part, (size_t)c->diag_blocks * 8 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->diag_out, 8 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->unstable, sizeof(int)) == hipSuccess &&
       hipMemset(c->unstable, 0, sizeof(int)) == hipSuccess;
  ok = ok && hipEventCreate(&c->ev0) == hipSuccess && hipEventCreate(&c->ev1) == hipSuccess;
  if (!ok) {
    lbm_destroy(c);
    return fail(nullptr, LBM_ENOMEM, "device allocation failed");
  }
  *out = c;
  return LBM_OK;
}

extern "C" void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  for (int k = 0; k < 2; ++k) {
    if (c->g[k]) (void)hipFree(c->g[k]);
    if (c->sc[k]) (void)hipFree(c->sc[k]);
    if (c->outlet[k]) (void)hipFree(c->outlet[k]);
  }
  if (c->init) (void)hipFree(c->init);
  if (c->dbuf) (void)hipFree(c->dbuf);
  if (c->diag_part) (void)hipFree(c->diag_part);
  if (c->diag_out) (void)hipFree(c->diag_out);
  if (c->unstable) (void)hipFree(c->unstable);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

extern "C" const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

extern "C" lbm_status lbm_set_inflow(lbm_ctx* c, double xc, double yc, double diameter, double u_normal,
                                     double noise_rel, unsigned long long seed) {
  if (!c) return LBM_EINVAL;
  if (c->geo.face_lo != FACE_FREESLIP && c->geo.face_lo != FACE_BOUNCEBACK)
    return fail(c, LBM_EINVAL, "the inflow disk needs a wall rule on the -z face");
  if (!(diameter > 0.0) || !(noise_rel >= 0.0 && noise_rel < 1.0)) return fail(c, LBM_EINVAL, "bad inflow parameters");
  Geo& G = c->geo;
  G.inflow = 1;
  G.xc = (float)xc;
  G.yc = (float)yc;
  G.r2 = (float)(0.25 * diameter * diameter);
  G.rho_r0 = (float)c->p.rho_r0;
  G.u_in = (float)u_normal;
  G.noise = (float)noise_rel;
  G.seed = seed;
  return LBM_OK;
}

extern "C" lbm_status lbm_set_tiling(lbm_ctx* c, int tx, int ty, int zchunk) {
  if (!c) return LBM_EINVAL;
  if (!step_tiling_supported(tx, ty) || zchunk < 0) return fail(c, LBM_EINVAL, "unsupported tiling");
  c->tx = tx;
  c->ty = ty;
  c->zchunk = zchunk;
  for (int& z : c->zchunk_set) z = 0;
  return LBM_OK;
}

static AuxArgs aux_args(const lbm_ctx* c) {
  AuxArgs a{};
  a.g_in = c->g[c->cur];
  a.sc_in = c->sc[c->cur];
  a.init = c->init;
  a.outlet_in = c->outlet[c->out_cur];
  a.outlet_out = c->outlet[1 - c->out_cur];
  a.step = c->step;
  a.init_mode = c->step == 0 ? 1 : 0;
  a.geo = c->geo;
  a.pc = c->pc;
  a.cp = c->cp;
  return a;
}

extern "C" lbm_status lbm_init_fields(lbm_ctx* c, const double* rho_r, const double* rho_b, const double* u) {
  if (!c || !rho_r || !rho_b) return LBM_EINVAL;
  const size_t n = (size_t)c->geo.n;
  // held as (e, psi, u): e = sum_k rho_k (1 - alpha_k) - E0 formed in FP64; psi the signed
  // minority-colour fraction (psi_encode)
  const double ar = 1.0 - (1.0 - kAlphaB) * c->p.rho_b0 / c->p.rho_r0, E0 = c->p.rho_b0 * (1.0 - kAlphaB);
  std::vector<float> h(5 * n, 0.0f);
  for (size_t k = 0; k < n; ++k) {
    if (!(rho_r[k] >= 0.0) || !(rho_b[k] >= 0.0) || !(rho_r[k] + rho_b[k] > 0.0))
      return fail(c, LBM_EINVAL, "initial densities must be >= 0 with a positive sum");
    h[k] = (float)(rho_r[k] * (1.0 - ar) + rho_b[k] * (1.0 - kAlphaB) - E0);
    const double rho = rho_r[k] + rho_b[k];
    h[n + k] = rho_r[k] <= rho_b[k] ? (float)(rho_r[k] / rho) : -(float)(rho_b[k] / rho);
    if (u)
      for (int d = 0; d < 3; ++d) h[(2 + d) * n + k] = (float)u[d * n + k];
  }
  if (!c->init) LBM_HIP(c, hipMalloc((void**)&c->init, 5 * n * sizeof(float)));
  LBM_HIP(c, hipMemcpyAsync(c->init, h.data(), 5 * n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  LBM_HIP(c, hipMemsetAsync(c->unstable, 0, sizeof(int), c->stream));
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  c->cur = 0;
  c->out_cur = 0;
  c->step = 0;
  c->initialised = true;
  c->frozen = false;
  return LBM_OK;
}

// Planes per workgroup when none is set: the number of z chunks that minimises
// (rounds of resident workgroups) x (planes per chunk + the 2 planes each chunk pulls first).
static int zchunk_for(const lbm_ctx* c, long long tiles) {
  const Geo& G = c->geo;
  if (tiles < 1) return G.nz;
  int dev = 0;
  (void)hipGetDevice(&dev);
  long long resident = step_resident_blocks((int)c->p.storage, c->tx, c->ty, dev);
  if (resident < 1) resident = 1024;
  long long best_cost = -1;
  int best = G.nz;
  for (int nch = 1; nch <= G.nz; ++nch) {
    const int zc = (G.nz + nch - 1) / nch;
    if ((G.nz + zc - 1) / zc != nch) continue;  // same chunking as a smaller count
    const long long rounds = (tiles * nch + resident - 1) / resident;
    const long long cost = rounds * (zc + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zc;
    }
  }
  return best;
}

static int auto_zchunk(const lbm_ctx* c) {
  const Geo& G = c->geo;
  return zchunk_for(c, (long long)((G.nx + c->tx - 1) / c->tx) * ((G.ny + c->ty - 1) / c->ty));
}

static void fill_step_args(const lbm_ctx* c, int cur, int out_cur, StepArgs& s);

static void choose_tiling(lbm_ctx* c) {
  if (c->tx == 0) {
    // measured on MI355X: 64 x 4 tiles on rows of 64 cells or more, 32 x 8 otherwise; with
    // lateral walls 64 x 4 and 32 x 8 are within 0.3 % of each other on the jet
    // (lbm_autotune times the shapes for a given lattice)
    const bool wide = c->geo.nx >= 64;
    c->tx = wide ? 64 : 32;
    c->ty = wide ? 4 : 8;
  }
  if (c->zchunk < 1) {
    c->zchunk = auto_zchunk(c);
    for (int& z : c->zchunk_set) z = 0;
    if (c->geo.wall_x || c->geo.wall_y) {
      // the interior and the parts of the frame run as launches one after the other: each is
      // chunked in z to fill the device by itself
      StepArgs s{};
      fill_step_args(c, 0, 0, s);
      int sets[kCorners + 1];
      const int nsets = wall_tile_sets((int)c->p.storage, sets);
      for (int k = 0; k < nsets; ++k) {
        s.tile_set = sets[k];
        c->zchunk_set[sets[k]] = zchunk_for(c, tiles_in_set(s));
      }
    }
  }
}

static void set_zchunk(const Geo& G, int zchunk, StepArgs& s) {
  s.zchunk = zchunk;
  s.nchunks = (G.nz + zchunk - 1) / zchunk;
}

// Arguments of the step kernel for the state of parity cur (outlet record out_cur).
static void fill_step_args(const lbm_ctx* c, int cur, int out_cur, StepArgs& s) {
  const Geo& G = c->geo;
  s.g_in = c->g[cur];
  s.sc_in = c->sc[cur];
  s.g_out = c->g[1 - cur];
  s.sc_out = c->sc[1 - cur];
  s.init = c->init;
  s.outlet = c->outlet[1 - out_cur];
  s.step = c->step;
  s.init_mode = c->step == 0 ? 1 : 0;
  s.zchunk = c->zchunk;
  s.tiles_x = (G.nx + c->tx - 1) / c->tx;
  s.tiles_y = (G.ny + c->ty - 1) / c->ty;
  s.nchunks = (G.nz + c->zchunk - 1) / c->zchunk;
  // interior rectangle: tiles whose own and ring cells are all off the lateral walls, i.e.
  // tile index >= 1 and (index + 1) * tile width <= n - 2 along each axis that has walls
  s.tile_set = kAllTiles;
  s.tx_lo = 0;
  s.tx_hi = s.tiles_x;
  s.ty_lo = 0;
  s.ty_hi = s.tiles_y;
  if (G.wall_x) {
    s.tx_lo = 1;
    s.tx_hi = (G.nx - 2) / c->tx;
  }
  if (G.wall_y) {
    s.ty_lo = 1;
    s.ty_hi = (G.ny - 2) / c->ty;
  }
  if (s.tx_hi <= s.tx_lo || s.ty_hi <= s.ty_lo) s.tx_lo = s.tx_hi = s.ty_lo = s.ty_hi = 0;
  s.unstable = c->unstable;
  s.skip_unstable = c->in_batch ? 1 : 0;
  s.geo = G;
  s.pc = c->pc;
  s.cp = c->cp;
  s.rates = c->rates;
}

// LBM_EUNSTABLE if the step kernel has flagged a NaN or non-positive density since the state
// was set (synchronises the context's stream).
static lbm_status check_unstable(lbm_ctx* c) {
  int h = 0;
  LBM_HIP(c, hipMemcpyAsync(&h, c->unstable, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  return h ? fail(c, LBM_EUNSTABLE, "the state holds a NaN or a non-positive density (flagged by the step kernel)")
           : LBM_OK;
}

static lbm_status enqueue_one(lbm_ctx* c) {
  Geo& G = c->geo;
  if (G.face_hi == FACE_OUTFLOW) {
    AuxArgs a = aux_args(c);
    hipError_t e = launch_outlet((int)c->p.storage, a, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "outlet kernel");
  }
  StepArgs s{};
  choose_tiling(c);
  fill_step_args(c, c->cur, c->out_cur, s);
  hipError_t e = hipSuccess;
  if (G.wall_x || G.wall_y) {
    // the interior tiles with the plain pull, the edges and corners of the frame with the
    // instances that reflect at their walls
    int sets[kCorners + 1];
    const int nsets = wall_tile_sets((int)c->p.storage, sets);
    for (int k = 0; k < nsets && e == hipSuccess; ++k) {
      const int set = sets[k];
      s.tile_set = set;
      if (tiles_in_set(s) == 0) continue;
      set_zchunk(G, c->zchunk_set[set] > 0 ? c->zchunk_set[set] : c->zchunk, s);
      e = launch_step((int)c->p.storage, s, c->tx, c->ty, c->stream);
    }
  } else {
    e = launch_step((int)c->p.storage, s, c->tx, c->ty, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "step kernel");
  if (G.inflow) {
    e = launch_inflow((int)c->p.storage, s, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "inflow kernel");
  }
  c->cur = 1 - c->cur;
  if (G.face_hi == FACE_OUTFLOW) c->out_cur = 1 - c->out_cur;
  c->step++;
  return LBM_OK;
}

extern "C" lbm_status lbm_step(lbm_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  if (!c->initialised) return fail(c, LBM_ESTATE, "lbm_step before lbm_init_fields");
  if (c->in_batch) return fail(c, LBM_ESTATE, "a case of a batch advances only with lbm_batch_step");
  if (nsteps == 0) return LBM_OK;
  LBM_HIP(c, hipEventRecord(c->ev0, c->stream));
  for (int k = 0; k < nsteps; ++k) {
    lbm_status st = enqueue_one(c);
    if (st != LBM_OK) return st;
  }
  LBM_HIP(c, hipEventRecord(c->ev1, c->stream));
  c->last_ms = -(double)nsteps;  // resolved lazily: negative = steps of a pending measurement
  return LBM_OK;
}

extern "C" lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  return c->initialised ? check_unstable(c) : LBM_OK;
}

extern "C" double lbm_last_step_kernel_ms(const lbm_ctx* cc) {
  lbm_ctx* c = const_cast<lbm_ctx*>(cc);
  if (!c) return 0.0;
  if (c->last_ms < 0.0) {
    const double steps = -c->last_ms;
    float ms = 0.0f;
    if (hipEventSynchronize(c->ev1) != hipSuccess || hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) return 0.0;
    c->last_ms = ms / steps;
  }
  return c->last_ms;
}

extern "C" long long lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

static lbm_status ensure_dbuf(lbm_ctx* c, size_t bytes) {
  if (c->dbuf_bytes >= bytes) return LBM_OK;
  if (c->dbuf) (void)hipFree(c->dbuf);
  c->dbuf = nullptr;
  c->dbuf_bytes = 0;
  LBM_HIP(c, hipMalloc((void**)&c->dbuf, bytes));
  c->dbuf_bytes = bytes;
  return LBM_OK;
}

extern "C" lbm_status lbm_read_field_box(lbm_ctx* c, int field, int x0, int y0, int z0, int wx, int wy, int wz,
                                         double* dst) {
  if (!c || !dst) return LBM_EINVAL;
  if (!c->initialised) return fail(c, LBM_ESTATE, "read before lbm_init_fields");
  if (field < 0 || field > 6) return fail(c, LBM_EINVAL, "unknown field");
  const Geo& G = c->geo;
  if (x0 < 0 || y0 < 0 || z0 < 0 || wx < 1 || wy < 1 || wz < 1 || x0 + wx > G.nx || y0 + wy > G.ny || z0 + wz > G.nz)
    return fail(c, LBM_EINVAL, "box outside the lattice");
  const size_t nb = (size_t)wx * wy * wz;
  // the box is done in z slices so the FP64 staging stays bounded
  const int zs = (int)std::max<size_t>(1, std::min<size_t>((size_t)wz, (64ull << 20) / ((size_t)wx * wy)));
  lbm_status st = ensure_dbuf(c, (size_t)wx * wy * zs * 7 * sizeof(double));
  if (st != LBM_OK) return st;
  AuxArgs a = aux_args(c);
  for (int z = 0; z < wz; z += zs) {
    const int h = std::min(zs, wz - z);
    const size_t ns = (size_t)wx * wy * h;
    hipError_t e = launch_fields((int)c->p.storage, a, x0, y0, z0 + z, wx, wy, h, c->dbuf, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "fields kernel");
    LBM_HIP(c, hipMemcpyAsync(dst + (size_t)z * wx * wy, c->dbuf + (size_t)field * ns, ns * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(c, hipStreamSynchronize(c->stream));
  }
  (void)nb;
  return check_unstable(c);
}

extern "C" lbm_status lbm_read_field_box_noalloc(lbm_ctx* c, int field, int x0, int y0, int z0, int wx, int wy,
                                                 int wz, double* dst) {
  if (!c || !dst) return LBM_EINVAL;
  if (!c->initialised) return fail(c, LBM_ESTATE, "read before lbm_init_fields");
  if (field < 0 || field > 6) return fail(c, LBM_EINVAL, "unknown field");
  const Geo& G = c->geo;
  if (x0 < 0 || y0 < 0 || z0 < 0 || wx < 1 || wy < 1 || wz < 1 || x0 + wx > G.nx || y0 + wy > G.ny || z0 + wz > G.nz)
    return fail(c, LBM_EINVAL, "box outside the lattice");
  const size_t slice = (size_t)wx * wy;
  if (slice * 7 > kScratchDoubles)
    return fail(c, LBM_EINVAL, "box too wide for the no-allocation staging: wx*wy must be at most " +
                                   std::to_string(kScratchDoubles / 7));
  double* stage = g_scratch_ptr[c->device];  // set up by lbm_create on this device
  if (!stage) return fail(c, LBM_EDEVICE, "no staging array on this device");
  const int zs = (int)std::min<size_t>((size_t)wz, kScratchDoubles / (slice * 7));
  AuxArgs a = aux_args(c);
  for (int z = 0; z < wz; z += zs) {
    const int h = std::min(zs, wz - z);
    const size_t ns = slice * h;
    hipError_t e = launch_fields((int)c->p.storage, a, x0, y0, z0 + z, wx, wy, h, stage, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "fields kernel");
    LBM_HIP(c, hipMemcpyAsync(dst + (size_t)z * slice, stage + (size_t)field * ns, ns * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(c, hipStreamSynchronize(c->stream));
  }
  return check_unstable(c);
}

extern "C" lbm_status lbm_coarse_state(lbm_ctx* c, int factor, double u_scale, float* dst, int pd, int ph, int pw) {
  if (!c || !dst) return LBM_EINVAL;
  if (!c->initialised) return fail(c, LBM_ESTATE, "read before lbm_init_fields");
  const Geo& G = c->geo;
  if (factor < 1 || G.nx % factor || G.ny % factor || G.nz % factor)
    return fail(c, LBM_EINVAL, "the lattice sizes must be multiples of the coarsening factor");
  if (!(u_scale > 0.0)) return fail(c, LBM_EINVAL, "u_scale must be > 0");
  if (G.nz / factor > pd || G.ny / factor > ph || G.nx / factor > pw)
    return fail(c, LBM_EINVAL, "the coarse state does not fit the padded box");
  if (reinterpret_cast<uintptr_t>(dst) % 16) return fail(c, LBM_EINVAL, "dst must be 16-byte aligned");
  AuxArgs a = aux_args(c);
  hipError_t e = launch_coarse((int)c->p.storage, a, factor, (float)(1.0 / u_scale), dst, ph, pw, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "coarse kernel");
  return LBM_OK;
}

extern "C" lbm_status lbm_read_field(lbm_ctx* c, int field, double* dst) {
  if (!c) return LBM_EINVAL;
  return lbm_read_field_box(c, field, 0, 0, 0, c->geo.nx, c->geo.ny, c->geo.nz, dst);
}

extern "C" lbm_status lbm_read_populations(lbm_ctx* c, double* dst) {
  if (!c || !dst) return LBM_EINVAL;
  if (!c->initialised) return fail(c, LBM_ESTATE, "read before lbm_init_fields");
  const size_t n = (size_t)c->geo.n;
  lbm_status st = ensure_dbuf(c, n * 2 * Q * sizeof(double));
  if (st != LBM_OK) return st;
  AuxArgs a = aux_args(c);
  hipError_t e = launch_populations((int)c->p.storage, a, c->dbuf, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "populations kernel");
  LBM_HIP(c, hipMemcpyAsync(dst, c->dbuf, n * 2 * Q * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  return check_unstable(c);
}

extern "C" lbm_status lbm_diagnostics(lbm_ctx* c, double xc, double yc, double zc, double r_in, double r_out,
                                      lbm_diag* out) {
  if (!c || !out) return LBM_EINVAL;
  if (!c->initialised) return fail(c, LBM_ESTATE, "diagnostics before lbm_init_fields");
  AuxArgs a = aux_args(c);
  DiagQuery q{xc, yc, zc, r_in, r_out};
  hipError_t e = launch_diag((int)c->p.storage, a, q, c->diag_part, c->diag_blocks, c->diag_out, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics kernel");
  double h[8];
  LBM_HIP(c, hipMemcpyAsync(h, c->diag_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  out->mass_r = h[0];
  out->mass_b = h[1];
  out->n_in = (long long)h[3];
  out->p_in = h[3] > 0 ? h[2] / h[3] : 0.0;
  out->n_out = (long long)h[5];
  out->p_out = h[5] > 0 ? h[4] / h[5] : 0.0;
  out->nan_cells = (long long)h[6];
  out->umax = h[7];
  out->step = c->step;
  if (out->nan_cells > 0) return fail(c, LBM_EUNSTABLE, "state holds NaN or non-positive density");
  return check_unstable(c);
}

// ---------------------------------------------------------------- checkpoint
// Header of a saved state (64 bytes): "LBMD3Q27", the step (int64), then nx, ny, nz, the
// storage and the six face rules (int32 each), then the instability flag (int32).  A state
// loads only into a context with the same lattice, storage and faces.
static void state_header(const lbm_ctx* c, char* h) {
  std::memcpy(h, "LBMD3Q27", 8);
  std::memcpy(h + 8, &c->step, sizeof(long long));
  const int geo[10] = {c->p.nx, c->p.ny, c->p.nz, (int)c->p.storage, c->p.face[0], c->p.face[1],
                       c->p.face[2], c->p.face[3], c->p.face[4], c->p.face[5]};
  std::memcpy(h + 16, geo, sizeof(geo));
}

extern "C" size_t lbm_state_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  const size_t n = (size_t)c->geo.n, plane = (size_t)c->geo.plane;
  size_t b = 64 + n * Q * c->elem + n * 5 * sizeof(float) + n * 5 * sizeof(float);
  if (c->geo.face_hi == FACE_OUTFLOW) b += plane * kOutletPlanes * sizeof(float);
  return b;
}

extern "C" lbm_status lbm_save_state(lbm_ctx* c, void* dst, size_t bytes) {
  if (!c || !dst) return LBM_EINVAL;
  if (!c->initialised) return fail(c, LBM_ESTATE, "save before lbm_init_fields");
  if (bytes < lbm_state_bytes(c)) return fail(c, LBM_EINVAL, "buffer too small");
  const size_t n = (size_t)c->geo.n, plane = (size_t)c->geo.plane;
  char* p = static_cast<char*>(dst);
  int flag = 0;
  LBM_HIP(c, hipMemcpyAsync(&flag, c->unstable, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  std::memset(p, 0, 64);
  state_header(c, p);
  std::memcpy(p + 56, &flag, sizeof(int));
  p += 64;
  LBM_HIP(c, hipMemcpyAsync(p, c->g[c->cur], n * Q * c->elem, hipMemcpyDeviceToHost, c->stream));
  p += n * Q * c->elem;
  LBM_HIP(c, hipMemcpyAsync(p, c->sc[c->cur], n * 5 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  p += n * 5 * sizeof(float);
  if (c->init)
    LBM_HIP(c, hipMemcpyAsync(p, c->init, n * 5 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  p += n * 5 * sizeof(float);
  if (c->geo.face_hi == FACE_OUTFLOW)
    LBM_HIP(c, hipMemcpyAsync(p, c->outlet[c->out_cur], plane * kOutletPlanes * sizeof(float), hipMemcpyDeviceToHost,
                              c->stream));
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

extern "C" lbm_status lbm_load_state(lbm_ctx* c, const void* src, size_t bytes) {
  if (!c || !src) return LBM_EINVAL;
  if (bytes < lbm_state_bytes(c)) return fail(c, LBM_EINVAL, "buffer too small");
  const char* p = static_cast<const char*>(src);
  if (std::memcmp(p, "LBMD3Q27", 8) != 0) return fail(c, LBM_EINVAL, "not a saved state");
  char mine[64] = {0};
  state_header(c, mine);
  if (std::memcmp(p + 16, mine + 16, 40) != 0)
    return fail(c, LBM_EINVAL, "the saved state belongs to another lattice (size, storage or faces differ)");
  long long step;
  int flag = 0;
  std::memcpy(&step, p + 8, sizeof(long long));
  std::memcpy(&flag, p + 56, sizeof(int));
  if (step < 0 || (flag != 0 && flag != 1)) return fail(c, LBM_EINVAL, "corrupt state header");
  const size_t n = (size_t)c->geo.n, plane = (size_t)c->geo.plane;
  p += 64;
  // into the buffers of the context's current parity, so that a case of a batch stays in
  // lock-step with the others
  LBM_HIP(c, hipMemcpyAsync(c->g[c->cur], p, n * Q * c->elem, hipMemcpyHostToDevice, c->stream));
  p += n * Q * c->elem;
  LBM_HIP(c, hipMemcpyAsync(c->sc[c->cur], p, n * 5 * sizeof(float), hipMemcpyHostToDevice, c->stream));
  p += n * 5 * sizeof(float);
  if (!c->init) LBM_HIP(c, hipMalloc((void**)&c->init, n * 5 * sizeof(float)));
  LBM_HIP(c, hipMemcpyAsync(c->init, p, n * 5 * sizeof(float), hipMemcpyHostToDevice, c->stream));
  p += n * 5 * sizeof(float);
  if (c->geo.face_hi == FACE_OUTFLOW)
    LBM_HIP(c, hipMemcpyAsync(c->outlet[c->out_cur], p, plane * kOutletPlanes * sizeof(float), hipMemcpyHostToDevice,
                              c->stream));
  LBM_HIP(c, hipMemcpyAsync(c->unstable, &flag, sizeof(int), hipMemcpyHostToDevice, c->stream));
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  c->step = step;
  c->initialised = true;
  c->frozen = flag != 0;
  return LBM_OK;
}

// ---------------------------------------------------------------- batches of lattices
// Cases that share a storage type and tile shape form a group; one launch per group and step
// advances all of them (batch_step_kernel).  Every case steps in lock-step, so the argument
// tables of a group take two forms only (state parity 0 or 1) and are uploaded once per
// lbm_batch_step call.
struct BatchGroup {
  int storage = 0, tx = 0, ty = 0;
  int lat = 0;                          // reflection mode of the instance (lat_mode_of)
  int tile_set = kAllTiles;             // the tiles of each case the group's launch covers
  std::vector<int> cases;               // indices into lbm_batch::c
  StepArgs* d_args[2] = {nullptr, nullptr};  // device tables for parity 0 and 1
  int* d_first = nullptr;               // device block offsets (ncases + 1)
  int nblocks = 0;
};

// The outlet or the inflow work of the cases of one storage type, launched once per step:
// device tables of per-case arguments for parity 0 and 1 and block offsets over each plane.
struct AuxGroup {
  int storage = 0;
  std::vector<int> cases;
  AuxArgs* d_aux[2] = {nullptr, nullptr};     // outlet groups
  StepArgs* d_step[2] = {nullptr, nullptr};   // inflow groups
  int* d_first = nullptr;
  int nblocks = 0;
};

struct lbm_batch {
  std::vector<lbm_ctx*> c;
  std::vector<BatchGroup> groups;
  std::vector<AuxGroup> outlets, inflows;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  std::string err;
};

static lbm_status batch_fail(lbm_batch* b, lbm_status st, const std::string& msg) {
  if (b) b->err = msg;
  return st;
}

static void free_groups(lbm_batch* b) {
  for (auto& g : b->groups) {
    for (int k = 0; k < 2; ++k)
      if (g.d_args[k]) (void)hipFree(g.d_args[k]);
    if (g.d_first) (void)hipFree(g.d_first);
  }
  b->groups.clear();
  for (auto* v : {&b->outlets, &b->inflows}) {
    for (auto& g : *v) {
      for (int k = 0; k < 2; ++k) {
        if (g.d_aux[k]) (void)hipFree(g.d_aux[k]);
        if (g.d_step[k]) (void)hipFree(g.d_step[k]);
      }
      if (g.d_first) (void)hipFree(g.d_first);
    }
    v->clear();
  }
}

extern "C" void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  free_groups(b);
  for (lbm_ctx* c : b->c) lbm_destroy(c);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete b;
}

extern "C" lbm_status lbm_batch_create(const lbm_params* params, int ncases, void* hip_stream, lbm_batch** out) {
  if (!params || !out || ncases < 1) return fail(nullptr, LBM_EINVAL, "bad batch arguments");
  *out = nullptr;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
  b->stream = static_cast<hipStream_t>(hip_stream);
  for (int k = 0; k < ncases; ++k) {
    lbm_ctx* c = nullptr;
    const lbm_status st = lbm_create(&params[k], hip_stream, &c);
    if (st != LBM_OK) {
      const std::string msg = "case " + std::to_string(k) + ": " + g_create_error;
      lbm_batch_destroy(b);
      return fail(nullptr, st, msg);
    }
    c->in_batch = true;
    b->c.push_back(c);
  }
  if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
    lbm_batch_destroy(b);
    return fail(nullptr, LBM_EDEVICE, "event creation failed");
  }
  *out = b;
  return LBM_OK;
}

extern "C" lbm_ctx* lbm_batch_case(lbm_batch* b, int k) {
  if (!b || k < 0 || k >= (int)b->c.size()) return nullptr;
  return b->c[k];
}

extern "C" int lbm_batch_size(const lbm_batch* b) { return b ? (int)b->c.size() : 0; }

extern "C" const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : ""; }

// Tile shapes and z chunks of the cases not set by the caller or the autotuner.  Many cases
// fill the GPU together; when the batch has at least as many columns as the device holds
// workgroups, every case is cut into chunks of kBatchChunk planes so that the workgroups of
// uneven cases carry equal work.
static constexpr int kBatchChunk = 64;

static void batch_tiling(lbm_batch* b) {
  long long columns = 0, resident = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  for (lbm_ctx* c : b->c) {
    if (c->tx == 0) {
      const bool wide = c->geo.nx >= 64;
      c->tx = wide ? 64 : 32;
      c->ty = wide ? 4 : 8;
    }
    columns += (long long)((c->geo.nx + c->tx - 1) / c->tx) * ((c->geo.ny + c->ty - 1) / c->ty);
    resident = std::max<long long>(resident, step_resident_blocks((int)c->p.storage, c->tx, c->ty, dev));
  }
  for (lbm_ctx* c : b->c)
    if (c->zchunk < 1) c->zchunk = columns >= resident ? std::min(c->geo.nz, kBatchChunk) : auto_zchunk(c);
}

static lbm_status build_groups(lbm_batch* b) {
  free_groups(b);
  auto add = [&](int k, int lat, int set) {
    const lbm_ctx* c = b->c[k];
    BatchGroup* g = nullptr;
    for (auto& x : b->groups)
      if (x.storage == (int)c->p.storage && x.tx == c->tx && x.ty == c->ty && x.lat == lat && x.tile_set == set) g = &x;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->storage = (int)c->p.storage;
      g->tx = c->tx;
      g->ty = c->ty;
      g->lat = lat;
      g->tile_set = set;
    }
    g->cases.push_back(k);
  };
  for (int k = 0; k < (int)b->c.size(); ++k) {
    const lbm_ctx* c = b->c[k];
    if (c->frozen) continue;
    if (c->geo.wall_x || c->geo.wall_y) {
      // with lateral walls: the interior tiles in a plain group, each part of the frame in the
      // group of its reflection mode
      StepArgs s{};
      fill_step_args(c, 0, 0, s);
      int sets[kCorners + 1];
      const int nsets = wall_tile_sets((int)c->p.storage, sets);
      for (int m = 0; m < nsets; ++m) {
        s.tile_set = sets[m];
        if (tiles_in_set(s) > 0) add(k, lat_mode_of(sets[m], true), sets[m]);
      }
    } else {
      add(k, 0, kAllTiles);
    }
  }
  for (auto& g : b->groups) {
    const int n = (int)g.cases.size();
    std::vector<StepArgs> h[2];
    std::vector<int> first(n + 1, 0);
    for (int j = 0; j < n; ++j) {
      const lbm_ctx* c = b->c[g.cases[j]];
      for (int par = 0; par < 2; ++par) {
        StepArgs s{};
        fill_step_args(c, par, par, s);
        s.tile_set = g.tile_set;
        h[par].push_back(s);
      }
      const StepArgs& s = h[0].back();
      const long long blocks = (long long)tiles_in_set(s) * s.nchunks;
      first[j + 1] = first[j] + (int)((blocks + 7) / 8 * 8);
    }
    g.nblocks = first[n];
    bool ok = true;
    for (int par = 0; par < 2 && ok; ++par) {
      ok = hipMalloc((void**)&g.d_args[par], n * sizeof(StepArgs)) == hipSuccess &&
           hipMemcpy(g.d_args[par], h[par].data(), n * sizeof(StepArgs), hipMemcpyHostToDevice) == hipSuccess;
    }
    ok = ok && hipMalloc((void**)&g.d_first, (n + 1) * sizeof(int)) == hipSuccess &&
         hipMemcpy(g.d_first, first.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return batch_fail(b, LBM_ENOMEM, "batch table allocation failed");
  }
  // outlet and inflow work per storage type (an outflow lattice's record shares its parity)
  for (int k = 0; k < (int)b->c.size(); ++k) {
    const lbm_ctx* c = b->c[k];
    if (c->frozen) continue;
    for (int which = 0; which < 2; ++which) {
      const bool has = which == 0 ? c->geo.face_hi == FACE_OUTFLOW : (bool)c->geo.inflow;
      if (!has) continue;
      auto& v = which == 0 ? b->outlets : b->inflows;
      AuxGroup* g = nullptr;
      for (auto& x : v)
        if (x.storage == (int)c->p.storage) g = &x;
      if (!g) {
        v.emplace_back();
        g = &v.back();
        g->storage = (int)c->p.storage;
      }
      g->cases.push_back(k);
    }
  }
  for (int which = 0; which < 2; ++which)
    for (auto& g : which == 0 ? b->outlets : b->inflows) {
      const int n = (int)g.cases.size();
      std::vector<int> first(n + 1, 0);
      std::vector<AuxArgs> ha[2];
      std::vector<StepArgs> hs[2];
      for (int j = 0; j < n; ++j) {
        lbm_ctx* c = b->c[g.cases[j]];
        first[j + 1] = first[j] + (int)((c->geo.plane + 255) / 256);
        for (int par = 0; par < 2; ++par) {
          if (which == 0) {
            AuxArgs a = aux_args(c);
            a.g_in = c->g[par];
            a.sc_in = c->sc[par];
            a.outlet_in = c->outlet[par];
            a.outlet_out = c->outlet[1 - par];
            ha[par].push_back(a);
          } else {
            StepArgs st{};
            fill_step_args(c, par, par, st);
            hs[par].push_back(st);
          }
        }
      }
      g.nblocks = first[n];
      bool ok = hipMalloc((void**)&g.d_first, (n + 1) * sizeof(int)) == hipSuccess &&
                hipMemcpy(g.d_first, first.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
      for (int par = 0; par < 2 && ok; ++par) {
        if (which == 0)
          ok = hipMalloc((void**)&g.d_aux[par], n * sizeof(AuxArgs)) == hipSuccess &&
               hipMemcpy(g.d_aux[par], ha[par].data(), n * sizeof(AuxArgs), hipMemcpyHostToDevice) == hipSuccess;
        else
          ok = hipMalloc((void**)&g.d_step[par], n * sizeof(StepArgs)) == hipSuccess &&
               hipMemcpy(g.d_step[par], hs[par].data(), n * sizeof(StepArgs), hipMemcpyHostToDevice) == hipSuccess;
      }
      if (!ok) return batch_fail(b, LBM_ENOMEM, "batch table allocation failed");
    }
  return LBM_OK;
}

// Reads the cases' instability flags (after the batch's stream has drained) and freezes the
// flagged cases: they are left out of every later launch.  Returns the number of unstable
// cases, or -1 if a copy failed.
static int refresh_unstable(lbm_batch* b) {
  int count = 0;
  for (lbm_ctx* c : b->c) {
    if (!c->frozen && c->initialised) {
      int h = 0;
      if (hipMemcpy(&h, c->unstable, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return -1;
      c->frozen = h != 0;
    }
    count += c->frozen ? 1 : 0;
  }
  return count;
}

extern "C" lbm_status lbm_batch_step(lbm_batch* b, int nsteps) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  if (nsteps == 0) return LBM_OK;
  for (const lbm_ctx* c : b->c)
    if (!c->initialised) return batch_fail(b, LBM_ESTATE, "every case needs lbm_init_fields before lbm_batch_step");
  if (hipStreamSynchronize(b->stream) != hipSuccess) return batch_fail(b, LBM_EDEVICE, "stream synchronisation failed");
  if (refresh_unstable(b) < 0) return batch_fail(b, LBM_EDEVICE, "reading the instability flags failed");
  std::vector<lbm_ctx*> active;
  for (lbm_ctx* c : b->c)
    if (!c->frozen) active.push_back(c);
  if (active.empty()) return batch_fail(b, LBM_EUNSTABLE, "every case of the batch is unstable");
  const lbm_ctx* c0 = active[0];
  for (const lbm_ctx* c : active) {
    // the outlet record of an outflow lattice flips with its state, so both share the parity
    if (c->step != c0->step || c->cur != c0->cur || (c->geo.face_hi == FACE_OUTFLOW && c->out_cur != c->cur))
      return batch_fail(b, LBM_ESTATE, "the cases of a batch must be at the same step");
  }
  batch_tiling(b);
  lbm_status st = build_groups(b);
  if (st != LBM_OK) return st;
  if (hipEventRecord(b->ev0, b->stream) != hipSuccess) return batch_fail(b, LBM_EDEVICE, "event record failed");
  for (int k = 0; k < nsteps; ++k) {
    const int par = active[0]->cur;
    const long long step = active[0]->step;
    const bool init = step == 0;
    for (const auto& g : b->outlets) {
      const hipError_t e =
          launch_batch_outlet(g.storage, g.d_aux[par], g.d_first, (int)g.cases.size(), g.nblocks, step, b->stream);
      if (e != hipSuccess) return batch_fail(b, LBM_EDEVICE, std::string("outlet kernel: ") + hipGetErrorString(e));
    }
    for (const auto& g : b->groups) {
      const hipError_t e = launch_batch(g.storage, g.d_args[par], g.d_first, (int)g.cases.size(), g.nblocks, init,
                                        g.tx, g.ty, g.lat, b->stream);
      if (e != hipSuccess) return batch_fail(b, LBM_EDEVICE, std::string("batch step kernel: ") + hipGetErrorString(e));
    }
    for (const auto& g : b->inflows) {
      const hipError_t e =
          launch_batch_inflow(g.storage, g.d_step[par], g.d_first, (int)g.cases.size(), g.nblocks, step, b->stream);
      if (e != hipSuccess) return batch_fail(b, LBM_EDEVICE, std::string("inflow kernel: ") + hipGetErrorString(e));
    }
    for (lbm_ctx* c : active) {
      c->cur = 1 - c->cur;
      if (c->geo.face_hi == FACE_OUTFLOW) c->out_cur = 1 - c->out_cur;
      c->step++;
    }
  }
  if (hipEventRecord(b->ev1, b->stream) != hipSuccess) return batch_fail(b, LBM_EDEVICE, "event record failed");
  b->last_ms = -(double)nsteps;
  return LBM_OK;
}

extern "C" int lbm_batch_unstable_cases(lbm_batch* b, int* flags) {
  if (!b) return -1;
  if (hipStreamSynchronize(b->stream) != hipSuccess) {
    batch_fail(b, LBM_EDEVICE, "stream synchronisation failed");
    return -1;
  }
  const int count = refresh_unstable(b);
  if (count < 0) {
    batch_fail(b, LBM_EDEVICE, "reading the instability flags failed");
    return -1;
  }
  if (flags)
    for (size_t k = 0; k < b->c.size(); ++k) flags[k] = b->c[k]->frozen ? 1 : 0;
  return count;
}

extern "C" lbm_status lbm_batch_sync(lbm_batch* b) {
  if (!b) return LBM_EINVAL;
  const hipError_t e = hipStreamSynchronize(b->stream);
  return e == hipSuccess ? LBM_OK : batch_fail(b, LBM_EDEVICE, hipGetErrorString(e));
}

extern "C" double lbm_batch_last_step_ms(const lbm_batch* cb) {
  lbm_batch* b = const_cast<lbm_batch*>(cb);
  if (!b) return 0.0;
  if (b->last_ms < 0.0) {
    const double steps = -b->last_ms;
    float ms = 0.0f;
    if (hipEventSynchronize(b->ev1) != hipSuccess || hipEventElapsedTime(&ms, b->ev0, b->ev1) != hipSuccess) return 0.0;
    b->last_ms = ms / steps;
  }
  return b->last_ms;
}

// Time every supported tile shape on a scratch lattice with the parameters of c (blue fluid
// at rest) for trial_steps steps each, on `stream`, and return the fastest in (tx, ty).  c's
// own state is not touched.
static lbm_status time_tile_shapes(const lbm_ctx* c, void* stream, int trial_steps, int& tx, int& ty,
                                   std::string& err) {
  static const int shapes[][2] = {{32, 8}, {64, 4}, {32, 4}};
  lbm_ctx* t = nullptr;
  lbm_status st = lbm_create(&c->p, stream, &t);
  if (st != LBM_OK) {
    err = g_create_error;
    return st;
  }
  const size_t n = (size_t)c->geo.n;
  std::vector<double> rr(n, 0.0), rb(n, c->p.rho_b0);
  st = lbm_init_fields(t, rr.data(), rb.data(), nullptr);
  double best = -1.0;
  tx = 32;
  ty = 8;
  for (const auto& sh : shapes) {
    if (st != LBM_OK) break;
    if ((st = lbm_set_tiling(t, sh[0], sh[1], 0)) != LBM_OK) break;
    t->zchunk = 0;
    if ((st = lbm_step(t, 1)) != LBM_OK || (st = lbm_step(t, trial_steps)) != LBM_OK) break;
    const double ms = lbm_last_step_kernel_ms(t);
    if (ms <= 0.0) {
      st = LBM_EDEVICE;
      t->err = "no kernel time recorded";
      break;
    }
    if (best < 0.0 || ms < best) {
      best = ms;
      tx = sh[0];
      ty = sh[1];
    }
  }
  err = t->err;
  lbm_destroy(t);
  return st;
}

extern "C" lbm_status lbm_autotune(lbm_ctx* c, int trial_steps) {
  if (!c) return LBM_EINVAL;
  if (trial_steps < 1) return fail(c, LBM_EINVAL, "trial_steps must be >= 1");
  int tx = 0, ty = 0;
  std::string err;
  const lbm_status st = time_tile_shapes(c, c->stream, trial_steps, tx, ty, err);
  if (st != LBM_OK) return fail(c, st, "autotune: " + err);
  c->tx = tx;
  c->ty = ty;
  c->zchunk = 0;
  return LBM_OK;
}

extern "C" lbm_status lbm_get_tiling(const lbm_ctx* c, int* tx, int* ty, int* zchunk) {
  if (!c || !tx || !ty || !zchunk) return LBM_EINVAL;
  *tx = c->tx;
  *ty = c->ty;
  *zchunk = c->zchunk;
  return LBM_OK;
}

// Autotuner of a batch: one timing per distinct (lattice shape, storage) of the batch.
extern "C" lbm_status lbm_batch_autotune(lbm_batch* b, int trial_steps) {
  if (!b || trial_steps < 1) return LBM_EINVAL;
  struct Pick {
    int nx, ny, nz, storage, tx, ty;
  };
  std::vector<Pick> picks;
  for (lbm_ctx* c : b->c) {
    const Geo& G = c->geo;
    const Pick* found = nullptr;
    for (const Pick& p : picks)
      if (p.nx == G.nx && p.ny == G.ny && p.nz == G.nz && p.storage == (int)c->p.storage) found = &p;
    if (!found) {
      Pick p{G.nx, G.ny, G.nz, (int)c->p.storage, 32, 8};
      std::string err;
      const lbm_status st = time_tile_shapes(c, b->stream, trial_steps, p.tx, p.ty, err);
      if (st != LBM_OK) return batch_fail(b, st, "autotune: " + err);
      picks.push_back(p);
      found = &picks.back();
    }
    c->tx = found->tx;
    c->ty = found->ty;
    c->zchunk = 0;
  }
  return LBM_OK;
}

// ---------------------------------------------------------------- host self-checks
extern "C" lbm_status lbm_selftest_tile_sets_host(const lbm_params* params, int tx, int ty, int* counts) {
  if (!params || !counts) return LBM_EINVAL;
  if (!((tx == 32 && (ty == 4 || ty == 8 || ty == 16)) || (tx == 64 && (ty == 4 || ty == 8)))) return LBM_EINVAL;
  lbm_ctx tmp;
  tmp.p = *params;
  std::string msg;
  lbm_status st = check_params(params, &tmp, msg);
  if (st != LBM_OK) return fail(nullptr, st, msg);
  tmp.tx = tx;
  tmp.ty = ty;
  tmp.zchunk = tmp.geo.nz;
  StepArgs s{};
  fill_step_args(&tmp, 0, 0, s);
  const int nt = s.tiles_x * s.tiles_y;
  for (int k = 0; k < 3 * nt; ++k) counts[k] = 0;
  const bool walls = tmp.geo.wall_x || tmp.geo.wall_y;
  // the launches enqueue_one makes: one over all tiles without walls, else the interior and
  // the edges and corners of the frame for the storage type (reported together as the frame)
  int sets[kCorners + 1];
  const int nsets = walls ? wall_tile_sets((int)tmp.p.storage, sets) : 1;
  if (!walls) sets[0] = kAllTiles;
  for (int m = 0; m < nsets; ++m) {
    const int set = sets[m];
    const int b = set == kAllTiles ? 0 : (set == kInteriorTiles ? 1 : 2);
    s.tile_set = set;
    const int n = tiles_in_set(s);
    for (int t = 0; t < n; ++t) {
      int i = -1, j = -1;
      tile_of(s, t, i, j);
      if (i < 0 || i >= s.tiles_x || j < 0 || j >= s.tiles_y) return fail(nullptr, LBM_EDEVICE, "tile out of range");
      // the walls (bits of wall_flags) that the tile's cells, and its ring cells inside the
      // lattice, lie on must be among those its instance reflects at (a ring cell beyond a
      // wall, wrapped to the opposite side, is never read: there the stencil takes the
      // boundary cell)
      const int x0 = i * tx, y0 = j * ty;
      const int touched = (tmp.geo.wall_x && x0 == 0 ? 1 : 0) | (tmp.geo.wall_x && x0 + tx > tmp.geo.nx - 2 ? 2 : 0) |
                          (tmp.geo.wall_y && y0 == 0 ? 4 : 0) | (tmp.geo.wall_y && y0 + ty > tmp.geo.ny - 2 ? 8 : 0);
      if (walls && (touched & ~lat_mode_of(set, true)) != 0) return fail(nullptr, LBM_EDEVICE, "tile in the wrong set");
      counts[b * nt + j * s.tiles_x + i]++;
    }
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_selftest_collide_host(const lbm_params* params, const double* fr, const double* fb,
                                                const double* grad_phi, const double* grad_rho, double* out_r,
                                                double* out_b) {
  if (!params || !fr || !fb || !grad_phi || !grad_rho || !out_r || !out_b) return LBM_EINVAL;
  lbm_ctx tmp;
  tmp.p = *params;
  std::string msg;
  lbm_status st = check_params(params, &tmp, msg);
  if (st != LBM_OK) return fail(nullptr, st, msg);
  double rr = 0.0, rb = 0.0;
  for (int i = 0; i < Q; ++i) {
    rr += fr[i];
    rb += fb[i];
  }
  const double rho = rr + rb, a = rr / rho;
  const double abar = tmp.pc.alpha_b + a * (tmp.pc.alpha_r - tmp.pc.alpha_b);
  float df[Q];
  for (int i = 0; i < Q; ++i) {
    const double ph = i == 0 ? abar : (1.0 - abar) * q_of(i);
    df[i] = (float)(fr[i] + fb[i] - rho * ph);
  }
  const float gp[3] = {(float)grad_phi[0], (float)grad_phi[1], (float)grad_phi[2]};
  const float gr[3] = {(float)grad_rho[0], (float)grad_rho[1], (float)grad_rho[2]};
  CellOut o;
  collide_cell(tmp.cp, tmp.rates, df, 0.0f, 0.0f, (float)rho, (float)rr, (float)rb, gp, gr, o);
  const double ab2 = tmp.pc.alpha_b + (double)o.a * (tmp.pc.alpha_r - tmp.pc.alpha_b);
  for (int i = 0; i < Q; ++i) {
    const double ph = i == 0 ? ab2 : (1.0 - ab2) * q_of(i);
    const double f = (double)o.g[i] + (double)o.rho * ph;
    const double fri = (double)o.a * f + qc_of(i) * (CX[i] * (double)o.wx + CY[i] * (double)o.wy + CZ[i] * (double)o.wz);
    out_r[i] = fri;
    out_b[i] = f - fri;
  }
  return LBM_OK;
}
