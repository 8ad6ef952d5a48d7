// surr_ops.hip -- operators of the learned surrogate (include/surrogate.h): 3x3x3
// convolutions as implicit GEMMs on the matrix cores, their data and weight gradients, and
// the small element-wise operators of the encoder-decoder and its training.
//
// Convolution.  out[v][co] = sum_tap sum_ci in[v + off(tap)][ci] w[tap][co][ci] is a GEMM with
// M = voxels, N = cout, K = 27 cin.  One wave owns 32 voxels x 32 output channels and issues
// one v_mfma_f32_32x32x8_bf16 per (tap, 8 input channels): lane l holds the 4 input channels
// kq..kq+3 (kq = 4 (l / 32)) of voxel l % 32 as the A fragment and the same 4 channels of
// weight row co = l % 32 as the B fragment (both 8-byte loads in the channels-last layout);
// the 16 accumulators of lane l are rows 8 (r / 4) + kq + r % 4, column l % 32, of the tile.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "surrogate.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int kTapOff[27][3] = {
    {-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, -1}, {-1, 1, 0}, {-1, 1, 1},
    {0, -1, -1},  {0, -1, 0},  {0, -1, 1},  {0, 0, -1},  {0, 0, 0},  {0, 0, 1},  {0, 1, -1},  {0, 1, 0},  {0, 1, 1},
    {1, -1, -1},  {1, -1, 0},  {1, -1, 1},  {1, 0, -1},  {1, 0, 0},  {1, 0, 1},  {1, 1, -1},  {1, 1, 0},  {1, 1, 1}};

// ---------------------------------------------------------------- forward convolution
// grid (ceil(nvox / 128), cout / 32), 256 threads: wave w of block b owns voxels
// [(4 b + w) 32, +32) and output channels [32 blockIdx.y, +32).
__global__ void __launch_bounds__(256) conv_fwd_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, uint16_t* __restrict__ out,
                                                       float* __restrict__ out_f32, int D, int H, int W, int cin,
                                                       int cout, int relu, long long nvox) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long v0 = ((long long)blockIdx.x * 4 + wave) * 32;
  if (v0 >= nvox) return;  // the whole wave leaves; the kernel has no barrier
  const int co0 = blockIdx.y * 32;
  const long long va = v0 + (lane & 31);
  const bool valid = va < nvox;
  int x = 0, y = 0, z = 0;
  long long nb = 0;
  if (valid) {
    long long t = va;
    x = (int)(t % W);
    t /= W;
    y = (int)(t % H);
    t /= H;
    z = (int)(t % D);
    nb = t / D;
  }
  const int kq = (lane >> 5) * 4;
  floatx16 acc = {};
  for (int tap = 0; tap < 27; ++tap) {
    const int zz = z + kTapOff[tap][0], yy = y + kTapOff[tap][1], xx = x + kTapOff[tap][2];
    const bool inb = valid && zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
    const long long src = inb ? ((nb * D + zz) * H + yy) * (long long)W + xx : 0;
    const uint16_t* arow = in + src * cin + kq;
    const uint16_t* brow = w + ((long long)tap * cout + co0 + (lane & 31)) * cin + kq;
    for (int c0 = 0; c0 < cin; c0 += 8) {
      bf16x4 a = {0, 0, 0, 0};
      if (inb) a = *reinterpret_cast<const bf16x4*>(arow + c0);
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(brow + c0);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
  }
  const int col = co0 + (lane & 31);
  const float bb = bias ? bias[col] : 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const long long v = v0 + (r / 4) * 8 + kq + (r & 3);
    if (v < nvox) {
      float val = acc[r] + bb;
      if (relu) val = fmaxf(val, 0.0f);
      if (out_f32)
        out_f32[v * cout + col] = val;
      else
        out[v * cout + col] = f2bf(val);
    }
  }
}

// w_t[tap'][ci][co] = w[26 - tap'][co][ci]
__global__ void flip_kernel(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int cin, int cout) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = 27LL * cin * cout;
  if (i >= total) return;
  const int co = (int)(i % cout);
  const int ci = (int)((i / cout) % cin);
  const int tap = (int)(i / ((long long)cout * cin));
  wt[i] = w[((long long)(26 - tap) * cout + co) * cin + ci];
}

// ---------------------------------------------------------------- weight gradient
// dw[tap][co][ci] = sum_v dout[v][co] in[v + off(tap)][ci]: GEMM with M = cout, N = cin,
// K = voxels.  The voxels are taken row by row (rows = (n, z, y), x fastest) in chunks of
// whole rows; one wave per (chunk, tap, co tile, ci tile) steps through its rows 8 voxels
// at a time, lane l holding voxels x0 + kq .. x0 + kq + 3.  Partial sums per chunk go to
// scratch and are added in chunk order by chunk_sum_kernel.
constexpr int kChunk = 16384;  // voxels per chunk (whole rows, at least one)

__host__ __device__ inline int rows_per_chunk(int W) { return W >= kChunk ? 1 : kChunk / W; }

__global__ void __launch_bounds__(64) wgrad_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ dout,
                                                   float* __restrict__ part, int D, int H, int W, int cin, int cout,
                                                   int nrows, int ci_tiles) {
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x, tap = blockIdx.y;
  const int co0 = (blockIdx.z / ci_tiles) * 32, ci0 = (blockIdx.z % ci_tiles) * 32;
  const int kq = (lane >> 5) * 4;
  const int co = co0 + (lane & 31), ci = ci0 + (lane & 31);
  const bool ci_ok = ci < cin;
  const int dz = kTapOff[tap][0], dy = kTapOff[tap][1], dx = kTapOff[tap][2];
  const int rpc = rows_per_chunk(W);
  const int r0 = chunk * rpc, r1 = min(r0 + rpc, nrows);
  floatx16 acc = {};
  for (int row = r0; row < r1; ++row) {
    const int y = row % H, z = (row / H) % D, nb = row / (H * D);
    const int yy = y + dy, zz = z + dz;
    const bool row_ok = ci_ok && yy >= 0 && yy < H && zz >= 0 && zz < D;
    const long long orow = (long long)row * W;                      // first voxel of this row
    const long long irow = ((long long)(nb * D + zz) * H + yy) * W;  // first voxel of the source row
    for (int x0 = 0; x0 < W; x0 += 8) {
      bf16x4 a, b;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = x0 + kq + j, xx = x + dx;
        uint16_t av = 0, bv = 0;
        if (x < W) {
          av = dout[(orow + x) * cout + co];
          if (row_ok && xx >= 0 && xx < W) bv = in[(irow + xx) * cin + ci];
        }
        a[j] = (short)av;
        b[j] = (short)bv;
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
  }
  // acc row m = co0 + 8 (r/4) + kq + r%4, column n = ci0 + lane % 32
  float* dst = part + (long long)chunk * 27 * cout * cin + (long long)tap * cout * cin;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = co0 + (r / 4) * 8 + kq + (r & 3);
    if (ci_ok) dst[(long long)m * cin + ci] = acc[r];
  }
}

// dbias partials: block = chunk of rows, thread t sums channel t % cout over its voxels.
__global__ void __launch_bounds__(256) bias_part_kernel(const uint16_t* __restrict__ dout, float* __restrict__ part,
                                                        int cout, int W, int nrows) {
  __shared__ float s[256];
  const int t = threadIdx.x;
  const int P = 256 / cout;
  const int c = t % cout, p = t / cout;
  const int rpc = rows_per_chunk(W);
  const long long vbeg = (long long)blockIdx.x * rpc * W, vend = (long long)min(blockIdx.x * rpc + rpc, nrows) * W;
  float acc = 0.0f;
  if (p < P)
    for (long long v = vbeg + p; v < vend; v += P) acc += bf2f(dout[v * cout + c]);
  s[t] = acc;
  __syncthreads();
  if (t < cout) {
    float sum = 0.0f;
    for (int q = 0; q < P; ++q) sum += s[q * cout + t];
    part[(long long)blockIdx.x * cout + t] = sum;
  }
}

__global__ void chunk_sum_kernel(const float* __restrict__ part, float* __restrict__ out, long long len, int nchunks) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.0f;
  for (int k = 0; k < nchunks; ++k) s += part[(long long)k * len + i];
  out[i] = s;
}

// ---------------------------------------------------------------- element-wise operators
__global__ void relu_bwd_kernel(const uint16_t* __restrict__ y, const uint16_t* __restrict__ dy,
                                uint16_t* __restrict__ dx, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dx[i] = bf2f(y[i]) > 0.0f ? dy[i] : (uint16_t)0;
}

// (d, h, w): dimensions of the fine lattice
__global__ void pool_fwd_kernel(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int d, int h, int w, int c,
                                long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int ch = (int)(i % c);
  long long t = i / c;
  const int x = (int)(t % (w / 2));
  t /= (w / 2);
  const int y = (int)(t % (h / 2));
  t /= (h / 2);
  const int z = (int)(t % (d / 2));
  const long long n = t / (d / 2);
  float s = 0.0f;
  for (int k = 0; k < 8; ++k) {
    const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
    s += bf2f(in[(((n * d + zz) * h + yy) * (long long)w + xx) * c + ch]);
  }
  out[i] = f2bf(0.125f * s);
}

__global__ void pool_bwd_kernel(const uint16_t* __restrict__ dout, uint16_t* __restrict__ din, int d, int h, int w,
                                int c, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int ch = (int)(i % c);
  long long t = i / c;
  const int x = (int)(t % w);
  t /= w;
  const int y = (int)(t % h);
  t /= h;
  const int z = (int)(t % d);
  const long long n = t / d;
  const float g = bf2f(dout[(((n * (d / 2) + z / 2) * (h / 2) + y / 2) * (long long)(w / 2) + x / 2) * c + ch]);
  din[i] = f2bf(0.125f * g);
}

// (d, h, w): dimensions of the coarse input; out and skip are 2d x 2h x 2w
__global__ void up_add_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ skip,
                              uint16_t* __restrict__ out, int d, int h, int w, int c, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int ch = (int)(i % c);
  long long t = i / c;
  const int x = (int)(t % (2 * w));
  t /= (2 * w);
  const int y = (int)(t % (2 * h));
  t /= (2 * h);
  const int z = (int)(t % (2 * d));
  const long long n = t / (2 * d);
  const float a = bf2f(in[(((n * d + z / 2) * h + y / 2) * (long long)w + x / 2) * c + ch]);
  out[i] = f2bf(a + bf2f(skip[i]));
}

__global__ void up_bwd_kernel(const uint16_t* __restrict__ dout, uint16_t* __restrict__ din, int d, int h, int w, int c,
                              long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int ch = (int)(i % c);
  long long t = i / c;
  const int x = (int)(t % w);
  t /= w;
  const int y = (int)(t % h);
  t /= h;
  const int z = (int)(t % d);
  const long long n = t / d;
  float s = 0.0f;
  for (int k = 0; k < 8; ++k) {
    const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
    s += bf2f(dout[(((n * 2 * d + zz) * (2 * h) + yy) * (long long)(2 * w) + xx) * c + ch]);
  }
  din[i] = f2bf(s);
}

__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ pred, const float* __restrict__ target,
                                                  uint16_t* __restrict__ dpred, float* __restrict__ loss_part,
                                                  long long count, int stride, int used) {
  __shared__ float s[256];
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  float e2 = 0.0f;
  if (v < count) {
    const float scale = 2.0f / ((float)count * (float)used);
    for (int k = 0; k < stride; ++k) {
      float g = 0.0f;
      if (k < used) {
        const float e = pred[v * stride + k] - target[v * used + k];
        e2 += e * e;
        g = scale * e;
      }
      dpred[v * stride + k] = f2bf(g);
    }
  }
  s[threadIdx.x] = e2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = s[0];
}

__global__ void adam_kernel(float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, long long count, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi, vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

__global__ void add_kernel(const uint16_t* __restrict__ a, const uint16_t* __restrict__ b, uint16_t* __restrict__ out,
                           long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = f2bf(bf2f(a[i]) + bf2f(b[i]));
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = f2bf(x[i]);
}

__global__ void to_f32_kernel(const uint16_t* __restrict__ x, float* __restrict__ y, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = bf2f(x[i]);
}

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }
inline unsigned blocks(long long count, int per) { return (unsigned)((count + per - 1) / per); }
inline int done() { return hipGetLastError() == hipSuccess ? 0 : -2; }

}  // namespace

extern "C" int surr_conv3d_fwd(const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, float* out_f32,
                               int n, int d, int h, int wd, int cin, int cout, int relu, void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cin % 8 || cout < 32 || cout % 32 || !in || !w ||
      (!out && !out_f32))
    return -1;
  const long long nvox = (long long)n * d * h * wd;
  hipLaunchKernelGGL(conv_fwd_kernel, dim3(blocks(nvox, 128), cout / 32), dim3(256), 0, S(stream), in, w, bias, out,
                     out_f32, d, h, wd, cin, cout, relu, nvox);
  return done();
}

extern "C" int surr_conv3d_flip_weights(const uint16_t* w, uint16_t* w_t, int cin, int cout, void* stream) {
  if (cin < 1 || cout < 1 || !w || !w_t) return -1;
  const long long total = 27LL * cin * cout;
  hipLaunchKernelGGL(flip_kernel, dim3(blocks(total, 256)), dim3(256), 0, S(stream), w, w_t, cin, cout);
  return done();
}

extern "C" int surr_conv3d_dgrad(const uint16_t* dout, const uint16_t* w_t, uint16_t* din, int n, int d, int h, int wd,
                                 int cin, int cout, void* stream) {
  // the forward convolution of dout (cout channels) with w_t gives din (cin channels)
  return surr_conv3d_fwd(dout, w_t, nullptr, din, nullptr, n, d, h, wd, cout, cin, 0, stream);
}

extern "C" size_t surr_conv3d_wgrad_scratch_bytes(int n, int d, int h, int wd, int cin, int cout) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || cin < 1 || cout < 1) return 0;
  const long long nrows = (long long)n * d * h;
  const long long nchunks = (nrows + rows_per_chunk(wd) - 1) / rows_per_chunk(wd);
  return (size_t)nchunks * ((size_t)27 * cout * cin + (size_t)cout) * sizeof(float);
}

extern "C" int surr_conv3d_wgrad(const uint16_t* in, const uint16_t* dout, float* dw, float* dbias, void* scratch, int n,
                                 int d, int h, int wd, int cin, int cout, void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cin % 8 || cout < 32 || cout % 32 || cout > 256 || !in ||
      !dout || !dw || !scratch)
    return -1;
  const long long nrows_ll = (long long)n * d * h;
  if (nrows_ll * wd >= (1LL << 31)) return -1;
  const int nrows = (int)nrows_ll;
  const int nchunks = (nrows + rows_per_chunk(wd) - 1) / rows_per_chunk(wd);
  const int ci_tiles = (cin + 31) / 32;
  float* part = static_cast<float*>(scratch);
  float* bpart = part + (size_t)nchunks * 27 * cout * cin;
  hipLaunchKernelGGL(wgrad_kernel, dim3(nchunks, 27, (cout / 32) * ci_tiles), dim3(64), 0, S(stream), in, dout, part, d,
                     h, wd, cin, cout, nrows, ci_tiles);
  const long long len = 27LL * cout * cin;
  hipLaunchKernelGGL(chunk_sum_kernel, dim3(blocks(len, 256)), dim3(256), 0, S(stream), part, dw, len, nchunks);
  if (dbias) {
    hipLaunchKernelGGL(bias_part_kernel, dim3(nchunks), dim3(256), 0, S(stream), dout, bpart, cout, wd, nrows);
    hipLaunchKernelGGL(chunk_sum_kernel, dim3(blocks(cout, 256)), dim3(256), 0, S(stream), bpart, dbias,
                       (long long)cout, nchunks);
  }
  return done();
}

extern "C" int surr_relu_bwd(const uint16_t* y, const uint16_t* dy, uint16_t* dx, long long count, void* stream) {
  if (count < 0 || !y || !dy || !dx) return -1;
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), y, dy, dx, count);
  return done();
}

extern "C" int surr_pool_fwd(const uint16_t* in, uint16_t* out, int n, int d, int h, int wd, int c, void* stream) {
  if (n < 1 || d < 2 || h < 2 || wd < 2 || (d | h | wd) & 1 || c < 1 || !in || !out) return -1;
  const long long count = (long long)n * (d / 2) * (h / 2) * (wd / 2) * c;
  hipLaunchKernelGGL(pool_fwd_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), in, out, d, h, wd, c, count);
  return done();
}

extern "C" int surr_pool_bwd(const uint16_t* dout, uint16_t* din, int n, int d, int h, int wd, int c, void* stream) {
  if (n < 1 || d < 2 || h < 2 || wd < 2 || (d | h | wd) & 1 || c < 1 || !dout || !din) return -1;
  const long long count = (long long)n * d * h * wd * c;
  hipLaunchKernelGGL(pool_bwd_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), dout, din, d, h, wd, c, count);
  return done();
}

extern "C" int surr_up_add_fwd(const uint16_t* in, const uint16_t* skip, uint16_t* out, int n, int d, int h, int wd,
                               int c, void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || c < 1 || !in || !skip || !out) return -1;
  const long long count = (long long)n * 8 * d * h * wd * c;
  hipLaunchKernelGGL(up_add_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), in, skip, out, d, h, wd, c,
                     count);
  return done();
}

extern "C" int surr_up_bwd(const uint16_t* dout, uint16_t* din, int n, int d, int h, int wd, int c, void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || c < 1 || !dout || !din) return -1;
  const long long count = (long long)n * d * h * wd * c;
  hipLaunchKernelGGL(up_bwd_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), dout, din, d, h, wd, c, count);
  return done();
}

extern "C" int surr_mse(const float* pred, const float* target, uint16_t* dpred, float* loss_part, long long count,
                        int stride, int used, void* stream) {
  if (count < 1 || stride < 1 || used < 1 || used > stride || !pred || !target || !dpred || !loss_part) return -1;
  hipLaunchKernelGGL(mse_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), pred, target, dpred, loss_part,
                     count, stride, used);
  return done();
}

extern "C" int surr_adam(float* w, uint16_t* w_bf16, const float* g, float* m, float* v, long long count, float lr,
                         float beta1, float beta2, float eps, int t, void* stream) {
  if (count < 0 || t < 1 || !w || !w_bf16 || !g || !m || !v) return -1;
  const float c1 = 1.0f / (1.0f - powf(beta1, (float)t)), c2 = 1.0f / (1.0f - powf(beta2, (float)t));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), w, w_bf16, g, m, v, count, lr,
                     beta1, beta2, eps, c1, c2);
  return done();
}

extern "C" int surr_add(const uint16_t* a, const uint16_t* b, uint16_t* out, long long count, void* stream) {
  if (count < 0 || !a || !b || !out) return -1;
  hipLaunchKernelGGL(add_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), a, b, out, count);
  return done();
}

extern "C" int surr_to_bf16(const float* x, uint16_t* y, long long count, void* stream) {
  if (count < 0 || !x || !y) return -1;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), x, y, count);
  return done();
}

extern "C" int surr_to_f32(const uint16_t* x, float* y, long long count, void* stream) {
  if (count < 0 || !x || !y) return -1;
  hipLaunchKernelGGL(to_f32_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), x, y, count);
  return done();
}
