// surr_ops.hip -- operators of the learned surrogate (include/surrogate.h): 3x3x3
// convolutions as implicit GEMMs on the matrix cores, their data and weight gradients, and
// the small element-wise operators of the encoder-decoder and its training.
//
// Convolution.  out[v][co] = sum_tap sum_ci in[v + off(tap)][ci] w[tap][co][ci] is a GEMM with
// M = voxels, N = cout, K = 27 cin.  The kernels that carry the network (conv_ring_kernel,
// conv_staged_kernel, wgrad_kernel) stage their operands through LDS and issue
// v_mfma_f32_32x32x16_bf16; conv_fwd_kernel, the direct form with one wave per 32 voxels x
// 32 output channels and v_mfma_f32_32x32x8_bf16 fed from global memory, serves channel
// counts the others do not take (cin = 128, and planes too large for 32-bit offsets).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "surrogate.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// v_mfma_f32_32x32x16_bf16: lane l supplies A[l % 32][8 (l / 32) + j] and B[8 (l / 32) + j][l % 32],
// j = 0..7, and holds D rows 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32, in accumulator r.
__device__ __forceinline__ floatx16 mfma16(uint4 a, uint4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                 0);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void unpack8(uint4 u, float (&f)[8]) {
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f[2 * i] = __uint_as_float(w[i] << 16);
    f[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
  }
}

__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = (uint32_t)f2bf(f[2 * i]) | ((uint32_t)f2bf(f[2 * i + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

constexpr int kTapOff[27][3] = {
    {-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, -1}, {-1, 1, 0}, {-1, 1, 1},
    {0, -1, -1},  {0, -1, 0},  {0, -1, 1},  {0, 0, -1},  {0, 0, 0},  {0, 0, 1},  {0, 1, -1},  {0, 1, 0},  {0, 1, 1},
    {1, -1, -1},  {1, -1, 0},  {1, -1, 1},  {1, 0, -1},  {1, 0, 0},  {1, 0, 1},  {1, 1, -1},  {1, 1, 0},  {1, 1, 1}};

// ---------------------------------------------------------------- forward convolution, direct
// v_mfma_f32_32x32x8_bf16: lane l holds the 4 input channels kq..kq+3 (kq = 4 (l / 32)) of
// voxel l % 32 as the A fragment and the same 4 channels of weight row co = l % 32 as the B
// fragment (8-byte loads in the channels-last layout); the 16 accumulators of lane l are rows
// 8 (r / 4) + kq + r % 4, column l % 32, of the tile.
// grid (ceil(nvox / 128), cout / (32 NT)), 256 threads: wave w of block b owns voxels
// [(4 b + w) 32, +32) and output channels [32 NT blockIdx.y, +32 NT).  CIN is the input
// channel count (a template constant, so the loads of a tap are issued ahead of its MFMAs);
// the A fragment of a tap is reused for the NT output-channel tiles.
template <int CIN, int NT>
__global__ void __launch_bounds__(256) conv_fwd_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, uint16_t* __restrict__ out,
                                                       float* __restrict__ out_f32, int D, int H, int W, int cout,
                                                       int relu, long long nvox) {
  constexpr int KS = CIN / 8;  // MFMA K steps per tap
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long v0 = ((long long)blockIdx.x * 4 + wave) * 32;
  if (v0 >= nvox) return;  // the whole wave leaves; the kernel has no barrier
  const int co0 = blockIdx.y * 32 * NT;
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
  floatx16 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = floatx16{};
  for (int tap = 0; tap < 27; ++tap) {
    const int zz = z + kTapOff[tap][0], yy = y + kTapOff[tap][1], xx = x + kTapOff[tap][2];
    const bool inb = valid && zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
    const long long src = inb ? ((nb * D + zz) * H + yy) * (long long)W + xx : 0;
    const uint16_t* arow = in + src * CIN + kq;
    bf16x4 a[KS], b[NT][KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      a[k] = bf16x4{0, 0, 0, 0};
      if (inb) a[k] = *reinterpret_cast<const bf16x4*>(arow + 8 * k);
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const uint16_t* brow = w + ((long long)tap * cout + co0 + 32 * j + (lane & 31)) * CIN + kq;
#pragma unroll
      for (int k = 0; k < KS; ++k) b[j][k] = *reinterpret_cast<const bf16x4*>(brow + 8 * k);
    }
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a[k], b[j][k], acc[j], 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int col = co0 + 32 * j + (lane & 31);
    const float bb = bias ? bias[col] : 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long long v = v0 + (r / 4) * 8 + kq + (r & 3);
      if (v < nvox) {
        float val = acc[j][r] + bb;
        if (relu) val = fmaxf(val, 0.0f);
        if (out_f32)
          out_f32[v * cout + col] = val;
        else
          out[v * cout + col] = f2bf(val);
      }
    }
  }
}

template <int CIN>
void launch_conv(const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, float* out_f32, int d, int h,
                 int wd, int cout, int relu, long long nvox, hipStream_t s) {
  if (cout % 64 == 0)
    hipLaunchKernelGGL((conv_fwd_kernel<CIN, 2>), dim3((unsigned)((nvox + 127) / 128), cout / 64), dim3(256), 0, s, in,
                       w, bias, out, out_f32, d, h, wd, cout, relu, nvox);
  else
    hipLaunchKernelGGL((conv_fwd_kernel<CIN, 1>), dim3((unsigned)((nvox + 127) / 128), cout / 32), dim3(256), 0, s, in,
                       w, bias, out, out_f32, d, h, wd, cout, relu, nvox);
}

// ---------------------------------------------------------------- forward convolution, staged
// For cin in {16, 32, 64}: a block of NW waves owns a co tile of 32 and walks tiles of two
// output rows x SEG voxels (grid-stride).  Per tile it stages into LDS every input voxel the
// tile reads -- 3 z-planes x 4 rows x (SEG + 2) voxels, all cin channels, zeros outside the
// volume -- with a voxel stride of cin + 8 elements (4 x an odd number of dwords, so each
// group of 8 lanes reading 16 bytes covers all banks once).  The K dimension of the GEMM,
// 27 cin / 16 steps of v_mfma_f32_32x32x16_bf16 over (tap, 16 input channels), is split
// evenly over the waves; each wave
// holds the weight fragments of its steps in registers for the whole kernel and accumulates
// every M-tile of the output tile over them.  The NW partial sums of an M-tile are added in
// wave order through LDS by the wave that finalizes it (m % NW).  NW = 8 for 64 channels
// keeps a wave's weight fragments at 56 registers.
template <int CIN>
struct StagedConv {
  static constexpr int SEG = CIN == 64 ? 32 : 64;  // voxels of an output row in a tile
  static constexpr int XT = SEG / 32;              // M-tiles per output row
  static constexpr int MT = 2 * XT;                // M-tiles per tile
  static constexpr int RV = SEG + 2;               // staged voxels per row
  static constexpr int VS = CIN + 8;               // staged voxel stride (elements)
  static constexpr int SL = CIN / 16;              // 16-channel slices (MFMA K-steps per tap)
  static constexpr int NW = CIN == 64 ? 8 : 4;     // waves per block
  static constexpr int KSTEPS = 27 * SL;
  static constexpr int IPW = (KSTEPS + NW - 1) / NW;  // K-steps of a wave, at most
  static constexpr int STAGE_BYTES = 12 * RV * VS * 2;
  static constexpr int RED_BYTES = (NW - 1) * MT * 4096;
  static constexpr int LDS_BYTES = STAGE_BYTES > RED_BYTES ? STAGE_BYTES : RED_BYTES;
  static_assert(LDS_BYTES <= 65536, "staged tile exceeds LDS");
};

template <int CIN>
__global__ void __launch_bounds__(64 * StagedConv<CIN>::NW, 2) conv_staged_kernel(const uint16_t* __restrict__ in,
                                                             const uint16_t* __restrict__ w,
                                                             const float* __restrict__ bias, uint16_t* __restrict__ out,
                                                             float* __restrict__ out_f32, int D, int H, int W, int cout,
                                                             int relu, long long ntiles) {
  using P = StagedConv<CIN>;
  __shared__ __align__(16) unsigned char lds[P::LDS_BYTES];
  uint16_t* st = reinterpret_cast<uint16_t*>(lds);
  float* red = reinterpret_cast<float*>(lds);
  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, c = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int co0 = blockIdx.y * 32;
  const int k0 = P::KSTEPS * wave / P::NW, nk = P::KSTEPS * (wave + 1) / P::NW - k0;

  uint4 wb[P::IPW];
#pragma unroll
  for (int i = 0; i < P::IPW; ++i) {
    wb[i] = make_uint4(0, 0, 0, 0);
    if (i < nk) {
      const int k = k0 + i, tap = k / P::SL, sl = k % P::SL;
      wb[i] = *reinterpret_cast<const uint4*>(w + ((long long)tap * cout + co0 + c) * CIN + sl * 16 + 8 * h);
    }
  }
  const float bb = bias ? bias[co0 + c] : 0.0f;
  const int lane_off = c * P::VS + 8 * h;
  const int nseg = (W + P::SEG - 1) / P::SEG, nyp = (H + 1) / 2;

  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int yp = (int)(tile % nyp);
    const long long col = tile / nyp;  // (n D + z) nseg + seg
    const int seg = (int)(col % nseg);
    const long long nz = col / nseg;
    const int z = (int)(nz % D);
    const int x0 = seg * P::SEG, y0 = 2 * yp;

    __syncthreads();  // the previous tile's reads of LDS are done
    constexpr int Q = CIN / 8;  // 16-byte chunks of a voxel
    for (int it = t; it < 12 * P::RV * Q; it += 64 * P::NW) {
      const int q = it % Q, v = (it / Q) % P::RV, row = it / (Q * P::RV);
      const int dz = row / 4 - 1, ys = y0 + row % 4 - 1, zs = z + dz, x = x0 + v - 1;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (zs >= 0 && zs < D && ys >= 0 && ys < H && x >= 0 && x < W)
        val = *reinterpret_cast<const uint4*>(in + (((nz + dz) * H + ys) * (long long)W + x) * CIN + 8 * q);
      *reinterpret_cast<uint4*>(st + (row * P::RV + v) * P::VS + 8 * q) = val;
    }
    __syncthreads();

    floatx16 acc[P::MT];
#pragma unroll
    for (int m = 0; m < P::MT; ++m) acc[m] = floatx16{};
#pragma unroll
    for (int i = 0; i < P::IPW; ++i) {
      if (i < nk) {
        const int k = k0 + i, tap = k / P::SL, sl = k % P::SL;
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;  // each offset + 1
        const uint16_t* a0 = st + ((dz * 4 + dy) * P::RV + dx) * P::VS + sl * 16 + lane_off;
#pragma unroll
        for (int m = 0; m < P::MT; ++m) {
          const int moff = (m / P::XT) * P::RV * P::VS + (m % P::XT) * 32 * P::VS;
          acc[m] = mfma16(*reinterpret_cast<const uint4*>(a0 + moff), wb[i], acc[m]);
        }
      }
    }

    __syncthreads();  // every wave is done with the staged rows; LDS now holds partial sums
#pragma unroll
    for (int m = 0; m < P::MT; ++m) {
      const int f = m % P::NW;
      if (wave != f) {
        float* slot = red + (m * (P::NW - 1) + (wave < f ? wave : wave - 1)) * 1024;
#pragma unroll
        for (int r = 0; r < 16; ++r) slot[r * 64 + lane] = acc[m][r];
      }
    }
    __syncthreads();
    if (wave < P::MT) {  // wave m finalizes tile m (MT <= NW): its partial plus the others' in wave order
      floatx16 mine = acc[0];
#pragma unroll
      for (int m = 1; m < P::MT; ++m)
        if (wave == m) mine = acc[m];
      const int m = wave;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        float sum = 0.0f;
#pragma unroll
        for (int ww = 0; ww < P::NW; ++ww)
          sum += ww == m ? mine[e] : red[(m * (P::NW - 1) + (ww < m ? ww : ww - 1)) * 1024 + e * 64 + lane];
        mine[e] = sum;
      }
      const int y = y0 + m / P::XT;
      if (y < H) {
        int co = cout;
        asm volatile("" : "+s"(co));  // keeps the per-element offsets from being hoisted as addresses
        const int xb = x0 + (m % P::XT) * 32 + 4 * h;
        const long long obase = ((nz * H + y) * (long long)W + xb) * co + co0 + c;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          if (xb + (e / 4) * 8 + (e & 3) < W) {
            float val = mine[e] + bb;
            if (relu) val = fmaxf(val, 0.0f);
            const long long o = obase + ((e / 4) * 8 + (e & 3)) * co;
            if (out_f32)
              out_f32[o] = val;
            else
              out[o] = f2bf(val);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- forward convolution, z ring
// For cin in {8, 16, 32}: as the staged kernel (four waves split the K-steps, weights in
// registers, output tiles of two rows x 64 voxels), but a block owns a column (n, row pair,
// segment) and sweeps a range of z: the three input planes z - 1, z, z + 1 (4 rows x 66
// voxels each) live in a ring in LDS, so each output plane stages one new plane, and the
// loads of plane z + 2 are issued before the MFMAs of plane z and stored after them.  The
// four partial sums of the four M-tiles are exchanged in three rounds through a separate
// buffer: in round r wave w passes its partial of tile (w + r + 1) % 4 to the wave that owns
// that tile, which adds it to its own (a fixed order per tile).  With 8 channels a K-step
// pairs two taps: lane half h takes tap 2 k + h (k = 13: tap 26 and a zero weight), and the
// voxel stride of 8 elements (4 dwords) is already conflict-free.
template <int CIN>
struct RingConv {
  static constexpr int SEG = 64, XT = 2, MT = 4, NW = 4;
  static constexpr int RV = SEG + 2;                 // staged voxels per row
  static constexpr int VS = CIN == 8 ? 8 : CIN + 8;  // staged voxel stride (elements)
  static constexpr int SL = CIN == 8 ? 1 : CIN / 16; // MFMA K-steps per tap (per tap pair for 8)
  static constexpr int Q = CIN / 8;                  // 16-byte chunks of a voxel
  static constexpr int KSTEPS = CIN == 8 ? 14 : 27 * SL, IPW = (KSTEPS + NW - 1) / NW;
  static constexpr int PLANE = 4 * RV * VS;          // elements of a staged plane
  static constexpr int CHUNKS = 4 * RV * Q;          // 16-byte chunks of a plane
  static constexpr int PF = (CHUNKS + 64 * NW - 1) / (64 * NW);  // chunks per thread
};

template <int CIN>
__global__ void __launch_bounds__(256, 2) conv_ring_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                           const float* __restrict__ bias, uint16_t* __restrict__ out,
                                                           float* __restrict__ out_f32, int D, int H, int W, int cout,
                                                           int relu, int nzc, int zlen, long long nitems) {
  using P = RingConv<CIN>;
  __shared__ __align__(16) uint16_t ring[3 * P::PLANE];
  __shared__ __align__(16) float xch[P::NW * 1024];
  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, c = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int co0 = blockIdx.y * 32;
  const int k0 = P::KSTEPS * wave / P::NW, nk = P::KSTEPS * (wave + 1) / P::NW - k0;

  uint4 wb[P::IPW];
#pragma unroll
  for (int i = 0; i < P::IPW; ++i) {
    wb[i] = make_uint4(0, 0, 0, 0);
    if (i < nk) {
      const int k = k0 + i;
      if constexpr (CIN == 8) {
        const int tap = 2 * k + h;
        if (tap < 27) wb[i] = *reinterpret_cast<const uint4*>(w + ((long long)tap * cout + co0 + c) * CIN);
      } else {
        const int tap = k / P::SL, sl = k % P::SL;
        wb[i] = *reinterpret_cast<const uint4*>(w + ((long long)tap * cout + co0 + c) * CIN + sl * 16 + 8 * h);
      }
    }
  }
  const float bb = bias ? bias[co0 + c] : 0.0f;
  const int lane_off = c * P::VS + (CIN == 8 ? 0 : 8 * h);
  const int nseg = (W + P::SEG - 1) / P::SEG, nyp = (H + 1) / 2;
  const long long plane_elems = (long long)H * W * CIN;
  // wave w owns output tile w: row y0 + w / 2, voxels x0 + 32 (w % 2) ..
  const int my_row = wave / P::XT, my_x = (wave % P::XT) * 32;

  // the staged chunks this thread moves: offset within an input plane (-1 where the voxel
  // is outside the plane or the chunk index is past the plane)
  int src_off[P::PF];

  auto store_plane = [&](int p, const uint4(&buf)[P::PF]) {
    uint16_t* dst = ring + ((p + 3) % 3) * P::PLANE;
#pragma unroll
    for (int k = 0; k < P::PF; ++k) {
      const int it = t + 64 * P::NW * k;
      if (it < P::CHUNKS) {
        const int q = it % P::Q, v = (it / P::Q) % P::RV, r = it / (P::Q * P::RV);
        *reinterpret_cast<uint4*>(dst + (r * P::RV + v) * P::VS + 8 * q) = buf[k];
      }
    }
  };

#pragma unroll 1
  for (long long item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int zc = (int)(item % nzc);
    const long long col = item / nzc;  // (n nyp + yp) nseg + seg
    const int seg = (int)(col % nseg);
    const int yp = (int)((col / nseg) % nyp);
    const long long nb = col / ((long long)nseg * nyp);
    const int x0 = seg * P::SEG, y0 = 2 * yp;
    const int za = zc * zlen, zb = min(D, za + zlen);
    const uint16_t* in_n = in + nb * D * plane_elems;
#pragma unroll
    for (int k = 0; k < P::PF; ++k) {
      const int it = t + 64 * P::NW * k;
      src_off[k] = -1;
      if (it < P::CHUNKS) {
        const int q = it % P::Q, v = (it / P::Q) % P::RV, r = it / (P::Q * P::RV);
        const int ys = y0 + r - 1, x = x0 + v - 1;
        if (ys >= 0 && ys < H && x >= 0 && x < W) src_off[k] = (ys * W + x) * CIN + 8 * q;
      }
    }
    auto load = [&](int p, uint4(&buf)[P::PF]) {
      const bool pin = p >= 0 && p < D;
      const uint16_t* base = in_n + (long long)p * plane_elems;
#pragma unroll
      for (int k = 0; k < P::PF; ++k) {
        buf[k] = make_uint4(0, 0, 0, 0);
        if (pin && src_off[k] >= 0) buf[k] = *reinterpret_cast<const uint4*>(base + src_off[k]);
      }
    };

    uint4 pf[P::PF];
    __syncthreads();  // the previous item's reads of the ring are done
    load(za - 1, pf);
    store_plane(za - 1, pf);
    load(za, pf);
    store_plane(za, pf);
    load(za + 1, pf);
    int sm = ((za + 2) % 3) * P::PLANE, s0 = (za % 3) * P::PLANE, sp = ((za + 1) % 3) * P::PLANE;  // z - 1, z, z + 1
#pragma unroll 1
    for (int z = za; z < zb; ++z) {
      store_plane(z + 1, pf);  // its slot held plane z - 2, last read before the previous exchange
      __syncthreads();
      if (z + 1 < zb) load(z + 2, pf);

      floatx16 acc[P::MT];
#pragma unroll
      for (int m = 0; m < P::MT; ++m) acc[m] = floatx16{};
      int lo = lane_off;
      asm volatile("" : "+v"(lo));  // keeps the per-step A addresses inside the z loop
#pragma unroll
      for (int i = 0; i < P::IPW; ++i) {
        if (i < nk) {
          const int k = k0 + i;
          int tap, sl;
          if constexpr (CIN == 8) {
            tap = min(2 * k + h, 26);  // lane-dependent; the zero weight of tap 27 reads tap 26
            sl = 0;
          } else {
            tap = k / P::SL;
            sl = k % P::SL;
          }
          const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;  // each offset + 1
          const int sb = dz == 0 ? sm : (dz == 1 ? s0 : sp);
          const uint16_t* a0 = ring + sb + (dy * P::RV + dx) * P::VS + sl * 16 + lo;
#pragma unroll
          for (int m = 0; m < P::MT; ++m) {
            const int moff = (m / P::XT) * P::RV * P::VS + (m % P::XT) * 32 * P::VS;
            acc[m] = mfma16(*reinterpret_cast<const uint4*>(a0 + moff), wb[i], acc[m]);
          }
        }
      }
      {
        const int tmp = sm;
        sm = s0;
        s0 = sp;
        sp = tmp;
      }

      // the partial sums: round r, wave w sends tile (w + r + 1) % 4 and adds the one from
      // wave (w - r - 1) % 4 to its own tile w (copies chosen by wave-uniform branches keep
      // the accumulators in registers)
      floatx16 mine = acc[0];
      if (wave == 1) mine = acc[1];
      if (wave == 2) mine = acc[2];
      if (wave == 3) mine = acc[3];
#pragma unroll
      for (int r = 0; r < P::NW - 1; ++r) {
        const int send = (wave + r + 1) % P::NW, from = (wave + P::NW - r - 1) % P::NW;
        floatx16 snd = acc[0];
        if (send == 1) snd = acc[1];
        if (send == 2) snd = acc[2];
        if (send == 3) snd = acc[3];
#pragma unroll
        for (int e = 0; e < 16; ++e) xch[wave * 1024 + e * 64 + lane] = snd[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) mine[e] += xch[from * 1024 + e * 64 + lane];
        __syncthreads();
      }
      const int y = y0 + my_row;
      if (y < H) {
        // element e of the tile is voxel xb + (e / 4) * 8 + e % 4; one base per step and
        // per-element offsets in multiples of cout (made opaque so they are not hoisted out
        // of the z loop as 16 separate 64-bit addresses)
        int co = cout;
        asm volatile("" : "+s"(co));
        const int xb = x0 + my_x + 4 * h;
        const long long obase = (((nb * D + z) * H + y) * (long long)W + xb) * co + co0 + c;
        if (out_f32) {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            if (xb + (e / 4) * 8 + (e & 3) < W) {
              const float val = mine[e] + bb;
              out_f32[obase + ((e / 4) * 8 + (e & 3)) * co] = relu ? fmaxf(val, 0.0f) : val;
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            if (xb + (e / 4) * 8 + (e & 3) < W) {
              const float val = mine[e] + bb;
              out[obase + ((e / 4) * 8 + (e & 3)) * co] = f2bf(relu ? fmaxf(val, 0.0f) : val);
            }
          }
        }
      }
    }
  }
}

template <int CIN>
void launch_ring(const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, float* out_f32, int n, int d,
                 int h, int wd, int cout, int relu, hipStream_t s) {
  using P = RingConv<CIN>;
  const int ctiles = cout / 32;
  const long long ncols = (long long)n * ((h + 1) / 2) * ((wd + P::SEG - 1) / P::SEG);
  const long long target = (512 + ctiles - 1) / ctiles;  // two resident blocks on each of 256 CUs
  long long nzc = (target + ncols - 1) / ncols;
  if (nzc > d) nzc = d;
  const int zlen = (int)((d + nzc - 1) / nzc);
  nzc = (d + zlen - 1) / zlen;
  const long long nitems = ncols * nzc;
  const unsigned gx = (unsigned)(nitems < target ? nitems : target);
  hipLaunchKernelGGL(conv_ring_kernel<CIN>, dim3(gx, ctiles), dim3(256), 0, s, in, w, bias, out, out_f32, d, h, wd, cout,
                     relu, (int)nzc, zlen, nitems);
}

template <int CIN>
void launch_staged(const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, float* out_f32, int n,
                   int d, int h, int wd, int cout, int relu, hipStream_t s) {
  using P = StagedConv<CIN>;
  const long long ntiles = (long long)n * d * ((wd + P::SEG - 1) / P::SEG) * ((h + 1) / 2);
  const int ctiles = cout / 32;
  const long long want = (512 + ctiles - 1) / ctiles;  // two resident blocks on each of 256 CUs
  const unsigned gx = (unsigned)(ntiles < want ? ntiles : want);
  hipLaunchKernelGGL(conv_staged_kernel<CIN>, dim3(gx, ctiles), dim3(64 * P::NW), 0, s, in, w, bias, out, out_f32, d, h, wd,
                     cout, relu, ntiles);
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
// dw[tap][co][ci] = sum_v dout[v][co] in[v + off(tap)][ci]: per tap a GEMM with M = cout,
// N = cin, K = voxels.  The voxels are walked as row segments of kSeg along x, ordered
// (n, z, segment, y) with y fastest; block (c, tile) of three waves owns the (co, ci) tile of
// 32 x 32 and the c-th of nchunks contiguous ranges of row segments.  Wave k accumulates
// the nine taps with dz = k - 1.  Per segment the block stages dout^T [co][x] into LDS, and
// wave k stages the source rows (z + dz, y') as in^T [ci][x] over x0 - 4 .. x0 + kSeg + 3;
// the three rows y - 1, y, y + 1 live in a ring, so the next segment of the same column
// stages only row y + 2.  The K order of an MFMA is free: with v_mfma_f32_32x32x16_bf16 lane
// half h takes voxels x0 + 32 h + 8 s + j at step s, so each lane walks its 32 voxels eight
// at a time and the dx = -1, +1 operands are its aligned 16-byte words shifted by one
// element, the word before or after coming from the previous or the next step.
constexpr int kSeg = 64;            // voxels per row segment
constexpr int kRsA = kSeg + 8;      // LDS row stride of dout^T (elements; 36 dwords)
constexpr int kRowB = kSeg + 16;    // staged source row, x0 - 8 .. x0 + kSeg + 7
constexpr int kRsB = kRowB + 8;     // LDS row stride of in^T (44 dwords)
// Channel row r of a staged tile starts at r * stride + (r / 8) * 16 elements: the 8-dword
// shift per group of 8 rows spreads the transposing 2-byte stores of the four 8-channel
// groups over distinct banks (stride * 8 is a multiple of 32 dwords); 16-byte reads along x
// keep their conflict-free pattern.
__host__ __device__ constexpr int trow(int r, int stride) { return r * stride + (r >> 3) * 16; }
constexpr int kTileA = 32 * kRsA + 4 * 16;  // elements of a staged dout^T tile
constexpr int kTileB = 32 * kRsB + 4 * 16;  // elements of a staged in^T row
constexpr int kWgradBlocks = 512;   // two resident blocks (LDS-bound) on each of 256 compute units

__host__ __device__ inline int nseg_of(int W) { return (W + kSeg - 1) / kSeg; }

struct WgradPlan {
  long long nsr;  // row segments
  int nchunks, ci_tiles, tiles;
};

inline WgradPlan wgrad_plan(int n, int d, int h, int wd, int cin, int cout) {
  WgradPlan p;
  p.nsr = (long long)n * d * h * nseg_of(wd);
  p.ci_tiles = (cin + 31) / 32;
  p.tiles = (cout / 32) * p.ci_tiles;
  const long long want = (kWgradBlocks + p.tiles - 1) / p.tiles;
  p.nchunks = (int)(want < p.nsr ? want : p.nsr);
  if (p.nchunks < 1) p.nchunks = 1;
  return p;
}

// [p.e7, c.e0 .. c.e6] and [c.e1 .. c.e7, n.e0] of 8-element BF16 words (element 2i in the
// low half of dword i)
__device__ __forceinline__ uint4 shift_in_prev(uint4 p, uint4 c) {
  return make_uint4((c.x << 16) | (p.w >> 16), (c.y << 16) | (c.x >> 16), (c.z << 16) | (c.y >> 16),
                    (c.w << 16) | (c.z >> 16));
}
__device__ __forceinline__ uint4 shift_in_next(uint4 c, uint4 n) {
  return make_uint4((c.x >> 16) | (c.y << 16), (c.y >> 16) | (c.z << 16), (c.z >> 16) | (c.w << 16),
                    (c.w >> 16) | (n.x << 16));
}

__global__ void __launch_bounds__(192, 2) wgrad_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ dout,
                                                       float* __restrict__ part, float* __restrict__ bpart, int D, int H,
                                                       int W, int cin, int cout, long long nsr, int nchunks,
                                                       int ci_tiles) {
  __shared__ __align__(16) uint16_t sA[kTileA];
  __shared__ __align__(16) uint16_t sB[3][3][kTileB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, dz = wave - 1;
  const int chunk = blockIdx.x;
  const int co0 = (blockIdx.y / ci_tiles) * 32, ci0 = (blockIdx.y % ci_tiles) * 32;
  const long long r0 = nsr * chunk / nchunks, r1 = nsr * (chunk + 1) / nchunks;
  const int nseg = nseg_of(W);
  const bool do_bias = bpart != nullptr && ci0 == 0;

  floatx16 acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = floatx16{};
  float bsum = 0.0f;  // wave 0, lane (h, c): channel co0 + c over voxels x0 + 32 h .. + 31

  // 16-byte chunks this thread moves, two voxels at a time so that the transposed stores are
  // whole dwords (one channel of both voxels, paired by v_perm): dout^T item it = t
  // (it < 128) -> voxels x0 + 2 (it / 4) + {0, 1}, channels co0 + 8 (it % 4) ..; in^T item
  // lane + 64 k -> voxels x0 - 8 + 2 ((lane + 64 k) / 4) + {0, 1}, channels ci0 + 8 ((lane + 64 k) % 4) ..
  constexpr int PB = (2 * kRowB + 63) / 64;  // voxel-pair items per lane of a source row
  auto pair_store = [&](uint16_t* base, int stride, int q, int xi, const uint4& A, const uint4& B) {
    const uint32_t a4[4] = {A.x, A.y, A.z, A.w}, b4[4] = {B.x, B.y, B.z, B.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      *reinterpret_cast<uint32_t*>(base + trow(8 * q + 2 * k, stride) + xi) = __builtin_amdgcn_perm(b4[k], a4[k], 0x05040100u);
      *reinterpret_cast<uint32_t*>(base + trow(8 * q + 2 * k + 1, stride) + xi) =
          __builtin_amdgcn_perm(b4[k], a4[k], 0x07060302u);
    }
  };
  auto load_dout = [&](long long nz, int y, int x0, uint4 (&buf)[2]) {
    buf[0] = buf[1] = make_uint4(0, 0, 0, 0);
    if (t < 128) {
      const int q = t & 3, x = x0 + 2 * (t >> 2);
      const uint16_t* src = dout + ((nz * H + y) * (long long)W + x) * cout + co0 + 8 * q;
      if (x < W) buf[0] = *reinterpret_cast<const uint4*>(src);
      if (x + 1 < W) buf[1] = *reinterpret_cast<const uint4*>(src + cout);
    }
  };
  auto store_dout = [&](const uint4 (&buf)[2]) {
    if (t < 128) pair_store(sA, kRsA, t & 3, 2 * (t >> 2), buf[0], buf[1]);
  };
  auto load_row = [&](long long nz, int z, int yy, int x0, uint4 (&buf)[PB][2]) {
    const int zz = z + dz;
    const bool row_ok = zz >= 0 && zz < D && yy >= 0 && yy < H;
    const long long base = ((nz + dz) * H + yy) * (long long)W;
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      const int it = lane + 64 * k;
      const int q = it & 3, x = x0 - 8 + 2 * (it >> 2);
      buf[k][0] = buf[k][1] = make_uint4(0, 0, 0, 0);
      if (it < 2 * kRowB && row_ok && ci0 + 8 * q < cin) {
        const uint16_t* src = in + (base + x) * cin + ci0 + 8 * q;
        if (x >= 0 && x < W) buf[k][0] = *reinterpret_cast<const uint4*>(src);
        if (x + 1 >= 0 && x + 1 < W) buf[k][1] = *reinterpret_cast<const uint4*>(src + cin);
      }
    }
  };
  auto store_row = [&](int yy, const uint4 (&buf)[PB][2]) {
    uint16_t* dst = sB[wave][(yy + 3) % 3];
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      const int it = lane + 64 * k;
      if (it < 2 * kRowB) pair_store(dst, kRsB, it & 3, 2 * (it >> 2), buf[k][0], buf[k][1]);
    }
  };

  // a segment continues the previous one's column when it is the next y of the same
  // (n, z, segment); its dout row and its one new source row are then loaded during the
  // previous segment's MFMAs
  uint4 pfa[2], pfb[PB][2];
  bool have = false;
  long long prev_col = -1;
  int prev_y = -2;
  for (long long r = r0; r < r1; ++r) {
    const int y = (int)(r % H);
    const long long col = r / H;  // (n D + z) nseg + seg
    const int seg = (int)(col % nseg);
    const long long nz = col / nseg;  // n D + z
    const int z = (int)(nz % D);
    const int x0 = seg * kSeg;
    const bool cont = col == prev_col && y == prev_y + 1;
    prev_col = col;
    prev_y = y;
    __syncthreads();  // the previous segment's reads of LDS are done

    if (have) {
      store_dout(pfa);
      store_row(y + 1, pfb);
    } else {
      uint4 tb[2];
      load_dout(nz, y, x0, tb);
      store_dout(tb);
      for (int yy = cont ? y + 1 : y - 1; yy <= y + 1; ++yy) {
        uint4 rb[PB][2];
        load_row(nz, z, yy, x0, rb);
        store_row(yy, rb);
      }
    }
    have = r + 1 < r1 && y + 1 < H;  // the next segment continues this column
    if (have) {
      load_dout(nz, y + 1, x0, pfa);
      load_row(nz, z, y + 2, x0, pfb);
    }
    __syncthreads();

    const int h = lane >> 5, c = lane & 31;
    const uint16_t* pa = sA + trow(c, kRsA) + 32 * h;
    if (do_bias && wave == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float f[8];
        unpack8(*reinterpret_cast<const uint4*>(pa + 8 * j), f);
#pragma unroll
        for (int i = 0; i < 8; ++i) bsum += f[i];
      }
    }
    const uint16_t* pb[3];
    uint4 prv[3], cur[3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      pb[dy] = sB[wave][(y + dy + 2) % 3] + trow(c, kRsB) + 32 * h;  // element 8 + 32 h is voxel x0 + 32 h
      prv[dy] = *reinterpret_cast<const uint4*>(pb[dy]);
      cur[dy] = *reinterpret_cast<const uint4*>(pb[dy] + 8);
    }
#pragma unroll
    for (int st = 0; st < kSeg / 16; ++st) {
      const uint4 a = *reinterpret_cast<const uint4*>(pa + 8 * st);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const uint4 nxt = *reinterpret_cast<const uint4*>(pb[dy] + 16 + 8 * st);
        acc[3 * dy + 0] = mfma16(a, shift_in_prev(prv[dy], cur[dy]), acc[3 * dy + 0]);  // voxels x - 1 ..
        acc[3 * dy + 1] = mfma16(a, cur[dy], acc[3 * dy + 1]);
        acc[3 * dy + 2] = mfma16(a, shift_in_next(cur[dy], nxt), acc[3 * dy + 2]);      // voxels x + 1 ..
        prv[dy] = cur[dy];
        cur[dy] = nxt;
      }
    }
  }

  // acc[3 dy + dx] row m = 8 (r / 4) + 4 h + r % 4 (co0 + m), column ci0 + lane % 32
  {
    const int h = lane >> 5, ci = ci0 + (lane & 31);
    if (ci < cin) {
      float* dst = part + ((long long)chunk * 27 + 9 * wave) * cout * cin;
#pragma unroll
      for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int co = co0 + (r / 4) * 8 + 4 * h + (r & 3);
          dst[((long long)k * cout + co) * cin + ci] = acc[k][r];
        }
    }
  }
  if (do_bias) {
    __syncthreads();
    float* red = reinterpret_cast<float*>(&sB[0][0][0]);
    if (t < 64) red[t] = bsum;
    __syncthreads();
    if (t < 32) bpart[(long long)chunk * cout + co0 + t] = red[t] + red[t + 32];
  }
}

// out[i] = sum over k of part[k][i], i < len.  A block of 256 threads covers OPB outputs with
// G = 256 / OPB groups; group g adds chunks g, g + G, ... in order, and the G group sums are
// added in group order, so the result does not depend on scheduling.
// Two sums share the launch: blocks [0, nb1) cover (part1, out1, len1), the rest (part2,
// out2, len2).
__global__ void __launch_bounds__(256) chunk_sum_kernel(const float* __restrict__ part1, float* __restrict__ out1,
                                                        long long len1, const float* __restrict__ part2,
                                                        float* __restrict__ out2, long long len2, long long nb1,
                                                        int nchunks, int opb) {
  __shared__ float sred[256];
  const bool first = blockIdx.x < nb1;
  const float* __restrict__ part = first ? part1 : part2;
  float* __restrict__ out = first ? out1 : out2;
  const long long len = first ? len1 : len2;
  const int t = threadIdx.x, o = t % opb, g = t / opb, G = 256 / opb;
  const long long i = (first ? (long long)blockIdx.x : (long long)blockIdx.x - nb1) * opb + o;
  float s = 0.0f;
  if (i < len) {
#pragma unroll 4
    for (int k = g; k < nchunks; k += G) s += part[(long long)k * len + i];
  }
  sred[t] = s;
  __syncthreads();
  if (g == 0 && i < len) {
    float sum = 0.0f;
    for (int q = 0; q < G; ++q) sum += sred[q * opb + o];
    out[i] = sum;
  }
}

// out1 = chunk sums of part1 (len1 >= 32), and of part2 into out2 when out2 is not null
inline void launch_chunk_sums(const float* part1, float* out1, long long len1, const float* part2, float* out2,
                              long long len2, int nchunks, hipStream_t s) {
  const int opb = 32;
  const long long nb1 = (len1 + opb - 1) / opb, nb2 = out2 ? (len2 + opb - 1) / opb : 0;
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)(nb1 + nb2)), dim3(256), 0, s, part1, out1, len1, part2, out2,
                     len2, nb1, nchunks, opb);
}

// ---------------------------------------------------------------- element-wise operators
// The element-wise operators move 8 channels (16 bytes) per thread; channel counts are
// multiples of 8 wherever they are called with voxel layouts, and the flat operators take a
// scalar tail.
// dx may alias dy: each thread reads its 8 elements before writing them
__global__ void relu_bwd_kernel(const uint16_t* __restrict__ y, const uint16_t* dy, uint16_t* dx, long long count,
                                int vec) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long e = 8 * i;
  if (vec && e + 8 <= count) {
    const uint4 yv = *reinterpret_cast<const uint4*>(y + e), gv = *reinterpret_cast<const uint4*>(dy + e);
    const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w}, gw[4] = {gv.x, gv.y, gv.z, gv.w};
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t lo = __uint_as_float(yw[k] << 16) > 0.0f ? 0x0000FFFFu : 0u;
      const uint32_t hi = __uint_as_float(yw[k] & 0xFFFF0000u) > 0.0f ? 0xFFFF0000u : 0u;
      o[k] = gw[k] & (lo | hi);
    }
    *reinterpret_cast<uint4*>(dx + e) = make_uint4(o[0], o[1], o[2], o[3]);
  } else {
    for (long long j = e; j < count && j < e + 8; ++j) dx[j] = bf2f(y[j]) > 0.0f ? dy[j] : (uint16_t)0;
  }
}

// (d, h, w): dimensions of the fine lattice; thread = (coarse voxel, 8 channels)
__global__ void pool_fwd_kernel(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int d, int h, int w, int c,
                                long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int c8 = c / 8, ch = 8 * (int)(i % c8);
  long long t = i / c8;
  const int x = (int)(t % (w / 2));
  t /= (w / 2);
  const int y = (int)(t % (h / 2));
  t /= (h / 2);
  const int z = (int)(t % (d / 2));
  const long long n = t / (d / 2);
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < 8; ++k) {
    const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
    float f[8];
    unpack8(*reinterpret_cast<const uint4*>(in + (((n * d + zz) * h + yy) * (long long)w + xx) * c + ch), f);
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += f[j];
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] *= 0.125f;
  *reinterpret_cast<uint4*>(out + (i / c8) * c + ch) = pack8(s);
}

// thread = (fine voxel, 8 channels)
__global__ void pool_bwd_kernel(const uint16_t* __restrict__ dout, uint16_t* __restrict__ din, int d, int h, int w,
                                int c, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int c8 = c / 8, ch = 8 * (int)(i % c8);
  long long t = i / c8;
  const long long vf = t;
  const int x = (int)(t % w);
  t /= w;
  const int y = (int)(t % h);
  t /= h;
  const int z = (int)(t % d);
  const long long n = t / d;
  float f[8];
  unpack8(*reinterpret_cast<const uint4*>(dout + (((n * (d / 2) + z / 2) * (h / 2) + y / 2) * (long long)(w / 2) + x / 2) *
                                                     c +
                                                 ch),
          f);
#pragma unroll
  for (int j = 0; j < 8; ++j) f[j] *= 0.125f;
  *reinterpret_cast<uint4*>(din + vf * c + ch) = pack8(f);
}

// (d, h, w): dimensions of the coarse input; out and skip are 2d x 2h x 2w; thread = (fine
// voxel, 8 channels)
__global__ void up_add_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ skip,
                              uint16_t* __restrict__ out, int d, int h, int w, int c, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int c8 = c / 8, ch = 8 * (int)(i % c8);
  long long t = i / c8;
  const long long vf = t;
  const int x = (int)(t % (2 * w));
  t /= (2 * w);
  const int y = (int)(t % (2 * h));
  t /= (2 * h);
  const int z = (int)(t % (2 * d));
  const long long n = t / (2 * d);
  float a[8], b[8];
  unpack8(*reinterpret_cast<const uint4*>(in + (((n * d + z / 2) * h + y / 2) * (long long)w + x / 2) * c + ch), a);
  unpack8(*reinterpret_cast<const uint4*>(skip + vf * c + ch), b);
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] += b[j];
  *reinterpret_cast<uint4*>(out + vf * c + ch) = pack8(a);
}

// thread = (coarse voxel, 8 channels); where mask (a ReLU output) is not positive the
// gradient is 0
__global__ void up_bwd_kernel(const uint16_t* __restrict__ dout, const uint16_t* __restrict__ mask,
                              uint16_t* __restrict__ din, int d, int h, int w, int c, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int c8 = c / 8, ch = 8 * (int)(i % c8);
  long long t = i / c8;
  const long long vc = t;
  const int x = (int)(t % w);
  t /= w;
  const int y = (int)(t % h);
  t /= h;
  const int z = (int)(t % d);
  const long long n = t / d;
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < 8; ++k) {
    const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
    float f[8];
    unpack8(*reinterpret_cast<const uint4*>(dout + (((n * 2 * d + zz) * (2 * h) + yy) * (long long)(2 * w) + xx) * c + ch),
            f);
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += f[j];
  }
  if (mask) {
    float mv[8];
    unpack8(*reinterpret_cast<const uint4*>(mask + vc * c + ch), mv);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (!(mv[j] > 0.0f)) s[j] = 0.0f;
  }
  *reinterpret_cast<uint4*>(din + vc * c + ch) = pack8(s);
}

__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ pred, const float* __restrict__ target,
                                                  uint16_t* __restrict__ dpred, float* __restrict__ loss_part,
                                                  long long count, int stride, int used) {
  __shared__ float s[256];
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  float e2 = 0.0f;
  if (v < count) {
    const float scale = 2.0f / ((float)count * (float)used);
    for (int k0 = 0; k0 < stride; k0 += 8) {
      float g[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        g[j] = 0.0f;
        if (k0 + j < used) {
          const float e = pred[v * stride + k0 + j] - target[v * used + k0 + j];
          e2 += e * e;
          g[j] = scale * e;
        }
      }
      *reinterpret_cast<uint4*>(dpred + v * stride + k0) = pack8(g);
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

// out may alias a or b: each thread reads its 8 elements before writing them.  Where mask (a
// ReLU output) is given and not positive the sum is 0.
__global__ void add_kernel(const uint16_t* a, const uint16_t* b, const uint16_t* mask, uint16_t* out, long long count,
                           int vec) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long e = 8 * i;
  if (vec && e + 8 <= count) {
    float fa[8], fb[8];
    unpack8(*reinterpret_cast<const uint4*>(a + e), fa);
    unpack8(*reinterpret_cast<const uint4*>(b + e), fb);
#pragma unroll
    for (int j = 0; j < 8; ++j) fa[j] += fb[j];
    if (mask) {
      float mv[8];
      unpack8(*reinterpret_cast<const uint4*>(mask + e), mv);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (!(mv[j] > 0.0f)) fa[j] = 0.0f;
    }
    *reinterpret_cast<uint4*>(out + e) = pack8(fa);
  } else {
    for (long long j = e; j < count && j < e + 8; ++j) {
      const float v = bf2f(a[j]) + bf2f(b[j]);
      out[j] = (mask && !(bf2f(mask[j]) > 0.0f)) ? (uint16_t)0 : f2bf(v);
    }
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = f2bf(x[i]);
}

// y[v][c] = bf16(x[v][c]) for c < c_src, 0 for c_src <= c < c_dst; thread = (voxel, 8
// output channels), with 16-byte stores when c_dst is a multiple of 8 and y is aligned
__global__ void pack_input_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, long long nvox, int c_src,
                                  int c_dst, int vec) {
  const int g8 = (c_dst + 7) / 8;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * g8) return;
  const long long v = i / g8;
  const int c0 = 8 * (int)(i % g8);
  float f[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) f[j] = c0 + j < c_src ? x[v * c_src + c0 + j] : 0.0f;
  if (vec) {
    *reinterpret_cast<uint4*>(y + v * c_dst + c0) = pack8(f);
  } else {
    for (int j = 0; j < 8 && c0 + j < c_dst; ++j) y[v * c_dst + c0 + j] = f2bf(f[j]);
  }
}

__global__ void to_f32_kernel(const uint16_t* __restrict__ x, float* __restrict__ y, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = bf2f(x[i]);
}

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }
inline unsigned blocks(long long count, int per) { return (unsigned)((count + per - 1) / per); }
inline bool aligned16(const void* p) { return p && ((uintptr_t)p & 15) == 0; }
inline int done() { return hipGetLastError() == hipSuccess ? 0 : -2; }

}  // namespace

namespace {
int conv_dispatch(const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, float* out_f32, int n, int d,
                  int h, int wd, int cin, int cout, int relu, void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cin % 8 || cout < 32 || cout % 32 || !in || !w ||
      (!out && !out_f32))
    return -1;
  const long long nvox = (long long)n * d * h * wd;
  const bool small_plane = (long long)h * wd * cin < (1LL << 31);
  switch (cin) {
    case 8:
      if (small_plane)
        launch_ring<8>(in, w, bias, out, out_f32, n, d, h, wd, cout, relu, S(stream));
      else
        launch_conv<8>(in, w, bias, out, out_f32, d, h, wd, cout, relu, nvox, S(stream));
      break;
    case 16:
      if (small_plane)
        launch_ring<16>(in, w, bias, out, out_f32, n, d, h, wd, cout, relu, S(stream));
      else
        launch_staged<16>(in, w, bias, out, out_f32, n, d, h, wd, cout, relu, S(stream));
      break;
    case 32:
      if (small_plane)
        launch_ring<32>(in, w, bias, out, out_f32, n, d, h, wd, cout, relu, S(stream));
      else
        launch_staged<32>(in, w, bias, out, out_f32, n, d, h, wd, cout, relu, S(stream));
      break;
    case 64: launch_staged<64>(in, w, bias, out, out_f32, n, d, h, wd, cout, relu, S(stream)); break;
    case 128: launch_conv<128>(in, w, bias, out, out_f32, d, h, wd, cout, relu, nvox, S(stream)); break;
    default: return -1;
  }
  return done();
}
}  // namespace

extern "C" int surr_conv3d_fwd(const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, float* out_f32,
                               int n, int d, int h, int wd, int cin, int cout, int relu, void* stream) {
  return conv_dispatch(in, w, bias, out, out_f32, n, d, h, wd, cin, cout, relu, stream);
}

extern "C" int surr_conv3d_flip_weights(const uint16_t* w, uint16_t* w_t, int cin, int cout, void* stream) {
  if (cin < 1 || cout < 1 || !w || !w_t) return -1;
  const long long total = 27LL * cin * cout;
  hipLaunchKernelGGL(flip_kernel, dim3(blocks(total, 256)), dim3(256), 0, S(stream), w, w_t, cin, cout);
  return done();
}

extern "C" int surr_conv3d_dgrad(const uint16_t* dout, const uint16_t* w_t, const uint16_t* relu_y, uint16_t* din, int n,
                                 int d, int h, int wd, int cin, int cout, void* stream) {
  // the forward convolution of dout (cout channels) with w_t gives din (cin channels); the
  // ReLU mask is a pass of its own (the convolution kernels have no registers to spare for it)
  if (!din) return -1;
  const int rc = conv_dispatch(dout, w_t, nullptr, din, nullptr, n, d, h, wd, cout, cin, 0, stream);
  if (rc != 0 || !relu_y) return rc;
  return surr_relu_bwd(relu_y, din, din, (long long)n * d * h * wd * cin, stream);
}

extern "C" size_t surr_conv3d_wgrad_scratch_bytes(int n, int d, int h, int wd, int cin, int cout) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cout < 32) return 0;
  const WgradPlan p = wgrad_plan(n, d, h, wd, cin, cout);
  return (size_t)p.nchunks * ((size_t)27 * cout * cin + (size_t)cout) * sizeof(float);
}

extern "C" int surr_conv3d_wgrad(const uint16_t* in, const uint16_t* dout, float* dw, float* dbias, void* scratch, int n,
                                 int d, int h, int wd, int cin, int cout, void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cin % 8 || cout < 32 || cout % 32 || !in || !dout || !dw ||
      !scratch)
    return -1;
  if ((long long)n * d * h * wd >= (1LL << 40)) return -1;
  const WgradPlan p = wgrad_plan(n, d, h, wd, cin, cout);
  float* part = static_cast<float*>(scratch);
  float* bpart = part + (size_t)p.nchunks * 27 * cout * cin;
  hipLaunchKernelGGL(wgrad_kernel, dim3(p.nchunks, p.tiles), dim3(192), 0, S(stream), in, dout, part,
                     dbias ? bpart : nullptr, d, h, wd, cin, cout, p.nsr, p.nchunks, p.ci_tiles);
  launch_chunk_sums(part, dw, 27LL * cout * cin, bpart, dbias, (long long)cout, p.nchunks, S(stream));
  return done();
}

extern "C" int surr_relu_bwd(const uint16_t* y, const uint16_t* dy, uint16_t* dx, long long count, void* stream) {
  if (count < 0 || !y || !dy || !dx) return -1;
  if (count == 0) return 0;
  const int vec = aligned16(y) && aligned16(dy) && aligned16(dx);
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks(count, 8 * 256)), dim3(256), 0, S(stream), y, dy, dx, count, vec);
  return done();
}

extern "C" int surr_pool_fwd(const uint16_t* in, uint16_t* out, int n, int d, int h, int wd, int c, void* stream) {
  if (n < 1 || d < 2 || h < 2 || wd < 2 || (d | h | wd) & 1 || c < 8 || c % 8 || !aligned16(in) || !aligned16(out))
    return -1;
  const long long count = (long long)n * (d / 2) * (h / 2) * (wd / 2) * (c / 8);
  hipLaunchKernelGGL(pool_fwd_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), in, out, d, h, wd, c, count);
  return done();
}

extern "C" int surr_pool_bwd(const uint16_t* dout, uint16_t* din, int n, int d, int h, int wd, int c, void* stream) {
  if (n < 1 || d < 2 || h < 2 || wd < 2 || (d | h | wd) & 1 || c < 8 || c % 8 || !aligned16(dout) || !aligned16(din))
    return -1;
  const long long count = (long long)n * d * h * wd * (c / 8);
  hipLaunchKernelGGL(pool_bwd_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), dout, din, d, h, wd, c, count);
  return done();
}

extern "C" int surr_up_add_fwd(const uint16_t* in, const uint16_t* skip, uint16_t* out, int n, int d, int h, int wd,
                               int c, void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || c < 8 || c % 8 || !aligned16(in) || !aligned16(skip) || !aligned16(out))
    return -1;
  const long long count = (long long)n * 8 * d * h * wd * (c / 8);
  hipLaunchKernelGGL(up_add_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), in, skip, out, d, h, wd, c,
                     count);
  return done();
}

extern "C" int surr_up_bwd(const uint16_t* dout, const uint16_t* relu_y, uint16_t* din, int n, int d, int h, int wd, int c,
                           void* stream) {
  if (n < 1 || d < 1 || h < 1 || wd < 1 || c < 8 || c % 8 || !aligned16(dout) || !aligned16(din) ||
      (relu_y && !aligned16(relu_y)))
    return -1;
  const long long count = (long long)n * d * h * wd * (c / 8);
  hipLaunchKernelGGL(up_bwd_kernel, dim3(blocks(count, 256)), dim3(256), 0, S(stream), dout, relu_y, din, d, h, wd, c,
                     count);
  return done();
}

extern "C" int surr_mse(const float* pred, const float* target, uint16_t* dpred, float* loss_part, long long count,
                        int stride, int used, void* stream) {
  if (count < 1 || stride < 8 || stride % 8 || used < 1 || used > stride || !pred || !target || !aligned16(dpred) ||
      !loss_part)
    return -1;
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

extern "C" int surr_add(const uint16_t* a, const uint16_t* b, const uint16_t* relu_y, uint16_t* out, long long count,
                        void* stream) {
  if (count < 0 || !a || !b || !out) return -1;
  if (count == 0) return 0;
  const int vec = aligned16(a) && aligned16(b) && aligned16(out) && (!relu_y || aligned16(relu_y));
  hipLaunchKernelGGL(add_kernel, dim3(blocks(count, 8 * 256)), dim3(256), 0, S(stream), a, b, relu_y, out, count, vec);
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

extern "C" int surr_pack_input(const float* x, uint16_t* y, long long nvox, int c_src, int c_dst, void* stream) {
  if (nvox < 0 || c_src < 1 || c_dst < c_src || !x || !y) return -1;
  if (nvox == 0) return 0;
  const int vec = c_dst % 8 == 0 && aligned16(y);
  hipLaunchKernelGGL(pack_input_kernel, dim3(blocks(nvox * ((c_dst + 7) / 8), 256)), dim3(256), 0, S(stream), x, y, nvox,
                     c_src, c_dst, vec);
  return done();
}
