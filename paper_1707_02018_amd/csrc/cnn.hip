// Warm-start CNN on gfx950: BF16 operands, FP32 accumulation.
//
// The 32 -> 32 layers are implicit GEMMs on v_mfma_f32_32x32x16_bf16 with M = 32 output
// channels, N = 32 pixels of one image row, K = 16 input channels per tap half.
// Each wave owns a 32-pixel column strip and slides down its rows: one input
// row's three shifted fragments feed the three output rows that need them, so
// every fragment is read once and used by three taps. The four waves of a
// workgroup own adjacent strips and stage each input row once in a ring of
// LDS rows (coalesced 16-byte loads issued two rows ahead), from which each
// wave reads its shifted fragments. The weights of all nine taps stay in
// registers for the whole strip. The same kernel runs the input gradient
// (mirrored, transposed weights) with the ReLU mask of the layer below applied
// in its epilogue.
//
// The weight gradient is a K = pixels contraction, so both operands are
// staged through LDS transposed to channel-major rows; the three horizontal
// tap shifts come from one aligned 16-byte read plus byte alignment.
//
// The 1 -> 32 input layer and the 32 -> 1 input gradient are VALU (nine
// products per output), as is the weight gradient of those two layers; the
// 32 -> 1 output layer is VALU on BF16 pair dot products (v_dot2c_f32_bf16).
// Every reduction is fixed-order: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "aw_internal.hpp"

namespace aw {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf2f(unsigned h) { return __uint_as_float(h << 16); }

// Round to nearest even; NaN stays a (quiet) NaN.
__device__ __forceinline__ unsigned f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Two values rounded to nearest even and packed (lo in the low half) by one
// v_cvt_pk_bf16_f32; equal to f2bf for every non-NaN input with FP32
// denormals kept (the default; a NaN stays a quiet NaN).
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned f2bf2(float lo, float hi) {
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}

__device__ __forceinline__ bool bf_positive(unsigned h) { return !(h & 0x8000u) && (h & 0x7fffu); }

__device__ __forceinline__ float rnd_bf(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ u32x4 ld16(const uint16_t* p) {
  return *reinterpret_cast<const u32x4*>(p);
}

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// ----------------------------------------------------------------- packing
__global__ void cnn_pack_kernel(const float* __restrict__ m, uint8_t* __restrict__ pk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int nW1 = 288, nB = 32, nMid = 9216;
  int r = i;
  if (r < nW1) {  // w1[t][c] = W1[c][0][t]
    const int t = r / 32, c = r % 32;
    reinterpret_cast<uint16_t*>(pk + CnnPack::w1)[r] = f2bf(m[kCnnMasterW1 + c * 9 + t]);
    return;
  }
  r -= nW1;
  if (r < nB) {
    reinterpret_cast<float*>(pk + CnnPack::b1)[r] = m[kCnnMasterB1 + r];
    return;
  }
  r -= nB;
  for (int l = 0; l < 4; ++l) {
    const long long base = cnn_master_mid(l);
    uint8_t* L = pk + CnnPack::mid + l * CnnPack::mid_size;
    if (r < nMid) {  // fwd[t][o][i] = W[o][i][t]
      const int t = r / 1024, o = (r / 32) % 32, c = r % 32;
      reinterpret_cast<uint16_t*>(L + CnnPack::mid_fwd)[r] = f2bf(m[base + (o * 32 + c) * 9 + t]);
      return;
    }
    r -= nMid;
    if (r < nMid) {  // dgrad[t][i][o] = W[o][i][8 - t]
      const int t = r / 1024, c = (r / 32) % 32, o = r % 32;
      reinterpret_cast<uint16_t*>(L + CnnPack::mid_dgrad)[r] =
          f2bf(m[base + (o * 32 + c) * 9 + (8 - t)]);
      return;
    }
    r -= nMid;
    if (r < nB) {
      reinterpret_cast<float*>(L + CnnPack::mid_bias)[r] = m[base + 9216 + r];
      return;
    }
    r -= nB;
  }
  if (r < nMid) {  // w6[t][o][i]: output 0 only
    const int t = r / 1024, o = (r / 32) % 32, c = r % 32;
    reinterpret_cast<uint16_t*>(pk + CnnPack::w6)[r] =
        o == 0 ? f2bf(m[kCnnMasterW6 + c * 9 + t]) : 0u;
    return;
  }
  r -= nMid;
  if (r < nB) {
    reinterpret_cast<float*>(pk + CnnPack::b6)[r] = r == 0 ? m[kCnnMasterB6] : 0.0f;
    return;
  }
  r -= nB;
  if (r < nW1) {  // w6d[t][c] = W6[0][c][8 - t]
    const int t = r / 32, c = r % 32;
    reinterpret_cast<uint16_t*>(pk + CnnPack::w6d)[r] = f2bf(m[kCnnMasterW6 + c * 9 + (8 - t)]);
  }
}
constexpr int kPackJobs = 288 + 32 + 4 * (2 * 9216 + 32) + 9216 + 32 + 288;

// ------------------------------------------------------- 1 -> 32 (VALU)
// FWD:  y[p][c] = relu(bias[c] + sum_t w[t][c] src[p + off(t)])   (src = the FP32 image)
// else: y[p][c] = [mask[p][c] > 0] sum_t w[t][c] rnd(src[p + off(t)])   (src = a gradient)
// One thread per (pixel column, group of 8 channels) and kInRows rows;
// off(t) = (t / 3 - 1, t % 3 - 1). No thread divides a pixel index.
// The image keeps FP32: its noise (1e-3) is below the BF16 step near 1 (2^-8).
constexpr int kInRows = 16;  // output rows per thread
constexpr int kInAhead = 4;  // rows of loads in flight per thread

template <bool FWD>
__global__ __launch_bounds__(256) void conv_in_kernel(const float* __restrict__ src,
                                                      const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ mask,
                                                      uint16_t* __restrict__ y, int H, int W) {
  // grid: (4 W / 256 rounded up, H / kInRows rounded up, images); a thread
  // walks kInRows rows of one (pixel column, channel group) with the weights
  // in registers and a sliding 3 x 3 window of inputs
  const int gx = blockIdx.x * 256 + threadIdx.x;
  const int x = gx >> 2, g = gx & 3;
  if (x >= W) return;
  const int r0 = blockIdx.y * kInRows;
  const int r1 = min(r0 + kInRows, H);
  const long long plane = (long long)H * W;
  const float* s = src + (long long)blockIdx.z * plane;
  const long long pbase = (long long)blockIdx.z * plane + x;
  float wf[9][8];  // the weights, widened once
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const u32x4 wv = ld16(w + t * 32 + 8 * g);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      wf[t][2 * j] = bf2f(wv[j] & 0xffffu);
      wf[t][2 * j + 1] = bf2f(wv[j] >> 16);
    }
  }
  float b8[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) b8[j] = FWD ? bias[8 * g + j] : 0.0f;
  auto in_row = [&](int rr, float (&v)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int cc = x + k - 1;
      const float u = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? s[(long long)rr * W + cc] : 0.0f;
      v[k] = FWD ? u : rnd_bf(u);
    }
  };
  // The input row below each output row and the output row's mask are
  // loaded kInAhead rows ahead of their use in a register ring, issued
  // unconditionally from clamped addresses with the bounds applied when a
  // value is used (a load under a condition would be waited for at once).
  auto raw_row = [&](int rr, float (&v)[3]) {
    const int rc = min(max(rr, 0), H - 1);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = s[(long long)rc * W + min(max(x + k - 1, 0), W - 1)];
  };
  auto use_row = [&](int rr, const float (&raw)[3], float (&v)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int cc = x + k - 1;
      const float u = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? raw[k] : 0.0f;
      v[k] = FWD ? u : rnd_bf(u);
    }
  };
  float in[3][3];  // rows r - 1, r, r + 1
  in_row(r0 - 1, in[0]);
  in_row(r0, in[1]);
  float qr[kInAhead][3];
  u32x4 qm[kInAhead];
#pragma unroll
  for (int d = 0; d < kInAhead; ++d) {
    raw_row(r0 + d + 1, qr[d]);
    qm[d] = FWD ? u32x4{0, 0, 0, 0}
                : ld16(mask + (pbase + (long long)min(r0 + d, r1 - 1) * W) * 32 + 8 * g);
  }
  for (int r4 = r0; r4 < r1; r4 += kInAhead) {
#pragma unroll
    for (int d = 0; d < kInAhead; ++d) {
      const int r = r4 + d;
      const float raw[3] = {qr[d][0], qr[d][1], qr[d][2]};
      const u32x4 mk = qm[d];
      const int rn = r + kInAhead;
      raw_row(rn + 1, qr[d]);
      if (!FWD) qm[d] = ld16(mask + (pbase + (long long)min(rn, r1 - 1) * W) * 32 + 8 * g);
      if (r >= r1) continue;
      use_row(r + 1, raw, in[2]);
      const long long p = pbase + (long long)r * W;
      float acc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = b8[j];
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const float iv = in[t / 3][t % 3];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += wf[t][j] * iv;
      }
      u32x4 out;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float a0 = acc[2 * j], a1 = acc[2 * j + 1];
        if (FWD) {
          a0 = fmaxf(a0, 0.0f);
          a1 = fmaxf(a1, 0.0f);
        } else {
          if (!bf_positive(mk[j] & 0xffffu)) a0 = 0.0f;
          if (!bf_positive(mk[j] >> 16)) a1 = 0.0f;
        }
        out[j] = f2bf2(a0, a1);
      }
      *reinterpret_cast<u32x4*>(y + p * 32 + 8 * g) = out;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        in[0][k] = in[1][k];
        in[1][k] = in[2][k];
      }
    }
  }
}

// ------------------------------------------------------- 32 -> 1 (VALU)
// u[p] = base[p] + bias + sum_t sum_c w[t][c] a[p + off(t)][c]: one output
// channel, so the MFMA tile of the 32 -> 32 layers would compute 31 zero rows.
// Four lanes (channel groups g of 8) share a pixel column and walk kInRows
// rows with a 3 x 3 window of 16-byte chunks in registers; the next rows'
// chunks are loaded kInAhead rows ahead, unconditionally from clamped
// positions, with the bounds applied at use. The four partial sums of a
// pixel are added across the lanes in a fixed order.
__global__ __launch_bounds__(256) void conv_out_kernel(const uint16_t* __restrict__ X,
                                                       const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       const float* __restrict__ base,
                                                       float* __restrict__ out, int H, int W) {
  const int gx = blockIdx.x * 256 + threadIdx.x;
  const int x = gx >> 2, g = gx & 3;
  if (x >= W) return;  // the four lanes of a pixel column leave together
  const int r0 = blockIdx.y * kInRows;
  const int r1 = min(r0 + kInRows, H);
  const long long plane = (long long)H * W;
  const uint16_t* Xi = X + (long long)blockIdx.z * plane * 32 + 8 * g;
  const long long obase = (long long)blockIdx.z * plane + x;
  u32x4 wp[9];  // w[t][0][c]: output channel 0, channel pairs packed as BF16
#pragma unroll
  for (int t = 0; t < 9; ++t) wp[t] = ld16(w + t * 1024 + 8 * g);
  const float b0 = bias[0];
  auto raw_row = [&](int rr, u32x4 (&v)[3]) {
    const int rc = min(max(rr, 0), H - 1);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      v[k] = ld16(Xi + ((long long)rc * W + min(max(x + k - 1, 0), W - 1)) * 32);
  };
  auto use_row = [&](int rr, const u32x4 (&raw)[3], u32x4 (&v)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int cc = x + k - 1;
      const bool ok = rr >= 0 && rr < H && cc >= 0 && cc < W;
      v[k] = ok ? raw[k] : u32x4{0, 0, 0, 0};
    }
  };
  u32x4 win[3][3];  // rows r - 1, r, r + 1; columns x - 1, x, x + 1
  {
    u32x4 raw[3];
    raw_row(r0 - 1, raw);
    use_row(r0 - 1, raw, win[0]);
    raw_row(r0, raw);
    use_row(r0, raw, win[1]);
  }
  u32x4 q[kInAhead][3];
  float qb[kInAhead];
#pragma unroll
  for (int d = 0; d < kInAhead; ++d) {
    raw_row(r0 + d + 1, q[d]);
    qb[d] = base[obase + (long long)min(r0 + d, H - 1) * W];
  }
  for (int r4 = r0; r4 < r1; r4 += kInAhead) {
#pragma unroll
    for (int d = 0; d < kInAhead; ++d) {
      const int r = r4 + d;
      const u32x4 raw[3] = {q[d][0], q[d][1], q[d][2]};
      const float bv = qb[d];
      const int rn = r + kInAhead;
      raw_row(rn + 1, q[d]);
      qb[d] = base[obase + (long long)min(rn, H - 1) * W];
      if (r >= r1) continue;
      use_row(r + 1, raw, win[2]);
      // BF16 pair dot products accumulated in FP32 (v_dot2c_f32_bf16)
      float acc = 0.0f;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const u32x4 v = win[t / 3][t % 3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // each element copied out first: a bit cast of the vector element
          // itself read element 0 every time
          const unsigned vj = v[j], wj = wp[t][j];
          acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, vj),
                                                __builtin_bit_cast(bf16x2_t, wj), acc, false);
        }
      }
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      if (g == 0) out[obase + (long long)r * W] = acc + b0 + bv;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        win[0][k] = win[1][k];
        win[1][k] = win[2][k];
      }
    }
  }
}

// ------------------------------------------------------- 32 -> 32 (MFMA)
enum ConvMode { kFwd = 0, kDgrad = 1 };

struct ConvArgs {
  const uint16_t* x;     // [n][H][W][32]
  const uint16_t* w;     // [9][32 out][32 in]
  const float* bias;     // [32] (kFwd)
  const uint16_t* mask;  // [n][H][W][32] (kDgrad)
  uint16_t* y;           // [n][H][W][32] (kFwd, kDgrad)
  int n, H, W, strips, bands, groups;  // groups: workgroups per band (kConvStrips strips each)
  int rows;                            // output rows per band (one of kConvRows)
};

// Output rows per band (per workgroup), tallest first; the host takes the
// tallest that still gives the grid kConvMinGrid workgroups (eight per CU),
// the shortest otherwise. A taller band stages fewer halo rows per output
// row and starts fewer workgroups: at 64 images of 512^2 the forward pass
// measured 2.81 ms at 16 rows, 2.63 at 31, 2.58-2.60 at 64 (the backward
// 7.03, 6.90, 6.81-6.87), 2.83 at 85 (too few workgroups); outputs are the
// same for every height (each output row sums its three input rows in the
// same order). Any height works with the row loop unrolled by three: rows
// past the band's end skip their loads, taps and stores.
constexpr int kConvRows[3] = {64, 31, 16};
constexpr long long kConvMinGrid = 2048;

struct Frags {
  u32x4 f[3][2];  // [kx][k half]
};

template <int I>
__device__ __forceinline__ f32x16& pick(f32x16& a, f32x16& b, f32x16& c) {
  if constexpr (I == 0) return a;
  else if constexpr (I == 1) return b;
  else return c;
}

// A workgroup (four waves) owns kConvStrips adjacent 32-pixel strips of one
// 16-row band. Its input rows are staged in a ring of three LDS rows: pixels
// x0 - 1 .. x0 + 128 (x0 = the first strip's first pixel), 32 channels each,
// at a pitch of 40 elements (80 bytes, so the 16-byte fragment reads of a
// wave spread over the banks). Staging is one 16-byte chunk per thread and
// load, coalesced; the three shifted fragments of a tap row then come from LDS.
constexpr int kConvStrips = 4;
constexpr int kConvPx = 32 * kConvStrips + 2;
constexpr int kConvPitch = 40;
constexpr int kConvRowElems = kConvPx * kConvPitch;
constexpr int kConvChunks = kConvPx * 4;
constexpr int kConvLoads = (kConvChunks + 255) / 256;

// Input row r, pixels xs .. xs + kConvPx - 1, into registers (zeros outside
// the image).
__device__ __forceinline__ void stage_load(u32x4 (&v)[kConvLoads], const uint16_t* X, int H, int W,
                                           int r, int xs) {
  const bool rv = r >= 0 && r < H;
#pragma unroll
  for (int i = 0; i < kConvLoads; ++i) {
    const int c = threadIdx.x + 256 * i;
    const int col = xs + c / 4;
    const bool ok = c < kConvChunks && rv && col >= 0 && col < W;
    v[i] = ok ? ld16(X + ((long long)r * W + col) * 32 + 8 * (c % 4)) : u32x4{0, 0, 0, 0};
  }
}

__device__ __forceinline__ void stage_store(uint16_t* B, const u32x4 (&v)[kConvLoads]) {
#pragma unroll
  for (int i = 0; i < kConvLoads; ++i) {
    const int c = threadIdx.x + 256 * i;
    if (c < kConvChunks) *reinterpret_cast<u32x4*>(B + (c / 4) * kConvPitch + 8 * (c % 4)) = v[i];
  }
}

// The lane's fragments of a staged row: pixel pw + kx of the row buffer
// (pw = the wave's strip offset + lane % 32), channels 8 h + 16 kb .. + 7.
__device__ __forceinline__ void lds_frags(Frags& F, const uint16_t* B, int pw, int h) {
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
      F.f[kx][kb] = *reinterpret_cast<const u32x4*>(B + (pw + kx) * kConvPitch + 8 * (h + 2 * kb));
}

// Output row o of the wave's strip. The 32 -> 1 layer stores channel 0
// (lanes of h = 0, one float per pixel, contiguous). The 32 -> 32 modes round
// to BF16 in registers (the bias read from LDS: its channels differ between
// the two half-waves, so a global read would be a vector load per value), then
// pass the 32 pixels x 32 channels through the
// wave's LDS tile ob (pitch kConvPitch) so that each lane stores 16
// contiguous bytes and each store instruction writes 1 KB of the row: lane l
// takes pixel 16 k + l / 4, channels 8 (l % 4) .. + 7 (k = 0, 1). The ReLU
// mask of the input gradient is applied to the rounded values (a zero rounds
// to zero), read with the same coalesced pattern (mk, loaded by the caller
// before the row's MFMAs).
template <int MODE>
__device__ __forceinline__ void conv_epilogue(const ConvArgs& a, f32x16& acc, long long img_off,
                                              int o, int h, uint16_t* ob, int xw,
                                              const float* sbias, const u32x4 (&mk)[2]) {
  const int xl = threadIdx.x & 31;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int co = 8 * g + 4 * h;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = acc[4 * g + i];
    if constexpr (MODE == kFwd) {
      const float4 bv = *reinterpret_cast<const float4*>(sbias + co);
      v[0] = fmaxf(v[0] + bv.x, 0.0f);
      v[1] = fmaxf(v[1] + bv.y, 0.0f);
      v[2] = fmaxf(v[2] + bv.z, 0.0f);
      v[3] = fmaxf(v[3] + bv.w, 0.0f);
    }
    u32x2 st;
    st[0] = f2bf2(v[0], v[1]);
    st[1] = f2bf2(v[2], v[3]);
    *reinterpret_cast<u32x2*>(ob + xl * kConvPitch + co) = st;
  }
  // the tile is private to the wave and LDS operations of a wave complete
  // in order; the barrier only keeps the compiler from reordering
  __builtin_amdgcn_wave_barrier();
  const int lane = threadIdx.x & 63;
  const long long row = img_off + (long long)o * a.W;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int p = 16 * k + (lane >> 2), c = lane & 3;
    u32x4 v = *reinterpret_cast<const u32x4*>(ob + p * kConvPitch + 8 * c);
    if (xw + p < a.W) {
      const long long pix = row + xw + p;
      if constexpr (MODE == kDgrad) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (!bf_positive(mk[k][j] & 0xffffu)) v[j] &= 0xffff0000u;
          if (!bf_positive(mk[k][j] >> 16)) v[j] &= 0x0000ffffu;
        }
      }
      *reinterpret_cast<u32x4*>(a.y + pix * 32 + 8 * c) = v;
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
}

// The three taps of kernel row KY on one input row's fragments.
template <int KY>
__device__ __forceinline__ void conv_taps(const bf16x8 (&wa)[9][2], const Frags& cur, f32x16& acc) {
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[KY * 3 + kx][kb], as_bf(cur.f[kx][kb]), acc,
                                                    0, 0, 0);
}

// One input row r (S = (r - y0 + 1) mod 3, also its ring buffer): contributions
// to output rows r + 1 (ky = 0), r (ky = 1), r - 1 (ky = 2); row r - 1 is then
// complete. The registers pre hold row r + 2, loaded one row earlier: they go
// to ring buffer (S + 2) mod 3 (row r - 1's, read by every wave before the
// last barrier), and the loads of row r + 3 are issued, in flight over two
// rows of MFMAs. Ends with the barrier that publishes row r + 2.
template <int MODE, int S>
__device__ __forceinline__ void conv_row(const ConvArgs& a, const uint16_t* X, long long img_off,
                                         const bf16x8 (&wa)[9][2], uint16_t* ring,
                                         u32x4 (&pre)[kConvLoads], f32x16& a0, f32x16& a1,
                                         f32x16& a2, int r, int y0, int yend, int x, int h, int pw,
                                         int xs, uint16_t* ob, const float* sbias) {
  const int o = r - 1;
  const bool emit = o >= y0 && o < yend;
  u32x4 mk[2] = {};
  if constexpr (MODE == kDgrad) {  // the epilogue's mask, in flight during the MFMAs
    if (emit) {
      const int lane = threadIdx.x & 63, xw = x - (threadIdx.x & 31);
      const long long row = img_off + (long long)o * a.W;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int p = 16 * k + (lane >> 2);
        if (xw + p < a.W) mk[k] = ld16(a.mask + (row + xw + p) * 32 + 8 * (lane & 3));
      }
    }
  }
  Frags cur;
  lds_frags(cur, ring + S * kConvRowElems, pw, h);
  if (r + 2 <= yend) stage_store(ring + ((S + 2) % 3) * kConvRowElems, pre);
  if (r + 3 <= yend) stage_load(pre, X, a.H, a.W, r + 3, xs);
  if (r >= 0 && r < a.H) {
    if (r + 1 < yend) conv_taps<0>(wa, cur, pick<S>(a0, a1, a2));
    if (r >= y0 && r < yend) conv_taps<1>(wa, cur, pick<(S + 2) % 3>(a0, a1, a2));
    if (r - 1 >= y0 && r - 1 < yend) conv_taps<2>(wa, cur, pick<(S + 1) % 3>(a0, a1, a2));
  }
  f32x16& done = pick<(S + 1) % 3>(a0, a1, a2);
  if (emit) conv_epilogue<MODE>(a, done, img_off, o, h, ob, x - (threadIdx.x & 31), sbias, mk);
  else {
#pragma unroll
    for (int i = 0; i < 16; ++i) done[i] = 0.0f;
  }
  __syncthreads();
}

template <int MODE>
__global__ __launch_bounds__(256, MODE == kDgrad ? 2 : 1) void conv32_kernel(ConvArgs a) {
  __shared__ __align__(16) uint16_t ring[3 * kConvRowElems];
  __shared__ __align__(16) uint16_t obuf[4][32 * kConvPitch];  // per wave: one output row
  __shared__ __align__(16) float sbias[32];
  if (MODE == kFwd && threadIdx.x < 32) sbias[threadIdx.x] = a.bias[threadIdx.x];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int sg = blockIdx.x % a.groups;
  const int rest = blockIdx.x / a.groups;
  const int band = rest % a.bands;
  const int img = rest / a.bands;
  const int h = lane >> 5;
  const int pw = w * 32 + (lane & 31);
  const int x = sg * 32 * kConvStrips + pw;  // beyond W for strips past the image: no stores
  const int xs = sg * 32 * kConvStrips - 1;  // first staged pixel
  const int y0 = band * a.rows;
  const int yend = min(y0 + a.rows, a.H);
  const long long img_off = (long long)img * a.H * a.W;
  const uint16_t* X = a.x + img_off * 32;

  bf16x8 wa[9][2];
  {
    const uint16_t* wp = a.w + (lane & 31) * 32 + 8 * h;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) wa[t][kb] = as_bf(ld16(wp + t * 1024 + 16 * kb));
  }
  f32x16 a0, a1, a2;
#pragma unroll
  for (int i = 0; i < 16; ++i) a0[i] = a1[i] = a2[i] = 0.0f;
  // rows y0 - 1 and y0 staged, row y0 + 1 in flight
  u32x4 pre[kConvLoads];
  stage_load(pre, X, a.H, a.W, y0 - 1, xs);
  stage_store(ring, pre);
  stage_load(pre, X, a.H, a.W, y0, xs);
  stage_store(ring + kConvRowElems, pre);
  if (y0 + 1 <= yend) stage_load(pre, X, a.H, a.W, y0 + 1, xs);
  __syncthreads();
  for (int r = y0 - 1; r <= yend; r += 3) {
    conv_row<MODE, 0>(a, X, img_off, wa, ring, pre, a0, a1, a2, r, y0, yend, x, h, pw, xs,
                        obuf[w], sbias);
    conv_row<MODE, 1>(a, X, img_off, wa, ring, pre, a0, a1, a2, r + 1, y0, yend, x, h, pw, xs,
                        obuf[w], sbias);
    conv_row<MODE, 2>(a, X, img_off, wa, ring, pre, a0, a1, a2, r + 2, y0, yend, x, h, pw, xs,
                        obuf[w], sbias);
  }
}

// --------------------------------------------- 32 -> 32 weight gradient
// part[wg][(o * 32 + i) * 9 + t] = sum over the tile's pixels p of
//   dz[p][o] * x[p + off(t)][i];   part[wg][9216 + o] = sum_p dz[p][o].
constexpr int kWgSW = 128;              // strip width (pixels): 4 waves x 2 chunks of 16
constexpr int kWgPD = kWgSW + 8;        // dz^T row pitch (elements)
constexpr int kWgPY = kWgSW + 24;       // x^T row pitch: columns x0 - 8 .. x0 + SW + 7
constexpr int kWgPairsY = (kWgSW + 16) / 2;
constexpr int kWgLds = 32 * kWgPD + 3 * 32 * kWgPY;  // elements
constexpr int kWgWidth = 9248;
static_assert(kWgLds * 2 >= 9216 * 4, "reduction buffer reuses the staging LDS");
static_assert(kWgLds * 2 >= 256 * 8 * 4, "bias reduction reuses the staging LDS");

struct WgradArgs {
  const uint16_t* dz;
  const uint16_t* x;
  float* part;
  int H, W, strips, bands, RB;
};

__device__ __forceinline__ u32x4 load_chunk(const uint16_t* P, int H, int W, int r, int c, int g) {
  if (r < 0 || r >= H || c < 0 || c >= W) return u32x4{0, 0, 0, 0};
  return ld16(P + ((long long)r * W + c) * 32 + 8 * g);
}

// Channels 8g..8g+7 of pixels col and col + 1 -> eight channel-major rows.
__device__ __forceinline__ void put_pair(uint16_t* T, int pitch, int col, int g, u32x4 a, u32x4 b) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned lo = (a[i] & 0xffffu) | (b[i] << 16);
    const unsigned hi = (a[i] >> 16) | (b[i] & 0xffff0000u);
    *reinterpret_cast<unsigned*>(T + (8 * g + 2 * i) * pitch + col) = lo;
    *reinterpret_cast<unsigned*>(T + (8 * g + 2 * i + 1) * pitch + col) = hi;
  }
}

__global__ __launch_bounds__(256, 2) void wgrad32_kernel(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[kWgLds];
  uint16_t* dzT = lds;
  uint16_t* xT = lds + 32 * kWgPD;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int wg = blockIdx.x;
  const int sx = wg % a.strips;
  const int rest = wg / a.strips;
  const int band = rest % a.bands;
  const int img = rest / a.bands;
  const int x0 = sx * kWgSW, y0 = band * a.RB, y1 = min(y0 + a.RB, a.H);
  const long long plane = (long long)a.H * a.W * 32;
  const uint16_t* DZ = a.dz + img * plane;
  const uint16_t* XS = a.x + img * plane;
  const int pp = tid >> 2, g = tid & 3;  // staging job: pixel pair, channel group

  float bsum[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) bsum[j] = 0.0f;
  f32x16 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;

  // x rows y0 - 1 and y0 into slots 0 and 1
  for (int s = 0; s < 2; ++s)
    for (int j = tid; j < kWgPairsY * 4; j += 256) {
      const int q = j >> 2, gg = j & 3, c = x0 - 8 + 2 * q;
      const u32x4 u0 = load_chunk(XS, a.H, a.W, y0 - 1 + s, c, gg);
      const u32x4 u1 = load_chunk(XS, a.H, a.W, y0 - 1 + s, c + 1, gg);
      put_pair(xT + s * 32 * kWgPY, kWgPY, 2 * q, gg, u0, u1);
    }

  // dz row o and x row o + 1 into registers; issued one row ahead, so they
  // are in flight during the previous row's MFMAs
  u32x4 d0, d1, e0[2], e1[2];
  auto fetch = [&](int o) {
    d0 = load_chunk(DZ, a.H, a.W, o, x0 + 2 * pp, g);
    d1 = load_chunk(DZ, a.H, a.W, o, x0 + 2 * pp + 1, g);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int j = tid + 256 * k;
      const int q = j >> 2, gg = j & 3, c = x0 - 8 + 2 * q;
      const bool on = j < kWgPairsY * 4;
      e0[k] = on ? load_chunk(XS, a.H, a.W, o + 1, c, gg) : u32x4{0, 0, 0, 0};
      e1[k] = on ? load_chunk(XS, a.H, a.W, o + 1, c + 1, gg) : u32x4{0, 0, 0, 0};
    }
  };
  if (y0 < y1) fetch(y0);
  for (int o = y0; o < y1; ++o) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bsum[2 * i] += bf2f(d0[i] & 0xffffu) + bf2f(d1[i] & 0xffffu);
      bsum[2 * i + 1] += bf2f(d0[i] >> 16) + bf2f(d1[i] >> 16);
    }
    const int s0 = (o - y0) % 3;  // slot of row o - 1
    const int snew = (s0 + 2) % 3;
    __syncthreads();  // the previous row's reads are done
    put_pair(dzT, kWgPD, 2 * pp, g, d0, d1);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int j = tid + 256 * k;
      if (j < kWgPairsY * 4) put_pair(xT + snew * 32 * kWgPY, kWgPY, 2 * (j >> 2), j & 3, e0[k], e1[k]);
    }
    __syncthreads();
    if (o + 1 < y1) fetch(o + 1);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int k0 = (wv * 2 + c) * 16;
      const bf16x8 A = as_bf(*reinterpret_cast<const u32x4*>(dzT + l32 * kWgPD + k0 + 8 * h));
      const int E = k0 + 8 * h + 8;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const uint16_t* row = xT + ((s0 + ky) % 3) * 32 * kWgPY + l32 * kWgPY;
        const u32x4 d = *reinterpret_cast<const u32x4*>(row + E);
        const unsigned pv = *reinterpret_cast<const unsigned*>(row + E - 2);
        const unsigned nv = *reinterpret_cast<const unsigned*>(row + E + 8);
        u32x4 b0, b2;
        b0[0] = __builtin_amdgcn_alignbyte(d[0], pv, 2);
        b0[1] = __builtin_amdgcn_alignbyte(d[1], d[0], 2);
        b0[2] = __builtin_amdgcn_alignbyte(d[2], d[1], 2);
        b0[3] = __builtin_amdgcn_alignbyte(d[3], d[2], 2);
        b2[0] = b0[1];
        b2[1] = b0[2];
        b2[2] = b0[3];
        b2[3] = __builtin_amdgcn_alignbyte(nv, d[3], 2);
        acc[3 * ky] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, as_bf(b0), acc[3 * ky], 0, 0, 0);
        acc[3 * ky + 1] =
            __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, as_bf(d), acc[3 * ky + 1], 0, 0, 0);
        acc[3 * ky + 2] =
            __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, as_bf(b2), acc[3 * ky + 2], 0, 0, 0);
      }
    }
  }

  float* part = a.part + (long long)wg * kWgWidth;
  float* red = reinterpret_cast<float*>(lds);
  __syncthreads();
  // bias sums: threads sharing a channel group, fixed order
#pragma unroll
  for (int j = 0; j < 8; ++j) red[tid * 8 + j] = bsum[j];
  __syncthreads();
  if (tid < 32) {
    const int gg = tid >> 3, j = tid & 7;
    float s = 0.0f;
    for (int q = 0; q < 64; ++q) s += red[(q * 4 + gg) * 8 + j];
    part[9216 + tid] = s;
  }
  __syncthreads();
  // weight sums over the four waves, fixed order
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int co = 8 * (v >> 2) + 4 * h + (v & 3);
          const int idx = t * 1024 + co * 32 + l32;
          red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[t][v];
        }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 9216; idx += 256) {
    const int co = idx / 288, rem = idx - co * 288, ci = rem / 9, t = rem - ci * 9;
    part[idx] = red[t * 1024 + co * 32 + ci];
  }
}

// ------------------------------ 1-channel weight gradients (VALU)
// out[c][t] = sum_p X32[p][c] x1'[p + off(t)] (stored at c * 9 + (flip ? 8 - t : t)),
// x1' = x1 for the input layer (the FP32 image), rnd(x1) for the output layer (a gradient);
// out[288 + c] = sum_p X32[p][c] (width 320)  or  out[288] = sum_p x1[p] (width 289).
// One workgroup per 64 x 64 tile of an image, one partial row per workgroup.
constexpr int kWinCols = 64, kWinRows = 64;  // workgroup tile: 64 columns x 64 rows
constexpr int kWinAhead = 4;                  // rows of loads in flight per thread

__global__ __launch_bounds__(256) void wgrad_in_kernel(const uint16_t* __restrict__ X32,
                                                       const float* __restrict__ x1,
                                                       float* __restrict__ part, int H, int W,
                                                       int tiles_x, int tiles_y, int flip,
                                                       int width) {
  __shared__ float red[4][4][81];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = tid & 3;
  float acc[72], s32[8], s1 = 0.0f;
#pragma unroll
  for (int i = 0; i < 72; ++i) acc[i] = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s32[j] = 0.0f;
  // tile (column block, row block, image); the thread walks one pixel column
  // (channel group g) down the tile's rows with a sliding 3 x 3 window of x1
  const int tx = blockIdx.x % tiles_x, rest = blockIdx.x / tiles_x;
  const int ty = rest % tiles_y, im = rest / tiles_y;
  const int x = tx * kWinCols + (tid >> 2);
  const int r0 = ty * kWinRows, r1 = min(r0 + kWinRows, H);
  if (x < W) {
    const long long plane = (long long)H * W;
    const float* s = x1 + (long long)im * plane;
    const uint16_t* X = X32 + ((long long)im * plane + x) * 32 + 8 * g;
    auto in_row = [&](int rr, float (&v)[3]) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int cc = x + k - 1;
        const float u = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? s[(long long)rr * W + cc] : 0.0f;
        v[k] = flip ? rnd_bf(u) : u;
      }
    };
    // Loads run kWinAhead rows ahead of their use in a register ring (the
    // layer input's 16-byte chunk, three x1 values, the centre value). They
    // are issued unconditionally from clamped addresses, with the bounds
    // applied when a value is used: a load under a condition would be waited
    // for at once.
    auto raw_row = [&](int rr, float (&v)[3]) {
      const int rc = min(max(rr, 0), H - 1);
#pragma unroll
      for (int k = 0; k < 3; ++k) v[k] = s[(long long)rc * W + min(max(x + k - 1, 0), W - 1)];
    };
    auto use_row = [&](int rr, const float (&raw)[3], float (&v)[3]) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int cc = x + k - 1;
        const float u = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? raw[k] : 0.0f;
        v[k] = flip ? rnd_bf(u) : u;
      }
    };
    float in[3][3];  // x1 rows r - 1, r, r + 1 around column x
    in_row(r0 - 1, in[0]);
    in_row(r0, in[1]);
    u32x4 qx[kWinAhead];
    float qr[kWinAhead][3], qs[kWinAhead];
#pragma unroll
    for (int d = 0; d < kWinAhead; ++d) {
      const int rr = r0 + d;
      qx[d] = ld16(X + (long long)min(rr, r1 - 1) * W * 32);
      raw_row(rr + 1, qr[d]);
      qs[d] = s[(long long)min(rr, H - 1) * W + x];
    }
    for (int r = r0; r < r1; r += kWinAhead) {
#pragma unroll
      for (int d = 0; d < kWinAhead; ++d) {
        const int rr = r + d;
        const u32x4 v = qx[d];
        const float raw[3] = {qr[d][0], qr[d][1], qr[d][2]};
        const float sv = qs[d];
        const int rn = rr + kWinAhead;
        qx[d] = ld16(X + (long long)min(rn, r1 - 1) * W * 32);
        raw_row(rn + 1, qr[d]);
        qs[d] = s[(long long)min(rn, H - 1) * W + x];
        if (rr < r1) {
          use_row(rr + 1, raw, in[2]);
          float xv[8];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            xv[2 * j] = bf2f(v[j] & 0xffffu);
            xv[2 * j + 1] = bf2f(v[j] >> 16);
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            s32[j] += xv[j];
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[j * 9 + t] += xv[j] * in[t / 3][t % 3];
          }
          if (g == 0) s1 += sv;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            in[0][k] = in[1][k];
            in[1][k] = in[2][k];
          }
        }
      }
    }
  }
  // lanes with the same g: reduce over lane bits 2..5 (fixed pattern)
#pragma unroll
  for (int i = 0; i < 72; ++i)
    for (int m = 4; m < 64; m <<= 1) acc[i] += __shfl_xor(acc[i], m);
#pragma unroll
  for (int j = 0; j < 8; ++j)
    for (int m = 4; m < 64; m <<= 1) s32[j] += __shfl_xor(s32[j], m);
  for (int m = 4; m < 64; m <<= 1) s1 += __shfl_xor(s1, m);
  if (lane < 4) {
#pragma unroll
    for (int i = 0; i < 72; ++i) red[wv][g][i] = acc[i];
#pragma unroll
    for (int j = 0; j < 8; ++j) red[wv][g][72 + j] = s32[j];
    red[wv][g][80] = s1;
  }
  __syncthreads();
  float* out = part + (long long)blockIdx.x * width;
  for (int i = tid; i < width; i += 256) {
    float v = 0.0f;
    if (i < 288) {
      const int c = i / 9, tt = i % 9, t = flip ? 8 - tt : tt;
      for (int w = 0; w < 4; ++w) v += red[w][c >> 3][(c & 7) * 9 + t];
    } else if (width == 320) {
      const int c = i - 288;
      for (int w = 0; w < 4; ++w) v += red[w][c >> 3][72 + (c & 7)];
    } else {
      for (int w = 0; w < 4; ++w) v += red[w][0][80];
    }
    out[i] = v;
  }
}

// ------------------------------------------------ column sums of partials
// out[j] = sum_r part[r][j], rows in fixed order (two stages, FP64).
constexpr int kRedRows = 32;

__global__ void col_sum_stage1(const float* __restrict__ part, int nrows, int width,
                               double* __restrict__ tmp) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= width) return;
  const int r0 = blockIdx.y * kRedRows, r1 = min(r0 + kRedRows, nrows);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += part[(long long)r * width + j];
  tmp[(long long)blockIdx.y * width + j] = s;
}

__global__ void col_sum_stage2(const double* __restrict__ tmp, int nchunks, int width,
                               float* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= width) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += tmp[(long long)c * width + j];
  out[j] = (float)s;
}

// ---------------------------------------------------------------- others
// b1, b2 and their complements (computed in FP64 on the host: 1 - 0.999f
// would lose four digits) enter separately.
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, long long n, float lr, float b1, float b2,
                            float omb1, float omb2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

constexpr int kSqBlock = 256, kSqPerThread = 16;

__global__ __launch_bounds__(kSqBlock) void sq_error_kernel(long long n, const float* __restrict__ c,
                                                            const float* __restrict__ t, float scale,
                                                            float* __restrict__ grad,
                                                            double* __restrict__ partials) {
  __shared__ double red[kSqBlock];
  const long long base = (long long)blockIdx.x * kSqBlock * kSqPerThread;
  double s = 0.0;
  for (int k = 0; k < kSqPerThread; ++k) {
    const long long i = base + (long long)k * kSqBlock + threadIdx.x;
    if (i < n) {
      const float r = c[i] - t[i];
      if (grad) grad[i] = scale * 2.0f * r;
      s += (double)r * r;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSqBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void soft_kernel(long long n, const float* __restrict__ in, float tau,
                            float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float v = in[i];
  const float a = fabsf(v) - tau;
  out[i] = a > 0.0f ? copysignf(a, v) : 0.0f;
}

// ------------------------------------------------------------ host side
ConvArgs conv_args(int n, int H, int W) {
  ConvArgs a{};
  a.H = H;
  a.W = W;
  a.strips = (W + 31) / 32;
  a.groups = (a.strips + kConvStrips - 1) / kConvStrips;
  a.n = n;
  for (int rows : kConvRows) {
    a.rows = rows;
    a.bands = (H + rows - 1) / rows;
    if ((long long)n * a.bands * a.groups >= kConvMinGrid) break;
  }
  return a;
}

template <int MODE>
hipError_t launch_conv32(const ConvArgs& a, hipStream_t s) {
  const long long blocks = (long long)a.n * a.bands * a.groups;
  hipLaunchKernelGGL(conv32_kernel<MODE>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_conv_in(bool fwd, const float* src, const uint16_t* w, const float* bias,
                          const uint16_t* mask, uint16_t* y, int n, int H, int W, hipStream_t s) {
  if (n > 65535) return hipErrorInvalidValue;  // grid z
  const dim3 grid((unsigned)((4LL * W + 255) / 256), (unsigned)((H + kInRows - 1) / kInRows),
                  (unsigned)n);
  if (fwd)
    hipLaunchKernelGGL(conv_in_kernel<true>, grid, dim3(256), 0, s, src, w, bias, mask, y, H, W);
  else
    hipLaunchKernelGGL(conv_in_kernel<false>, grid, dim3(256), 0, s, src, w, bias, mask, y, H, W);
  return hipGetLastError();
}

struct WgradPlan {
  int strips, bands, RB, nwg;
};

WgradPlan wgrad_plan(int n, int H, int W) {
  WgradPlan p{};
  p.strips = (W + kWgSW - 1) / kWgSW;
  const int per = n * p.strips;
  // about one round of workgroups at two per CU: at 64 images of 512^2 the
  // backward pass measured 6.67-6.71 ms with 512, 6.79-6.81 with 1024,
  // 7.10-7.14 with 768 and 7.02-7.04 with 2048
  const int want = 512;
  int bands = (want + per - 1) / per;
  bands = bands < 1 ? 1 : (bands > H ? H : bands);
  p.RB = (H + bands - 1) / bands;
  p.bands = (H + p.RB - 1) / p.RB;
  p.nwg = per * p.bands;
  return p;
}

long long win_blocks(int n, int H, int W) {
  return (long long)n * ((H + kWinRows - 1) / kWinRows) * ((W + kWinCols - 1) / kWinCols);
}

hipError_t col_sum(const float* part, int nrows, int width, double* tmp, float* out,
                   hipStream_t s) {
  const int chunks = (nrows + kRedRows - 1) / kRedRows;
  const int bx = (width + 255) / 256;
  hipLaunchKernelGGL(col_sum_stage1, dim3(bx, chunks), dim3(256), 0, s, part, nrows, width, tmp);
  hipLaunchKernelGGL(col_sum_stage2, dim3(bx), dim3(256), 0, s, tmp, chunks, width, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cnn_pack(const float* master, void* packed, hipStream_t s) {
  hipLaunchKernelGGL(cnn_pack_kernel, dim3((kPackJobs + 255) / 256), dim3(256), 0, s, master,
                     static_cast<uint8_t*>(packed));
  return hipGetLastError();
}

hipError_t launch_cnn_forward(const void* packed, int n, int H, int W, const float* b, void* acts,
                              float* u, hipStream_t s) {
  const uint8_t* pk = static_cast<const uint8_t*>(packed);
  uint16_t* A = static_cast<uint16_t*>(acts);
  const long long layer = (long long)n * H * W * kCnnCh;
  hipError_t e = launch_conv_in(true, b, reinterpret_cast<const uint16_t*>(pk + CnnPack::w1),
                                reinterpret_cast<const float*>(pk + CnnPack::b1), nullptr, A, n, H,
                                W, s);
  if (e != hipSuccess) return e;
  for (int m = 0; m < 4; ++m) {
    const uint8_t* L = pk + CnnPack::mid + m * CnnPack::mid_size;
    ConvArgs a = conv_args(n, H, W);
    a.x = A + m * layer;
    a.w = reinterpret_cast<const uint16_t*>(L + CnnPack::mid_fwd);
    a.bias = reinterpret_cast<const float*>(L + CnnPack::mid_bias);
    a.y = A + (m + 1) * layer;
    if ((e = launch_conv32<kFwd>(a, s)) != hipSuccess) return e;
  }
  if (n > 65535) return hipErrorInvalidValue;  // grid z
  const dim3 grid((unsigned)((4LL * W + 255) / 256), (unsigned)((H + kInRows - 1) / kInRows),
                  (unsigned)n);
  hipLaunchKernelGGL(conv_out_kernel, grid, dim3(256), 0, s, A + 4 * layer,
                     reinterpret_cast<const uint16_t*>(pk + CnnPack::w6),
                     reinterpret_cast<const float*>(pk + CnnPack::b6), b, u, H, W);
  return hipGetLastError();
}

size_t cnn_backward_scratch(int n, int H, int W) {
  const WgradPlan p = wgrad_plan(n, H, W);
  const long long rows = p.nwg > win_blocks(n, H, W) ? p.nwg : win_blocks(n, H, W);
  const size_t part = (size_t)rows * kWgWidth * sizeof(float);
  const size_t tmp = (size_t)((rows + kRedRows - 1) / kRedRows) * kWgWidth * sizeof(double);
  return ((part + 255) / 256) * 256 + tmp;
}

hipError_t launch_cnn_backward(const void* packed, int n, int H, int W, const float* b,
                               const void* acts, const float* du, void* dacts, float* grad,
                               void* scratch, hipStream_t s) {
  const uint8_t* pk = static_cast<const uint8_t*>(packed);
  const uint16_t* A = static_cast<const uint16_t*>(acts);
  uint16_t* D = static_cast<uint16_t*>(dacts);
  const long long layer = (long long)n * H * W * kCnnCh;
  const WgradPlan wp = wgrad_plan(n, H, W);
  const long long wb = win_blocks(n, H, W);
  const long long rows = wp.nwg > wb ? wp.nwg : wb;
  float* part = static_cast<float*>(scratch);
  double* tmp = reinterpret_cast<double*>(static_cast<uint8_t*>(scratch) +
                                          ((size_t)rows * kWgWidth * sizeof(float) + 255) / 256 * 256);
  hipError_t e;
  // output layer: weights, then the gradient at layer 5's pre-activation
  const int wtx = (W + kWinCols - 1) / kWinCols, wty = (H + kWinRows - 1) / kWinRows;
  hipLaunchKernelGGL(wgrad_in_kernel, dim3((unsigned)wb), dim3(256), 0, s, A + 4 * layer, du, part,
                     H, W, wtx, wty, 1, 289);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = col_sum(part, (int)wb, 289, tmp, grad + kCnnMasterW6, s)) != hipSuccess) return e;
  if ((e = launch_conv_in(false, du, reinterpret_cast<const uint16_t*>(pk + CnnPack::w6d), nullptr,
                          A + 4 * layer, D + 4 * layer, n, H, W, s)) != hipSuccess)
    return e;
  for (int m = 3; m >= 0; --m) {  // layer m + 2: input acts[m], output gradient dacts[m + 1]
    WgradArgs g{};
    g.dz = D + (m + 1) * layer;
    g.x = A + m * layer;
    g.part = part;
    g.H = H;
    g.W = W;
    g.strips = wp.strips;
    g.bands = wp.bands;
    g.RB = wp.RB;
    hipLaunchKernelGGL(wgrad32_kernel, dim3(wp.nwg), dim3(256), 0, s, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = col_sum(part, wp.nwg, kWgWidth, tmp, grad + cnn_master_mid(m), s)) != hipSuccess)
      return e;
    const uint8_t* L = pk + CnnPack::mid + m * CnnPack::mid_size;
    ConvArgs a = conv_args(n, H, W);
    a.x = D + (m + 1) * layer;
    a.w = reinterpret_cast<const uint16_t*>(L + CnnPack::mid_dgrad);
    a.mask = A + m * layer;
    a.y = D + m * layer;
    if ((e = launch_conv32<kDgrad>(a, s)) != hipSuccess) return e;
  }
  // input layer: weights only (no gradient is needed at the image)
  hipLaunchKernelGGL(wgrad_in_kernel, dim3((unsigned)wb), dim3(256), 0, s, D, b, part, H, W, wtx, wty,
                     0, 320);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return col_sum(part, (int)wb, 320, tmp, grad + kCnnMasterW1, s);
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, long long n, double lr,
                       double beta1, double beta2, double eps, double c1, double c2,
                       hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, m, v, g, n,
                     (float)lr, (float)beta1, (float)beta2, (float)(1.0 - beta1),
                     (float)(1.0 - beta2), (float)eps, (float)c1, (float)c2);
  return hipGetLastError();
}

int sq_error_blocks(long long n) {
  const long long per = (long long)kSqBlock * kSqPerThread;
  return (int)((n + per - 1) / per);
}

hipError_t launch_sq_error(long long n, const float* c, const float* t, float scale, float* grad,
                           double* partials, hipStream_t s) {
  hipLaunchKernelGGL(sq_error_kernel, dim3(sq_error_blocks(n)), dim3(kSqBlock), 0, s, n, c, t, scale,
                     grad, partials);
  return hipGetLastError();
}

hipError_t launch_soft_threshold(long long n, const float* in, float tau, float* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(soft_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in, tau,
                     out);
  return hipGetLastError();
}

}  // namespace aw
