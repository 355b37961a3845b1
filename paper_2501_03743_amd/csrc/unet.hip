// The warm-start network: a 3-level U-shaped 3D conv net that maps the
// coefficient field and source of a variable-coefficient Poisson problem to
// an initial guess x0 for the s-step solver (the learned-warm-start
// extension).  Training and inference run in these kernels:
//
//   * 3x3x3 convolutions (stride 1 or 2, zero padding 1) as implicit GEMMs on
//     the BF16 matrix cores (v_mfma_f32_16x16x32_bf16), FP32 accumulation;
//     the input gradient is the same kernel run on the transposed problem;
//   * weight gradients as FP32 tile reductions (fixed order, deterministic);
//   * nearest-neighbour upsampling, channel concatenation, ReLU masks, a 1x1
//     head, the squared-error loss and Adam, as streaming kernels.
//
// Tensors are channels-last [B, D, H, W, C]; activations are BF16, gradients
// FP32, master weights and Adam moments FP32.  Layer table (Ci -> Co, stride);
// the three levels are 4x apart, so the coarsest sees the whole domain:
//   level 1: e1a 8->16, e1b 16->16;  down: d1a 16->16 /2, d1b 16->32 /2
//   level 2: e2 32->32;              down: d2a 32->32 /2, d2b 32->48 /2
//   level 3: bott 48->32
//   up: u2 64->32 (up4(bott) ++ e2), u1 48->16 (up4(u2) ++ e1b), head 16->1.
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

#include "engine.hpp"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

using namespace ssp;

constexpr int kLayers = 10;
constexpr int kHeadC = 16;
struct LayerDef {
  int ci, co, stride;
};
constexpr LayerDef kDef[kLayers] = {{8, 16, 1},  {16, 16, 1}, {16, 16, 2}, {16, 32, 2},
                                    {32, 32, 1}, {32, 32, 2}, {32, 48, 2}, {48, 32, 1},
                                    {64, 32, 1}, {48, 16, 1}};
enum { L_E1A, L_E1B, L_D1A, L_D1B, L_E2, L_D2A, L_D2B, L_BOTT, L_U2, L_U1 };
constexpr int kUp = 4;   // levels are 4x apart (two stride-2 convolutions down)

struct Grid3 {
  int B, D, H, W;
  __host__ __device__ int64_t points() const { return (int64_t)B * D * H * W; }
};

__device__ __forceinline__ void decode(int64_t p, const Grid3 &g, int &b, int &z, int &y,
                                       int &x) {
  x = (int)(p % g.W);
  int64_t t = p / g.W;
  y = (int)(t % g.H);
  t /= g.H;
  z = (int)(t % g.D);
  b = (int)(t / g.D);
}

// The same split for point indices below 2^31, in 32-bit arithmetic (the
// 64-bit divisions cost several times more instructions).
__device__ __forceinline__ void decode32(uint32_t p, const Grid3 &g, int &b, int &z, int &y,
                                         int &x) {
  const uint32_t W = (uint32_t)g.W, H = (uint32_t)g.H, D = (uint32_t)g.D;
  const uint32_t t = p / W, t2 = t / H, bb = t2 / D;
  x = (int)(p - t * W);
  y = (int)(t - t2 * H);
  z = (int)(t2 - bb * D);
  b = (int)bb;
}

__device__ __forceinline__ int64_t encode(int b, int z, int y, int x, const Grid3 &g) {
  return (((int64_t)b * g.D + z) * g.H + y) * g.W + x;
}

// --------------------------------------------------------------------------
// Convolution as an implicit GEMM on the matrix cores
// --------------------------------------------------------------------------
//
// out[p, n] = sum_k A[p, k] Wt[n, k] with k = tap * Cin + c over the 27 taps
// (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)) and Cin input channels, padded to a
// multiple of 32.  Each wavefront owns 16 output points and all NS*16 output
// channels; one v_mfma_f32_16x16x32_bf16 per 32-wide k chunk and 16 channels.
// Operand layout of the instruction (per lane l, m = l % 16, g = l / 16):
//   A: row m, k = 8g .. 8g+7        B: column m, k = 8g .. 8g+7
//   D: rows 4g .. 4g+3, column m
// MODE 0 (forward):  input point q = stride * p + (dz, dy, dx)
// MODE 1 (input gradient of a stride-s convolution): q = (p - (dz, dy, dx)) / s
//   when divisible; here "in" is the output gradient and Wt holds W
//   transposed to [Ci][tap * Co + co].
template <int MODE, int NS>
__global__ __launch_bounds__(256) void k_conv_mfma(const bf16 *__restrict__ in, int cin, Grid3 gi,
                                                   Grid3 go, int stride,
                                                   const bf16 *__restrict__ wt, int kp,
                                                   const float *__restrict__ bias, int relu,
                                                   float *__restrict__ out_f, bf16 *__restrict__ out_b) {
  __shared__ int s_tap[512];      // k/8 -> tap
  __shared__ int s_ci[512];       // k/8 -> channel offset
  const int nk8 = kp / 8;
  for (int i = threadIdx.x; i < nk8; i += 256) {
    const int k = i * 8;
    const int t = k / cin;
    s_tap[i] = t;
    s_ci[i] = k - t * cin;
  }
  __syncthreads();
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int m = lane % 16, g = lane / 16;
  const int64_t P = go.points();
  const int64_t p = (int64_t)blockIdx.x * 64 + wave * 16 + m;
  const bool valid = p < P;
  int b = 0, z = 0, y = 0, x = 0;
  if (valid) decode(p, go, b, z, y, x);
  f32x4 acc[NS];
#pragma unroll
  for (int n = 0; n < NS; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero8 = {};
  // KU k chunks per step: every gather and weight load of the step is issued
  // before its matrix-core operations.  A tap outside the grid, the padding
  // past 27 taps and a point past the end load nothing and use zero (for
  // the stride-2 input gradient most taps are such).  Fewer chunks for the
  // wide input gradients (registers; measured).
  constexpr int KU = (MODE == 1 && NS >= 3) ? 2 : 4;
  for (int kc = 0; kc < kp; kc += 32 * KU) {
    bf16x8 a[KU], w[KU][NS];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = kc + 32 * u < kp ? kc + 32 * u : kp - 32;
      const int i8 = (k >> 3) + g;
      const int t = s_tap[i8];
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      int qz, qy, qx;
      bool ok = valid && t < 27;
      if (MODE == 0) {
        qz = stride * z + dz;
        qy = stride * y + dy;
        qx = stride * x + dx;
      } else {
        qz = z - dz;
        qy = y - dy;
        qx = x - dx;
        if (stride == 2) {
          ok = ok && ((qz | qy | qx) & 1) == 0;
          qz >>= 1;
          qy >>= 1;
          qx >>= 1;
        }
      }
      ok = ok && qz >= 0 && qz < gi.D && qy >= 0 && qy < gi.H && qx >= 0 && qx < gi.W;
      a[u] = zero8;
      if (ok) a[u] = *(const bf16x8 *)(in + encode(b, qz, qy, qx, gi) * cin + s_ci[i8]);
#pragma unroll
      for (int n = 0; n < NS; ++n)
        w[u][n] = *(const bf16x8 *)(wt + (int64_t)(n * 16 + m) * kp + k + g * 8);
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (kc + 32 * u < kp) {
#pragma unroll
        for (int n = 0; n < NS; ++n)
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], w[u][n], acc[n], 0, 0, 0);
      }
    }
  }
  const int cout = NS * 16;
#pragma unroll
  for (int n = 0; n < NS; ++n) {
    const int c = n * 16 + m;
    const float bs = bias ? bias[c] : 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t po = (int64_t)blockIdx.x * 64 + wave * 16 + 4 * g + i;
      if (po < P) {
        float v = acc[n][i] + bs;
        if (relu) v = v > 0.0f ? v : 0.0f;
        if (out_f) out_f[po * cout + c] = v;
        if (out_b) out_b[po * cout + c] = (bf16)v;
      }
    }
  }
}

// Stride-1 convolutions (and their input gradients) with the input tile in
// LDS: a workgroup computes a CTZ x CTY x CTX block of output points (eight
// 16-point rows along x, two per wavefront) and first stages the block plus
// a one-cell halo, all channels, in LDS (zero outside the grid).  Each input
// value then serves all 27 taps from LDS instead of being gathered from the
// caches 27 times; the weight fragment of a k chunk is loaded once per
// wavefront and used for both of its rows.  Same operands, same k order and
// same matrix-core sequence per output as k_conv_mfma, so the results are
// identical.  MODE 1 reads the taps mirrored (q = p - o).  Dynamic LDS:
// (CTZ+2)(CTY+2)(CTX+2) * cin BF16 values.
constexpr int CTX = 16, CTY = 4, CTZ = 2;
constexpr int kTiledMaxCin = 64;   // widest input the staged form takes
// A convolution input formed on the fly as the concatenation of a coarser
// tensor upsampled by kUp (nearest neighbour: channels 0 .. cu-1) and the
// tensor `in` (channels cu .. cin-1), the buffer that k_up_concat writes,
// read in the staging loop instead; up == nullptr: `in` holds all cin.
struct UpSrc {
  const bf16 *up;
  Grid3 gu;
  int cu;
};

template <int MODE, int NS, int KU>
__global__ __launch_bounds__(256) void k_conv_tiled(const bf16 *__restrict__ in, int cin, Grid3 g,
                                                    const bf16 *__restrict__ wt, int kp,
                                                    const float *__restrict__ bias, int relu,
                                                    float *__restrict__ out_f,
                                                    bf16 *__restrict__ out_b, UpSrc us) {
  constexpr int HX = CTX + 2, HY = CTY + 2, HZ = CTZ + 2;
  extern __shared__ __align__(16) bf16 s_in[];
  // per 8-wide k group: the LDS offset of its tap and channel relative to a
  // lane's own point (negative for taps behind it; kPadOff for the zero
  // padding past 27 taps), so the inner loop does no index arithmetic
  constexpr int kPadOff = -(1 << 30);
  __shared__ int s_off[512];
  const int nk8 = kp / 8;
  for (int i = threadIdx.x; i < nk8; i += 256) {
    const int k = i * 8;
    const int t = k / cin;
    int off = kPadOff;
    if (t < 27) {
      int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      if (MODE == 1) {
        dz = -dz;
        dy = -dy;
        dx = -dx;
      }
      off = ((dz * HY + dy) * HX + dx) * cin + (k - t * cin);
    }
    s_off[i] = off;
  }
  const int ntx = (g.W + CTX - 1) / CTX, nty = (g.H + CTY - 1) / CTY, ntz = (g.D + CTZ - 1) / CTZ;
  int64_t bi = blockIdx.x;
  const int tx = (int)(bi % ntx);
  bi /= ntx;
  const int ty = (int)(bi % nty);
  bi /= nty;
  const int tz = (int)(bi % ntz);
  const int b = (int)(bi / ntz);
  const int x0 = tx * CTX, y0 = ty * CTY, z0 = tz * CTZ;
  const int ng = cin / 8;
  const bf16x8 zero8 = {};
  // loads are issued in batches of kStageBatch per thread before their LDS
  // stores, so a 48-channel tile costs three round trips to memory instead
  // of ten (a larger batch costs registers and occupancy; measured)
  constexpr int kStageBatch = 4;
  const int total = HZ * HY * HX * ng;
  for (int e0 = threadIdx.x; e0 < total; e0 += 256 * kStageBatch) {
    bf16x8 sv[kStageBatch];
#pragma unroll
    for (int i = 0; i < kStageBatch; ++i) {
      const int e = e0 + 256 * i;
      sv[i] = zero8;
      if (e < total) {
        const int pi = e / ng, cg = e - pi * ng;
        const int hx = pi % HX, hy = (pi / HX) % HY, hz = pi / (HX * HY);
        const int qx = x0 + hx - 1, qy = y0 + hy - 1, qz = z0 + hz - 1;
        if (qx >= 0 && qx < g.W && qy >= 0 && qy < g.H && qz >= 0 && qz < g.D) {
          const bf16 *src;
          if (!us.up)
            src = in + encode(b, qz, qy, qx, g) * cin + cg * 8;
          else if (cg * 8 < us.cu)
            src = us.up + encode(b, qz / kUp, qy / kUp, qx / kUp, us.gu) * us.cu + cg * 8;
          else
            src = in + encode(b, qz, qy, qx, g) * (cin - us.cu) + (cg * 8 - us.cu);
          sv[i] = *(const bf16x8 *)src;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kStageBatch; ++i) {
      const int e = e0 + 256 * i;
      if (e < total) {
        const int pi = e / ng, cg = e - pi * ng;
        *(bf16x8 *)(s_in + (int64_t)pi * cin + cg * 8) = sv[i];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int m = lane % 16, gq = lane / 16;
  int rz[2], ry[2], base[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int r = wave * 2 + mt;   // 0..7: (z, y) row of the block
    rz[mt] = r / CTY;
    ry[mt] = r % CTY;
    base[mt] = (((rz[mt] + 1) * HY + (ry[mt] + 1)) * HX + (m + 1)) * cin;   // the lane's point
  }
  f32x4 acc[2][NS];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int n = 0; n < NS; ++n) acc[mt][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  // K k chunks of 32 per step: every offset, weight and operand load of the
  // step is issued before its products, so one round trip serves 2 K NS
  // matrix-core operations.  Whole steps of KU chunks first, then one step
  // of the remaining chunks: no branch inside a step, so the accumulators
  // stay in the matrix-core registers.  The chunk order is the same as a
  // plain loop's, whatever KU.
  const bf16 *wl = wt + (int64_t)m * kp + gq * 8;   // this lane's weight row, n = 0
  auto step = [&](int kc, auto kcount) {
    constexpr int K = decltype(kcount)::value;
    int off[K];
    bf16x8 w[K][NS], a[K][2];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int k = kc + 32 * u;
      off[u] = s_off[(k >> 3) + gq];
#pragma unroll
      for (int n = 0; n < NS; ++n) w[u][n] = *(const bf16x8 *)(wl + (int64_t)n * 16 * kp + k);
    }
#pragma unroll
    for (int u = 0; u < K; ++u)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        // padding groups read the lane's own point (always staged) and use zero
        const bool pad = off[u] == kPadOff;
        const bf16x8 v = *(const bf16x8 *)(s_in + base[mt] + (pad ? 0 : off[u]));
        a[u][mt] = pad ? zero8 : v;
      }
#pragma unroll
    for (int u = 0; u < K; ++u)
#pragma unroll
      for (int n = 0; n < NS; ++n)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          acc[mt][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][mt], w[u][n], acc[mt][n], 0, 0, 0);
  };
  const int kfull = kp - kp % (32 * KU);
  for (int kc = 0; kc < kfull; kc += 32 * KU) step(kc, std::integral_constant<int, KU>{});
  // the remaining chunks (fewer than KU) as one step
  switch ((kp - kfull) / 32) {
    case 1: step(kfull, std::integral_constant<int, 1>{}); break;
    case 2: if constexpr (KU > 2) step(kfull, std::integral_constant<int, 2>{}); break;
    case 3: if constexpr (KU > 3) step(kfull, std::integral_constant<int, 3>{}); break;
    default: break;
  }
  const int cout = NS * 16;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int z = z0 + rz[mt], y = y0 + ry[mt];
    if (z >= g.D || y >= g.H) continue;
#pragma unroll
    for (int n = 0; n < NS; ++n) {
      const int c = n * 16 + m;
      const float bs = bias ? bias[c] : 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + 4 * gq + i;
        if (x < g.W) {
          const int64_t po = encode(b, z, y, x, g);
          float v = acc[mt][n][i] + bs;
          if (relu) v = v > 0.0f ? v : 0.0f;
          if (out_f) out_f[po * cout + c] = v;
          if (out_b) out_b[po * cout + c] = (bf16)v;
        }
      }
    }
  }
}

// Weight and bias gradients of one tap on the matrix cores: a GEMM with
// M = ci, N = co and K = the block's output points,
//   part[blk][t][ci][co] = sum_p x[q_t(p), ci] dz[p, co].
// Points are staged KC at a time in LDS transposed to [channel][point]
// (BF16), so a lane's operand (8 consecutive points of one channel) is one
// 16-byte LDS read; the 16 x 16 output tiles are spread over the four waves
// (TPW tiles per wave).  ci is padded to 16 with zero rows.  Tap-0 blocks
// also sum dz per channel for the bias gradient (bpart[blk][co]).  KC
// points per chunk, for at most CX input and CD output channels: the
// narrow layers take longer chunks in the same LDS, and every load of a
// chunk is issued before its LDS stores, so a round trip to memory moves
// more points (the chunk loop waits for one round trip per chunk).  The
// points are multiplied in the same order whatever KC, so the sums are too.
template <int TPW, int KC, int CX, int CD>
__global__ __launch_bounds__(256) void k_wgrad_mfma(const bf16 *__restrict__ xin, int ci_n,
                                                    Grid3 gi, Grid3 go, int stride,
                                                    const bf16 *__restrict__ dz, int co_n,
                                                    int64_t pts_per_blk, float *__restrict__ part,
                                                    float *__restrict__ bpart) {
  constexpr int LDP = KC + 8;   // padded LDS row, in BF16 elements
  __shared__ __align__(16) bf16 sx[CX][LDP];
  __shared__ __align__(16) bf16 sd[CD][LDP];
  const int t = blockIdx.y;
  const int dz_ = t / 9 - 1, dy_ = (t / 3) % 3 - 1, dx_ = t % 3 - 1;
  const int cim = (ci_n + 15) / 16 * 16;
  const int NN = co_n / 16, ntile = (cim / 16) * NN;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int m = lane % 16, g = lane / 16;
  f32x4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.0f;
  const int64_t P = go.points();
  const int64_t p0 = (int64_t)blockIdx.x * pts_per_blk;
  const int64_t p1 = p0 + pts_per_blk < P ? p0 + pts_per_blk : P;
  for (int e = threadIdx.x; e < (cim - ci_n) * LDP; e += 256)
    sx[ci_n + e / LDP][e % LDP] = (bf16)0.0f;
  const bf16x8 zero8 = {};
  const int ngx = ci_n / 8, ngd = co_n / 8;
  constexpr int NX = (KC * (CX / 8) + 255) / 256;   // x loads per thread per chunk
  constexpr int ND = (KC * (CD / 8) + 255) / 256;   // dz loads per thread per chunk
  for (int64_t pb = p0; pb < p1; pb += KC) {
    bf16x8 vx[NX], vd[ND];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = threadIdx.x + 256 * i;
      vx[i] = zero8;
      if (e < KC * ngx) {
        const int j = e / ngx, cg = e - j * ngx;
        const int64_t p = pb + j;
        if (p < p1) {
          int b, z, y, x;
          decode32((uint32_t)p, go, b, z, y, x);   // P < 2^31 (host check)
          const int qz = stride * z + dz_, qy = stride * y + dy_, qx = stride * x + dx_;
          if (qz >= 0 && qz < gi.D && qy >= 0 && qy < gi.H && qx >= 0 && qx < gi.W)
            vx[i] = *(const bf16x8 *)(xin + encode(b, qz, qy, qx, gi) * ci_n + cg * 8);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const int e = threadIdx.x + 256 * i;
      vd[i] = zero8;
      if (e < KC * ngd) {
        const int j = e / ngd, cg = e - j * ngd;
        const int64_t p = pb + j;
        if (p < p1) vd[i] = *(const bf16x8 *)(dz + p * co_n + cg * 8);
      }
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < KC * ngx) {
        const int j = e / ngx, cg = e - j * ngx;
#pragma unroll
        for (int u = 0; u < 8; ++u) sx[cg * 8 + u][j] = vx[i][u];
      }
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < KC * ngd) {
        const int j = e / ngd, cg = e - j * ngd;
#pragma unroll
        for (int u = 0; u < 8; ++u) sd[cg * 8 + u][j] = vd[i][u];
      }
    }
    __syncthreads();
    if (t == 0 && threadIdx.x < co_n)
      for (int j = 0; j < KC; ++j) bacc += (float)sd[threadIdx.x][j];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int tile = wave + 4 * i;
      if (tile < ntile) {
        const int mi = tile / NN, ni = tile - (tile / NN) * NN;
#pragma unroll
        for (int ks = 0; ks < KC; ks += 32) {
          const bf16x8 a = *(const bf16x8 *)&sx[mi * 16 + m][ks + 8 * g];
          const bf16x8 bb = *(const bf16x8 *)&sd[ni * 16 + m][ks + 8 * g];
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[i], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (t == 0 && threadIdx.x < co_n) bpart[(int64_t)blockIdx.x * co_n + threadIdx.x] = bacc;
  float *o = part + ((int64_t)blockIdx.x * 27 + t) * ci_n * co_n;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int tile = wave + 4 * i;
    if (tile < ntile) {
      const int mi = tile / NN, ni = tile - (tile / NN) * NN;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ci = mi * 16 + 4 * g + r;
        if (ci < ci_n) o[ci * co_n + ni * 16 + m] = acc[i][r];
      }
    }
  }
}

// grad[i] += sum over blocks of part[blk][i] (fixed order: four running
// sums over blocks k = 0, 1, 2, 3 mod 4, then combined).
__global__ __launch_bounds__(256) void k_sum_blocks(const float *__restrict__ part, int nblk,
                                                    int64_t m, float *__restrict__ grad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  int k = 0;
  for (; k + 4 <= nblk; k += 4) {
    s0 += part[(int64_t)k * m + i];
    s1 += part[(int64_t)(k + 1) * m + i];
    s2 += part[(int64_t)(k + 2) * m + i];
    s3 += part[(int64_t)(k + 3) * m + i];
  }
  for (; k < nblk; ++k) s0 += part[(int64_t)k * m + i];
  grad[i] += (s0 + s1) + (s2 + s3);
}

// Packs FP32 weights W[27][Ci][Co] into BF16 GEMM operands:
//   fwd: wf[co][t*Ci + ci]   (k padded to kpf with zeros)
//   bwd: wb[ci][t*Co + co]   (k padded to kpb with zeros)
__device__ __forceinline__ void pack_elem(const float *__restrict__ w, int ci_n, int co_n,
                                          bf16 *__restrict__ wf, int kpf, bf16 *__restrict__ wb,
                                          int kpb, int64_t i) {
  const int64_t nf = (int64_t)co_n * kpf, nb = (int64_t)ci_n * kpb;
  if (i < nf) {
    const int co = (int)(i / kpf), k = (int)(i % kpf);
    float v = 0.0f;
    if (k < 27 * ci_n) {
      const int t = k / ci_n, ci = k % ci_n;
      v = w[((int64_t)t * ci_n + ci) * co_n + co];
    }
    wf[i] = (bf16)v;
  }
  if (wb && i < nb) {
    const int ci = (int)(i / kpb), k = (int)(i % kpb);
    float v = 0.0f;
    if (k < 27 * co_n) {
      const int t = k / co_n, co = k % co_n;
      v = w[((int64_t)t * ci_n + ci) * co_n + co];
    }
    wb[i] = (bf16)v;
  }
}

__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ w, int ci_n, int co_n,
                                              bf16 *__restrict__ wf, int kpf,
                                              bf16 *__restrict__ wb, int kpb) {
  pack_elem(w, ci_n, co_n, wf, kpf, wb, kpb, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// Every layer's packing in one launch (the per-layer launches were mostly
// launch overhead): element i belongs to the layer L with
// start[L] <= i < start[L + 1].
constexpr int kPackLayers = 10;
struct PackTable {
  const float *w[kPackLayers];
  bf16 *wf[kPackLayers], *wb[kPackLayers];
  int ci[kPackLayers], co[kPackLayers], kpf[kPackLayers], kpb[kPackLayers];
  int64_t start[kPackLayers + 1];
};
__global__ __launch_bounds__(256) void k_pack_all(PackTable t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= t.start[kPackLayers]) return;
  int L = 0;
  while (L + 1 < kPackLayers && i >= t.start[L + 1]) ++L;
  pack_elem(t.w[L], t.ci[L], t.co[L], t.wf[L], t.kpf[L], t.wb[L], t.kpb[L], i - t.start[L]);
}

// --------------------------------------------------------------------------
// Streaming kernels
// --------------------------------------------------------------------------

// x0[p, 0..7] = (in[p, 0], in[p, 1], 0, ...) in BF16.
__global__ __launch_bounds__(256) void k_input(const float *__restrict__ in, int64_t P,
                                               bf16 *__restrict__ x0) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  for (int c = 0; c < 8; ++c) x0[p * 8 + c] = (bf16)(c < 2 ? in[p * 2 + c] : 0.0f);
}

// Concatenation buffer: buf[p, 0:cu] = up_f(coarse)[p] (nearest neighbour,
// factor f), buf[p, cu:cu+cs] = skip[p]; one thread per (fine point, group
// of 8 channels), 16-byte copies (cu and cs are multiples of 8).
__global__ __launch_bounds__(256) void k_up_concat(const bf16 *__restrict__ coarse, Grid3 gc,
                                                   int cu, const bf16 *__restrict__ skip, int cs,
                                                   Grid3 gf, int f, bf16 *__restrict__ buf) {
  const int ng = (cu + cs) / 8;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= gf.points() * ng) return;
  const int64_t p = i / ng;
  const int cg = (int)(i - p * ng);
  bf16x8 v;
  if (cg * 8 < cu) {
    int b, z, y, x;
    decode(p, gf, b, z, y, x);
    const int64_t q = encode(b, z / f, y / f, x / f, gc);
    v = *(const bf16x8 *)(coarse + q * cu + cg * 8);
  } else {
    v = *(const bf16x8 *)(skip + p * cs + (cg * 8 - cu));
  }
  *(bf16x8 *)(buf + p * (cu + cs) + cg * 8) = v;
}

// Upsampling backward: g_coarse[q, c] = sum over the f^3 fine children of
// g_fine[p, off + c] (fine tensor has ct channels); one thread per (q, c).
__global__ __launch_bounds__(256) void k_up_backward(const float *__restrict__ gfine, Grid3 gf,
                                                     int ct, int off, int c_n, Grid3 gc, int f,
                                                     float *__restrict__ gcoarse) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= gc.points() * c_n) return;
  const int64_t q = i / c_n;
  const int c = (int)(i - q * c_n);
  int b, z, y, x;
  decode(q, gc, b, z, y, x);
  float s = 0.0f;
  for (int oz = 0; oz < f; ++oz)
    for (int oy = 0; oy < f; ++oy)
      for (int ox = 0; ox < f; ++ox) {
        const int fz = f * z + oz, fy = f * y + oy, fx = f * x + ox;
        if (fz < gf.D && fy < gf.H && fx < gf.W) s += gfine[encode(b, fz, fy, fx, gf) * ct + off + c];
      }
  gcoarse[i] = s;
}

// dz = BF16((g1[:, off1:] + g2[:, off2:]) * (act > 0)) over c_n channels.
__global__ __launch_bounds__(256) void k_relu_grad(int64_t P, int c_n, const float *__restrict__ g1,
                                                   int ct1, int off1, const float *__restrict__ g2,
                                                   int ct2, int off2, const bf16 *__restrict__ act,
                                                   bf16 *__restrict__ dz) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= P * c_n) return;
  const int64_t p = i / c_n;
  const int c = (int)(i - p * c_n);
  float g = g1[p * ct1 + off1 + c];
  if (g2) g += g2[p * ct2 + off2 + c];
  dz[i] = (bf16)((float)act[i] > 0.0f ? g : 0.0f);
}

// dst[p, 0:c_n] = src[p, off:off+c_n] (src has ct channels).
__global__ __launch_bounds__(256) void k_slice(const float *__restrict__ src, int ct, int off,
                                               int c_n, int64_t P, float *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= P * c_n) return;
  const int64_t p = i / c_n;
  dst[i] = src[p * ct + off + (i - p * c_n)];
}

// 1x1 head of point p: sum over the 16 channels in order, then the bias.
__device__ __forceinline__ float head_out(const bf16 *__restrict__ a, int64_t p,
                                          const float *__restrict__ w, const float *__restrict__ b) {
  float s = 0.0f;
  for (int c = 0; c < kHeadC; ++c) s += (float)a[p * kHeadC + c] * w[c];
  return s + b[0];
}

// 1x1 head: y[p] = sum_c a[p, c] w[c] + b.
__global__ __launch_bounds__(256) void k_head(const bf16 *__restrict__ a, int64_t P,
                                              const float *__restrict__ w, const float *__restrict__ b,
                                              float *__restrict__ y) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  y[p] = head_out(a, p, w, b);
}

// Inference input and output for one problem (batch 1), in the form the
// training data take: input channels log k and f / rms(f) (the rest zero),
// output x0 = y rms(f) out_scale in FP64.  rms(f) = sqrt(sum f^2 / P) in
// FP64 from per-block partial sums added in block order (1 if it is 0).
__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ f, int64_t P,
                                               double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double v = p < P ? f[p] : 0.0;
  red[threadIdx.x] = v * v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_rms(const double *__restrict__ part, int nblk, int64_t P,
                                             double *__restrict__ rms) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = sqrt(red[0] / (double)P);
    rms[0] = r > 0.0 ? r : 1.0;
  }
}

// double -> FP32 -> BF16 with both roundings, as the FP32 input pair of
// the training path gets them (left alone, the compiler turns the pair into
// one rounding of the double, which differs where the FP32 value sits on a
// BF16 tie); the empty asm keeps the FP32 value opaque
__device__ __forceinline__ bf16 bf16_via_f32(double d) {
  float t = (float)d;
  asm volatile("" : "+v"(t));
  return (bf16)t;
}

__global__ __launch_bounds__(256) void k_input_fields(const double *__restrict__ logk,
                                                      const double *__restrict__ f, int64_t P,
                                                      const double *__restrict__ rms,
                                                      bf16 *__restrict__ x0) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  bf16x8 v = {};
  v[0] = bf16_via_f32(logk[p]);
  v[1] = bf16_via_f32(f[p] / rms[0]);
  *(bf16x8 *)(x0 + p * 8) = v;
}

__global__ __launch_bounds__(256) void k_head_scaled(const bf16 *__restrict__ a, int64_t P,
                                                     const float *__restrict__ w,
                                                     const float *__restrict__ b,
                                                     const double *__restrict__ rms,
                                                     double out_scale, double *__restrict__ x) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  x[p] = (double)head_out(a, p, w, b) * (rms[0] * out_scale);
}

// Head backward: g_a[p, c] = dy[p] w[c]; per-block partial sums of the head
// weight and bias gradients (part[blk][0..16]).
__global__ __launch_bounds__(256) void k_head_backward(const bf16 *__restrict__ a, int64_t P,
                                                       const float *__restrict__ w,
                                                       const float *__restrict__ dy,
                                                       float *__restrict__ ga,
                                                       float *__restrict__ part) {
  __shared__ float red[256][kHeadC + 1];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float d = 0.0f;
  float av[kHeadC];
  for (int c = 0; c < kHeadC; ++c) av[c] = 0.0f;
  if (p < P) {
    d = dy[p];
    for (int c = 0; c < kHeadC; ++c) {
      ga[p * kHeadC + c] = d * w[c];
      av[c] = (float)a[p * kHeadC + c];
    }
  }
  for (int c = 0; c < kHeadC; ++c) red[threadIdx.x][c] = av[c] * d;
  red[threadIdx.x][kHeadC] = d;
  __syncthreads();
  if (threadIdx.x <= kHeadC) {
    float s = 0.0f;
    for (int j = 0; j < 256; ++j) s += red[j][threadIdx.x];
    part[(int64_t)blockIdx.x * (kHeadC + 1) + threadIdx.x] = s;
  }
}

// Squared error: dy = 2 (y - t) / N and per-block partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                             int64_t N, float *__restrict__ dy,
                                             double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (i < N) {
    const float d = y[i] - t[i];
    dy[i] = 2.0f * d / (float)N;
    e = (double)d * (double)d;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Energy-type loss of the error e = y - t on each sample's grid:
// per point l_p = e_p (L e)_p + lambda e_p^2 with L the 7-point Laplacian
// (6 e_p minus the in-grid neighbours; zero outside), so that sum_p l_p =
// e^T (L + lambda I) e; dy = 2 (L e + lambda e) / N, and per-block partial
// sums of l_p.  Penalising the error's gradients matches what CG started
// from y pays for: its energy norm, not its mean square.
__global__ __launch_bounds__(256) void k_loss_h1(const float *__restrict__ y,
                                                 const float *__restrict__ t, Grid3 g, float lam,
                                                 float *__restrict__ dy, double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t N = g.points();
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (p < N) {
    int b, z, yy, x;
    decode(p, g, b, z, yy, x);
    const int64_t sy = g.W, sz = (int64_t)g.W * g.H;
    const float ep = y[p] - t[p];
    float nb = 0.0f;
    if (x > 0) nb += y[p - 1] - t[p - 1];
    if (x < g.W - 1) nb += y[p + 1] - t[p + 1];
    if (yy > 0) nb += y[p - sy] - t[p - sy];
    if (yy < g.H - 1) nb += y[p + sy] - t[p + sy];
    if (z > 0) nb += y[p - sz] - t[p - sz];
    if (z < g.D - 1) nb += y[p + sz] - t[p + sz];
    const float le = 6.0f * ep - nb;
    dy[p] = 2.0f * (le + lam * ep) / (float)N;
    l = (double)ep * ((double)le + (double)lam * (double)ep);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam with bias correction (Kingma & Ba), FP32 master parameters.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }
// Point blocks of a weight-gradient launch (x 27 taps): at least 1024 points
// each, at most 64 blocks, so the partial sums stay small.
int wgrad_blocks(int64_t P) { return (int)std::max<int64_t>(1, std::min<int64_t>(64, P / 1024)); }
int pad32(int k) { return (k + 31) / 32 * 32; }

}  // namespace

// ===========================================================================
// Network object
// ===========================================================================

struct ssp_net {
  ssp_handle *h = nullptr;
  int D = 0, H = 0, W = 0, max_batch = 0;
  int64_t nparam = 0;
  float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  int64_t w_off[kLayers], b_off[kLayers], head_w_off = 0, head_b_off = 0;
  bf16 *wf[kLayers] = {}, *wb[kLayers] = {};
  int kpf[kLayers], kpb[kLayers];
  // activations (BF16)
  bf16 *x0 = nullptr, *a1 = nullptr, *a2 = nullptr, *h1 = nullptr, *d1 = nullptr, *a3 = nullptr,
       *h2 = nullptr, *d2 = nullptr, *a4 = nullptr, *c2 = nullptr, *a5 = nullptr, *c1 = nullptr,
       *a6 = nullptr;
  // backward scratch
  float *g_big = nullptr, *g_big2 = nullptr, *g_skip1 = nullptr, *g_skip2 = nullptr;
  bf16 *dz = nullptr;
  float *wpart = nullptr, *bpart = nullptr;
  int64_t wpart_len = 0;
  double *loss_part = nullptr;
  double *fstat = nullptr;   // inference: per-block sums of f^2, then rms(f)
  float *head_part = nullptr;
  int batch = 0;  // batch of the last forward
  std::vector<void *> allocs;
};

namespace {

int net_alloc(ssp_net *net, void **p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return SSP_ENOMEM;
  }
  net->allocs.push_back(*p);
  return SSP_OK;
}

Grid3 grid_level(const ssp_net *n, int level, int batch) {
  int D = n->D, H = n->H, W = n->W;
  for (int i = 0; i < level; ++i) {
    D = (D - 1) / 2 + 1;
    H = (H - 1) / 2 + 1;
    W = (W - 1) / 2 + 1;
  }
  return Grid3{batch, D, H, W};
}

template <int MODE>
int launch_conv(ssp_handle *h, const bf16 *in, int cin, Grid3 gi, Grid3 go, int stride,
                const bf16 *wt, int kp, const float *bias, int relu, float *out_f, bf16 *out_b,
                int cout, UpSrc us = UpSrc{nullptr, Grid3{}, 0}) {
  const bool tiled = stride == 1 && cin <= kTiledMaxCin && cin % 8 == 0;
  if (us.up && (!tiled || us.cu <= 0 || us.cu >= cin || us.cu % 8 != 0))
    return fail(h, SSP_EINVAL, "conv: the fused upsampled input needs the staged form");
  if (tiled) {
    // LDS-staged input tile (same results, far fewer cache gathers)
    const unsigned tiles = (unsigned)(((gi.W + CTX - 1) / CTX) * ((gi.H + CTY - 1) / CTY) *
                                      ((gi.D + CTZ - 1) / CTZ) * gi.B);
    const size_t lds = sizeof(bf16) * (CTZ + 2) * (CTY + 2) * (CTX + 2) * cin;
    // k chunks per step (KU): 2 for the wide outputs (registers) and for
    // narrow inputs (fewer chunks; the occupancy that fewer registers allow
    // hides more latency), 4 otherwise (measured)
    const bool narrow = cin <= 16;
    switch (cout / 16) {
      case 1:
        if (narrow)
          k_conv_tiled<MODE, 1, 2><<<tiles, 256, lds, h->stream>>>(in, cin, gi, wt, kp, bias, relu, out_f, out_b, us);
        else
          k_conv_tiled<MODE, 1, 4><<<tiles, 256, lds, h->stream>>>(in, cin, gi, wt, kp, bias, relu, out_f, out_b, us);
        break;
      case 2: k_conv_tiled<MODE, 2, 4><<<tiles, 256, lds, h->stream>>>(in, cin, gi, wt, kp, bias, relu, out_f, out_b, us); break;
      case 3: k_conv_tiled<MODE, 3, 2><<<tiles, 256, lds, h->stream>>>(in, cin, gi, wt, kp, bias, relu, out_f, out_b, us); break;
      case 4: k_conv_tiled<MODE, 4, 2><<<tiles, 256, lds, h->stream>>>(in, cin, gi, wt, kp, bias, relu, out_f, out_b, us); break;
      default: return fail(h, SSP_EINVAL, "conv: unsupported channel count");
    }
    LAUNCHCHK(h);
    return SSP_OK;
  }
  const unsigned grid = (unsigned)((go.points() + 63) / 64);
  switch (cout / 16) {
    case 1: k_conv_mfma<MODE, 1><<<grid, 256, 0, h->stream>>>(in, cin, gi, go, stride, wt, kp, bias, relu, out_f, out_b); break;
    case 2: k_conv_mfma<MODE, 2><<<grid, 256, 0, h->stream>>>(in, cin, gi, go, stride, wt, kp, bias, relu, out_f, out_b); break;
    case 3: k_conv_mfma<MODE, 3><<<grid, 256, 0, h->stream>>>(in, cin, gi, go, stride, wt, kp, bias, relu, out_f, out_b); break;
    case 4: k_conv_mfma<MODE, 4><<<grid, 256, 0, h->stream>>>(in, cin, gi, go, stride, wt, kp, bias, relu, out_f, out_b); break;
    case 5: k_conv_mfma<MODE, 5><<<grid, 256, 0, h->stream>>>(in, cin, gi, go, stride, wt, kp, bias, relu, out_f, out_b); break;
    default: return fail(h, SSP_EINVAL, "conv: unsupported channel count");
  }
  LAUNCHCHK(h);
  return SSP_OK;
}

// Weight/bias-gradient partials of one convolution (nblk point blocks x 27
// taps) on the matrix cores.
int launch_wgrad(ssp_handle *h, const bf16 *x, int ci, Grid3 gi, Grid3 go, int stride,
                 const bf16 *dz, int co, int nblk, int64_t per, float *part, float *bpart) {
  const int ntile = ((ci + 15) / 16) * (co / 16);
  if (go.points() > INT32_MAX || gi.points() > INT32_MAX)
    return fail(h, SSP_EINVAL, "weight gradient: grids of 2^31 points or more are not supported");
  const dim3 grid(nblk, 27);
  // chunk length by channel counts (about 17 KB of LDS per workgroup each)
  if (ci <= 16 && co <= 16) {
    k_wgrad_mfma<1, 256, 16, 16><<<grid, 256, 0, h->stream>>>(x, ci, gi, go, stride, dz, co, per, part, bpart);
  } else if (ci <= 48 && co <= 16) {
    k_wgrad_mfma<1, 128, 48, 16><<<grid, 256, 0, h->stream>>>(x, ci, gi, go, stride, dz, co, per, part, bpart);
  } else {
    switch ((ntile + 3) / 4) {
      case 1: k_wgrad_mfma<1, 64, 80, 48><<<grid, 256, 0, h->stream>>>(x, ci, gi, go, stride, dz, co, per, part, bpart); break;
      case 2: k_wgrad_mfma<2, 64, 80, 48><<<grid, 256, 0, h->stream>>>(x, ci, gi, go, stride, dz, co, per, part, bpart); break;
      case 3: k_wgrad_mfma<3, 64, 80, 48><<<grid, 256, 0, h->stream>>>(x, ci, gi, go, stride, dz, co, per, part, bpart); break;
      case 4: k_wgrad_mfma<4, 64, 80, 48><<<grid, 256, 0, h->stream>>>(x, ci, gi, go, stride, dz, co, per, part, bpart); break;
      default: return fail(h, SSP_EINVAL, "weight gradient: unsupported channel counts");
    }
  }
  LAUNCHCHK(h);
  return SSP_OK;
}

// Forward of conv layer L: out = relu(conv(in) + b) in BF16.
int layer_forward(ssp_net *n, int L, const bf16 *in, Grid3 gi, Grid3 go, bf16 *out,
                  UpSrc us = UpSrc{nullptr, Grid3{}, 0}) {
  const LayerDef &d = kDef[L];
  return launch_conv<0>(n->h, in, d.ci, gi, go, d.stride, n->wf[L], n->kpf[L],
                        n->params + n->b_off[L], 1, nullptr, out, d.co, us);
}

// Backward of conv layer L given dz (BF16, after the ReLU mask): weight and
// bias gradients, and (if gx) the FP32 input gradient.
int layer_backward(ssp_net *n, int L, const bf16 *in, Grid3 gi, Grid3 go, const bf16 *dz,
                   float *gx) {
  ssp_handle *h = n->h;
  const LayerDef &d = kDef[L];
  const int64_t P = go.points();
  const int nblk = wgrad_blocks(P);
  const int64_t per = (P + nblk - 1) / nblk;
  const int64_t m = 27LL * d.ci * d.co;
  if ((int64_t)nblk * m > n->wpart_len) return fail(h, SSP_EINVAL, "weight-gradient scratch too small");
  int rc = launch_wgrad(h, in, d.ci, gi, go, d.stride, dz, d.co, nblk, per, n->wpart, n->bpart);
  if (rc) return rc;
  k_sum_blocks<<<nblocks(m), 256, 0, h->stream>>>(n->wpart, nblk, m, n->grads + n->w_off[L]);
  LAUNCHCHK(h);
  k_sum_blocks<<<1, 256, 0, h->stream>>>(n->bpart, nblk, d.co, n->grads + n->b_off[L]);
  LAUNCHCHK(h);
  if (gx) {
    rc = launch_conv<1>(h, dz, d.co, go, gi, d.stride, n->wb[L], n->kpb[L], nullptr, 0, gx,
                            nullptr, d.ci);
    if (rc) return rc;
  }
  return SSP_OK;
}

}  // namespace

namespace {

// BF16 GEMM operands from the FP32 master weights, all layers in one launch.
int pack_weights(ssp_net *n) {
  ssp_handle *h = n->h;
  static_assert(kLayers == kPackLayers, "one packing table entry per layer");
  PackTable t;
  t.start[0] = 0;
  for (int L = 0; L < kLayers; ++L) {
    const int64_t nf = (int64_t)kDef[L].co * n->kpf[L], nb = (int64_t)kDef[L].ci * n->kpb[L];
    t.w[L] = n->params + n->w_off[L];
    t.wf[L] = n->wf[L];
    t.wb[L] = n->wb[L];
    t.ci[L] = kDef[L].ci;
    t.co[L] = kDef[L].co;
    t.kpf[L] = n->kpf[L];
    t.kpb[L] = n->kpb[L];
    t.start[L + 1] = t.start[L] + std::max(nf, nb);
  }
  k_pack_all<<<nblocks(t.start[kLayers]), 256, 0, h->stream>>>(t);
  LAUNCHCHK(h);
  return SSP_OK;
}

// Encoder (x0 -> e1b, the 32-channel level and the bottleneck) of the
// network on the grids g.
int encoder_forward(ssp_net *n, const Grid3 *g) {
  int rc;
  if ((rc = layer_forward(n, L_E1A, n->x0, g[0], g[0], n->a1))) return rc;
  if ((rc = layer_forward(n, L_E1B, n->a1, g[0], g[0], n->a2))) return rc;
  if ((rc = layer_forward(n, L_D1A, n->a2, g[0], g[1], n->h1))) return rc;
  if ((rc = layer_forward(n, L_D1B, n->h1, g[1], g[2], n->d1))) return rc;
  if ((rc = layer_forward(n, L_E2, n->d1, g[2], g[2], n->a3))) return rc;
  if ((rc = layer_forward(n, L_D2A, n->a3, g[2], g[3], n->h2))) return rc;
  if ((rc = layer_forward(n, L_D2B, n->h2, g[3], g[4], n->d2))) return rc;
  return layer_forward(n, L_BOTT, n->d2, g[4], g[4], n->a4);
}

}  // namespace

extern "C" {

int ssp_net_create(ssp_handle *h, int D, int H, int W, int max_batch, uint64_t seed,
                   ssp_net **out) {
  if (!h || !out) return SSP_EINVAL;
  *out = nullptr;
  if (D < 4 || H < 4 || W < 4 || max_batch < 1 || (int64_t)D * H * W * max_batch > (1LL << 28))
    return fail(h, SSP_EINVAL, "ssp_net_create: invalid grid or batch");
  HIPCHK(h, hipSetDevice(h->device));
  ssp_net *n = new (std::nothrow) ssp_net();
  if (!n) return SSP_ENOMEM;
  n->h = h;
  n->D = D;
  n->H = H;
  n->W = W;
  n->max_batch = max_batch;
  // parameter layout: per layer W[27][Ci][Co] then b[Co]; head w[16], b[1]
  int64_t off = 0;
  for (int L = 0; L < kLayers; ++L) {
    n->w_off[L] = off;
    off += 27LL * kDef[L].ci * kDef[L].co;
    n->b_off[L] = off;
    off += kDef[L].co;
    n->kpf[L] = pad32(27 * kDef[L].ci);
    n->kpb[L] = pad32(27 * kDef[L].co);
  }
  n->head_w_off = off;
  off += kHeadC;
  n->head_b_off = off;
  off += 1;
  n->nparam = off;
  // grids: g0 full, g1 = /2, g2 = /4 (level 2), g3 = /8, g4 = /16 (level 3)
  int64_t P[5];
  for (int l = 0; l < 5; ++l) P[l] = grid_level(n, l, max_batch).points();
  int rc = SSP_OK;
  auto A = [&](void **p, size_t bytes) {
    if (rc == SSP_OK) rc = net_alloc(n, p, bytes);
  };
  A((void **)&n->params, sizeof(float) * off);
  A((void **)&n->grads, sizeof(float) * off);
  A((void **)&n->adam_m, sizeof(float) * off);
  A((void **)&n->adam_v, sizeof(float) * off);
  for (int L = 0; L < kLayers; ++L) {
    A((void **)&n->wf[L], sizeof(bf16) * kDef[L].co * n->kpf[L]);
    A((void **)&n->wb[L], sizeof(bf16) * kDef[L].ci * n->kpb[L]);
  }
  A((void **)&n->x0, sizeof(bf16) * P[0] * 8);
  A((void **)&n->a1, sizeof(bf16) * P[0] * 16);
  A((void **)&n->a2, sizeof(bf16) * P[0] * 16);
  A((void **)&n->h1, sizeof(bf16) * P[1] * 16);
  A((void **)&n->d1, sizeof(bf16) * P[2] * 32);
  A((void **)&n->a3, sizeof(bf16) * P[2] * 32);
  A((void **)&n->h2, sizeof(bf16) * P[3] * 32);
  A((void **)&n->d2, sizeof(bf16) * P[4] * 48);
  A((void **)&n->a4, sizeof(bf16) * P[4] * 32);
  A((void **)&n->c2, sizeof(bf16) * P[2] * 64);
  A((void **)&n->a5, sizeof(bf16) * P[2] * 32);
  A((void **)&n->c1, sizeof(bf16) * P[0] * 48);
  A((void **)&n->a6, sizeof(bf16) * P[0] * 16);
  const int64_t big = std::max({P[0] * 48, P[1] * 16, P[2] * 64, P[3] * 32, P[4] * 48});
  A((void **)&n->g_big, sizeof(float) * big);
  A((void **)&n->g_big2, sizeof(float) * big);
  A((void **)&n->g_skip1, sizeof(float) * P[0] * 16);
  A((void **)&n->g_skip2, sizeof(float) * P[2] * 32);
  A((void **)&n->dz, sizeof(bf16) * std::max({P[0] * 16, P[1] * 16, P[2] * 32, P[3] * 32, P[4] * 48}));
  n->wpart_len = 64LL * 27 * 80 * 32;
  A((void **)&n->wpart, sizeof(float) * n->wpart_len);
  A((void **)&n->bpart, sizeof(float) * 64 * 48);
  A((void **)&n->loss_part, sizeof(double) * nblocks(P[0]));
  A((void **)&n->fstat, sizeof(double) * (nblocks((int64_t)D * H * W) + 1));
  A((void **)&n->head_part, sizeof(float) * nblocks(P[0]) * (kHeadC + 1));
  if (rc) {
    ssp_net_destroy(n);
    return fail(h, rc, "ssp_net_create: allocation failed");
  }
  // He-normal initial weights, zero biases (host RNG, seeded)
  std::vector<float> hp(off, 0.0f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int L = 0; L < kLayers; ++L) {
    const double sd = std::sqrt(2.0 / (27.0 * kDef[L].ci));
    for (int64_t i = 0; i < 27LL * kDef[L].ci * kDef[L].co; ++i)
      hp[n->w_off[L] + i] = (float)(nd(rng) * sd);
  }
  for (int c = 0; c < kHeadC; ++c) hp[n->head_w_off + c] = (float)(nd(rng) * std::sqrt(1.0 / kHeadC));
  HIPCHK(h, hipMemcpy(n->params, hp.data(), sizeof(float) * off, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemset(n->grads, 0, sizeof(float) * off));
  HIPCHK(h, hipMemset(n->adam_m, 0, sizeof(float) * off));
  HIPCHK(h, hipMemset(n->adam_v, 0, sizeof(float) * off));
  *out = n;
  return SSP_OK;
}

int ssp_net_destroy(ssp_net *n) {
  if (!n) return SSP_OK;
  if (n->h) (void)hipStreamSynchronize(n->h->stream);
  for (void *p : n->allocs) (void)hipFree(p);
  delete n;
  return SSP_OK;
}

int ssp_net_params(ssp_net *n, float **params, float **grads, int64_t *count) {
  if (!n) return SSP_EINVAL;
  if (params) *params = n->params;
  if (grads) *grads = n->grads;
  if (count) *count = n->nparam;
  return SSP_OK;
}

int ssp_net_forward(ssp_net *n, const float *in, int batch, float *out) {
  if (!n || !in || !out || batch < 1 || batch > n->max_batch) return SSP_EINVAL;
  ssp_handle *h = n->h;
  HIPCHK(h, hipSetDevice(h->device));
  int rc = pack_weights(n);
  if (rc) return rc;
  Grid3 g[5];
  for (int l = 0; l < 5; ++l) g[l] = grid_level(n, l, batch);
  k_input<<<nblocks(g[0].points()), 256, 0, h->stream>>>(in, g[0].points(), n->x0);
  LAUNCHCHK(h);
  if ((rc = encoder_forward(n, g))) return rc;
  k_up_concat<<<nblocks(g[2].points() * 8), 256, 0, h->stream>>>(n->a4, g[4], 32, n->a3, 32, g[2],
                                                                 kUp, n->c2);
  LAUNCHCHK(h);
  if ((rc = layer_forward(n, L_U2, n->c2, g[2], g[2], n->a5))) return rc;
  k_up_concat<<<nblocks(g[0].points() * 6), 256, 0, h->stream>>>(n->a5, g[2], 32, n->a2, 16, g[0],
                                                                 kUp, n->c1);
  LAUNCHCHK(h);
  if ((rc = layer_forward(n, L_U1, n->c1, g[0], g[0], n->a6))) return rc;
  k_head<<<nblocks(g[0].points()), 256, 0, h->stream>>>(n->a6, g[0].points(), n->params + n->head_w_off,
                                                        n->params + n->head_b_off, out);
  LAUNCHCHK(h);
  n->batch = batch;
  return SSP_OK;
}

int ssp_net_predict(ssp_net *n, const double *logk, const double *f, double out_scale,
                    double *x0) {
  if (!n || !logk || !f || !x0 || !std::isfinite(out_scale)) return SSP_EINVAL;
  ssp_handle *h = n->h;
  HIPCHK(h, hipSetDevice(h->device));
  int rc = pack_weights(n);
  if (rc) return rc;
  Grid3 g[5];
  for (int l = 0; l < 5; ++l) g[l] = grid_level(n, l, 1);
  const int64_t P = g[0].points();
  const unsigned nb = nblocks(P);
  k_sumsq<<<nb, 256, 0, h->stream>>>(f, P, n->fstat + 1);
  LAUNCHCHK(h);
  k_rms<<<1, 256, 0, h->stream>>>(n->fstat + 1, (int)nb, P, n->fstat);
  LAUNCHCHK(h);
  k_input_fields<<<nb, 256, 0, h->stream>>>(logk, f, P, n->fstat, n->x0);
  LAUNCHCHK(h);
  if ((rc = encoder_forward(n, g))) return rc;
  // the decoder reads its concatenated inputs straight from the two levels
  if ((rc = layer_forward(n, L_U2, n->a3, g[2], g[2], n->a5, UpSrc{n->a4, g[4], 32}))) return rc;
  if ((rc = layer_forward(n, L_U1, n->a2, g[0], g[0], n->a6, UpSrc{n->a5, g[2], 32}))) return rc;
  k_head_scaled<<<nb, 256, 0, h->stream>>>(n->a6, P, n->params + n->head_w_off,
                                          n->params + n->head_b_off, n->fstat, out_scale, x0);
  LAUNCHCHK(h);
  n->batch = 0;   // the activations are not a training forward's
  return SSP_OK;
}

int ssp_net_zero_grad(ssp_net *n) {
  if (!n) return SSP_EINVAL;
  HIPCHK(n->h, hipMemsetAsync(n->grads, 0, sizeof(float) * n->nparam, n->h->stream));
  return SSP_OK;
}

int ssp_net_backward(ssp_net *n, const float *dy) {
  if (!n || !dy || n->batch < 1) return SSP_EINVAL;
  ssp_handle *h = n->h;
  HIPCHK(h, hipSetDevice(h->device));
  const int batch = n->batch;
  Grid3 g[5];
  int64_t P[5];
  for (int l = 0; l < 5; ++l) {
    g[l] = grid_level(n, l, batch);
    P[l] = g[l].points();
  }
  float *A = n->g_big, *B = n->g_big2;   // ping-pong FP32 gradient buffers
  int rc;
  auto relu_grad = [&](int64_t Pn, int c, const float *g1, const float *g2, const bf16 *act) {
    k_relu_grad<<<nblocks(Pn * c), 256, 0, h->stream>>>(Pn, c, g1, c, 0, g2, c, 0, act, n->dz);
    return hipGetLastError() == hipSuccess ? SSP_OK : fail(h, SSP_EHIP, "kernel launch failed");
  };
  // head
  k_head_backward<<<nblocks(P[0]), 256, 0, h->stream>>>(n->a6, P[0], n->params + n->head_w_off, dy,
                                                        A, n->head_part);
  LAUNCHCHK(h);
  k_sum_blocks<<<1, 256, 0, h->stream>>>(n->head_part, (int)nblocks(P[0]), kHeadC + 1,
                                         n->grads + n->head_w_off);
  LAUNCHCHK(h);
  // u1: c1 = [up4(a5), a2] (48 channels) -> a6
  if ((rc = relu_grad(P[0], 16, A, nullptr, n->a6))) return rc;
  if ((rc = layer_backward(n, L_U1, n->c1, g[0], g[0], n->dz, B))) return rc;
  k_up_backward<<<nblocks(P[2] * 32), 256, 0, h->stream>>>(B, g[0], 48, 0, 32, g[2], kUp, A);
  LAUNCHCHK(h);
  // the a2 skip gradient, channels 32..47, must survive the reuse of B
  k_slice<<<nblocks(P[0] * 16), 256, 0, h->stream>>>(B, 48, 32, 16, P[0], n->g_skip1);
  LAUNCHCHK(h);
  // u2: c2 = [up4(a4), a3] (64 channels) -> a5
  if ((rc = relu_grad(P[2], 32, A, nullptr, n->a5))) return rc;
  if ((rc = layer_backward(n, L_U2, n->c2, g[2], g[2], n->dz, B))) return rc;
  k_up_backward<<<nblocks(P[4] * 32), 256, 0, h->stream>>>(B, g[2], 64, 0, 32, g[4], kUp, A);
  LAUNCHCHK(h);
  k_slice<<<nblocks(P[2] * 32), 256, 0, h->stream>>>(B, 64, 32, 32, P[2], n->g_skip2);
  LAUNCHCHK(h);
  // bott: d2 -> a4
  if ((rc = relu_grad(P[4], 32, A, nullptr, n->a4))) return rc;
  if ((rc = layer_backward(n, L_BOTT, n->d2, g[4], g[4], n->dz, B))) return rc;
  // d2b: h2 -> d2 (stride 2)
  if ((rc = relu_grad(P[4], 48, B, nullptr, n->d2))) return rc;
  if ((rc = layer_backward(n, L_D2B, n->h2, g[3], g[4], n->dz, A))) return rc;
  // d2a: a3 -> h2 (stride 2)
  if ((rc = relu_grad(P[3], 32, A, nullptr, n->h2))) return rc;
  if ((rc = layer_backward(n, L_D2A, n->a3, g[2], g[3], n->dz, B))) return rc;
  // e2: d1 -> a3 (a3 also feeds the u2 skip)
  if ((rc = relu_grad(P[2], 32, B, n->g_skip2, n->a3))) return rc;
  if ((rc = layer_backward(n, L_E2, n->d1, g[2], g[2], n->dz, A))) return rc;
  // d1b: h1 -> d1 (stride 2)
  if ((rc = relu_grad(P[2], 32, A, nullptr, n->d1))) return rc;
  if ((rc = layer_backward(n, L_D1B, n->h1, g[1], g[2], n->dz, B))) return rc;
  // d1a: a2 -> h1 (stride 2)
  if ((rc = relu_grad(P[1], 16, B, nullptr, n->h1))) return rc;
  if ((rc = layer_backward(n, L_D1A, n->a2, g[0], g[1], n->dz, A))) return rc;
  // e1b: a1 -> a2 (a2 also feeds the u1 skip)
  if ((rc = relu_grad(P[0], 16, A, n->g_skip1, n->a2))) return rc;
  if ((rc = layer_backward(n, L_E1B, n->a1, g[0], g[0], n->dz, B))) return rc;
  // e1a: x0 -> a1
  if ((rc = relu_grad(P[0], 16, B, nullptr, n->a1))) return rc;
  if ((rc = layer_backward(n, L_E1A, n->x0, g[0], g[0], n->dz, nullptr))) return rc;
  return SSP_OK;
}

namespace {
int finish_loss(ssp_net *n, unsigned nb, int64_t N, double *loss) {
  ssp_handle *h = n->h;
  LAUNCHCHK(h);
  if (loss) {
    std::vector<double> part(nb);
    HIPCHK(h, hipMemcpyAsync(part.data(), n->loss_part, sizeof(double) * nb, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double s = 0.0;
    for (double v : part) s += v;
    *loss = s / (double)N;
  }
  return SSP_OK;
}
}  // namespace

int ssp_net_loss(ssp_net *n, const float *y, const float *target, float *dy, double *loss) {
  if (!n || !y || !target || !dy || n->batch < 1) return SSP_EINVAL;
  const int64_t N = grid_level(n, 0, n->batch).points();
  const unsigned nb = nblocks(N);
  k_mse<<<nb, 256, 0, n->h->stream>>>(y, target, N, dy, n->loss_part);
  return finish_loss(n, nb, N, loss);
}

int ssp_net_loss_h1(ssp_net *n, const float *y, const float *target, float lambda, float *dy,
                    double *loss) {
  if (!n || !y || !target || !dy || n->batch < 1 || !(lambda >= 0.0f)) return SSP_EINVAL;
  const Grid3 g = grid_level(n, 0, n->batch);
  const int64_t N = g.points();
  const unsigned nb = nblocks(N);
  k_loss_h1<<<nb, 256, 0, n->h->stream>>>(y, target, g, lambda, dy, n->loss_part);
  return finish_loss(n, nb, N, loss);
}

int ssp_net_adam_step(ssp_net *n, float lr, float beta1, float beta2, float eps, int step) {
  if (!n || step < 1) return SSP_EINVAL;
  ssp_handle *h = n->h;
  const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
  k_adam<<<nblocks(n->nparam), 256, 0, h->stream>>>(n->params, n->grads, n->adam_m, n->adam_v,
                                                    n->nparam, lr, beta1, beta2, eps, c1, c2);
  LAUNCHCHK(h);
  return SSP_OK;
}

int ssp_net_get_state(ssp_net *n, float *host, int64_t cap) {
  if (!n || !host || cap < 3 * n->nparam) return SSP_EINVAL;
  HIPCHK(n->h, hipStreamSynchronize(n->h->stream));
  HIPCHK(n->h, hipMemcpy(host, n->params, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
  HIPCHK(n->h, hipMemcpy(host + n->nparam, n->adam_m, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
  HIPCHK(n->h, hipMemcpy(host + 2 * n->nparam, n->adam_v, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
  return SSP_OK;
}

int ssp_net_set_state(ssp_net *n, const float *host, int64_t len) {
  if (!n || !host || len < n->nparam) return SSP_EINVAL;
  HIPCHK(n->h, hipStreamSynchronize(n->h->stream));
  HIPCHK(n->h, hipMemcpy(n->params, host, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
  if (len >= 3 * n->nparam) {
    HIPCHK(n->h, hipMemcpy(n->adam_m, host + n->nparam, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
    HIPCHK(n->h, hipMemcpy(n->adam_v, host + 2 * n->nparam, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
  }
  return SSP_OK;
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float *a, int64_t n, bf16 *b) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = (bf16)a[i];
}

// One 3x3x3 convolution on its own (inputs rounded to BF16, FP32 result):
// mode 0: out = conv(in, w) (no bias, no ReLU), in [B,D,H,W,ci] -> out on the
// strided grid with co channels; mode 1: out = input gradient of that
// convolution for the output gradient `in` ([B, Do, Ho, Wo, co]) -> [B,D,H,W,ci].
// w is FP32 [27][ci][co].  All DEVICE pointers; allocates temporaries.
int ssp_conv3d(ssp_handle *h, int mode, const float *in, int B, int D, int H, int W, int ci,
               const float *w, int co, int stride, float *out) {
  if (!h || !in || !w || !out || (mode != 0 && mode != 1) || (stride != 1 && stride != 2) ||
      ci % 8 || co % 16 || (mode == 1 && (ci % 16 || co % 8)) || ci > 80 || co > 80)
    return SSP_EINVAL;
  HIPCHK(h, hipSetDevice(h->device));
  const Grid3 gi{B, D, H, W};
  const Grid3 go{B, (D - 1) / stride + 1, (H - 1) / stride + 1, (W - 1) / stride + 1};
  const int kpf = pad32(27 * ci), kpb = pad32(27 * co);
  const int64_t nin = (mode == 0 ? gi.points() * ci : go.points() * co);
  bf16 *ib = nullptr, *wf = nullptr, *wb = nullptr;
  HIPCHK(h, hipMalloc(&ib, sizeof(bf16) * nin));
  HIPCHK(h, hipMalloc(&wf, sizeof(bf16) * co * kpf));
  HIPCHK(h, hipMalloc(&wb, sizeof(bf16) * ci * kpb));
  k_f32_to_bf16<<<nblocks(nin), 256, 0, h->stream>>>(in, nin, ib);
  k_pack<<<nblocks(std::max<int64_t>((int64_t)co * kpf, (int64_t)ci * kpb)), 256, 0, h->stream>>>(
      w, ci, co, wf, kpf, wb, kpb);
  int rc = (mode == 0) ? launch_conv<0>(h, ib, ci, gi, go, stride, wf, kpf, nullptr, 0, out, nullptr, co)
                       : launch_conv<1>(h, ib, co, go, gi, stride, wb, kpb, nullptr, 0, out, nullptr, ci);
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(ib);
  (void)hipFree(wf);
  (void)hipFree(wb);
  return rc;
}

// Weight and bias gradients of one convolution (inputs rounded to BF16):
// dw[27][ci][co] = sum_p x[q(p,t), ci] dz[p, co], db[co] = sum_p dz[p, co].
int ssp_conv3d_wgrad(ssp_handle *h, const float *x, int B, int D, int H, int W, int ci,
                     const float *dz, int co, int stride, float *dw, float *db) {
  if (!h || !x || !dz || !dw || !db || (stride != 1 && stride != 2) || ci % 8 || co % 16 ||
      ci > 80 || co > 48)
    return SSP_EINVAL;
  HIPCHK(h, hipSetDevice(h->device));
  const Grid3 gi{B, D, H, W};
  const Grid3 go{B, (D - 1) / stride + 1, (H - 1) / stride + 1, (W - 1) / stride + 1};
  const int64_t P = go.points();
  const int nblk = wgrad_blocks(P);
  const int64_t per = (P + nblk - 1) / nblk;
  const int64_t m = 27LL * ci * co;
  bf16 *xb = nullptr, *db16 = nullptr;
  float *part = nullptr, *bpart = nullptr;
  HIPCHK(h, hipMalloc(&xb, sizeof(bf16) * gi.points() * ci));
  HIPCHK(h, hipMalloc(&db16, sizeof(bf16) * P * co));
  HIPCHK(h, hipMalloc(&part, sizeof(float) * nblk * m));
  HIPCHK(h, hipMalloc(&bpart, sizeof(float) * nblk * co));
  k_f32_to_bf16<<<nblocks(gi.points() * ci), 256, 0, h->stream>>>(x, gi.points() * ci, xb);
  k_f32_to_bf16<<<nblocks(P * co), 256, 0, h->stream>>>(dz, P * co, db16);
  HIPCHK(h, hipMemsetAsync(dw, 0, sizeof(float) * m, h->stream));
  HIPCHK(h, hipMemsetAsync(db, 0, sizeof(float) * co, h->stream));
  const int lrc = launch_wgrad(h, xb, ci, gi, go, stride, db16, co, nblk, per, part, bpart);
  if (lrc == SSP_OK) k_sum_blocks<<<nblocks(m), 256, 0, h->stream>>>(part, nblk, m, dw);
  k_sum_blocks<<<1, 256, 0, h->stream>>>(bpart, nblk, co, db);
  const hipError_t e = hipGetLastError();
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(xb);
  (void)hipFree(db16);
  (void)hipFree(part);
  (void)hipFree(bpart);
  if (lrc) return lrc;
  return e == hipSuccess ? SSP_OK : SSP_EHIP;
}

// Matrix-core self test: D = A B for a 16 x 32 A and a 32 x 16 B (FP32 in
// and out, BF16 operands), one v_mfma_f32_16x16x32_bf16 with the operand
// layout the convolutions assume.  DEVICE pointers: A row-major 16 x 32,
// B row-major 32 x 16, D row-major 16 x 16.
static __global__ void k_mfma_selftest(const float *A, const float *B, float *D) {
  const int l = threadIdx.x, m = l % 16, g = l / 16;
  bf16x8 a, b;
  for (int j = 0; j < 8; ++j) {
    a[j] = (bf16)A[m * 32 + 8 * g + j];
    b[j] = (bf16)B[(8 * g + j) * 16 + m];
  }
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  for (int i = 0; i < 4; ++i) D[(4 * g + i) * 16 + m] = acc[i];
}

int ssp_net_mfma_selftest(ssp_handle *h, const float *A, const float *B, float *D) {
  if (!h || !A || !B || !D) return SSP_EINVAL;
  HIPCHK(h, hipSetDevice(h->device));
  k_mfma_selftest<<<1, 64, 0, h->stream>>>(A, B, D);
  LAUNCHCHK(h);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return SSP_OK;
}

}  // extern "C"
