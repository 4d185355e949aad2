// decoder.hip -- the reconstruction network of TRIPS (Sec. 3.3, Fig. conv) for gfx950.
//
// One block per pyramid layer, coarsest first: the layer's D feature channels and (below
// the coarsest layer) the bilinear doubling of the coarser block's 32 output features go
// through one gated 3x3 convolution (ELU of 32 feature outputs times the sigmoid of 32 gate
// outputs), plus the doubled coarser features as a bypass; the finest block's features go
// through a 1x1 output convolution.
//
// The convolution is the one dense contraction of the pipeline, so it runs on the matrix
// cores: an implicit GEMM with M = output texels, N = 64 outputs (feature and gate),
// K = 9 taps x input channels, binary16 operands and float32 accumulation
// (v_mfma_f32_16x16x32_f16).  A workgroup owns a 16x16 tile of output texels per step
// (persistent over tiles) and keeps the layer's packed kernel in LDS for all of them:
//  - the 18x18 input halo is built in LDS straight from the feature pyramid (float32 ->
//    binary16) and from the coarser block's output (doubled on the fly), 80 bytes per
//    texel: 32 doubled features, then the D layer features, zero padded;
//  - K is ordered as nine steps of 32 (one per tap: the doubled features) followed by
//    ceil(9 D / 32) steps over (tap, layer channel), so every A fragment is one or two
//    LDS reads at 16-byte granularity; B fragments are stored lane-major (packed once by
//    k_dec_pack) and read without bank conflicts;
//  - a wave owns four rows of the tile: 4 x 4 accumulator tiles of 16 outputs x 16 texels
//    (kernel fragments as the A operand); outputs 16j + 4(lane/16) + i (feature, j = 0, 1)
//    and 32 + the same (gate) of texel lane%16 sit in the same lane, so the gating needs no
//    exchange and every lane reads and writes four consecutive channels at once;
//  - the epilogue gates, adds the bypass, rounds to binary16 and writes the tile through LDS
//    in 16-byte rows (or applies the output layer and writes float32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "trips.h"

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int FEAT = TRIPS_DEC_FEATURES;  // 32
constexpr int NOUT = 2 * FEAT;            // feature + gate outputs of a convolution
constexpr int TILE = 16;                  // output tile is TILE x TILE texels
constexpr int HALO = TILE + 2;
constexpr int HPIX = HALO * HALO;         // 324 halo texels
constexpr int PSTRIDE = 40;               // halves per halo texel: 32 doubled + 8 layer channels
constexpr int CREG = TILE / 2 + 2;        // coarser texels under the halo, per row and column
constexpr int OSTRIDE = 40;               // halves per texel of the output staging (32 used)
constexpr int DEC_THREADS = 256;
constexpr int MAX_OUT = 8;
constexpr int MAXL = TRIPS_MAX_LAYERS;

int32_t g_dec_last_hip = 0;

// K steps of one layer's convolution: nine over the doubled features (absent for the
// coarsest layer), then ceil(9 D / 32) over (tap, layer channel).
__host__ __device__ constexpr int feat_steps(int D) { return (9 * D + 31) / 32; }
__host__ __device__ constexpr int conv_steps(int D, bool coarse) {
  return (coarse ? 9 : 0) + feat_steps(D);
}
// Packed layer: steps x 4 N-blocks x 64 lanes x 8 halves, then the bias (64 floats).
__host__ __device__ constexpr size_t packed_kernel_bytes(int D, bool coarse) {
  return size_t(conv_steps(D, coarse)) * 4 * 64 * 16;
}
__host__ __device__ constexpr size_t packed_layer_bytes(int D, bool coarse) {
  return packed_kernel_bytes(D, coarse) + NOUT * 4;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct DecLayout {
  int nl, D, out_dim, W[MAXL], H[MAXL];
  size_t layer_off[MAXL];  // packed weights
  size_t out_off;          // output layer: wo [32][out_dim], bo [out_dim] (float32)
  size_t packed_bytes;
  size_t h_off[MAXL];      // workspace: block outputs of layers 1..n-1, binary16 [H][W][32]
  size_t ws_bytes;
};

trips_status dec_layout(const trips_decoder_config* c, DecLayout& d) {
  if (!c) return TRIPS_ERR_INVALID_ARG;
  if (c->num_layers < 1 || c->num_layers > MAXL) return TRIPS_ERR_INVALID_ARG;
  if (c->desc_dim != 4 && c->desc_dim != 8) return TRIPS_ERR_UNSUPPORTED;
  if (c->out_dim < 1 || c->out_dim > MAX_OUT) return TRIPS_ERR_INVALID_ARG;
  if (c->width < 1 || c->height < 1 || c->width > (1 << 16) || c->height > (1 << 16))
    return TRIPS_ERR_INVALID_ARG;
  std::memset(&d, 0, sizeof(d));
  d.nl = c->num_layers;
  d.D = c->desc_dim;
  d.out_dim = c->out_dim;
  size_t o = 0, w = 0;
  for (int L = 0; L < d.nl; ++L) {
    d.W[L] = int((int64_t(c->width) + (int64_t(1) << L) - 1) >> L);
    d.H[L] = int((int64_t(c->height) + (int64_t(1) << L) - 1) >> L);
    d.layer_off[L] = o;
    o = align256(o + packed_layer_bytes(d.D, L + 1 < d.nl));
    d.h_off[L] = w;
    if (L > 0) w = align256(w + size_t(d.W[L]) * d.H[L] * FEAT * 2);
  }
  d.out_off = o;
  d.packed_bytes = align256(o + size_t(FEAT + 1) * d.out_dim * 4);
  d.ws_bytes = std::max<size_t>(w, 256);
  return TRIPS_OK;
}

// ---------------------------------------------------------------------------------------
// Weight packing: B fragment (step s, N-block j, lane l) holds K indices 32 s + 8 (l / 16)
// + e, e = 0..7, of output 16 j + l % 16.  Step s < 9 (with a coarser layer): tap s,
// doubled feature channel 8 (l / 16) + e (input channel D + that).  Other steps: K index
// k' = 32 (s - s0) + 8 (l / 16) + e over (tap k' / D, layer channel k' % D), zero past 9 D.
__global__ void k_dec_pack(const uint16_t* __restrict__ kern, const float* __restrict__ bias,
                           int D, int coarse, uint16_t* __restrict__ packed) {
  const int steps = conv_steps(D, coarse != 0);
  const int cin = coarse ? D + FEAT : D;
  const int n_frag = steps * 4 * 64;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < n_frag; f += gridDim.x * blockDim.x) {
    const int l = f & 63, j = (f >> 6) & 3, s = f >> 8;
    const int o = 16 * j + (l & 15);
    const int s0 = coarse ? 9 : 0;
    for (int e = 0; e < 8; ++e) {
      uint16_t v = 0;
      if (s < s0) {
        const int ci = D + 8 * (l >> 4) + e;
        v = kern[(size_t(s) * cin + ci) * NOUT + o];
      } else {
        const int k = 32 * (s - s0) + 8 * (l >> 4) + e;
        if (k < 9 * D) v = kern[(size_t(k / D) * cin + (k % D)) * NOUT + o];
      }
      packed[size_t(f) * 8 + e] = v;
    }
  }
  float* pb = reinterpret_cast<float*>(reinterpret_cast<char*>(packed) +
                                       packed_kernel_bytes(D, coarse != 0));
  if (blockIdx.x == 0 && threadIdx.x < NOUT) pb[threadIdx.x] = bias[threadIdx.x];
}

__global__ void k_dec_pack_out(const float* __restrict__ wo, const float* __restrict__ bo,
                               int out_dim, float* __restrict__ dst) {
  const int t = threadIdx.x;
  if (t < FEAT * out_dim) dst[t] = wo[t];
  if (t < out_dim) dst[FEAT * out_dim + t] = bo[t];
}

// ---------------------------------------------------------------------------------------
// The gating's exponentials use the hardware exp2 (a few float32 ulps): the results are
// rounded to binary16, whose spacing is 2^13 float32 ulps.
__device__ __forceinline__ float elu_f(float x) { return x > 0.0f ? x : __expf(x) - 1.0f; }
__device__ __forceinline__ float sigmoid_f(float x) {
  const float e = __expf(-fabsf(x));
  const float r = __builtin_amdgcn_rcpf(1.0f + e);  // (the hardware reciprocal, 1 ulp)
  return x >= 0.0f ? r : e * r;
}

// Doubling along one axis: finer index i sits at coarser position i/2 - 1/4: the nearer
// coarser texel (weight 3/4) is i/2, the farther (1/4) i/2 - 1 for even i, i/2 + 1 for odd i,
// both clamped to the layer.
__device__ __forceinline__ void up_taps(int i, int n, int& near, int& far) {
  const int k = i >> 1;
  near = min(k, n - 1);
  far = min(max((i & 1) ? k + 1 : k - 1, 0), n - 1);
}

// FO: 0 = write the block output; 3 = apply a 3-channel output layer; MAX_OUT = apply an
// output layer of out_dim <= MAX_OUT channels (zero padded)
template <int D, bool COARSE, int FO>
__global__ __launch_bounds__(DEC_THREADS, 2) void k_dec_block(
    const float* __restrict__ feat, const uint16_t* __restrict__ coarse,
    const uint16_t* __restrict__ packed, const float* __restrict__ outw, int W, int H, int Wc,
    int Hc, int out_dim, uint16_t* __restrict__ hout, float* __restrict__ image) {
  constexpr int STEPS = conv_steps(D, COARSE);
  constexpr int S0 = COARSE ? 9 : 0;
  // B fragments; of the last step only lanes 0..15 hold K indices below 9 D (both for D = 4
  // and D = 8), so only those are staged
  __shared__ __align__(16) half8 s_b[(STEPS - 1) * 4 * 64 + 4 * 16];
  __shared__ __align__(16) _Float16 s_in[HPIX * PSTRIDE];  // also the output staging
  __shared__ __align__(16) half8 s_c[COARSE ? CREG * CREG * 4 : 4];  // coarser texels under the halo
  __shared__ float s_bias[NOUT];
  constexpr bool FINAL = FO > 0;
  __shared__ float s_ow[FINAL ? (FEAT + 1) * FO : 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  {  // the packed kernel, once per workgroup
    const uint4* src = reinterpret_cast<const uint4*>(packed);
    uint4* dst = reinterpret_cast<uint4*>(s_b);
    for (int i = t; i < (STEPS - 1) * 256; i += DEC_THREADS) dst[i] = src[i];
    if (t < 64) dst[(STEPS - 1) * 256 + t] = src[(STEPS - 1) * 256 + (t >> 4) * 64 + (t & 15)];
    const float* pb = reinterpret_cast<const float*>(reinterpret_cast<const char*>(packed) +
                                                     packed_kernel_bytes(D, COARSE));
    if (t < NOUT) s_bias[t] = pb[t];
    if (FINAL) {  // output layer [c][k] padded to FO outputs (zeros), then its bias
      for (int u = t; u < (FEAT + 1) * FO; u += DEC_THREADS) {
        const int c = u / FO, k = u % FO;
        s_ow[u] = k < out_dim ? outw[c * out_dim + k] : 0.0f;
      }
    }
  }
  const int tx_n = (W + TILE - 1) / TILE, ty_n = (H + TILE - 1) / TILE;
  const int tiles = tx_n * ty_n;
  // ---- halo, phase 1: every global load of a tile issued at once, into registers (the next
  // tile's while this one is on the matrix cores).  The coarser block's texels under the
  // halo (rows and columns (y0 >> 1) - 1 .. + CREG - 1, clamped to the layer on load) go to
  // LDS as they are; the layer's features go to the halo as binary16.
  half8 cv[2];
  float4 fv[2][D / 4];
  auto fetch = [&](int tile) {
    const int y0 = (tile / tx_n) * TILE, x0 = (tile % tx_n) * TILE;
    const int cy0 = (y0 >> 1) - 1, cx0 = (x0 >> 1) - 1;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int u = t + r * DEC_THREADS;
      if (COARSE && u < CREG * CREG * 4) {
        const int p = u >> 2, g = u & 3;
        const int cy = min(max(cy0 + p / CREG, 0), Hc - 1);
        const int cx = min(max(cx0 + p % CREG, 0), Wc - 1);
        cv[r] = reinterpret_cast<const half8*>(coarse)[(size_t(cy) * Wc + cx) * 4 + g];
      }
      if (u < HPIX) {
        const int y = y0 + u / HALO - 1, x = x0 + u % HALO - 1;
        const bool in = y >= 0 && y < H && x >= 0 && x < W;
        const float4* fp =
            reinterpret_cast<const float4*>(feat + (size_t(in ? y : 0) * W + (in ? x : 0)) * D);
#pragma unroll
        for (int q = 0; q < D / 4; ++q) fv[r][q] = in ? fp[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  };
  if (int(blockIdx.x) < tiles) fetch(blockIdx.x);
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int y0 = (tile / tx_n) * TILE, x0 = (tile % tx_n) * TILE;
    const int cy0 = (y0 >> 1) - 1, cx0 = (x0 >> 1) - 1;
    __syncthreads();  // previous tile's staging is consumed (and the kernel is in LDS)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int u = t + r * DEC_THREADS;
      if (COARSE && u < CREG * CREG * 4) s_c[u] = cv[r];
      if (u < HPIX) {
        half8 h;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float4 v = q < D / 4 ? fv[r][q < D / 4 ? q : 0] : make_float4(0.f, 0.f, 0.f, 0.f);
          h[4 * q + 0] = _Float16(v.x); h[4 * q + 1] = _Float16(v.y);
          h[4 * q + 2] = _Float16(v.z); h[4 * q + 3] = _Float16(v.w);
        }
        reinterpret_cast<half8*>(s_in + u * PSTRIDE)[4] = h;
      }
    }
    __syncthreads();
    // ---- halo, phase 2 (below the coarsest layer only; the coarsest reads no doubled
    // features): the doubled features from LDS, two halo rows by four halo columns per unit.
    // Unit (ur, uc2) covers layer rows 2k and 2k + 1 (halo rows 2 ur - 1, 2 ur), k = y0/2 - 1
    // + ur = cy0 + ur, and the layer columns of the coarser columns 2 uc2 and 2 uc2 + 1 (halo
    // columns 4 uc2 - 1 .. 4 uc2 + 2): it reads the 3x4 staged coarser texels around them once,
    // blends each of the four coarser columns along the rows once, and forms its eight texels
    // exactly as the per-texel formula (rows first at the near and the far column, each 3/4
    // near + 1/4 far, then columns).  Staged slots outside the region (clamped) only feed halo
    // texels outside the halo, which are skipped.
    if (COARSE) {
      constexpr int CP = CREG / 2;  // column pairs
      for (int u = t; u < CREG * CP * 4; u += DEC_THREADS) {
        const int g = u & 3, q = u >> 2, ur = q / CP, uc2 = q % CP;
        half8 cr[3][4];
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int ry = min(max(ur - 1 + a2, 0), CREG - 1);
            const int rx = min(max(2 * uc2 - 1 + j, 0), CREG - 1);
            cr[a2][j] = s_c[(ry * CREG + rx) * 4 + g];
          }
        // 3/4 near + 1/4 far is (3 near + far) / 4, and a power-of-two scale is exact: each
        // pass forms 3 near + far with one rounding (from the binary16 values directly along
        // the rows), and the doubled value is the column pass's result times 1/16, the same
        // float32 as 3/4 near + 1/4 far taken twice, then rounded to binary16
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          // even layer row (dy = 0): far row above; odd (dy = 1): far row below
          float v[4][8];
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 8; ++e)
              v[j][e] = fmaf(3.0f, float(cr[1][j][e]), float(cr[dy ? 2 : 0][j][e]));
#pragma unroll
          for (int w = 0; w < 2; ++w) {  // coarser column 2 uc2 + w: near j = 1 + w
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {  // far column j = w (dx = 0) or 2 + w (dx = 1)
              const int hy = 2 * ur - 1 + dy, hx = 2 * (2 * uc2 + w) - 1 + dx;
              if (hy < 0 || hy >= HALO || hx < 0 || hx >= HALO) continue;
              const int y = y0 - 1 + hy, x = x0 - 1 + hx;
              const bool inimg = y >= 0 && y < H && x >= 0 && x < W;
              half8 hv;
#pragma unroll
              for (int e = 0; e < 8; ++e)
                hv[e] = _Float16(0.0625f * fmaf(3.0f, v[1 + w][e], v[dx ? 2 + w : w][e]));
              uint4 hw = *reinterpret_cast<const uint4*>(&hv);
              hw.x = inimg ? hw.x : 0u; hw.y = inimg ? hw.y : 0u;
              hw.z = inimg ? hw.z : 0u; hw.w = inimg ? hw.w : 0u;
              reinterpret_cast<uint4*>(s_in + (hy * HALO + hx) * PSTRIDE)[g] = hw;
            }
          }
        }
      }
    }
    __syncthreads();
    if (tile + int(gridDim.x) < tiles) fetch(tile + gridDim.x);  // in flight during the MFMAs
    // ---- implicit GEMM: wave owns tile rows 4 wave .. 4 wave + 3
    // The kernel fragments go in as the A operand and the texels as B, so the accumulator is
    // the transposed tile: lane (grp, col) holds outputs 16 j + 4 grp + i of texel col.
    const int col = lane & 15, grp = lane >> 4;
    floatx4 acc[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      floatx4 bj;
#pragma unroll
      for (int i = 0; i < 4; ++i) bj[i] = s_bias[16 * j + 4 * grp + i];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r][j] = bj;
    }
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      half8 b[4];
      if (s < STEPS - 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = s_b[(s * 4 + j) * 64 + lane];
      } else {  // (its A fragments are zero past lane 15 too)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          b[j] = s_b[(STEPS - 1) * 256 + j * 16 + (lane & 15)];
          if (lane >= 16) {
#pragma unroll
            for (int e = 0; e < 8; ++e) b[j][e] = _Float16(0.0f);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * wave + r;
        half8 a;
        if (s < S0) {  // tap s, doubled channels 8 grp .. 8 grp + 7
          const int dy = s / 3, dx = s % 3;
          a = *reinterpret_cast<const half8*>(s_in + ((row + dy) * HALO + col + dx) * PSTRIDE +
                                              8 * grp);
        } else if (D == 8) {  // tap 4 (s - S0) + grp, all eight layer channels
          const int tap = 4 * (s - S0) + grp;
          if (tap < 9) {
            a = *reinterpret_cast<const half8*>(
                s_in + ((row + tap / 3) * HALO + col + tap % 3) * PSTRIDE + FEAT);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = _Float16(0.0f);
          }
        } else {  // D == 4: taps 8 (s - S0) + 2 grp and the next, four channels each
          const int tap0 = 8 * (s - S0) + 2 * grp;
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) {
            const int tap = tap0 + h2;
            half4 v;
            if (tap < 9) {
              v = *reinterpret_cast<const half4*>(
                  s_in + ((row + tap / 3) * HALO + col + tap % 3) * PSTRIDE + FEAT);
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e) v[e] = _Float16(0.0f);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) a[4 * h2 + e] = v[e];
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(b[j], a, acc[r][j], 0, 0, 0);
      }
    }
    // ---- epilogue: lane holds outputs 16 j + 4 grp + i (features j = 0, 1; gates j + 2) of
    // texel (row, col): four consecutive channels, read and written as 8-byte pieces
    half4 hv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * wave + r;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        half4 up;
        if (COARSE)
          up = *reinterpret_cast<const half4*>(s_in + ((row + 1) * HALO + col + 1) * PSTRIDE +
                                               16 * j + 4 * grp);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = elu_f(acc[r][j][i]) * sigmoid_f(acc[r][j + 2][i]);
          if (COARSE) v += float(up[i]);
          hv[r][j][i] = _Float16(v);
        }
      }
    }
    __syncthreads();  // every wave is done with the halo; it becomes the output staging
    _Float16* s_out = s_in;  // [256 texels][OSTRIDE]: texels 80 bytes apart hit other banks
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        *reinterpret_cast<half4*>(s_out + ((4 * wave + r) * TILE + col) * OSTRIDE + 16 * j +
                                  4 * grp) = hv[r][j];
    __syncthreads();
    if (!FINAL) {  // 16-byte pieces: four per texel, tile rows contiguous in memory
      for (int u = t; u < TILE * TILE * 4; u += DEC_THREADS) {
        const int p = u >> 2, g = u & 3;
        const int y = y0 + p / TILE, x = x0 + p % TILE;
        if (y < H && x < W)
          reinterpret_cast<uint4*>(hout)[(size_t(y) * W + x) * 4 + g] =
              *reinterpret_cast<const uint4*>(s_out + p * OSTRIDE + 8 * g);
      }
    } else {  // the output layer, one texel per thread (weights from LDS, FO-padded)
      const int y = y0 + t / TILE, x = x0 + t % TILE;
      if (y < H && x < W) {
        float o[FINAL ? FO : 1];
#pragma unroll
        for (int k = 0; k < FO; ++k) o[k] = s_ow[FEAT * FO + k];
        const half8* hp = reinterpret_cast<const half8*>(s_out + t * OSTRIDE);
        constexpr int CU = FO == 3 ? FEAT / 8 : 1;  // (the generic width stays rolled)
#pragma unroll CU
        for (int c8 = 0; c8 < FEAT / 8; ++c8) {
          const half8 hv8 = hp[c8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float h = float(hv8[e]);
#pragma unroll
            for (int k = 0; k < FO; ++k) o[k] = fmaf(h, s_ow[(8 * c8 + e) * FO + k], o[k]);
          }
        }
        float* dst = image + (size_t(y) * W + x) * out_dim;
#pragma unroll
        for (int k = 0; k < FO; ++k)
          if (k < out_dim) dst[k] = o[k];
      }
    }
  }
}

#define DEC_HIP(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) { g_dec_last_hip = int32_t(e_); return TRIPS_ERR_HIP; } \
  } while (0)

bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Workgroups of one block launch: one per tile up to two per CU (the residency the kernel's
// LDS allows), each looping over tiles with the layer's packed kernel staged once.
uint32_t dec_grid(int W, int H) {
  const uint32_t tiles = uint32_t((W + TILE - 1) / TILE) * uint32_t((H + TILE - 1) / TILE);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return std::min<uint32_t>(tiles, 2u * uint32_t(std::max(cus, 1)));
}

template <int D>
trips_status launch_block(const DecLayout& d, const char* packed, int L, const float* feat,
                          const uint16_t* coarse, uint16_t* hout, float* image,
                          hipStream_t st) {
  const bool has_coarse = L + 1 < d.nl;
  const uint16_t* pk = reinterpret_cast<const uint16_t*>(packed + d.layer_off[L]);
  const float* ow = reinterpret_cast<const float*>(packed + d.out_off);
  const int W = d.W[L], H = d.H[L];
  const int Wc = has_coarse ? d.W[L + 1] : 1, Hc = has_coarse ? d.H[L + 1] : 1;
  const dim3 grid(dec_grid(W, H)), blk(DEC_THREADS);
  const int fo = image ? (d.out_dim == 3 ? 3 : MAX_OUT) : 0;
#define DEC_LAUNCH(C, F)                                                                   \
  hipLaunchKernelGGL((k_dec_block<D, C, F>), grid, blk, 0, st, feat, coarse, pk, ow, W, H, \
                     Wc, Hc, d.out_dim, hout, image)
  if (has_coarse) {
    if (fo == 3) DEC_LAUNCH(true, 3);
    else if (fo) DEC_LAUNCH(true, MAX_OUT);
    else DEC_LAUNCH(true, 0);
  } else {
    if (fo == 3) DEC_LAUNCH(false, 3);
    else if (fo) DEC_LAUNCH(false, MAX_OUT);
    else DEC_LAUNCH(false, 0);
  }
#undef DEC_LAUNCH
  DEC_HIP(hipGetLastError());
  return TRIPS_OK;
}

}  // namespace

extern "C" {

trips_status trips_decoder_sizes(const trips_decoder_config* cfg, size_t* packed_bytes,
                                 size_t* workspace_bytes) {
  DecLayout d;
  trips_status s = dec_layout(cfg, d);
  if (s != TRIPS_OK) return s;
  if (packed_bytes) *packed_bytes = d.packed_bytes;
  if (workspace_bytes) *workspace_bytes = d.ws_bytes;
  return TRIPS_OK;
}

trips_status trips_decoder_pack(const trips_decoder_config* cfg, const trips_decoder_weights* w,
                                void* packed, size_t packed_bytes, hipStream_t st) {
  DecLayout d;
  trips_status s = dec_layout(cfg, d);
  if (s != TRIPS_OK) return s;
  if (!w || !packed || (reinterpret_cast<uintptr_t>(packed) & 255u)) return TRIPS_ERR_INVALID_ARG;
  if (packed_bytes < d.packed_bytes) return TRIPS_ERR_WORKSPACE;
  for (int L = 0; L < d.nl; ++L)
    if (!w->kernel[L] || !w->bias[L]) return TRIPS_ERR_INVALID_ARG;
  if (!w->out_weight || !w->out_bias) return TRIPS_ERR_INVALID_ARG;
  char* p = static_cast<char*>(packed);
  for (int L = 0; L < d.nl; ++L) {
    const int coarse = L + 1 < d.nl ? 1 : 0;
    hipLaunchKernelGGL(k_dec_pack, dim3(conv_steps(d.D, coarse != 0)), dim3(256), 0, st,
                       w->kernel[L], w->bias[L], d.D, coarse,
                       reinterpret_cast<uint16_t*>(p + d.layer_off[L]));
    DEC_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_dec_pack_out, dim3(1), dim3(FEAT * MAX_OUT), 0, st, w->out_weight,
                     w->out_bias, d.out_dim, reinterpret_cast<float*>(p + d.out_off));
  DEC_HIP(hipGetLastError());
  return TRIPS_OK;
}

trips_status trips_decoder_block(const trips_decoder_config* cfg, const void* packed,
                                 size_t packed_bytes, int32_t layer, const float* features,
                                 const uint16_t* coarse, uint16_t* out, float* image,
                                 hipStream_t st) {
  DecLayout d;
  trips_status s = dec_layout(cfg, d);
  if (s != TRIPS_OK) return s;
  if (!packed || (reinterpret_cast<uintptr_t>(packed) & 255u)) return TRIPS_ERR_INVALID_ARG;
  if (packed_bytes < d.packed_bytes) return TRIPS_ERR_WORKSPACE;
  if (layer < 0 || layer >= d.nl) return TRIPS_ERR_INVALID_ARG;
  if (!features || !al16(features)) return TRIPS_ERR_INVALID_ARG;
  if (layer + 1 < d.nl && (!coarse || !al16(coarse))) return TRIPS_ERR_INVALID_ARG;
  if (!out && !image) return TRIPS_ERR_INVALID_ARG;
  if (out && image) return TRIPS_ERR_INVALID_ARG;
  if (out && !al16(out)) return TRIPS_ERR_INVALID_ARG;
  const char* p = static_cast<const char*>(packed);
  return d.D == 4 ? launch_block<4>(d, p, layer, features, coarse, out, image, st)
                  : launch_block<8>(d, p, layer, features, coarse, out, image, st);
}

trips_status trips_decoder_forward(const trips_decoder_config* cfg, const void* packed,
                                   size_t packed_bytes, const float* pyramid, float* image,
                                   void* workspace, size_t workspace_bytes, hipStream_t st) {
  DecLayout d;
  trips_status s = dec_layout(cfg, d);
  if (s != TRIPS_OK) return s;
  if (!packed || (reinterpret_cast<uintptr_t>(packed) & 255u)) return TRIPS_ERR_INVALID_ARG;
  if (packed_bytes < d.packed_bytes) return TRIPS_ERR_WORKSPACE;
  if (!pyramid || !al16(pyramid) || !image) return TRIPS_ERR_INVALID_ARG;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u)) return TRIPS_ERR_INVALID_ARG;
  if (workspace_bytes < d.ws_bytes) return TRIPS_ERR_WORKSPACE;
  const char* p = static_cast<const char*>(packed);
  char* ws = static_cast<char*>(workspace);
  size_t off = 0;
  size_t layer_feat[MAXL];
  for (int L = 0; L < d.nl; ++L) {
    layer_feat[L] = off;
    off += size_t(d.W[L]) * d.H[L] * d.D;
  }
  for (int L = d.nl - 1; L >= 0; --L) {
    const uint16_t* coarse =
        L + 1 < d.nl ? reinterpret_cast<const uint16_t*>(ws + d.h_off[L + 1]) : nullptr;
    uint16_t* hout = L > 0 ? reinterpret_cast<uint16_t*>(ws + d.h_off[L]) : nullptr;
    const float* feat = pyramid + layer_feat[L];
    s = d.D == 4 ? launch_block<4>(d, p, L, feat, coarse, hout, L == 0 ? image : nullptr, st)
                 : launch_block<8>(d, p, L, feat, coarse, hout, L == 0 ? image : nullptr, st);
    if (s != TRIPS_OK) return s;
  }
  return TRIPS_OK;
}

int32_t trips_decoder_last_hip_error(void) { return g_dec_last_hip; }

}  // extern "C"
