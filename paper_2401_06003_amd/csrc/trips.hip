// trips.hip -- HIP kernels and C ABI of the trilinear point-splatting renderer for gfx950.
//
// Method (TRIPS, Sec. 3.1-3.2, Eq. 1-7): every point is projected with a pinhole camera,
// written with one trilinear write (a bilinear 2x2 footprint in each of the two pyramid
// layers floor/ceil(log2 s)) and every (layer, texel) blends its 16 front-most fragments
// front to back.  The backward pass is the analytic adjoint.
//
// Design for MI355X (no global atomics on the data path; random device atomics run at
// ~27 G/s on this part, 1.3 G/s when contended, far below scattered stores):
//   count      one workgroup per (point block, view): LDS histogram of tile entries
//              (entry = one point's footprint part inside one 256-texel tile of one layer)
//              -> one row of a per-block histogram matrix H16[block][bin] (16-bit counts).
//   colscan    per bin, exclusive prefix of H16 over blocks (32-bit, into H) and bin totals.
//   binscan    exclusive scans of bin totals -> bin starts, and of work items -> item starts.
//   scatter    same blocks again: LDS ranks, entry written at bin_start + H + rank.
//   fwd_items  persistent: one workgroup per work item (a bin, or a chunk of a heavy bin);
//              entries -> fragments in LDS, counting sort by texel, per-texel top-16 kept
//              in registers (thread = texel); blend, or write a partial top-16.
//   fwd_merge  heavy bins: merge the partial top-16 lists, blend.
//   bwd_pixels per texel: recompute T_m, reverse recurrence -> (dgamma_m, T_m gamma_m).
//   bwd_items  per work item: every entry looks its corners up in the tile's kept lists
//              (LDS) and writes one partial-gradient row per (view, slot, point).
//   bwd_points per point: sum its rows, chain rule through the projection, write grads.
// Every result is deterministic: ordering keys are unique (depth bits, point index) and
// every sum is taken in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "trips.h"

namespace {

constexpr int KEEP = TRIPS_KEEP;
constexpr int TP = 256;    // texels per tile == threads of a tile workgroup
constexpr int NSLOT = 8;   // (layer entry 0/1) x (tile touch 0..3)
constexpr int MAXV = TRIPS_MAX_VIEWS;
constexpr int MAXL = TRIPS_MAX_LAYERS;
constexpr uint64_t KEY_NONE = ~0ull;
// A tile with at most FINE_E entries ("fine" tile, typical of the finest layers) is rendered
// by one workgroup with one entry per thread: its lists are sorted in LDS, and the kept slot
// of every corner is stored in the entry for the backward pass.  With coarser-layer
// inclusion only empty tiles take that path (the backward of every other tile then reads
// per-slot adjoints that the inclusion pass accumulates).
constexpr uint32_t FINE_E = 256;
// The backward needs no merge, so its workgroups take smaller parts of the work items.
constexpr uint32_t BWD_SPLIT = 2;
// Workgroups are dealt to the chip's 8 dies (XCDs, each with its own L2) in turn by index;
// kernels that share data between workgroups place them 8 indices apart.  The work-item
// capacity is a multiple of it.
constexpr uint32_t XCDS = 8;
constexpr uint32_t PT_GROUP = 16;  // point chunks of the point pass kept on one die
// Tile (tx, ty) of a layer with tiles_x x tiles_y tiles for workgroup b of a per-tile pass
// whose tiles read the lists of the next coarser layer: the 2x2 tiles under one coarser tile
// share them, so they go to one die.  Quads are numbered row-major; quad q's four tiles are
// workgroups (q / XCDS) 4 XCDS + XCDS m + q % XCDS, m = 2 (row in quad) + column.  False
// for a workgroup past the layer's tiles.
__device__ __forceinline__ bool quad_tile(uint32_t b, int tiles_x, int tiles_y, int& tx, int& ty) {
  constexpr uint32_t span = 4 * XCDS;
  const uint32_t q = b / span * XCDS + b % XCDS, m = b % span / XCDS;
  const uint32_t qx_n = uint32_t(tiles_x + 1) / 2;
  const uint32_t qy = q / qx_n, qx = q % qx_n;
  tx = int(2 * qx + (m & 1u));
  ty = int(2 * qy + (m >> 1));
  return tx < tiles_x && ty < tiles_y;
}
// Work items are ordered by size class, largest first: class q holds items of more than
// (NBUCKET - 1 - q) / NBUCKET of item_e entries.  info[INFO_BUCKET + q] is the first work
// slot of class q, info[INFO_BUCKET + NBUCKET + q] its fill counter.
constexpr int NBUCKET = 8;
constexpr int INFO_BUCKET = 8;
__device__ __forceinline__ uint32_t size_class(uint32_t entries, uint32_t item_e) {
  const uint32_t short_by = item_e - min(entries, item_e);  // 0 for a full item
  return min(uint32_t(NBUCKET - 1), uint32_t((uint64_t(short_by) * NBUCKET) / item_e));
}

struct ViewP {
  float R[9], t[3];
  float fx, fy, cx, cy, znear;
  int32_t W, H;
  uint32_t bin_base, nbins;
  uint32_t lbin[MAXL + 1];  // absolute first bin of each layer; [nl] = end of the view
  uint32_t lout[MAXL];      // first texel of each layer in the pyramid of all views
};

struct Params {
  int32_t V, nl, D, ltw;  // ltw = log2(tile width); tile height = 256 >> ltw
  float eps;
  uint32_t pb, nblk, NB, item_e;
  int32_t coarser;        // coarser-layer inclusion on
  uint32_t fine_e;        // tiles with at most fine_e entries take the fine path
  int64_t n;
  ViewP view[MAXV];
};

struct __align__(4) Entry {
  uint32_t idx;    // point index
  uint32_t zbits;  // bits of the camera depth (positive float: order preserving)
  float u, v;      // layer-texel coordinates of the point, x / 2^L - 0.5
  float ia;        // iota * alpha
};
static_assert(sizeof(Entry) == 20, "entry layout");

// ------------------------------------------------------------------------------------
// Geometry shared by every kernel that needs a point's footprint.  Compiled without
// floating-point contraction: these operations decide integers (culling, layers,
// texels, which corners exist) and must match any other correct single-precision
// evaluation of the same sequence.

__host__ __device__ __forceinline__ int layer_dim(int W, int L) { return (W + (1 << L) - 1) >> L; }
__device__ __forceinline__ float pow2i(int e) { return __int_as_float((127 + e) << 23); }

struct Geo {
  float x, y, zc, s, qx, qy;  // screen x, y, depth, screen size, X_c/Z_c, Y_c/Z_c
  int nl, L0;                 // number of layers (1 or 2) and the finer one
  float io[2], dio[2];        // iota and d iota / d s per layer entry
};

__device__ bool project(const ViewP& c, float X, float Y, float Z, float sw, int nlayers,
                        float eps, Geo& g) {
  // Sec. 3.1, Eq. 2: pinhole projection and screen size s = f s_w / z
  float Xc = __builtin_fmaf(c.R[0], X, __builtin_fmaf(c.R[1], Y, __builtin_fmaf(c.R[2], Z, c.t[0])));
  float Yc = __builtin_fmaf(c.R[3], X, __builtin_fmaf(c.R[4], Y, __builtin_fmaf(c.R[5], Z, c.t[1])));
  float Zc = __builtin_fmaf(c.R[6], X, __builtin_fmaf(c.R[7], Y, __builtin_fmaf(c.R[8], Z, c.t[2])));
  if (!(Zc > c.znear)) return false;
  float qx = Xc / Zc, qy = Yc / Zc;
  float x = __builtin_fmaf(c.fx, qx, c.cx);
  float y = __builtin_fmaf(c.fy, qy, c.cy);
  float s = (c.fx * sw) / Zc;
  if (!isfinite(x) || !isfinite(y) || !isfinite(s) || !(s > 0.0f)) return false;
  g.x = x; g.y = y; g.zc = Zc; g.s = s; g.qx = qx; g.qy = qy;
  // Sec. 3.1, Eq. 5: layers floor(log2 s) and ceil(log2 s) with linear layer weights
  if (s < 1.0f) {
    g.nl = 1; g.L0 = 0;
    g.io[0] = __builtin_fmaf(1.0f - eps, s, eps);
    g.dio[0] = 1.0f - eps;
  } else if (s >= pow2i(nlayers - 1)) {
    g.nl = 1; g.L0 = nlayers - 1; g.io[0] = 1.0f; g.dio[0] = 0.0f;
  } else {
    uint32_t b = __float_as_uint(s);
    int e = int(b >> 23) - 127;                               // exact floor(log2 s), s normal
    float t = __uint_as_float((b & 0x7fffffu) | (127u << 23));  // s / 2^e in [1, 2), exact
    if (t == 1.0f) {
      g.nl = 1; g.L0 = e; g.io[0] = 1.0f; g.dio[0] = 0.0f;
    } else {
      g.nl = 2; g.L0 = e;
      g.io[0] = 2.0f - t; g.io[1] = t - 1.0f;  // exact (Sterbenz)
      float inv = pow2i(-e);
      g.dio[0] = -inv; g.dio[1] = inv;
    }
  }
  return true;
}

struct Foot {
  int i0, j0;       // texel of the lower-left corner
  float fu, fv;     // fractional offsets inside the 2x2 footprint
  float u, v;
  uint32_t cmask;   // bit (2*dj + di) set if corner (i0+di, j0+dj) is written
};

// Sec. 3.1, Eq. 4: bilinear 2x2 footprint of a point in layer L (texel centres at
// integer u, v in layer-texel units).  A corner is written iff it lies inside the layer
// and both of its 1-D weights are non-zero.
__device__ bool footprint(float x, float y, int L, int WL, int HL, Foot& f) {
  float sc = pow2i(-L);
  float u = x * sc - 0.5f;
  float v = y * sc - 0.5f;
  if (!(u > -1.0f && u < float(WL) && v > -1.0f && v < float(HL))) return false;
  float flu = floorf(u), flv = floorf(v);
  int i0 = int(flu), j0 = int(flv);
  float fu = u - flu, fv = v - flv;
  uint32_t m = 0;
#pragma unroll
  for (int dj = 0; dj < 2; ++dj)
#pragma unroll
    for (int di = 0; di < 2; ++di) {
      int i = i0 + di, j = j0 + dj;
      float wx = di ? fu : 1.0f - fu;
      float wy = dj ? fv : 1.0f - fv;
      bool in = (i >= 0) & (i < WL) & (j >= 0) & (j < HL) & (wx != 0.0f) & (wy != 0.0f);
      m |= uint32_t(in) << (2 * dj + di);
    }
  f.i0 = i0; f.j0 = j0; f.fu = fu; f.fv = fv; f.u = u; f.v = v; f.cmask = m;
  return m != 0;
}

// Corners of a footprint grouped by the 256-texel tile they fall in.  touch = dx + 2 dy
// relative to the tile of corner (i0, j0) (floor division, so i0 = -1 is tile -1).
__device__ __forceinline__ void touches(const Foot& f, int ltw, uint32_t (&tm)[4]) {
  int lth = 8 - ltw;
  int txb = f.i0 >> ltw, tyb = f.j0 >> lth;
  int tc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int di = c & 1, dj = c >> 1;
    tc[c] = (((f.i0 + di) >> ltw) - txb) + 2 * (((f.j0 + dj) >> lth) - tyb);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    uint32_t m = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) m |= uint32_t(((f.cmask >> c) & 1u) && tc[c] == t) << c;
    tm[t] = m;
  }
}

// Decode a bin index into view, layer and tile coordinates (wave-uniform).
struct BinInfo { int v, L, tx, ty, WL, HL; };
__device__ BinInfo decode_bin(const Params& P, uint32_t b) {
  BinInfo r;
  int v = 0;
  while (v + 1 < P.V && b >= P.view[v + 1].bin_base) ++v;
  const ViewP& c = P.view[v];
  int L = 0;
  while (L + 1 < P.nl && b >= c.lbin[L + 1]) ++L;
  r.v = v; r.L = L;
  r.WL = layer_dim(c.W, L); r.HL = layer_dim(c.H, L);
  int tiles_x = (r.WL + (1 << P.ltw) - 1) >> P.ltw;
  int local = int(b - c.lbin[L]);
  r.ty = local / tiles_x;
  r.tx = local - r.ty * tiles_x;
  return r;
}

// ------------------------------------------------------------------------------------
// Wave and workgroup scans (wavefront of 64 lanes).

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan over a workgroup of NW waves; `ws` holds NW words of LDS.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* ws, uint32_t& total) {
  uint32_t inc = wave_incl_scan(x);
  int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    uint32_t s = ws[k];
    off += (k < w) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + inc - x;
}

// The same for four independent counters at once; `ws` holds NW uint4 of LDS.
template <int NW>
__device__ __forceinline__ uint4 block_excl_scan4(uint4 x, uint4* ws, uint4& total) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint4 inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t a = __shfl_up(inc.x, d, 64), b = __shfl_up(inc.y, d, 64);
    const uint32_t c = __shfl_up(inc.z, d, 64), e = __shfl_up(inc.w, d, 64);
    if (lane >= d) { inc.x += a; inc.y += b; inc.z += c; inc.w += e; }
  }
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint4 off = make_uint4(0u, 0u, 0u, 0u), tot = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint4 s = ws[k];
    if (k < w) { off.x += s.x; off.y += s.y; off.z += s.z; off.w += s.w; }
    tot.x += s.x; tot.y += s.y; tot.z += s.z; tot.w += s.w;
  }
  __syncthreads();
  total = tot;
  return make_uint4(off.x + inc.x - x.x, off.y + inc.y - x.y, off.z + inc.z - x.z,
                    off.w + inc.w - x.w);
}

// ------------------------------------------------------------------------------------
// Per-texel top-16 in registers: keys ascending; insertion is a fixed compare network.

__device__ __forceinline__ void top_insert(uint64_t (&k)[KEEP], float (&g)[KEEP], uint64_t nk,
                                           float ng) {
  if (!(nk < k[KEEP - 1])) return;
  // b[i] = nk < k[i] is false below the insertion point and true from it on: slot i takes
  // k[i-1] if b[i-1], nk if only b[i], and keeps k[i] otherwise
  bool b[KEEP];
#pragma unroll
  for (int i = 0; i < KEEP; ++i) b[i] = nk < k[i];
#pragma unroll
  for (int i = KEEP - 1; i > 0; --i) {
    const uint64_t ki = b[i - 1] ? k[i - 1] : nk;
    const float gi = b[i - 1] ? g[i - 1] : ng;
    k[i] = b[i] ? ki : k[i];
    g[i] = b[i] ? gi : g[i];
  }
  k[0] = b[0] ? nk : k[0];
  g[0] = b[0] ? ng : g[0];
}

// ------------------------------------------------------------------------------------
// LDS counters packed two per word (16 bits each): add one to counter c, return its old value.
__device__ __forceinline__ uint32_t add16(uint32_t* words, uint32_t c) {
  const uint32_t sh = (c & 1u) * 16u;
  return (atomicAdd(&words[c >> 1], 1u << sh) >> sh) & 0xffffu;
}

// ------------------------------------------------------------------------------------
// Kernels.

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t value) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// Emits every tile entry of one point for view c; calls f(bin, slot, sel, foot, geo).
// SELECT: take the layer's first tile from a select over the view's (wave-uniform, scalar)
// table instead of indexing it with the per-lane layer, which is a vector memory load; a
// caller that stores between entries needs that (the load would wait for its stores).
template <bool SELECT, class F>
__device__ __forceinline__ void for_each_entry(const Params& P, const ViewP& c, float X, float Y,
                                               float Z, float sw, F&& f) {
  Geo g;
  if (!project(c, X, Y, Z, sw, P.nl, P.eps, g)) return;
#pragma unroll
  for (int sel = 0; sel < 2; ++sel) {
    if (sel >= g.nl) break;
    int L = g.L0 + sel;
    int WL = layer_dim(c.W, L), HL = layer_dim(c.H, L);
    Foot ft;
    if (!footprint(g.x, g.y, L, WL, HL, ft)) continue;
    uint32_t tm[4];
    touches(ft, P.ltw, tm);
    int tiles_x = (WL + (1 << P.ltw) - 1) >> P.ltw;
    int txb = ft.i0 >> P.ltw, tyb = ft.j0 >> (8 - P.ltw);
    uint32_t lbase;
    if (SELECT) {
      lbase = c.lbin[0];
#pragma unroll
      for (int k = 1; k < MAXL; ++k) lbase = L == k ? c.lbin[k] : lbase;
    } else {
      lbase = c.lbin[L];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (!tm[t]) continue;
      int tx = txb + (t & 1), ty = tyb + (t >> 1);
      uint32_t bin = lbase + uint32_t(ty * tiles_x + tx);
      f(bin, uint32_t(sel * 4 + t), sel, ft, g);
    }
  }
}

constexpr int BIN_THREADS = 1024;  // threads of a count / scatter workgroup

// count: LDS histogram (two 16-bit counters per word) of the entries of one point block
// in one view; writes row `blk` of H for the bins of that view.
__global__ __launch_bounds__(BIN_THREADS) void k_count(const Params P, const float* __restrict__ X,
                                                       const float* __restrict__ Y,
                                                       const float* __restrict__ Z,
                                                       const float* __restrict__ SW,
                                                       uint16_t* __restrict__ H16) {
  extern __shared__ uint32_t hist[];
  const int v = blockIdx.x % P.V;
  const uint32_t blk = blockIdx.x / P.V;
  const ViewP& c = P.view[v];
  const uint32_t nw = (c.nbins + 1) >> 1;
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t p0 = int64_t(blk) * P.pb;
  const int64_t p1 = min(P.n, p0 + int64_t(P.pb));
  // the next point of this thread is loaded while the current one is binned (the index is
  // clamped to the block's last point, a valid address)
  int64_t p = p0 + threadIdx.x;
  int64_t pc = min(p, p1 - 1);
  float x = 0.f, y = 0.f, z = 0.f, sw = 0.f;
  if (p < p1) { x = X[pc]; y = Y[pc]; z = Z[pc]; sw = SW[pc]; }
  for (; p < p1; p += blockDim.x) {
    pc = min(p + int64_t(blockDim.x), p1 - 1);
    const float xn = X[pc], yn = Y[pc], zn = Z[pc], swn = SW[pc];
    for_each_entry<false>(P, c, x, y, z, sw,
                   [&](uint32_t bin, uint32_t, int, const Foot&, const Geo&) {
                     add16(hist, bin - c.bin_base);
                   });
    x = xn; y = yn; z = zn; sw = swn;
  }
  __syncthreads();
  // 16-bit counts: a block holds at most P.pb < 2^16 points, each with at most one entry
  // per tile
  uint16_t* row = H16 + size_t(blk) * P.NB + c.bin_base;
  for (uint32_t i = threadIdx.x; i < c.nbins; i += blockDim.x)
    row[i] = uint16_t((hist[i >> 1] >> ((i & 1u) * 16u)) & 0xffffu);
}

// The tile scan over chunks of 64 tiles (one wavefront each): the chunk sums (written by the
// column scan, whose workgroups cover the same chunks), then two short passes.  A tile
// of at most FINE_E entries is listed in fine_work; every other tile is listed in coarse_bins
// and cut into ceil(total / item_e) work items; tiles with more than one item are listed in
// multi_bins (their partial lists are merged), with the first of their items' consecutive
// partial-list slots NB words further on.  bin_start and item_start are the exclusive scans
// of entries and items.
constexpr uint32_t CHUNK = 64;
constexpr int CSUM = 4 + NBUCKET;  // per chunk: entries, items, multi tiles, fine tiles, classes

// ceil(a / b) for b > 0: the correctly rounded double quotient of integers below 2^33 is
// never rounded across an integer (a quotient just below k is at least 1/b below it), so its
// ceiling is exact.
__device__ __forceinline__ uint32_t ceil_div(uint32_t a, uint32_t b) {
  return uint32_t(ceil(double(a) / double(b)));
}

struct TileCount { uint32_t e, it, multi, fine; };
__device__ __forceinline__ TileCount tile_count_of(uint32_t e, bool valid, uint32_t item_e,
                                                   uint32_t fine_e) {
  TileCount r{0u, 0u, 0u, 0u};
  if (valid) {
    r.e = e;
    r.fine = r.e <= fine_e ? 1u : 0u;
    r.it = r.fine ? 0u : ceil_div(r.e, item_e);
    r.multi = r.it > 1 ? 1u : 0u;
  }
  return r;
}
__device__ __forceinline__ TileCount tile_count(const uint32_t* __restrict__ tot, uint32_t b,
                                                uint32_t NB, uint32_t item_e, uint32_t fine_e) {
  return tile_count_of(b < NB ? tot[b] : 0u, b < NB, item_e, fine_e);
}
// Size class of every item of a tile: the forward takes the items of a tile as strided
// blocks of its entries, so they are of equal size (within a block), e / it on average.
__device__ __forceinline__ uint32_t item_class(const TileCount& c, uint32_t item_e) {
  return c.it ? size_class(ceil_div(c.e, c.it), item_e) : 0u;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// The sums of one chunk (a wavefront, a tile per lane): entries, items, multi-item tiles,
// fine tiles and the items per size class; lane 0 writes them.
__device__ __forceinline__ void chunk_sums(const TileCount& c, uint32_t item_e,
                                           uint32_t* __restrict__ out) {
  const uint32_t cls = item_class(c, item_e);  // (all items of a tile)
  uint32_t v[CSUM];
  v[0] = c.e; v[1] = c.it; v[2] = c.multi; v[3] = c.fine;
#pragma unroll
  for (int q = 0; q < NBUCKET; ++q) v[4 + q] = cls == uint32_t(q) ? c.it : 0u;
#pragma unroll
  for (int q = 0; q < CSUM; ++q) {
    const uint32_t w = wave_sum_u32(v[q]);
    if ((threadIdx.x & 63) == 0) out[q] = w;
  }
}

// chunksum: the chunk sums from the tile totals (used when there are no points, so the
// column scan, which otherwise writes them, does not run).
__global__ __launch_bounds__(64) void k_chunksum(const uint32_t* __restrict__ tot,
                                                 uint32_t* __restrict__ csum, uint32_t NB,
                                                 uint32_t item_e, uint32_t fine_e) {
  const uint32_t b = blockIdx.x * CHUNK + threadIdx.x;
  chunk_sums(tile_count(tot, b, NB, item_e, fine_e), item_e, csum + size_t(blockIdx.x) * CSUM);
}

// colscan: per bin, exclusive prefix of H16 over point blocks (into H) and the bin total;
// the wavefront that finishes the totals of its 64 bins (one chunk) also writes the chunk's
// sums.  Workgroup = 64 bins x 16 block segments.
constexpr int CS_SEG = 16;
static_assert(CHUNK == 64, "a column-scan workgroup covers one chunk");
__global__ __launch_bounds__(64 * CS_SEG) void k_colscan(const uint16_t* __restrict__ H16,
                                                         uint32_t* __restrict__ H,
                                                         uint32_t* __restrict__ tot, uint32_t NB,
                                                         uint32_t nblk, uint32_t* __restrict__ csum,
                                                         uint32_t item_e, uint32_t fine_e) {
  __shared__ uint32_t ssum[CS_SEG][64];
  const uint32_t lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const uint32_t b = blockIdx.x * 64 + lane;
  const uint32_t per = (nblk + CS_SEG - 1) / CS_SEG;
  const uint32_t k0 = min(nblk, seg * per), k1 = min(nblk, k0 + per);
  // A segment of at most RC rows is read once, all rows at a time, and kept in registers for
  // the prefix pass; longer segments are read eight rows at a time, twice.  Rows past the
  // segment read its last row (a valid address) and are not used.
  constexpr uint32_t RB = 8, RC = 32;
  const bool cached = per <= RC;  // uniform over the workgroup
  uint32_t c[RC];
  uint32_t sum = 0;
  if (cached) {
    const uint32_t bb = min(b, NB - 1);
#pragma unroll
    for (uint32_t q = 0; q < RC; ++q) c[q] = H16[size_t(min(k0 + q, k1 - 1)) * NB + bb];
#pragma unroll
    for (uint32_t q = 0; q < RC; ++q) sum += k0 + q < k1 && b < NB ? c[q] : 0u;
  } else if (b < NB) {
    for (uint32_t k = k0; k < k1; k += RB) {
      uint32_t v[RB];
#pragma unroll
      for (uint32_t q = 0; q < RB; ++q) v[q] = H16[size_t(min(k + q, k1 - 1)) * NB + b];
#pragma unroll
      for (uint32_t q = 0; q < RB; ++q) sum += k + q < k1 ? v[q] : 0u;
    }
  }
  ssum[seg][lane] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (uint32_t s = 0; s < seg; ++s) run += ssum[s][lane];
  if (seg == CS_SEG - 1)  // the whole wavefront (lanes past NB count nothing)
    chunk_sums(tile_count_of(run + sum, b < NB, item_e, fine_e), item_e,
               csum + size_t(blockIdx.x) * CSUM);
  if (b < NB && cached) {
    if (seg == CS_SEG - 1) tot[b] = run + sum;
#pragma unroll
    for (uint32_t q = 0; q < RC; ++q)
      if (k0 + q < k1) {
        H[size_t(k0 + q) * NB + b] = run;
        run += c[q];
      }
  } else if (b < NB) {
    if (seg == CS_SEG - 1) tot[b] = run + sum;
    for (uint32_t k = k0; k < k1; k += RB) {
      uint32_t v[RB];
#pragma unroll
      for (uint32_t q = 0; q < RB; ++q) v[q] = H16[size_t(min(k + q, k1 - 1)) * NB + b];
#pragma unroll
      for (uint32_t q = 0; q < RB; ++q)
        if (k + q < k1) {
          H[size_t(k + q) * NB + b] = run;
          run += v[q];
        }
    }
  }
}

// chunkscan (one workgroup): exclusive scan of the chunk sums, the totals and the first work
// slot of each size class.
__global__ __launch_bounds__(1024) void k_chunkscan(const uint32_t* __restrict__ csum,
                                                    uint32_t* __restrict__ coff,
                                                    uint32_t* __restrict__ bin_start,
                                                    uint32_t* __restrict__ item_start,
                                                    uint32_t* __restrict__ info, uint32_t NB,
                                                    uint32_t nchunks) {
  __shared__ uint4 ws[16];
  __shared__ uint32_t s_cls[NBUCKET];
  if (threadIdx.x < NBUCKET) s_cls[threadIdx.x] = 0;
  __syncthreads();
  uint4 carry = make_uint4(0u, 0u, 0u, 0u);
  uint32_t cls[NBUCKET];
#pragma unroll
  for (int q = 0; q < NBUCKET; ++q) cls[q] = 0;
  for (uint32_t c0 = 0; c0 < nchunks; c0 += 1024) {
    const uint32_t c = c0 + threadIdx.x;
    uint4 x = make_uint4(0u, 0u, 0u, 0u);
    if (c < nchunks) {
      const uint32_t* r = csum + size_t(c) * CSUM;
      x = make_uint4(r[0], r[1], r[2], r[3]);
#pragma unroll
      for (int q = 0; q < NBUCKET; ++q) cls[q] += r[4 + q];
    }
    uint4 t4;
    const uint4 o = block_excl_scan4<16>(x, ws, t4);
    if (c < nchunks) {
      uint32_t* w = coff + size_t(c) * 4;
      w[0] = carry.x + o.x; w[1] = carry.y + o.y; w[2] = carry.z + o.z; w[3] = carry.w + o.w;
    }
    carry.x += t4.x; carry.y += t4.y; carry.z += t4.z; carry.w += t4.w;
  }
#pragma unroll
  for (int q = 0; q < NBUCKET; ++q) {
    const uint32_t w = wave_sum_u32(cls[q]);
    if ((threadIdx.x & 63) == 0 && w) atomicAdd(&s_cls[q], w);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bin_start[NB] = carry.x;
    item_start[NB] = carry.y;
    info[0] = carry.x;
    info[1] = carry.y;
    info[2] = 0;  // visible (point, view) pairs, accumulated by the scatter pass
    info[3] = carry.z;
    info[4] = carry.w;
    info[5] = NB - carry.w;
    uint32_t o = 0;
    for (int q = 0; q < NBUCKET; ++q) {  // first work slot of each size class; fill counters
      info[INFO_BUCKET + q] = o;
      info[INFO_BUCKET + NBUCKET + q] = 0;
      o += s_cls[q];
    }
  }
}

// binscan: per chunk (one wavefront), the tiles' starts, list entries and work items.  The
// work table is in processing order, largest items first (size classes of item_e / NBUCKET
// entries; the order within a class is whatever the atomics give, which changes no result:
// every item writes its own outputs).  A slot describes item it as
// {tile, first entry, end entry, it | (tile has several items) << 31}; slots are reserved per
// chunk and class, with LDS counters and then one global atomic per class.
// With FUSED (at most FUSE_CHUNKS chunks), every wavefront instead derives its chunk's
// offsets, and the first slot of each class, from the chunk sums of all chunks (the chunk
// scan does not run), and wavefront 0 writes the totals.
constexpr uint32_t FUSE_CHUNKS = 512;
template <bool FUSED>
__global__ __launch_bounds__(64) void k_binscan(const uint32_t* __restrict__ tot,
                                                const uint32_t* __restrict__ csum,
                                                const uint32_t* __restrict__ coff,
                                                uint32_t* __restrict__ bin_start,
                                                uint32_t* __restrict__ item_start,
                                                uint32_t* __restrict__ multi_bins,
                                                uint4* __restrict__ fine_work,
                                                uint32_t* __restrict__ coarse_bins,
                                                uint32_t* __restrict__ info, uint4* __restrict__ work,
                                                uint32_t NB, uint32_t nch, uint32_t item_e,
                                                uint32_t fine_e) {
  __shared__ uint32_t s_cnt[NBUCKET], s_base[NBUCKET];
  const int t = threadIdx.x;
  if (t < NBUCKET) s_cnt[t] = 0;
  const uint32_t b = blockIdx.x * CHUNK + t;
  const TileCount c = tile_count(tot, b, NB, item_e, fine_e);
  uint32_t co[4];
  if (FUSED) {
    uint32_t pre[CSUM], all[CSUM];  // sums over the chunks before this one, over all chunks
#pragma unroll
    for (int q = 0; q < CSUM; ++q) pre[q] = all[q] = 0u;
    for (uint32_t k = t; k < nch; k += 64) {
      const uint32_t* r = csum + size_t(k) * CSUM;
      const bool before = k < blockIdx.x;
#pragma unroll
      for (int q = 0; q < CSUM; ++q) {
        const uint32_t x = r[q];
        all[q] += x;
        pre[q] += before ? x : 0u;
      }
    }
#pragma unroll
    for (int q = 0; q < CSUM; ++q) {
      pre[q] = wave_sum_u32(pre[q]);
      all[q] = wave_sum_u32(all[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) co[q] = pre[q];
    const bool lead = blockIdx.x == 0 && t == 0;
    uint32_t o = 0;
#pragma unroll
    for (int q = 0; q < NBUCKET; ++q) {
      if (t == 0) s_base[q] = o + pre[4 + q];
      if (lead) {
        info[INFO_BUCKET + q] = o;
        info[INFO_BUCKET + NBUCKET + q] = 0;
      }
      o += all[4 + q];
    }
    if (lead) {
      bin_start[NB] = all[0];
      item_start[NB] = all[1];
      info[0] = all[0];
      info[1] = all[1];
      info[2] = 0;  // visible (point, view) pairs, accumulated by the scatter pass
      info[3] = all[2];
      info[4] = all[3];
      info[5] = NB - all[3];
    }
  } else {
    const uint32_t* cp = coff + size_t(blockIdx.x) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) co[q] = cp[q];
  }
  const uint32_t oe = co[0] + wave_incl_scan(c.e) - c.e;
  const uint32_t oi = co[1] + wave_incl_scan(c.it) - c.it;
  const uint32_t om = co[2] + wave_incl_scan(c.multi) - c.multi;
  const uint32_t of = co[3] + wave_incl_scan(c.fine) - c.fine;
  if (b < NB) {
    bin_start[b] = oe;
    item_start[b] = oi;
    if (c.multi) {  // the tile and the first of its items' partial-list slots
      multi_bins[om] = b;
      multi_bins[NB + om] = oi - (b - om - of);
    }
    if (c.fine) fine_work[of] = make_uint4(b, oe, oe + c.e, 0u);
    else coarse_bins[b - of] = b;  // tiles before b that are not fine
  }
  // work items: consecutive ranges of item_e entries (the last holds the rest), all in the
  // class of the tile's average item (the forward takes them as strided blocks)
  const uint32_t q = item_class(c, item_e);
  __syncthreads();
  const uint32_t rf = c.it ? atomicAdd(&s_cnt[q], c.it) : 0u;
  __syncthreads();
  if (!FUSED && t < NBUCKET && s_cnt[t])
    s_base[t] = info[INFO_BUCKET + t] + atomicAdd(&info[INFO_BUCKET + NBUCKET + t], s_cnt[t]);
  __syncthreads();
  if (!c.it) return;
  // items of multi-item tiles carry their partial-list slot: the items of such tiles before
  // this one (oi counts one item for each of the b - om - of single-item tiles before it)
  const uint32_t multi = c.it > 1 ? 0x80000000u : 0u;
  const uint32_t pslot = multi ? oi - (b - om - of) : 0u;
  for (uint32_t k = 0; k < c.it; ++k) {
    const uint32_t e0 = oe + k * item_e;
    work[s_base[q] + rf + k] = make_uint4(b, e0, min(e0 + item_e, oe + c.e), (pslot + k) | multi);
  }
}

// scatter: the count pass again, with LDS ranks; entry -> bin_start + H (column prefix) + rank.
// With STAGED, the block's first position in every bin of its view is staged in LDS first;
// otherwise it is read per entry (views whose tables exceed 64 KB of LDS).
template <bool STAGED>
__global__ __launch_bounds__(BIN_THREADS) void k_scatter(const Params P, const float* __restrict__ X,
                                                         const float* __restrict__ Y,
                                                         const float* __restrict__ Z,
                                                         const float* __restrict__ SW,
                                                         const float* __restrict__ A,
                                                         const uint32_t* __restrict__ H,
                                                         const uint32_t* __restrict__ bin_start,
                                                         Entry* __restrict__ ent,
                                                         uint32_t* __restrict__ epos,
                                                         uint32_t* __restrict__ info) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t s_vis;
  const int v = blockIdx.x % P.V;
  const uint32_t blk = blockIdx.x / P.V;
  const ViewP& c = P.view[v];
  const uint32_t nw = (c.nbins + 1) >> 1;
  uint32_t* hist = lds;            // packed 16-bit ranks
  uint32_t* base = lds + nw;       // first slot of this block in each bin
  const uint32_t* row = H + size_t(blk) * P.NB + c.bin_base;
  const uint32_t* bs = bin_start + c.bin_base;
  if (threadIdx.x == 0) s_vis = 0;
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) hist[i] = 0;
  if (STAGED) {  // SB bins per thread in flight (a 1080p view's tiles in one batch)
    constexpr int SB = 12;
    for (uint32_t i0 = threadIdx.x; i0 < c.nbins; i0 += SB * blockDim.x) {
      uint32_t va[SB], vb[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        const uint32_t i = min(i0 + q * blockDim.x, c.nbins - 1);  // a valid bin, used if in range
        va[q] = bs[i];
        vb[q] = row[i];
      }
#pragma unroll
      for (int q = 0; q < SB; ++q)
        if (i0 + q * blockDim.x < c.nbins) base[i0 + q * blockDim.x] = va[q] + vb[q];
    }
  }
  __syncthreads();
  const int64_t p0 = int64_t(blk) * P.pb;
  const int64_t p1 = min(P.n, p0 + int64_t(P.pb));
  uint32_t vis = 0;
  // two points ahead: a load issued after this point's entry stores would wait for them
  // (one in-order counter), so the point used next was requested a point earlier
  const int64_t pn = p0 + threadIdx.x;
  const int64_t st = blockDim.x;
  float x = 0.f, y = 0.f, z = 0.f, sw = 0.f, al = 0.f;
  float x1 = 0.f, y1 = 0.f, z1 = 0.f, sw1 = 0.f, al1 = 0.f;
  if (pn < p1) {
    const int64_t q0 = pn, q1 = min(pn + st, p1 - 1);
    x = X[q0]; y = Y[q0]; z = Z[q0]; sw = SW[q0]; al = A[q0];
    x1 = X[q1]; y1 = Y[q1]; z1 = Z[q1]; sw1 = SW[q1]; al1 = A[q1];
  }
  for (int64_t p = pn; p < p1; p += st) {
    const int64_t pc = min(p + 2 * st, p1 - 1);
    const float xn = X[pc], yn = Y[pc], zn = Z[pc], swn = SW[pc], aln = A[pc];
    const float alpha = al;
    bool any = false;
    uint32_t er[NSLOT];  // the point's entry positions, written as one 32-byte record
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) er[k] = 0u;
    for_each_entry<true>(P, c, x, y, z, sw,
                   [&](uint32_t bin, uint32_t slot, int sel, const Foot& ft, const Geo& g) {
                     any = true;
                     const uint32_t lb = bin - c.bin_base;
                     const uint32_t rank = add16(hist, lb);
                     Entry e;
                     e.idx = uint32_t(p);
                     e.zbits = __float_as_uint(g.zc);
                     e.u = ft.u;
                     e.v = ft.v;
                     e.ia = g.io[sel] * alpha;
                     const uint32_t at = (STAGED ? base[lb] : bs[lb] + row[lb]) + rank;
                     ent[at] = e;
#pragma unroll
                     for (int k = 0; k < NSLOT; ++k) er[k] = slot == uint32_t(k) ? at : er[k];
                   });
    if (any) {  // where the backward finds the rows of this point's entries
      uint4* ep4 = reinterpret_cast<uint4*>(epos + (size_t(v) * size_t(P.n) + size_t(p)) * NSLOT);
      ep4[0] = make_uint4(er[0], er[1], er[2], er[3]);
      ep4[1] = make_uint4(er[4], er[5], er[6], er[7]);
    }
    vis += any ? 1u : 0u;
    x = x1; y = y1; z = z1; sw = sw1; al = al1;
    x1 = xn; y1 = yn; z1 = zn; sw1 = swn; al1 = aln;
  }
  // number of (point, view) pairs with at least one entry, for reports
  atomicAdd(&s_vis, vis);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&info[2], s_vis);
}

// Corners of entry e that lie in tile (tx, ty): corner c = 2 dj + di is present iff bit c
// of the returned mask is set; cs[c] then holds its local texel id and weights.
struct Corner { int p; float wx, wy; float sx, sy; };
__device__ __forceinline__ uint32_t entry_corners(const Entry& e, const BinInfo& bi, int ltw,
                                                  Corner (&cs)[4]) {
  const int lth = 8 - ltw;
  float flu = floorf(e.u), flv = floorf(e.v);
  int i0 = int(flu), j0 = int(flv);
  float fu = e.u - flu, fv = e.v - flv;
  uint32_t mask = 0;
#pragma unroll
  for (int dj = 0; dj < 2; ++dj)
#pragma unroll
    for (int di = 0; di < 2; ++di) {
      const int c = 2 * dj + di;
      int i = i0 + di, j = j0 + dj;
      float wx = di ? fu : 1.0f - fu;
      float wy = dj ? fv : 1.0f - fv;
      bool in = (i >= 0) & (i < bi.WL) & (j >= 0) & (j < bi.HL) & (wx != 0.0f) & (wy != 0.0f) &
                ((i >> ltw) == bi.tx) & ((j >> lth) == bi.ty);
      cs[c].p = ((j - (bi.ty << lth)) << ltw) + (i - (bi.tx << ltw));
      cs[c].wx = wx; cs[c].wy = wy;
      cs[c].sx = di ? 1.0f : -1.0f; cs[c].sy = dj ? 1.0f : -1.0f;
      mask |= uint32_t(in) << c;
    }
  return mask;
}

// Optional inputs and outputs around the blend (any may be null): a background composited
// behind the kept fragments, C += T_K bg with T_K the transmittance left after them; the
// coverage 1 - T_K of every texel; in the backward pass the upstream gradient of the
// coverage, the gradient of the background (T_K G) and the camera gradient.
struct Extras {
  float* alpha;               // [P]
  const float* bg;            // [P][D], 16-byte aligned
  const float* galpha;        // [P]
  float* gbg;                 // [P][D], 16-byte aligned
  float* gcam;                // [V][16]
};

// Write the composited colour and the coverage of texel `tex` (pyramid texel index).
template <int D>
__device__ __forceinline__ void write_texel(float (&C)[D], float T, size_t tex, float* __restrict__ pyr,
                                            const float* __restrict__ bg, float* __restrict__ alpha) {
  if (bg) {
    const float4* bp = reinterpret_cast<const float4*>(bg + tex * D);
#pragma unroll
    for (int q = 0; q < D / 4; ++q) {
      const float4 bv = bp[q];
      C[4 * q + 0] += T * bv.x;
      C[4 * q + 1] += T * bv.y;
      C[4 * q + 2] += T * bv.z;
      C[4 * q + 3] += T * bv.w;
    }
  }
  float4* op = reinterpret_cast<float4*>(pyr + tex * D);
#pragma unroll
  for (int q = 0; q < D / 4; ++q) op[q] = make_float4(C[4 * q], C[4 * q + 1], C[4 * q + 2], C[4 * q + 3]);
  if (alpha) alpha[tex] = 1.0f - T;
}

// Blend the kept fragments of one texel front to back (Eq. 6-7) and write its outputs.
template <int D>
__device__ __forceinline__ void finalize_texel(const Params& P, const BinInfo& bi, uint32_t b,
                                               const uint64_t (&kk)[KEEP], const float (&kg)[KEEP],
                                               uint32_t n, const float* __restrict__ desc,
                                               float* __restrict__ pyr, uint32_t* __restrict__ npix,
                                               uint64_t* __restrict__ kkey, float* __restrict__ kgam,
                                               const float* __restrict__ bg, float* __restrict__ alpha,
                                               int t) {
  const int lth = 8 - P.ltw;
  const int i = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
  const int j = (bi.ty << lth) + (t >> P.ltw);
  const uint32_t k = min(n, uint32_t(KEEP));
  float C[D];
#pragma unroll
  for (int d = 0; d < D; ++d) C[d] = 0.0f;
  float T = 1.0f;
  // descriptor gathers are issued in batches of GB before they are used
  constexpr int GB = D > 4 ? 4 : 8;
#pragma unroll
  for (int m0 = 0; m0 < KEEP; m0 += GB) {
    float4 tv[GB][D / 4];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int m = m0 + q;
      const float4* tp = reinterpret_cast<const float4*>(desc + size_t(uint32_t(kk[m])) * D);
#pragma unroll
      for (int r = 0; r < D / 4; ++r)
        tv[q][r] = uint32_t(m) < k ? tp[r] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int m = m0 + q;
      if (uint32_t(m) < k) {
        const float w = T * kg[m];
#pragma unroll
        for (int r = 0; r < D / 4; ++r) {
          C[4 * r + 0] += w * tv[q][r].x;
          C[4 * r + 1] += w * tv[q][r].y;
          C[4 * r + 2] += w * tv[q][r].z;
          C[4 * r + 3] += w * tv[q][r].w;
        }
        T = T * (1.0f - kg[m]);
      }
    }
  }
  if (i < bi.WL && j < bi.HL)
    write_texel<D>(C, T, size_t(P.view[bi.v].lout[bi.L]) + size_t(j) * bi.WL + i, pyr, bg, alpha);
  npix[size_t(b) * TP + t] = n;
#pragma unroll
  for (int m = 0; m < KEEP; ++m)
    if (uint32_t(m) < k) {
      kkey[(size_t(b) * KEEP + m) * TP + t] = kk[m];
      kgam[(size_t(b) * KEEP + m) * TP + t] = kg[m];
    }
}

constexpr int EPT = 2;                // entries per thread per LDS round
constexpr int SUB_E = EPT * TP;       // entries per LDS round
constexpr int SUB_F = 4 * SUB_E;      // fragments per LDS round (at most 4 per entry)
constexpr uint32_t ENT_BLK = 4;       // consecutive entries taken together by fwd_items
constexpr uint32_t RND_BLK = SUB_E / ENT_BLK;  // blocks per round

// Compare-exchange of (key, gamma) pairs: afterwards a holds the smaller key.
__device__ __forceinline__ void cswap(uint64_t& ka, float& ga, uint64_t& kb, float& gb) {
  const bool sw = kb < ka;
  const uint64_t k0 = sw ? kb : ka, k1 = sw ? ka : kb;
  const float g0 = sw ? gb : ga, g1 = sw ? ga : gb;
  ka = k0; kb = k1; ga = g0; gb = g1;
}

// Lowest 16 of two ascending lists: c[i] = min(a[i], b[15-i]) is bitonic and holds them;
// half-cleaners of width 8, 4, 2, 1 sort it.
__device__ __forceinline__ void merge16(uint64_t (&k)[KEEP], float (&g)[KEEP],
                                        const uint64_t (&ok)[KEEP], const float (&og)[KEEP]) {
#pragma unroll
  for (int i = 0; i < KEEP; ++i) {
    const bool take = ok[KEEP - 1 - i] < k[i];
    k[i] = take ? ok[KEEP - 1 - i] : k[i];
    g[i] = take ? og[KEEP - 1 - i] : g[i];
  }
#pragma unroll
  for (int w = KEEP / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int i = 0; i < KEEP; ++i)
      if ((i & w) == 0) cswap(k[i], g[i], k[i + w], g[i + w]);
}

// fwd_items: one workgroup per work item (largest first).  Each LDS round expands SUB_E
// entries into fragments, counting-sorts them by texel and lets the thread owning the texel
// insert them into its register top-16; in the first round, whose lists are all empty, the
// fragments' depth ranks are counted in LDS instead and the first 16 ranks loaded in order.
// The entries are taken in blocks of ENT_BLK consecutive ones, strided over the tile: item i
// of a tile with I items takes blocks i, i + I, ..., and round r of an item with R rounds
// its blocks r, r + R, ...  A round then mixes entries from the whole tile whatever the
// order of the points (consecutive points of a spatially ordered cloud crowd a few texels,
// whose threads would insert long runs while the others idle), and the loads stay
// coalesced per block.  The result does not depend on the order.
// A fragment whose depth bits are above those of the texel's current 16th key is only
// counted, never sorted (the insertion makes the exact comparison).  A texel's tally and its
// count of sorted fragments share one LDS word, so a fragment costs one LDS atomic.
constexpr uint32_t TALLY_BITS = 20;  // per-texel word: all fragments of the item (low bits),
constexpr uint32_t TALLY_MASK = (1u << TALLY_BITS) - 1u;  // and this round's sorted ones or
                                                          // the start of the texel's run
static_assert(4u * SUB_E < (1u << (32 - TALLY_BITS)), "run starts fit the high bits");
template <int D>
__global__ __launch_bounds__(256) void k_fwd_items(
    const Params P, const uint32_t* __restrict__ info, const uint4* __restrict__ work,
    const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ item_start,
    const Entry* __restrict__ ent, const float* __restrict__ desc, float* __restrict__ pyr,
    uint32_t* __restrict__ npix, uint64_t* __restrict__ kkey, float* __restrict__ kgam,
    uint32_t* __restrict__ pcnt, uint64_t* __restrict__ pkey, float* __restrict__ pgam,
    const float* __restrict__ bg, float* __restrict__ alpha) {
  __shared__ uint32_t th[TP];      // tally | (sorted fragments, then run start) << TALLY_BITS
  __shared__ uint32_t thz[TP];     // depth bits of the current 16th key per texel
  __shared__ uint64_t skey[SUB_F];
  __shared__ float sgam[SUB_F];
  __shared__ uint8_t stex[SUB_F];   // texel of each sorted fragment (first round)
  // at run start + r: run position of rank r (first round); its first words also serve the
  // run-start scan, which is done with them before the first round writes ranks
  __shared__ uint32_t sord_w[SUB_F / 2];
  uint16_t* sord = reinterpret_cast<uint16_t*>(sord_w);
  uint32_t* ws = sord_w;
  const int t = threadIdx.x;
  const uint32_t total = info[1];
  const uint4 wk = work[blockIdx.x];  // in bounds (grid = capacity); used only if valid
  if (blockIdx.x >= total) return;
  const uint32_t b = wk.x, it = wk.w & 0x7fffffffu;
  const bool multi = (wk.w >> 31) != 0;
  const BinInfo bi = decode_bin(P, b);
  // the item's blocks (uniform): the tile's entries t0..t1, item ii of ni
  uint32_t t0 = wk.y, t1 = wk.z, ni = 1, ii = 0;
  if (multi) {
    t0 = bin_start[b];
    t1 = bin_start[b + 1];
    ni = item_start[b + 1] - item_start[b];
    ii = (wk.y - t0) / P.item_e;
  }
  const uint32_t nbt = (t1 - t0 + ENT_BLK - 1) / ENT_BLK;  // the tile's blocks (ii < ni <= nbt)
  const uint32_t nbi = (nbt - ii + ni - 1) / ni;           // the item's
  const uint32_t nr = (nbi + RND_BLK - 1) / RND_BLK;       // rounds
  // position of entry slot s (0 .. SUB_E - 1) of round r, or t1 if the slot is empty
  auto entry_at = [&](uint32_t r, uint32_t s) {
    const uint32_t kb = r + nr * (s / ENT_BLK);
    const uint32_t pos = t0 + (ii + ni * kb) * ENT_BLK + s % ENT_BLK;
    return kb < nbi && pos < t1 ? pos : t1;
  };
  uint64_t kk[KEEP];
  float kg[KEEP];
#pragma unroll
  for (int m = 0; m < KEEP; ++m) { kk[m] = KEY_NONE; kg[m] = 0.0f; }
  th[t] = 0;
  thz[t] = ~0u;
  // entries of the current round, loaded one round ahead
  Entry en[EPT];
  uint32_t ep[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    ep[q] = entry_at(0, q * TP + t);
    if (ep[q] < t1) en[q] = ent[ep[q]];
  }
  for (uint32_t r = 0; r < nr; ++r) {
    th[t] &= TALLY_MASK;
    __syncthreads();
    uint32_t cm[EPT], rank[EPT][2];  // corner masks; 16-bit ranks, two per word
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      cm[q] = 0;
      rank[q][0] = rank[q][1] = 0;
      Corner cs[4];
      if (ep[q] < t1) cm[q] = entry_corners(en[q], bi, P.ltw, cs);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if ((cm[q] >> c) & 1u) {
          const int px = cs[c].p;
          const bool pass = en[q].zbits <= thz[px];
          const uint32_t old = atomicAdd(&th[px], pass ? 1u + (1u << TALLY_BITS) : 1u);
          if (pass) rank[q][c >> 1] |= (old >> TALLY_BITS) << ((c & 1) * 16);
          else cm[q] &= ~(1u << c);
        }
      }
    }
    Entry nx[EPT];  // next round's entries
    uint32_t np[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      np[q] = r + 1 < nr ? entry_at(r + 1, q * TP + t) : t1;
      if (np[q] < t1) nx[q] = ent[np[q]];
    }
    __syncthreads();
    const uint32_t cnt = th[t] >> TALLY_BITS;
    uint32_t tot;
    const uint32_t base = block_excl_scan<4>(cnt, ws, tot);
    th[t] = (th[t] & TALLY_MASK) | (base << TALLY_BITS);  // counts were read before the scan
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      if (!cm[q]) continue;
      Corner cs[4];
      entry_corners(en[q], bi, P.ltw, cs);
      const uint64_t key = (uint64_t(en[q].zbits) << 32) | en[q].idx;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if ((cm[q] >> c) & 1u) {
          const uint32_t o =
              (th[cs[c].p] >> TALLY_BITS) + ((rank[q][c >> 1] >> ((c & 1) * 16)) & 0xffffu);
          skey[o] = key;
          sgam[o] = (cs[c].wx * cs[c].wy) * en[q].ia;
          stex[o] = uint8_t(cs[c].p);
        }
    }
    __syncthreads();
    if (r == 0) {
      // first round: every list is empty, so a texel's list is simply the first ranks of its
      // run.  Every fragment counts the smaller keys of its run (its depth rank; keys are
      // distinct in a texel), then each thread loads its first 16 ranks in order.
      for (uint32_t o = t; o < tot; o += TP) {
        const uint32_t p = stex[o];
        const uint32_t r0 = th[p] >> TALLY_BITS;
        const uint32_t r1 = p + 1 < TP ? th[p + 1] >> TALLY_BITS : tot;
        const uint64_t ko = skey[o];
        uint32_t rk = 0;
        // eight keys per step, every read inside the run (the compares past its end are
        // masked): long runs of crowded texels are latency-bound LDS chains
        for (uint32_t r = r0; r < r1; r += 8) {
          uint64_t kq[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) kq[q] = skey[min(r + q, r1 - 1)];
#pragma unroll
          for (int q = 0; q < 8; ++q) rk += (r + q < r1 && kq[q] < ko) ? 1u : 0u;
        }
        if (rk < KEEP) sord[r0 + rk] = uint16_t(o - r0);
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < KEEP; ++m) {
        const bool v = uint32_t(m) < cnt;
        // (the clamp only guards LDS: ranks are a permutation of the run)
        const uint32_t o = base + (v ? min(uint32_t(sord[base + m]), cnt - 1) : 0u);
        kk[m] = v ? skey[o] : KEY_NONE;
        kg[m] = v ? sgam[o] : 0.0f;
      }
    } else {
      // the texel's run, read from LDS four fragments at a time
      for (uint32_t r = 0; r < cnt; r += 4) {
        uint64_t rk[4];
        float rg[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool v = r + q < cnt;
          rk[q] = v ? skey[base + r + q] : KEY_NONE;
          rg[q] = v ? sgam[base + r + q] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) top_insert(kk, kg, rk[q], rg[q]);
      }
    }
    thz[t] = uint32_t(kk[KEEP - 1] >> 32);
#pragma unroll
    for (int q = 0; q < EPT; ++q) { en[q] = nx[q]; ep[q] = np[q]; }
    __syncthreads();
  }
  const uint32_t n = th[t] & TALLY_MASK;
  if (!multi) {
    finalize_texel<D>(P, bi, b, kk, kg, n, desc, pyr, npix, kkey, kgam, bg, alpha, t);
  } else {
    // partial list of this texel: 16 keys and gammas stored contiguously (unused slots hold
    // KEY_NONE), read back as whole lists by the merge
    pcnt[size_t(it) * TP + t] = n;
    uint4* pk = reinterpret_cast<uint4*>(pkey + (size_t(it) * TP + t) * KEEP);
    float4* pg = reinterpret_cast<float4*>(pgam + (size_t(it) * TP + t) * KEEP);
#pragma unroll
    for (int m = 0; m < KEEP; m += 2)
      pk[m / 2] = make_uint4(uint32_t(kk[m]), uint32_t(kk[m] >> 32), uint32_t(kk[m + 1]),
                             uint32_t(kk[m + 1] >> 32));
#pragma unroll
    for (int m = 0; m < KEEP; m += 4) pg[m / 4] = make_float4(kg[m], kg[m + 1], kg[m + 2], kg[m + 3]);
  }
}

// Kept slots of the entries of a fine tile, once the forward pass ran (kslot[fine tile][entry
// of the tile]): bits 5c .. 5c + 4 hold the kept slot (0..15) of corner c, 31 if absent or
// not kept.
constexpr uint32_t KSLOT_NONE = 31;

// fwd_fine: one workgroup per fine tile, one entry per thread.  Fragments are counting-sorted
// by texel in LDS; every fragment then counts the smaller keys of its texel's run (its
// depth rank, computed by the threads in parallel whatever the run lengths), the first 16
// ranks are the kept list, and the thread owning a texel blends it (Eq. 6-7) and writes
// the same outputs as the item path.  Each entry's descriptor is loaded at the start and
// read from LDS by the blend.  Every entry then records the kept slot of each of its
// corners.
template <int D>
__global__ __launch_bounds__(256) void k_fwd_fine(
    const Params P, const uint32_t* __restrict__ info, const uint4* __restrict__ fine_work,
    const Entry* __restrict__ ent, uint32_t* __restrict__ kslot, const float* __restrict__ desc,
    float* __restrict__ pyr, uint32_t* __restrict__ npix, uint64_t* __restrict__ kkey,
    float* __restrict__ kgam, const float* __restrict__ bg, float* __restrict__ alpha) {
  constexpr int NF = 4 * FINE_E;     // fragment capacity
  __shared__ uint32_t hist[TP];      // fragments per texel, then the start of its run
  __shared__ uint32_t ws[4];
  __shared__ uint64_t skey[NF];
  __shared__ float sgam[NF];
  __shared__ uint16_t sord[NF];      // at run start + m: run position of the m-th kept fragment
  __shared__ uint8_t sslot[NF];      // kept slot (depth rank) of each fragment, 0xff if not kept
  __shared__ uint8_t stex[NF];       // texel of each fragment
  __shared__ uint8_t sent[NF];       // entry (thread) of each fragment
  __shared__ float4 sdesc[FINE_E][D / 4];  // descriptor of each entry's point
  static_assert(FINE_E == TP, "one entry per thread");
  const int t = threadIdx.x;
  const uint4 wk = fine_work[blockIdx.x];  // in bounds (grid = bin count); used only if valid
  if (blockIdx.x >= info[4]) return;
  if (wk.y == wk.z) {  // an empty tile (uniform): only the background shows
    const BinInfo bi = decode_bin(P, wk.x);
    const int lth = 8 - P.ltw;
    const int i = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
    const int j = (bi.ty << lth) + (t >> P.ltw);
    float C[D];
#pragma unroll
    for (int d = 0; d < D; ++d) C[d] = 0.0f;
    if (i < bi.WL && j < bi.HL)
      write_texel<D>(C, 1.0f, size_t(P.view[bi.v].lout[bi.L]) + size_t(j) * bi.WL + i, pyr, bg, alpha);
    npix[size_t(wk.x) * TP + t] = 0;
    return;
  }
  const bool has = wk.y + uint32_t(t) < wk.z;
  Entry en = {};
  if (has) en = ent[wk.y + t];
  {
    // every entry's descriptor is loaded now and used after the sort (in a fine tile
    // nearly every fragment is kept)
    float4 dv[D / 4];
#pragma unroll
    for (int r4 = 0; r4 < D / 4; ++r4) dv[r4] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (has) {
      const float4* dp = reinterpret_cast<const float4*>(desc + size_t(en.idx) * D);
#pragma unroll
      for (int r4 = 0; r4 < D / 4; ++r4) dv[r4] = dp[r4];
    }
    const uint32_t b = wk.x;
    const BinInfo bi = decode_bin(P, b);
    hist[t] = 0;
    __syncthreads();
    Corner cs[4];
    uint32_t cm = 0, rank[4] = {0u, 0u, 0u, 0u};
    if (has) cm = entry_corners(en, bi, P.ltw, cs);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if ((cm >> c) & 1u) rank[c] = atomicAdd(&hist[cs[c].p], 1u);
    __syncthreads();
    const uint32_t cnt = hist[t];
    uint32_t tot;
    const uint32_t base = block_excl_scan<4>(cnt, ws, tot);
    hist[t] = base;  // all counts were read before the scan's first barrier
    __syncthreads();
    const uint64_t key = (uint64_t(en.zbits) << 32) | en.idx;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if ((cm >> c) & 1u) {
        const uint32_t o = hist[cs[c].p] + rank[c];
        skey[o] = key;
        sgam[o] = (cs[c].wx * cs[c].wy) * en.ia;
        stex[o] = uint8_t(cs[c].p);
        sent[o] = uint8_t(t);
      }
#pragma unroll
    for (int r4 = 0; r4 < D / 4; ++r4) sdesc[t][r4] = dv[r4];
    __syncthreads();
    // depth rank of every fragment within its texel (keys are distinct within a texel)
    for (uint32_t o = t; o < tot; o += TP) {
      const uint32_t p = stex[o];
      const uint32_t r0 = hist[p], r1 = p + 1 < TP ? hist[p + 1] : tot;
      const uint64_t ko = skey[o];
      uint32_t rk = 0;
      for (uint32_t r = r0; r < r1; r += 4) {
        uint64_t kq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) kq[q] = r + q < r1 ? skey[r + q] : KEY_NONE;
#pragma unroll
        for (int q = 0; q < 4; ++q) rk += kq[q] < ko ? 1u : 0u;
      }
      sslot[o] = rk < KEEP ? uint8_t(rk) : uint8_t(0xff);
      if (rk < KEEP) sord[r0 + rk] = uint16_t(o - r0);
    }
    __syncthreads();
    if (has) {  // the kept slot of every corner, for the backward pass
      uint32_t packed = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        uint32_t m = KSLOT_NONE;
        if ((cm >> c) & 1u) {
          const uint32_t s8 = sslot[hist[cs[c].p] + rank[c]];
          m = s8 < KEEP ? s8 : KSLOT_NONE;
        }
        packed |= m << (5 * c);
      }
      kslot[size_t(blockIdx.x) * TP + t] = packed;
    }
    // blend front to back
    const uint32_t k = min(cnt, uint32_t(KEEP));
    {
      const int lth = 8 - P.ltw;
      const int i = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
      const int j = (bi.ty << lth) + (t >> P.ltw);
      float C[D];
#pragma unroll
      for (int d = 0; d < D; ++d) C[d] = 0.0f;
      float T = 1.0f;
#pragma unroll 1
      for (uint32_t m = 0; m < k; ++m) {
        const uint32_t o = base + min(uint32_t(sord[base + m]), cnt - 1);  // guards LDS only
        const uint64_t kq = skey[o];
        const float gq = sgam[o];
        const uint32_t eo = sent[o];
        const float w = T * gq;
#pragma unroll
        for (int r4 = 0; r4 < D / 4; ++r4) {
          const float4 tv = sdesc[eo][r4];
          C[4 * r4 + 0] += w * tv.x;
          C[4 * r4 + 1] += w * tv.y;
          C[4 * r4 + 2] += w * tv.z;
          C[4 * r4 + 3] += w * tv.w;
        }
        T = T * (1.0f - gq);
        kkey[(size_t(b) * KEEP + m) * TP + t] = kq;
        kgam[(size_t(b) * KEEP + m) * TP + t] = gq;
      }
      if (i < bi.WL && j < bi.HL)
        write_texel<D>(C, T, size_t(P.view[bi.v].lout[bi.L]) + size_t(j) * bi.WL + i, pyr, bg, alpha);
      npix[size_t(b) * TP + t] = cnt;
    }
  }
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor(uint32_t(v), m, 64);
  const uint32_t hi = __shfl_xor(uint32_t(v >> 32), m, 64);
  return (uint64_t(hi) << 32) | lo;
}

// fwd_merge: bins that were cut into several items.  A workgroup takes 64 texels of one
// such bin; its four wavefronts each merge every fourth item's partial lists (thread =
// texel; each list is read whole with independent loads), the four results are combined
// through LDS and the first wavefront blends.  Work units (bin, 64 texels) are strided over
// the grid.
template <int D>
__global__ __launch_bounds__(256) void k_fwd_merge(
    const Params P, const uint32_t* __restrict__ item_start, const uint32_t* __restrict__ multi_bins,
    const uint32_t* __restrict__ info, const uint32_t* __restrict__ pcnt,
    const uint64_t* __restrict__ pkey, const float* __restrict__ pgam,
    const float* __restrict__ desc, float* __restrict__ pyr, uint32_t* __restrict__ npix,
    uint64_t* __restrict__ kkey, float* __restrict__ kgam, const float* __restrict__ bg,
    float* __restrict__ alpha) {
  __shared__ uint64_t s_key[3][KEEP][64];
  __shared__ float s_gam[3][KEEP][64];
  __shared__ uint32_t s_n[3][64];
  const uint32_t units = info[3] * (TP / 64);
  const int lane = threadIdx.x & 63;
  const int slice = threadIdx.x >> 6;
  for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
    const uint32_t mb = u / (TP / 64);
    const uint32_t b = multi_bins[mb];
    const int t = int(u % (TP / 64)) * 64 + lane;  // texel
    // the tile's items' partial lists: consecutive slots from multi_bins[NB + mb]
    const uint32_t i0 = multi_bins[P.NB + mb], i1 = i0 + (item_start[b + 1] - item_start[b]);
    uint64_t kk[KEEP];
    float kg[KEEP];
#pragma unroll
    for (int m = 0; m < KEEP; ++m) { kk[m] = KEY_NONE; kg[m] = 0.0f; }
    uint32_t n = 0;
    // a partial list holds min(count, 16) ascending keys, then KEY_NONE; the next item's list
    // is loaded while the current one is merged
    auto load = [&](uint32_t it, uint4 (&k4)[KEEP / 2], float4 (&g4)[KEEP / 4], uint32_t& c) {
      const uint4* pk = reinterpret_cast<const uint4*>(pkey + (size_t(it) * TP + t) * KEEP);
      const float4* pg = reinterpret_cast<const float4*>(pgam + (size_t(it) * TP + t) * KEEP);
#pragma unroll
      for (int m = 0; m < KEEP / 2; ++m) k4[m] = pk[m];
#pragma unroll
      for (int m = 0; m < KEEP / 4; ++m) g4[m] = pg[m];
      c = pcnt[size_t(it) * TP + t];
    };
    uint4 k4[KEEP / 2];
    float4 g4[KEEP / 4];
    uint32_t c = 0;
    uint32_t it = i0 + slice;
    if (it < i1) load(it, k4, g4, c);
    while (it < i1) {
      uint64_t ok[KEEP];
      float og[KEEP];
#pragma unroll
      for (int m = 0; m < KEEP; m += 2) {
        ok[m] = (uint64_t(k4[m / 2].y) << 32) | k4[m / 2].x;
        ok[m + 1] = (uint64_t(k4[m / 2].w) << 32) | k4[m / 2].z;
      }
#pragma unroll
      for (int m = 0; m < KEEP; m += 4) {
        og[m] = g4[m / 4].x; og[m + 1] = g4[m / 4].y; og[m + 2] = g4[m / 4].z; og[m + 3] = g4[m / 4].w;
      }
      n += c;
      it += 4;
      if (it < i1) load(it, k4, g4, c);
      merge16(kk, kg, ok, og);
    }
    if (slice > 0) {
#pragma unroll
      for (int m = 0; m < KEEP; ++m) {
        s_key[slice - 1][m][lane] = kk[m];
        s_gam[slice - 1][m][lane] = kg[m];
      }
      s_n[slice - 1][lane] = n;
    }
    __syncthreads();
    if (slice == 0) {
#pragma unroll 1
      for (int q = 0; q < 3; ++q) {
        uint64_t ok[KEEP];
        float og[KEEP];
#pragma unroll
        for (int m = 0; m < KEEP; ++m) { ok[m] = s_key[q][m][lane]; og[m] = s_gam[q][m][lane]; }
        merge16(kk, kg, ok, og);
        n += s_n[q][lane];
      }
      finalize_texel<D>(P, decode_bin(P, b), b, kk, kg, n, desc, pyr, npix, kkey, kgam, bg, alpha, t);
    }
    __syncthreads();  // LDS is reused by the next unit
  }
}

// export: counts and blended ids in pyramid texel order (with coarser-layer inclusion the
// blended list is fkey, its length in fcnt).
__global__ __launch_bounds__(256) void k_export(const Params P, const uint32_t* __restrict__ npix,
                                                const uint64_t* __restrict__ kkey,
                                                const uint64_t* __restrict__ fkey,
                                                const uint32_t* __restrict__ fcnt,
                                                int32_t* __restrict__ counts,
                                                int32_t* __restrict__ ids) {
  const uint32_t b = blockIdx.x;
  const int t = threadIdx.x;
  const BinInfo bi = decode_bin(P, b);
  const int lth = 8 - P.ltw;
  const int i = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
  const int j = (bi.ty << lth) + (t >> P.ltw);
  if (i >= bi.WL || j >= bi.HL) return;
  const size_t o = size_t(P.view[bi.v].lout[bi.L]) + size_t(j) * bi.WL + i;
  const uint32_t n = npix[size_t(b) * TP + t];
  counts[o] = int32_t(n);
  const uint32_t fc = P.coarser ? fcnt[size_t(b) * TP + t] : 0u;
  const uint32_t k = P.coarser ? (fc & 31u) + ((fc >> 5) & 31u) : n;
  if (!P.coarser) {
    for (int m = 0; m < KEEP; ++m)
      ids[o * KEEP + m] = uint32_t(m) < k ? int32_t(uint32_t(kkey[(size_t(b) * KEEP + m) * TP + t])) : -1;
    return;
  }
  // layer 0's blended lists are not stored (below a coarser layer): rebuilt from the own list
  // and the covering layer-1 texel's list (pb, pt) by the origin mask
  const bool rebuilt = bi.L == 0 && P.nl > 1;
  uint32_t pb = 0;
  int pt = 0;
  if (rebuilt) {
    const int pi = i >> 1, pj = j >> 1;
    const int tiles_x1 = (layer_dim(P.view[bi.v].W, 1) + (1 << P.ltw) - 1) >> P.ltw;
    pb = P.view[bi.v].lbin[1] + uint32_t((pj >> lth) * tiles_x1 + (pi >> P.ltw));
    pt = ((pj & ((1 << lth) - 1)) << P.ltw) | (pi & ((1 << P.ltw) - 1));
  }
  const uint32_t mask = fc >> 16;
  for (int m = 0; m < KEEP; ++m) {
    uint64_t key = 0;
    if (uint32_t(m) < k) {
      if (rebuilt) {
        const uint32_t ip = __popc(mask & ((1u << m) - 1u));
        key = ((mask >> m) & 1u) ? fkey[(size_t(pb) * KEEP + ip) * TP + pt]
                                 : kkey[(size_t(b) * KEEP + (uint32_t(m) - ip)) * TP + t];
      } else {
        key = fkey[(size_t(b) * KEEP + m) * TP + t];
      }
    }
    ids[o * KEEP + m] = uint32_t(m) < k ? int32_t(uint32_t(key)) : -1;
  }
}

// g_m = G . tau_m, summed in one fixed order.
template <int D>
__device__ __forceinline__ float dot_g(const float (&G)[D], const float4 (&tv)[D / 4]) {
  float acc = 0.0f;
#pragma unroll
  for (int r = 0; r < D / 4; ++r)
    acc += G[4 * r] * tv[r].x + G[4 * r + 1] * tv[r].y + G[4 * r + 2] * tv[r].z + G[4 * r + 3] * tv[r].w;
  return acc;
}

// dst[0..D) = s * G (16-byte aligned).
template <int D>
__device__ __forceinline__ void write_scaled(float* dst, float s, const float (&G)[D]) {
  float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int q = 0; q < D / 4; ++q) d4[q] = make_float4(s * G[4 * q], s * G[4 * q + 1], s * G[4 * q + 2], s * G[4 * q + 3]);
}

// One step of the reverse blend recurrence for kept fragment m (B holds B_m on entry and
// B_{m-1} on return): returns (dL/dgamma_m, T_m gamma_m).
__device__ __forceinline__ float2 blend_adjoint_step(float Tm, float gam, float gm, float& B) {
  const float dgam = Tm * (gm - B);
  B = gam * gm + (1.0f - gam) * B;
  return make_float2(dgam, Tm * gam);
}

// bwd_pixels: per texel, recompute transmittance T_m front to back and run the reverse
// recurrence B_{m-1} = gamma_m g_m + (1 - gamma_m) B_m (g_m = G . tau_m, B_last = 0):
// dL/dgamma_m = T_m (g_m - B_m); the descriptor gets T_m gamma_m G.
template <int D>
__global__ __launch_bounds__(256) void k_bwd_pixels(const Params P, const uint32_t* __restrict__ info,
                                                    const uint32_t* __restrict__ coarse_bins,
                                                    const uint32_t* __restrict__ npix,
                                                    const uint64_t* __restrict__ kkey,
                                                    const float* __restrict__ kgam,
                                                    const float* __restrict__ desc,
                                                    const float* __restrict__ gpyr,
                                                    float2* __restrict__ bst, const Extras X) {
  const int t = threadIdx.x;
  const uint32_t b = coarse_bins[blockIdx.x];  // in bounds (grid = bin count); used if valid
  if (blockIdx.x >= info[5]) return;
  const uint32_t n = npix[size_t(b) * TP + t];
  if (n == 0 && !X.gbg) return;
  const BinInfo bi = decode_bin(P, b);
  const int lth = 8 - P.ltw;
  const int i = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
  const int j = (bi.ty << lth) + (t >> P.ltw);
  if (!(i < bi.WL && j < bi.HL)) return;  // (such texels hold no fragments)
  const size_t tex = size_t(P.view[bi.v].lout[bi.L]) + size_t(j) * bi.WL + i;
  const size_t o = tex * D;
  float G[D];
  const float4* gp = reinterpret_cast<const float4*>(gpyr + o);
#pragma unroll
  for (int q = 0; q < D / 4; ++q) {
    float4 gv = gp[q];
    G[4 * q] = gv.x; G[4 * q + 1] = gv.y; G[4 * q + 2] = gv.z; G[4 * q + 3] = gv.w;
  }
  if (n == 0) {  // only the background shows
    float4* gb = reinterpret_cast<float4*>(X.gbg + o);
#pragma unroll
    for (int q = 0; q < D / 4; ++q) gb[q] = make_float4(G[4 * q], G[4 * q + 1], G[4 * q + 2], G[4 * q + 3]);
    return;
  }
  const uint32_t k = min(n, uint32_t(KEEP));
  float gam[KEEP], Tm[KEEP], gm[KEEP];
  uint32_t idx[KEEP];
  // kept entries first (independent loads), then the descriptor gathers in batches
#pragma unroll
  for (int m = 0; m < KEEP; ++m) {
    const size_t ko = (size_t(b) * KEEP + m) * TP + t;
    const bool v = uint32_t(m) < k;
    idx[m] = v ? uint32_t(kkey[ko]) : 0u;
    gam[m] = v ? kgam[ko] : 0.0f;
  }
  float T = 1.0f;
#pragma unroll
  for (int m = 0; m < KEEP; ++m) {
    Tm[m] = T;
    if (uint32_t(m) < k) T = T * (1.0f - gam[m]);
  }
  constexpr int GB = D > 4 ? 4 : 8;
#pragma unroll
  for (int m0 = 0; m0 < KEEP; m0 += GB) {
    float4 tv[GB][D / 4];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const float4* tp = reinterpret_cast<const float4*>(desc + size_t(idx[m0 + q]) * D);
#pragma unroll
      for (int r = 0; r < D / 4; ++r)
        tv[q][r] = uint32_t(m0 + q) < k ? tp[r] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < GB; ++q) gm[m0 + q] = dot_g<D>(G, tv[q]);
  }
  if (X.galpha) {  // the coverage blends a constant 1 through the same weights
    const float ga = X.galpha[tex];
#pragma unroll
    for (int m = 0; m < KEEP; ++m) gm[m] += ga;
  }
  float B = X.bg ? dot_g<D>(G, *reinterpret_cast<const float4(*)[D / 4]>(X.bg + o)) : 0.0f;
#pragma unroll
  for (int m = KEEP - 1; m >= 0; --m)
    if (uint32_t(m) < k) bst[(size_t(b) * KEEP + m) * TP + t] = blend_adjoint_step(Tm[m], gam[m], gm[m], B);
  if (X.gbg) write_scaled<D>(X.gbg + o, T, G);
}

// bwd_items: per work item, each entry finds its corners in the tile's kept lists and writes
// its partial-gradient row: (A, Bx, By, 0, tau[D]) with A = sum dgamma wx wy,
// Bx = sum dgamma sx wy, By = sum dgamma wx sy, tau = sum T_m gamma_m G over its corners.
// A corner is kept iff its key is not above the texel's last kept key (the kept set is the
// 16 smallest keys); its position among the kept is found by point index.  With
// coarser-layer inclusion (INC) the kept own fragments are those the blended list took
// (a prefix of the own list), and each one's totals (dL/dgamma, tau part) are read from
// itot instead of being formed from the blend adjoint and G.
template <int D, bool INC>
__global__ __launch_bounds__(256) void k_bwd_items(
    const Params P, const uint32_t* __restrict__ info, const uint4* __restrict__ work,
    const Entry* __restrict__ ent,
    const uint32_t* __restrict__ npix, const uint64_t* __restrict__ kkey,
    const float2* __restrict__ bst, const float* __restrict__ gpyr, float* __restrict__ rows,
    uint32_t split, const uint32_t* __restrict__ fcnt, const float* __restrict__ itot) {
  constexpr int RW = 4 + D;
  constexpr int S = D + 1;
  constexpr int EB = 3;  // entries per thread in flight
  __shared__ uint32_t s_k[TP];
  __shared__ uint64_t s_last[TP];
  // kept point ids, four per 16 bytes, quarter-list major: the reads of one quarter by lanes
  // of random texels then fall on eight bank groups rather than two (texel-major rows are
  // 64 bytes apart)
  __shared__ uint4 s_idx[KEEP / 4][TP];
  __shared__ float s_G[TP][D + 1];
  const int t = threadIdx.x;
  const uint32_t total = info[1];
  // every work item is shared by `split` workgroups, each taking an equal part of its entries;
  // the parts of an item are XCDS indices apart (the same die, so the tile's lists and blend
  // adjoints are fetched into one L2): workgroup g XCDS split + XCDS p + q takes part p of
  // item g XCDS + q
  const uint32_t grp = blockIdx.x / (XCDS * split), rem = blockIdx.x % (XCDS * split);
  const uint32_t wi = grp * XCDS + rem % XCDS, part = rem / XCDS;
  const uint4 wk = work[wi];  // in bounds (grid = split x capacity); used only if valid
  if (wi >= total) return;
  const uint32_t b = wk.x;
  const uint32_t chunk = (wk.z - wk.y + split - 1) / split;
  const uint32_t e0 = wk.y + min(wk.z - wk.y, part * chunk);
  const uint32_t e1 = wk.y + min(wk.z - wk.y, (part + 1) * chunk);
  if (e0 == e1) return;
  // the first entries of this thread, loaded while the tile is staged
  Entry nx[EB];
#pragma unroll
  for (int q = 0; q < EB; ++q)
    if (e0 + q * TP + t < e1) nx[q] = ent[e0 + q * TP + t];
  const BinInfo bi = decode_bin(P, b);
  const int lth = 8 - P.ltw;
  {  // stage the tile's kept point ids, last kept keys and upstream gradient
    const uint32_t k = INC ? (fcnt[size_t(b) * TP + t] & 31u) : min(npix[size_t(b) * TP + t], uint32_t(KEEP));
    s_k[t] = k;
    uint64_t last = 0;
    uint32_t ids[KEEP];
    uint64_t raw[KEEP];
    // all 16 loads are issued together: slots past the list read slot 0 of the same texel
    // (a valid address) and are discarded
#pragma unroll
    for (int m = 0; m < KEEP; ++m) raw[m] = kkey[(size_t(b) * KEEP + (uint32_t(m) < k ? m : 0)) * TP + t];
#pragma unroll
    for (int m = 0; m < KEEP; ++m) {
      const uint64_t key = uint32_t(m) < k ? raw[m] : KEY_NONE;
      ids[m] = uint32_t(key);
      last = uint32_t(m) < k ? key : last;
    }
#pragma unroll
    for (int m = 0; m < KEEP; m += 4) s_idx[m / 4][t] = make_uint4(ids[m], ids[m + 1], ids[m + 2], ids[m + 3]);
    s_last[t] = last;
    const int i = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
    const int j = (bi.ty << lth) + (t >> P.ltw);
    if (!INC && k > 0) {  // texels with fragments lie inside the layer
      const size_t o = (size_t(P.view[bi.v].lout[bi.L]) + size_t(j) * bi.WL + i) * D;
#pragma unroll
      for (int d = 0; d < D; ++d) s_G[t][d] = gpyr[o + d];
    }
  }
  __syncthreads();
  for (uint32_t e = e0 + t; e < e1; e += EB * TP) {
    Entry en[EB];
    bool valid[EB];
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      en[q] = nx[q];
      valid[q] = e + q * TP < e1;
      if (e + (EB + q) * TP < e1) nx[q] = ent[e + (EB + q) * TP];  // next round of entries
    }
    // find the kept slot of every corner, then gather the blend adjoints of all of them
    Corner cs[EB][4];
    uint32_t cm[EB];
    size_t pos[EB][4];
#pragma unroll
    for (int h = 0; h < EB; ++h) {
      cm[h] = valid[h] ? entry_corners(en[h], bi, P.ltw, cs[h]) : 0u;
      const uint64_t key = (uint64_t(en[h].zbits) << 32) | en[h].idx;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pos[h][q] = 0;
        if (!((cm[h] >> q) & 1u)) continue;
        const int p = cs[h][q].p;
        const uint32_t kp = s_k[p];
        uint32_t m = kp;
        if (kp != 0 && !(key > s_last[p])) {  // among the kept fragments: find its position
#pragma unroll
          for (int j = 0; j < KEEP / 4; ++j) {
            const uint4 v = s_idx[j][p];
            m = (v.x == en[h].idx && uint32_t(4 * j) < kp) ? uint32_t(4 * j) : m;
            m = (v.y == en[h].idx && uint32_t(4 * j + 1) < kp) ? uint32_t(4 * j + 1) : m;
            m = (v.z == en[h].idx && uint32_t(4 * j + 2) < kp) ? uint32_t(4 * j + 2) : m;
            m = (v.w == en[h].idx && uint32_t(4 * j + 3) < kp) ? uint32_t(4 * j + 3) : m;
          }
        }
        if (m == kp) cm[h] &= ~(1u << q);
        else pos[h][q] = INC ? (size_t(b) * KEEP + m) * S * TP + uint32_t(p)
                             : (size_t(b) * KEEP + m) * TP + uint32_t(p);
      }
    }
    float2 st[EB][4];
    float itau[INC ? EB : 1][4][INC ? D : 1];
#pragma unroll
    for (int h = 0; h < EB; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool on = (cm[h] >> q) & 1u;
        if (INC) {
          st[h][q] = make_float2(on ? itot[pos[h][q]] : 0.0f, 0.0f);
#pragma unroll
          for (int d = 0; d < D; ++d)
            itau[INC ? h : 0][q][INC ? d : 0] = on ? itot[pos[h][q] + size_t(1 + d) * TP] : 0.0f;
        } else {
          st[h][q] = on ? bst[pos[h][q]] : make_float2(0.f, 0.f);
        }
      }
#pragma unroll
    for (int h = 0; h < EB; ++h) {
      if (!valid[h]) continue;
      float A = 0.0f, Bx = 0.0f, By = 0.0f;
      float tau[D];
#pragma unroll
      for (int d = 0; d < D; ++d) tau[d] = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!((cm[h] >> q) & 1u)) continue;
        const int p = cs[h][q].p;
        const float dg = st[h][q].x;
        A += dg * (cs[h][q].wx * cs[h][q].wy);
        Bx += dg * (cs[h][q].sx * cs[h][q].wy);
        By += dg * (cs[h][q].wx * cs[h][q].sy);
#pragma unroll
        for (int d = 0; d < D; ++d) tau[d] += INC ? itau[INC ? h : 0][q][INC ? d : 0] : st[h][q].y * s_G[p][d];
      }
      float* r = rows + size_t(e + h * TP) * RW;  // rows in entry order
      float4* r4 = reinterpret_cast<float4*>(r);
      r4[0] = make_float4(A, Bx, By, 0.0f);
#pragma unroll
      for (int q = 0; q < D / 4; ++q)
        r4[1 + q] = make_float4(tau[4 * q], tau[4 * q + 1], tau[4 * q + 2], tau[4 * q + 3]);
    }
  }
}

// bwd_fine: the backward of fine tiles, one workgroup per tile and one entry per thread.
// The kept slot of every corner was recorded by the forward pass, so the kept lists are
// rebuilt in LDS from the entries themselves (compact: texel t's list starts at s_off[t]);
// each texel's thread runs the blend adjoint (as bwd_pixels does) and every entry then
// writes its row (as bwd_items does).
template <int D>
__global__ __launch_bounds__(256) void k_bwd_fine(
    const Params P, const uint32_t* __restrict__ info, const uint4* __restrict__ fine_work,
    const Entry* __restrict__ ent, const uint32_t* __restrict__ kslot,
    const uint32_t* __restrict__ npix, const float* __restrict__ desc,
    const float* __restrict__ gpyr, float* __restrict__ rows, const Extras X) {
  constexpr int RW = 4 + D;
  constexpr int NF = 4 * FINE_E;  // at most one kept fragment per fragment
  __shared__ float s_G[TP][D + 1];
  __shared__ uint32_t s_off[TP];
  __shared__ uint32_t ws[4];
  __shared__ float s_gam[NF];
  __shared__ uint8_t s_ent[NF];
  __shared__ float2 s_bst[NF];
  __shared__ float4 s_desc[FINE_E][D / 4];
  const int t = threadIdx.x;
  const uint4 wk = fine_work[blockIdx.x];  // in bounds (grid = bin count); used only if valid
  if (blockIdx.x >= info[4]) return;
  const uint32_t b = wk.x, e0 = wk.y, e1 = wk.z;
  const BinInfo bi = decode_bin(P, b);
  if (e0 == e1) {  // an empty tile (uniform): only the background gradient, T G with T = 1
    if (X.gbg) {
      const int lth = 8 - P.ltw;
      const int ti = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
      const int tj = (bi.ty << lth) + (t >> P.ltw);
      if (ti < bi.WL && tj < bi.HL) {
        const size_t tex = size_t(P.view[bi.v].lout[bi.L]) + size_t(tj) * bi.WL + ti;
        float G[D];
#pragma unroll
        for (int d = 0; d < D; ++d) G[d] = gpyr[tex * D + d];
        write_scaled<D>(X.gbg + tex * D, 1.0f, G);
      }
    }
    return;
  }
  const bool has = e0 + uint32_t(t) < e1;
  Entry en = {};
  uint32_t packed = 0;  // kept slots of the entry's corners, as the forward pass recorded them
  if (has) {
    en = ent[e0 + t];
    packed = kslot[size_t(blockIdx.x) * TP + t];
  }
  const uint32_t k = min(npix[size_t(b) * TP + t], uint32_t(KEEP));
  // upstream gradient of the tile's texels inside the layer
  const int lth = 8 - P.ltw;
  const int ti = (bi.tx << P.ltw) + (t & ((1 << P.ltw) - 1));
  const int tj = (bi.ty << lth) + (t >> P.ltw);
  const bool inl = ti < bi.WL && tj < bi.HL;
  const size_t tex = size_t(P.view[bi.v].lout[bi.L]) + size_t(tj) * bi.WL + ti;
  if (inl) {
#pragma unroll
    for (int d = 0; d < D; ++d) s_G[t][d] = gpyr[tex * D + d];
  }
  float4 dv[D / 4];
#pragma unroll
  for (int r4 = 0; r4 < D / 4; ++r4) dv[r4] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (has) {
    const float4* dp = reinterpret_cast<const float4*>(desc + size_t(en.idx) * D);
#pragma unroll
    for (int r4 = 0; r4 < D / 4; ++r4) dv[r4] = dp[r4];
  }
  uint32_t kt;
  s_off[t] = block_excl_scan<4>(k, ws, kt);
#pragma unroll
  for (int r4 = 0; r4 < D / 4; ++r4) s_desc[t][r4] = dv[r4];
  __syncthreads();
  Corner cs[4];
  uint32_t cm = has ? entry_corners(en, bi, P.ltw, cs) : 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t m = (packed >> (5 * q)) & 31u;
    if (((cm >> q) & 1u) && m < KEEP) {
      const uint32_t o = s_off[cs[q].p] + m;
      s_gam[o] = (cs[q].wx * cs[q].wy) * en.ia;
      s_ent[o] = uint8_t(t);
    } else {
      cm &= ~(1u << q);
    }
  }
  __syncthreads();
  if (inl && (k > 0 || X.gbg)) {  // blend adjoint of texel t (as in bwd_pixels)
    const uint32_t o0 = s_off[t];
    float G[D];
#pragma unroll
    for (int d = 0; d < D; ++d) G[d] = s_G[t][d];
    const float ga = X.galpha ? X.galpha[tex] : 0.0f;
    float T = 1.0f;
    for (uint32_t m = 0; m < k; ++m) {  // front to back: T_m and g_m
      float4 tv[D / 4];
#pragma unroll
      for (int r4 = 0; r4 < D / 4; ++r4) tv[r4] = s_desc[s_ent[o0 + m]][r4];
      float gm = dot_g<D>(G, tv);
      if (X.galpha) gm += ga;
      s_bst[o0 + m] = make_float2(gm, T);
      T = T * (1.0f - s_gam[o0 + m]);
    }
    float B = X.bg ? dot_g<D>(G, *reinterpret_cast<const float4(*)[D / 4]>(X.bg + tex * D)) : 0.0f;
    for (uint32_t m = k; m-- > 0;) {  // back to front
      const float2 gt = s_bst[o0 + m];
      s_bst[o0 + m] = blend_adjoint_step(gt.y, s_gam[o0 + m], gt.x, B);
    }
    if (X.gbg) write_scaled<D>(X.gbg + tex * D, T, G);
  }
  __syncthreads();
  if (!has) return;
  float2 st[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    st[q] = ((cm >> q) & 1u) ? s_bst[s_off[cs[q].p] + ((packed >> (5 * q)) & 31u)] : make_float2(0.f, 0.f);
  float A = 0.0f, Bx = 0.0f, By = 0.0f;
  float tau[D];
#pragma unroll
  for (int d = 0; d < D; ++d) tau[d] = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!((cm >> q) & 1u)) continue;
    const int p = cs[q].p;
    const float dg = st[q].x;
    A += dg * (cs[q].wx * cs[q].wy);
    Bx += dg * (cs[q].sx * cs[q].wy);
    By += dg * (cs[q].wx * cs[q].sy);
#pragma unroll
    for (int d = 0; d < D; ++d) tau[d] += st[q].y * s_G[p][d];
  }
  float* r = rows + size_t(e0 + t) * RW;  // rows in entry order
  float4* r4 = reinterpret_cast<float4*>(r);
  r4[0] = make_float4(A, Bx, By, 0.0f);
#pragma unroll
  for (int q = 0; q < D / 4; ++q)
    r4[1 + q] = make_float4(tau[4 * q], tau[4 * q + 1], tau[4 * q + 2], tau[4 * q + 3]);
}

// Sum of v over the 64 lanes of a wavefront (a fixed butterfly, so the order never changes).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// ------------------------------------------------------------------------------------
// Coarser-layer inclusion (Sec. 3.6).  The list blended at texel (i, j) of layer L is the
// texel's own kept list merged with the blended list of the covering texel (i/2, j/2) of
// layer L + 1, which by induction holds the fragments of every coarser layer: the 16
// smallest of a union are the 16 smallest of the union of the parts' 16 smallest.  The
// merge is stable and takes the own fragment first on equal keys (a point written to two
// layers meets itself; the finer layer comes first), so the order inside the covering
// list is kept.  Per texel the blended list is saved as fkey / fgam and
// fcnt = own count | coarser count << 5 | (bit m: item m came from the coarser list) << 16;
// the items taken from either side are a prefix of that side.

// Tile and texel slot of texel (i, j) of layer L of view v.
__device__ __forceinline__ void texel_bin(const Params& P, int v, int L, int i, int j,
                                          uint32_t& b, int& t) {
  const int lth = 8 - P.ltw;
  const int WL = layer_dim(P.view[v].W, L);
  const int tiles_x = (WL + (1 << P.ltw) - 1) >> P.ltw;
  b = P.view[v].lbin[L] + uint32_t((j >> lth) * tiles_x + (i >> P.ltw));
  t = ((j & ((1 << lth) - 1)) << P.ltw) | (i & ((1 << P.ltw) - 1));
}

constexpr int PT = TP / 4;  // covering texels of one tile in the next coarser layer

// incl_fwd: one launch per layer, coarsest first; one workgroup per tile of the layer
// (grid.y = view).  The coarsest layer's blended list is its own (copied); every finer
// texel merges its own list (staged in LDS) with its covering texel's blended list
// (the tile's 64 covering texels staged in LDS), blends the result (Eq. 6-7) and rewrites
// its outputs.
template <int D>
__global__ __launch_bounds__(256) void k_incl_fwd(
    const Params P, int L, const uint32_t* __restrict__ npix, const uint64_t* __restrict__ kkey,
    const float* __restrict__ kgam, uint64_t* __restrict__ fkey, float* __restrict__ fgam,
    uint32_t* __restrict__ fcnt, const float* __restrict__ desc, float* __restrict__ pyr,
    const float* __restrict__ bg, float* __restrict__ alpha) {
  __shared__ uint64_t s_ok[KEEP][TP];
  __shared__ float s_og[KEEP][TP];
  __shared__ uint64_t s_pk[KEEP][PT];
  __shared__ float s_pg[KEEP][PT];
  __shared__ uint32_t s_pn[PT];
  const int v = blockIdx.y;
  const ViewP& c = P.view[v];
  const int t = threadIdx.x;
  const int lth = 8 - P.ltw;
  const int WL = layer_dim(c.W, L), HL = layer_dim(c.H, L);
  const int tiles_x = (WL + (1 << P.ltw) - 1) >> P.ltw, tiles_y = (HL + (1 << lth) - 1) >> lth;
  int tx, ty;  // the four tiles under one covering tile on one die
  if (!quad_tile(blockIdx.x, tiles_x, tiles_y, tx, ty)) return;  // uniform per workgroup
  const uint32_t b = c.lbin[L] + uint32_t(ty * tiles_x + tx);
  const int i = (tx << P.ltw) + (t & ((1 << P.ltw) - 1));
  const int j = (ty << lth) + (t >> P.ltw);
  const bool in = i < WL && j < HL;
  const size_t tb = size_t(b) * KEEP;
  const uint32_t ko = in ? min(npix[size_t(b) * TP + t], uint32_t(KEEP)) : 0u;
  if (L == P.nl - 1) {  // uniform: the coarsest layer blends its own list (already written)
    uint64_t ck[KEEP];
    float cg[KEEP];
#pragma unroll
    for (int m = 0; m < KEEP; ++m) {
      ck[m] = kkey[(tb + m) * TP + t];
      cg[m] = kgam[(tb + m) * TP + t];
    }
#pragma unroll
    for (int m = 0; m < KEEP; ++m)
      if (uint32_t(m) < ko) {
        fkey[(tb + m) * TP + t] = ck[m];
        fgam[(tb + m) * TP + t] = cg[m];
      }
    fcnt[size_t(b) * TP + t] = ko;
    return;
  }
  // slots are staged whatever the list length (stale values past it are never read), so
  // their loads do not wait on one another: all 16 in the coarser layers, the first four in
  // the two finest (longer own lists are rare there and load the rest)
#pragma unroll
  for (int m = 0; m < KEEP; ++m) {
    if (m < 4 || L >= 2 || uint32_t(m) < ko) {
      s_ok[m][t] = kkey[(tb + m) * TP + t];
      s_og[m][t] = kgam[(tb + m) * TP + t];
    }
  }
  {  // the covering texels: (tw/2) x (th/2) texels of one tile of layer L + 1
    const int hw = 1 << (P.ltw - 1);
    const int q = t & (PT - 1), g = t >> 6;  // texel q, slots g, g+4, g+8, g+12
    const int pi = (tx << (P.ltw - 1)) + (q & (hw - 1));
    const int pj = (ty << (lth - 1)) + (q >> (P.ltw - 1));
    const bool pin = pi < layer_dim(c.W, L + 1) && pj < layer_dim(c.H, L + 1);
    uint32_t pb = 0;
    int pt = 0;
    if (pin) texel_bin(P, v, L + 1, pi, pj, pb, pt);
    const uint32_t pc = pin ? fcnt[size_t(pb) * TP + pt] : 0u;
    const uint32_t kp = (pc & 31u) + ((pc >> 5) & 31u);
    if (g == 0) s_pn[q] = kp;
#pragma unroll
    for (int r = 0; r < KEEP / 4; ++r) {  // slots past kp read slot 0 again (a cache hit)
      const uint32_t m = uint32_t(g + 4 * r);
      const size_t ms = m < kp ? m : 0u;
      s_pk[m][q] = fkey[(size_t(pb) * KEEP + ms) * TP + pt];
      s_pg[m][q] = fgam[(size_t(pb) * KEEP + ms) * TP + pt];
    }
  }
  __syncthreads();
  if (!in) return;  // (no later barrier)
  const int hw = 1 << (P.ltw - 1);
  const int q = ((j >> 1) & ((1 << (lth - 1)) - 1)) * hw + ((i >> 1) & (hw - 1));
  const uint32_t kp = s_pn[q];
  // stable merge of the two sorted lists, own first on equal keys
  uint32_t io = 0, ip = 0, mask = 0;
  uint64_t fk[KEEP];
  float fg[KEEP];
#pragma unroll
  for (int m = 0; m < KEEP; ++m) {
    const uint64_t ok = io < ko ? s_ok[min(io, uint32_t(KEEP - 1))][t] : KEY_NONE;
    const uint64_t pk = ip < kp ? s_pk[min(ip, uint32_t(KEEP - 1))][q] : KEY_NONE;
    const bool take_o = io < ko && !(pk < ok);
    const bool take_p = !take_o && ip < kp;
    fk[m] = take_o ? ok : (take_p ? pk : KEY_NONE);
    fg[m] = take_o ? s_og[min(io, uint32_t(KEEP - 1))][t]
                   : (take_p ? s_pg[min(ip, uint32_t(KEEP - 1))][q] : 0.0f);
    mask |= (take_p ? 1u : 0u) << m;
    io += take_o ? 1u : 0u;
    ip += take_p ? 1u : 0u;
  }
  const uint32_t k = io + ip;
  float C[D];
#pragma unroll
  for (int d = 0; d < D; ++d) C[d] = 0.0f;
  float T = 1.0f;
  constexpr int GB = D > 4 ? 4 : 8;
  // without points every list is empty and there is no point 0 to read (uniform branch)
  if (P.n > 0) {
#pragma unroll
  for (int m0 = 0; m0 < KEEP; m0 += GB) {
    // a batch of descriptor gathers, all issued before use (an empty slot reads point 0)
    float4 tv[GB][D / 4];
#pragma unroll
    for (int r = 0; r < GB; ++r) {
      const int m = m0 + r;
      const uint32_t id = uint32_t(m) < k ? uint32_t(fk[m]) : 0u;
      const float4* tp = reinterpret_cast<const float4*>(desc + size_t(id) * D);
#pragma unroll
      for (int e = 0; e < D / 4; ++e) tv[r][e] = tp[e];
    }
#pragma unroll
    for (int r = 0; r < GB; ++r) {
      const int m = m0 + r;
      if (uint32_t(m) < k) {
        const float w = T * fg[m];
#pragma unroll
        for (int e = 0; e < D / 4; ++e) {
          C[4 * e + 0] += w * tv[r][e].x;
          C[4 * e + 1] += w * tv[r][e].y;
          C[4 * e + 2] += w * tv[r][e].z;
          C[4 * e + 3] += w * tv[r][e].w;
        }
        T = T * (1.0f - fg[m]);
      }
    }
  }
  }
  // layer 0's list is rebuilt where it is read (own list, covering list, origin mask): no
  // finer layer merges it, and it is the largest layer
  if (L > 0) {
#pragma unroll
    for (int m = 0; m < KEEP; ++m)
      if (uint32_t(m) < k) {
        fkey[(tb + m) * TP + t] = fk[m];
        fgam[(tb + m) * TP + t] = fg[m];
      }
  }
  fcnt[size_t(b) * TP + t] = io | (ip << 5) | (mask << 16);
  write_texel<D>(C, T, size_t(c.lout[L]) + size_t(j) * WL + i, pyr, bg, alpha);
}

// incl_fwd_group: layers Lb..Lt in one launch, Lt - Lb at most log2 of the tile's shorter
// side; one workgroup per tile of layer Lb (grid.y = view).  The texels of layer Lb + k over
// that tile form a (tw >> k) x (th >> k) block that lies over no other tile of layer Lb, so
// the workgroup runs the layers itself, coarsest first, with a barrier between layers: each
// layer merges and blends exactly as k_incl_fwd does, stores its blended lists, and hands
// them to the next finer layer through LDS.  Layer Lt reads its covering lists (layer Lt + 1,
// an earlier launch) from memory; the coarsest layer of the pyramid keeps its own lists.
template <int D>
__global__ __launch_bounds__(256) void k_incl_fwd_group(
    const Params P, int Lb, int Lt, const uint32_t* __restrict__ npix,
    const uint64_t* __restrict__ kkey, const float* __restrict__ kgam, uint64_t* __restrict__ fkey,
    float* __restrict__ fgam, uint32_t* __restrict__ fcnt, const float* __restrict__ desc,
    float* __restrict__ pyr, const float* __restrict__ bg, float* __restrict__ alpha) {
  __shared__ uint64_t s_k[2][KEEP][PT];  // blended lists of a layer's block, for the next layer
  __shared__ float s_g[2][KEEP][PT];
  __shared__ uint32_t s_n[2][PT];
  const int v = blockIdx.y;
  const ViewP& c = P.view[v];
  const uint32_t local = blockIdx.x;
  if (local >= c.lbin[Lb + 1] - c.lbin[Lb]) return;  // uniform per workgroup
  const int t = threadIdx.x;
  const int ltw = P.ltw, lth = 8 - P.ltw;
  const int tiles_x = (layer_dim(c.W, Lb) + (1 << ltw) - 1) >> ltw;
  const int ty = int(local) / tiles_x, tx = int(local) - ty * tiles_x;
  for (int L = Lt; L >= Lb; --L) {
    const int k = L - Lb;
    const int rw = (1 << ltw) >> k, rh = (1 << lth) >> k;  // this layer's block
    const int cur = k & 1, prev = cur ^ 1;  // LDS lists written here / by layer L + 1
    if (t < rw * rh) {
      const int i = tx * rw + t % rw, j = ty * rh + t / rw;
      const int WL = layer_dim(c.W, L), HL = layer_dim(c.H, L);
      uint32_t kout = 0;
      uint64_t fk[KEEP];
      float fg[KEEP];
      if (i < WL && j < HL) {
        uint32_t b;
        int tt;
        texel_bin(P, v, L, i, j, b, tt);
        const size_t tb = size_t(b) * KEEP;
        const uint32_t ko = min(npix[size_t(b) * TP + tt], uint32_t(KEEP));
        uint64_t ok[KEEP];
        float og[KEEP];
#pragma unroll
        for (int m = 0; m < KEEP; ++m) {  // every slot read (those past ko read slot 0 again, a
          const size_t ms = uint32_t(m) < ko ? m : 0;  // cache hit) and left unused
          ok[m] = kkey[(tb + ms) * TP + tt];
          og[m] = kgam[(tb + ms) * TP + tt];
        }
        if (L == P.nl - 1) {  // the coarsest layer keeps its own lists (already blended)
#pragma unroll
          for (int m = 0; m < KEEP; ++m) {
            fk[m] = uint32_t(m) < ko ? ok[m] : KEY_NONE;
            fg[m] = uint32_t(m) < ko ? og[m] : 0.0f;
            if (uint32_t(m) < ko) {
              fkey[(tb + m) * TP + tt] = ok[m];
              fgam[(tb + m) * TP + tt] = og[m];
            }
          }
          fcnt[size_t(b) * TP + tt] = ko;
          kout = ko;
        } else {
          uint64_t pk[KEEP];
          float pg[KEEP];
          uint32_t kp = 0;
          if (L == Lt) {  // covering lists of an earlier launch
            const int pi = i >> 1, pj = j >> 1;
            uint32_t pb = 0;
            int pt = 0;
            const bool pin = pi < layer_dim(c.W, L + 1) && pj < layer_dim(c.H, L + 1);
            if (pin) texel_bin(P, v, L + 1, pi, pj, pb, pt);
            const uint32_t pc = pin ? fcnt[size_t(pb) * TP + pt] : 0u;
            kp = (pc & 31u) + ((pc >> 5) & 31u);
#pragma unroll
            for (int m = 0; m < KEEP; ++m) {  // (past kp: slot 0 again, unused)
              const size_t ms = uint32_t(m) < kp ? m : 0;
              pk[m] = fkey[(size_t(pb) * KEEP + ms) * TP + pt];
              pg[m] = fgam[(size_t(pb) * KEEP + ms) * TP + pt];
            }
          } else {  // the block of layer L + 1 above, from LDS
            const int q = ((j >> 1) - ty * (rh >> 1)) * (rw >> 1) + ((i >> 1) - tx * (rw >> 1));
            kp = s_n[prev][q];
#pragma unroll
            for (int m = 0; m < KEEP; ++m) {
              pk[m] = s_k[prev][m][q];
              pg[m] = s_g[prev][m][q];
            }
          }
          // stable merge of the two sorted lists, own first on equal keys
          uint32_t io = 0, ip = 0, mask = 0;
#pragma unroll
          for (int m = 0; m < KEEP; ++m) {
            uint64_t okm = KEY_NONE, pkm = KEY_NONE;
            float ogm = 0.0f, pgm = 0.0f;
#pragma unroll
            for (int r = 0; r < KEEP; ++r) {  // register lists: select slots io and ip
              okm = uint32_t(r) == io ? ok[r] : okm;
              ogm = uint32_t(r) == io ? og[r] : ogm;
              pkm = uint32_t(r) == ip ? pk[r] : pkm;
              pgm = uint32_t(r) == ip ? pg[r] : pgm;
            }
            const uint64_t okv = io < ko ? okm : KEY_NONE;
            const uint64_t pkv = ip < kp ? pkm : KEY_NONE;
            const bool take_o = io < ko && !(pkv < okv);
            const bool take_p = !take_o && ip < kp;
            fk[m] = take_o ? okv : (take_p ? pkv : KEY_NONE);
            fg[m] = take_o ? ogm : (take_p ? pgm : 0.0f);
            mask |= (take_p ? 1u : 0u) << m;
            io += take_o ? 1u : 0u;
            ip += take_p ? 1u : 0u;
          }
          kout = io + ip;
          float C[D];
#pragma unroll
          for (int d = 0; d < D; ++d) C[d] = 0.0f;
          float T = 1.0f;
          constexpr int GB = D > 4 ? 4 : 8;
          if (P.n > 0) {  // without points every list is empty and there is no point 0
#pragma unroll
            for (int m0 = 0; m0 < KEEP; m0 += GB) {
              float4 tv[GB][D / 4];
#pragma unroll
              for (int r = 0; r < GB; ++r) {
                const int m = m0 + r;
                const uint32_t id = uint32_t(m) < kout ? uint32_t(fk[m]) : 0u;
                const float4* tp = reinterpret_cast<const float4*>(desc + size_t(id) * D);
#pragma unroll
                for (int e = 0; e < D / 4; ++e) tv[r][e] = tp[e];
              }
#pragma unroll
              for (int r = 0; r < GB; ++r) {
                const int m = m0 + r;
                if (uint32_t(m) < kout) {
                  const float w = T * fg[m];
#pragma unroll
                  for (int e = 0; e < D / 4; ++e) {
                    C[4 * e + 0] += w * tv[r][e].x;
                    C[4 * e + 1] += w * tv[r][e].y;
                    C[4 * e + 2] += w * tv[r][e].z;
                    C[4 * e + 3] += w * tv[r][e].w;
                  }
                  T = T * (1.0f - fg[m]);
                }
              }
            }
          }
          if (L > 0) {  // (layer 0's lists are rebuilt where they are read)
#pragma unroll
            for (int m = 0; m < KEEP; ++m)
              if (uint32_t(m) < kout) {
                fkey[(tb + m) * TP + tt] = fk[m];
                fgam[(tb + m) * TP + tt] = fg[m];
              }
          }
          fcnt[size_t(b) * TP + tt] = io | (ip << 5) | (mask << 16);
          write_texel<D>(C, T, size_t(c.lout[L]) + size_t(j) * WL + i, pyr, bg, alpha);
        }
      }
      if (k > 0) {  // the next finer layer reads this block's lists
#pragma unroll
        for (int m = 0; m < KEEP; ++m) {
          s_k[cur][m][t] = uint32_t(m) < kout ? fk[m] : KEY_NONE;
          s_g[cur][m][t] = uint32_t(m) < kout ? fg[m] : 0.0f;
        }
        s_n[cur][t] = kout;
      }
    }
    __syncthreads();
  }
}

// Slot m of the blended list of texel (b, t), as the forward pass made it: stored in fkey /
// fgam, or (layer 0 below a coarser layer, whose lists are not stored) rebuilt from the own
// list (kkey / kgam of the texel) and the covering texel's stored list (pb, pt): by the
// origin mask, slot m is the covering list's item popc(mask below m), else the own list's
// item m minus that.  Every address is in bounds whatever m.
struct BlendedSrc {
  const uint64_t* fkey;
  const float* fgam;
  const uint64_t* kkey;  // null: the list is stored
  const float* kgam;
  uint32_t pb;
  int pt;
};
// REBUILT is known at compile time, so every slot is one unconditional load from a selected
// address (a load under a branch would wait on its own).
template <bool REBUILT>
__device__ __forceinline__ void blended_slot(const BlendedSrc& S, uint32_t b, int t, uint32_t fc,
                                             int m, uint64_t& key, float& gam) {
  if (!REBUILT) {
    const size_t o = (size_t(b) * KEEP + m) * TP + t;
    key = S.fkey[o];
    gam = S.fgam[o];
    return;
  }
  const uint32_t mask = fc >> 16;
  const uint32_t ip = __popc(mask & ((1u << m) - 1u));
  const bool up = (mask >> m) & 1u;
  const size_t o = up ? (size_t(S.pb) * KEEP + ip) * TP + S.pt
                      : (size_t(b) * KEEP + (uint32_t(m) - ip)) * TP + t;
  const uint64_t* kp = up ? S.fkey : S.kkey;
  const float* gp = up ? S.fgam : S.kgam;
  key = kp[o];
  gam = gp[o];
}

// Blend adjoint of the blended list of one texel (tile b, slot t, pyramid texel tex; fc its
// count word): G, and per item m < k dg[m] = dL/dgamma_m and tg[m] = T_m gamma_m (zero past
// k); writes the background gradient.  Returns k.  has_points: the cloud is not empty (an
// empty slot then reads point 0's descriptor, which exists).
template <int D, bool REBUILT>
__device__ __forceinline__ uint32_t blended_adjoint(const BlendedSrc& S, uint32_t b,
                                                    int t, uint32_t fc, size_t tex, bool has_points,
                                                    const float* __restrict__ desc,
                                                    const float* __restrict__ gpyr, const Extras& X,
                                                    float (&G)[D], float (&dg)[KEEP],
                                                    float (&tg)[KEEP]) {
  const uint32_t k = (fc & 31u) + ((fc >> 5) & 31u);
  {
    const float4* gp = reinterpret_cast<const float4*>(gpyr + tex * D);
#pragma unroll
    for (int q = 0; q < D / 4; ++q) {
      const float4 gv = gp[q];
      G[4 * q] = gv.x; G[4 * q + 1] = gv.y; G[4 * q + 2] = gv.z; G[4 * q + 3] = gv.w;
    }
  }
  float gam[KEEP], Tm[KEEP], gm[KEEP];
  uint32_t idx[KEEP];
#pragma unroll
  for (int m = 0; m < KEEP; ++m) {  // every slot is read: those past k read slot 0 again (a
    uint64_t kr;                    // cache hit, not a row of memory) and are dropped
    float gr;
    blended_slot<REBUILT>(S, b, t, fc, uint32_t(m) < k ? m : 0, kr, gr);
    const bool ok = uint32_t(m) < k;
    idx[m] = ok ? uint32_t(kr) : 0u;
    gam[m] = ok ? gr : 0.0f;
  }
  float T = 1.0f;
#pragma unroll
  for (int m = 0; m < KEEP; ++m) {
    Tm[m] = T;
    if (uint32_t(m) < k) T = T * (1.0f - gam[m]);
  }
  constexpr int GB = D > 4 ? 4 : 8;
#pragma unroll
  for (int m = 0; m < KEEP; ++m) gm[m] = 0.0f;
  if (has_points) {  // uniform; without points k is 0
#pragma unroll
    for (int m0 = 0; m0 < KEEP; m0 += GB) {
      float4 tv[GB][D / 4];  // empty slots read point 0 and are dropped
#pragma unroll
      for (int q = 0; q < GB; ++q) {
        const float4* tp = reinterpret_cast<const float4*>(desc + size_t(idx[m0 + q]) * D);
#pragma unroll
        for (int r = 0; r < D / 4; ++r) tv[q][r] = tp[r];
      }
#pragma unroll
      for (int q = 0; q < GB; ++q) gm[m0 + q] = dot_g<D>(G, tv[q]);
    }
  }
  if (X.galpha) {
    const float ga = X.galpha[tex];
#pragma unroll
    for (int m = 0; m < KEEP; ++m) gm[m] += ga;
  }
  float B = X.bg ? dot_g<D>(G, *reinterpret_cast<const float4(*)[D / 4]>(X.bg + tex * D)) : 0.0f;
#pragma unroll
  for (int m = KEEP - 1; m >= 0; --m) {
    dg[m] = 0.0f; tg[m] = 0.0f;
    if (uint32_t(m) < k) {
      const float2 st = blend_adjoint_step(Tm[m], gam[m], gm[m], B);
      dg[m] = st.x; tg[m] = st.y;
    }
  }
  if (X.gbg) write_scaled<D>(X.gbg + tex * D, T, G);
  return k;
}

// incl_bwd: one launch per layer, finest first; four threads per texel, a quarter of a tile
// (64 texels) per workgroup (grid.x = 4 x the layer's tiles, grid.y = view).  All four
// threads of a texel run the blend adjoint of its blended list (as bwd_pixels; their loads
// are the same addresses, merged by the memory system), which gives every item dL/dgamma
// and T gamma G; thread g then completes items g, g + 4, g + 8 and g + 12: the blend part,
// then what each of the four finer texels the texel covers passed up for the item, in
// child order.  Each item's total goes to the own slot it came from (itot, read by the rows
// of the entries) or, for items of the coarser list, up to the covering texel (iup, read by
// the next launch).  Per slot the D + 1 values are (dL/dgamma, dL/dtau contribution [D]),
// each row of 256 texels contiguous.
constexpr int INCL_LANES = 4;  // threads per texel in incl_bwd
template <int D>
__global__ __launch_bounds__(256) void k_incl_bwd(
    const Params P, int L, const uint64_t* __restrict__ fkey, const float* __restrict__ fgam,
    const uint32_t* __restrict__ fcnt, const float* __restrict__ desc,
    const float* __restrict__ gpyr, float* __restrict__ itot, const float* __restrict__ iup_in,
    float* __restrict__ iup_out, const Extras X) {
  // iup_in and iup_out are the same table: this launch reads the rows of layer L - 1 and
  // writes those of layer L, which never overlap
  constexpr int S = D + 1;
  constexpr int NH = KEEP / INCL_LANES;  // items per thread
  const int v = blockIdx.y;
  const ViewP& c = P.view[v];
  const uint32_t local = blockIdx.x / INCL_LANES;
  if (local >= c.lbin[L + 1] - c.lbin[L]) return;
  const uint32_t b = c.lbin[L] + local;
  const int g = threadIdx.x % INCL_LANES;
  const int t = int(blockIdx.x % INCL_LANES) * (TP / INCL_LANES) + int(threadIdx.x) / INCL_LANES;
  const int lth = 8 - P.ltw;
  const int WL = layer_dim(c.W, L), HL = layer_dim(c.H, L);
  const int tiles_x = (WL + (1 << P.ltw) - 1) >> P.ltw;
  const int ty = int(local) / tiles_x, tx = int(local) - ty * tiles_x;
  const int i = (tx << P.ltw) + (t & ((1 << P.ltw) - 1));
  const int j = (ty << lth) + (t >> P.ltw);
  if (!(i < WL && j < HL)) return;
  const size_t tb = size_t(b) * KEEP;
  const uint32_t fc = fcnt[size_t(b) * TP + t];
  const uint32_t mask = fc >> 16;
  const size_t tex = size_t(c.lout[L]) + size_t(j) * WL + i;
  // the finer texels this texel covers, and how many of its items each of them took
  size_t cbase[4];
  uint32_t cup[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cbase[q] = 0; cup[q] = 0;
    if (L > 0) {
      const int ci = 2 * i + (q & 1), cj = 2 * j + (q >> 1);
      if (ci < layer_dim(c.W, L - 1) && cj < layer_dim(c.H, L - 1)) {
        uint32_t cb;
        int ct;
        texel_bin(P, v, L - 1, ci, cj, cb, ct);
        cup[q] = (fcnt[size_t(cb) * TP + ct] >> 5) & 31u;
        cbase[q] = size_t(cb) * KEEP * S * TP + size_t(ct);
      }
    }
  }
  float tot[NH][S];
  uint32_t k;
  {
    Extras Xg = X;  // the background gradient is written by one thread of the four
    if (g != 0) Xg.gbg = nullptr;
    float G[D], dg[KEEP], tg[KEEP];
    const BlendedSrc src{fkey, fgam, nullptr, nullptr, 0u, 0};
    k = blended_adjoint<D, false>(src, b, t, fc, tex, P.n > 0, desc, gpyr, Xg, G, dg, tg);
    // this thread's items, selected without indexing registers by g
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int m0 = INCL_LANES * h;
      const float d0 = g == 0 ? dg[m0] : g == 1 ? dg[m0 + 1] : g == 2 ? dg[m0 + 2] : dg[m0 + 3];
      const float t0 = g == 0 ? tg[m0] : g == 1 ? tg[m0 + 1] : g == 2 ? tg[m0 + 2] : tg[m0 + 3];
      tot[h][0] = d0;
#pragma unroll
      for (int d = 0; d < D; ++d) tot[h][1 + d] = t0 * G[d];
    }
  }
  // what each finer texel passed up, in child order; every row is read (in bounds: a
  // missing child reads tile 0; an item the child did not take reads the child's slot 0,
  // which the cache holds) and used only for the items that child took
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float u[NH][S];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const uint32_t m = uint32_t(INCL_LANES * h + g);
      const size_t ms = m < cup[q] ? m : 0u;
#pragma unroll
      for (int r = 0; r < S; ++r) u[h][r] = iup_in[cbase[q] + (ms * S + r) * TP];
    }
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const bool take = uint32_t(INCL_LANES * h + g) < cup[q];
#pragma unroll
      for (int r = 0; r < S; ++r) tot[h][r] += take ? u[h][r] : 0.0f;
    }
  }
  // item m of the list is the popc(mask below m)-th item taken from the coarser list, or
  // the (m - that)-th own item
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const uint32_t m = uint32_t(INCL_LANES * h + g);
    if (m < k) {
      const bool up = (mask >> m) & 1u;
      const uint32_t sp = __popc(mask & ((1u << m) - 1u)), so = m - sp;
      float* dst = up ? iup_out + ((tb + sp) * S) * TP + t : itot + ((tb + so) * S) * TP + t;
#pragma unroll
      for (int r = 0; r < S; ++r) dst[size_t(r) * TP] = tot[h][r];
    }
  }
}

// incl_bwd_group: layers Lb..Lt in one launch (Lt - Lb at most log2 of the tile's shorter
// side), finest first, one workgroup per tile of layer Lb (grid.y = view); the texels of
// layer Lb + k over the tile form a (tw >> k) x (th >> k) block over no other tile.  Every
// texel's total per item is its own blend part, then what each of its four finer texels
// passed up, in child order (as k_incl_bwd): the own parts of the layers above Lb are put
// in LDS first; then, layer by layer, each texel completes its totals, writes its own
// items' totals to itot and adds its items of the coarser list to its covering texel's LDS
// totals, one child position at a time.  Layer Lb reads what layer Lb - 1 passed up from
// memory; layer Lt passes its coarser items up through memory (iup).
constexpr int GROUP_PARENTS = 64 + 16 + 4 + 1;  // texels of the layers above a 16x16 tile
template <int D>
__global__ __launch_bounds__(256, 1) void k_incl_bwd_group(
    const Params P, int Lb, int Lt, const uint64_t* __restrict__ fkey,
    const float* __restrict__ fgam, const uint32_t* __restrict__ fcnt,
    const float* __restrict__ desc, const float* __restrict__ gpyr, float* __restrict__ itot,
    float* __restrict__ iup, const Extras X) {
  constexpr int S = D + 1;
  __shared__ float s_tot[GROUP_PARENTS][KEEP][S];
  const int v = blockIdx.y;
  const ViewP& c = P.view[v];
  const uint32_t local = blockIdx.x;
  if (local >= c.lbin[Lb + 1] - c.lbin[Lb]) return;  // uniform per workgroup
  const int t = threadIdx.x;
  const int ltw = P.ltw, lth = 8 - P.ltw;
  const int tiles_x = (layer_dim(c.W, Lb) + (1 << ltw) - 1) >> ltw;
  const int ty = int(local) / tiles_x, tx = int(local) - ty * tiles_x;
  const BlendedSrc src{fkey, fgam, nullptr, nullptr, 0u, 0};
  // block k's first slot in s_tot (layer Lb + k, k >= 1): blocks of 64, 16, 4 and 1 texels
  auto slot0 = [](int k) { int o = 0; for (int q = 1; q < k; ++q) o += TP >> (2 * q); return o; };
  // texel q of this workgroup's block of layer Lb + k (false: outside the block or the layer)
  auto texel_at = [&](int k, int q, int& i, int& j, int& WL, int& HL) {
    const int rw = (1 << ltw) >> k, rh = (1 << lth) >> k;
    if (q >= rw * rh) return false;
    i = tx * rw + q % rw;
    j = ty * rh + q / rw;
    WL = layer_dim(c.W, Lb + k);
    HL = layer_dim(c.H, Lb + k);
    return i < WL && j < HL;
  };
  auto texel_of = [&](int k, int& i, int& j, int& WL, int& HL) {
    return texel_at(k, t, i, j, WL, HL);
  };
  // own parts of the layers above Lb, all at once: thread t takes slot t of s_tot (block k
  // of the slot, texel t - slot0(k) of it)
  if (t < slot0(Lt - Lb + 1)) {
    int k = 1;
    while (k < Lt - Lb && t >= slot0(k + 1)) ++k;
    int i, j, WL, HL;
    const bool in = texel_at(k, t - slot0(k), i, j, WL, HL);
    float (*tot)[S] = s_tot[t];
    float G[D], dg[KEEP], tg[KEEP];
#pragma unroll
    for (int d = 0; d < D; ++d) G[d] = 0.0f;
#pragma unroll
    for (int m = 0; m < KEEP; ++m) { dg[m] = 0.0f; tg[m] = 0.0f; }
    if (in) {
      uint32_t b;
      int tt;
      texel_bin(P, v, Lb + k, i, j, b, tt);
      const uint32_t fc = fcnt[size_t(b) * TP + tt];
      blended_adjoint<D, false>(src, b, tt, fc, size_t(c.lout[Lb + k]) + size_t(j) * WL + i, P.n > 0,
                         desc, gpyr, X, G, dg, tg);
    }
#pragma unroll
    for (int m = 0; m < KEEP; ++m) {
      tot[m][0] = dg[m];
#pragma unroll
      for (int d = 0; d < D; ++d) tot[m][1 + d] = tg[m] * G[d];
    }
  }
  __syncthreads();
  for (int k = 0; k <= Lt - Lb; ++k) {
    const int L = Lb + k;
    int i = 0, j = 0, WL = 0, HL = 0;
    const bool in = texel_of(k, i, j, WL, HL);
    float tot[KEEP][S];
    uint32_t kk = 0, mask = 0, b = 0;
    int tt = 0;
    if (in) {
      texel_bin(P, v, L, i, j, b, tt);
      const uint32_t fc = fcnt[size_t(b) * TP + tt];
      mask = fc >> 16;
      kk = (fc & 31u) + ((fc >> 5) & 31u);
      if (k == 0) {  // own part, then what layer L - 1 passed up (memory, an earlier launch)
        float G[D], dg[KEEP], tg[KEEP];
        blended_adjoint<D, false>(src, b, tt, fc, size_t(c.lout[L]) + size_t(j) * WL + i, P.n > 0, desc,
                           gpyr, X, G, dg, tg);
#pragma unroll
        for (int m = 0; m < KEEP; ++m) {
          tot[m][0] = dg[m];
#pragma unroll
          for (int d = 0; d < D; ++d) tot[m][1 + d] = tg[m] * G[d];
        }
        // the four finer texels (a missing one reads tile 0 and takes nothing), then their
        // rows, every load issued whatever it is used for
        size_t cbase[4];
        uint32_t cup[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ci = 2 * i + (q & 1), cj = 2 * j + (q >> 1);
          const bool cin = ci < layer_dim(c.W, L - 1) && cj < layer_dim(c.H, L - 1);
          uint32_t cb = 0;
          int ct = 0;
          if (cin) texel_bin(P, v, L - 1, ci, cj, cb, ct);
          cup[q] = cin ? (fcnt[size_t(cb) * TP + ct] >> 5) & 31u : 0u;
          cbase[q] = size_t(cb) * KEEP * S * TP + size_t(ct);
        }
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {  // one finer texel's rows in flight at a time
          float u[KEEP][S];  // (items the child did not take read its slot 0 again)
#pragma unroll
          for (int m = 0; m < KEEP; ++m)
#pragma unroll
            for (int r = 0; r < S; ++r)
              u[m][r] = iup[cbase[q] + (size_t(uint32_t(m) < cup[q] ? m : 0) * S + r) * TP];
#pragma unroll
          for (int m = 0; m < KEEP; ++m) {
            const bool take = uint32_t(m) < cup[q];
#pragma unroll
            for (int r = 0; r < S; ++r) tot[m][r] += take ? u[m][r] : 0.0f;
          }
        }
      } else {  // own part and every child's, already summed in LDS
        const float (*st)[S] = s_tot[slot0(k) + t];
#pragma unroll
        for (int m = 0; m < KEEP; ++m)
#pragma unroll
          for (int r = 0; r < S; ++r) tot[m][r] = st[m][r];
      }
      // own items to their slots; coarser items up (through memory from the top layer)
      const size_t tb = size_t(b) * KEEP;
      uint32_t so = 0, sp = 0;
#pragma unroll
      for (int m = 0; m < KEEP; ++m) {
        if (uint32_t(m) < kk) {
          const bool up = (mask >> m) & 1u;
          if (!up) {
            float* dst = itot + ((tb + so) * S) * TP + tt;
#pragma unroll
            for (int r = 0; r < S; ++r) dst[size_t(r) * TP] = tot[m][r];
            ++so;
          } else {
            if (k == Lt - Lb) {
              float* dst = iup + ((tb + sp) * S) * TP + tt;
#pragma unroll
              for (int r = 0; r < S; ++r) dst[size_t(r) * TP] = tot[m][r];
            }
            ++sp;
          }
        }
      }
    }
    if (k < Lt - Lb) {  // coarser items to the covering texel's totals, one child position at a time
      const int rw = (1 << ltw) >> k;
      const int q = (t / rw & 1) * 2 + (t % rw & 1);  // position among the covering texel's four
      const int pq = (t / rw >> 1) * (rw >> 1) + (t % rw >> 1);
#pragma unroll 1
      for (int qd = 0; qd < 4; ++qd) {
        __syncthreads();
        if (in && q == qd) {
          float (*pt)[S] = s_tot[slot0(k + 1) + pq];
          uint32_t sp = 0;
#pragma unroll
          for (int m = 0; m < KEEP; ++m) {
            if (uint32_t(m) < kk && ((mask >> m) & 1u)) {
#pragma unroll
              for (int r = 0; r < S; ++r) pt[sp][r] += tot[m][r];
              ++sp;
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// incl_bwd012: layers 0, 1 and 2 in one launch, one workgroup per tile of layer 1 (the
// texels of layer 2 over it form a (tw/2) x (th/2) block whose finer texels all lie in the
// tile).  Each thread runs the blend adjoint of its layer-1 texel and then of the four
// layer-0 texels it covers, whose items taken from it are added to its totals straight from
// registers (through a per-thread LDS column), so layer 0 passes nothing up through memory;
// then, one child position at a time, the layer-1 texels add their items of the coarser
// list to the totals of their layer-2 texel in LDS, which start as that texel's own blend
// part (computed first by the first PT threads); those threads finish layer 2, whose items
// of the coarser list go up to layer 3 through memory (iup).  Same totals and summation
// order as one launch of incl_bwd per layer.
template <int D>
__global__ __launch_bounds__(256) void k_incl_bwd012(
    const Params P, const uint64_t* __restrict__ fkey, const float* __restrict__ fgam,
    const uint64_t* __restrict__ kkey, const float* __restrict__ kgam,
    const uint32_t* __restrict__ fcnt, const float* __restrict__ desc,
    const float* __restrict__ gpyr, float* __restrict__ itot, float* __restrict__ iup,
    const Extras X) {
  constexpr int S = D + 1;
  __shared__ float s_dg[KEEP][TP];  // a child's items taken from this texel, in order
  __shared__ float s_tg[KEEP][TP];
  __shared__ float s_up[PT][KEEP][S];  // totals of the block's layer-2 texels
  const int v = blockIdx.y;
  const ViewP& c = P.view[v];
  const int t = threadIdx.x;
  const int ltw = P.ltw, lth = 8 - P.ltw;
  const int W1 = layer_dim(c.W, 1), H1 = layer_dim(c.H, 1);
  const int W0 = layer_dim(c.W, 0), H0 = layer_dim(c.H, 0);
  const int tiles_x = (W1 + (1 << ltw) - 1) >> ltw, tiles_y = (H1 + (1 << lth) - 1) >> lth;
  int tx, ty;  // the four tiles under one layer-2 tile on one die
  if (!quad_tile(blockIdx.x, tiles_x, tiles_y, tx, ty)) return;  // uniform per workgroup
  const uint32_t b = c.lbin[1] + uint32_t(ty * tiles_x + tx);
  const int i = (tx << ltw) + (t & ((1 << ltw) - 1));
  const int j = (ty << lth) + (t >> ltw);
  const bool in = i < W1 && j < H1;
  const bool two = P.nl > 2;  // uniform: layer 2 exists and is finished here
  const BlendedSrc src{fkey, fgam, nullptr, nullptr, 0u, 0};
  // layer 2, own blend parts: thread t < PT takes texel t of the block
  const int hw = 1 << (ltw - 1), hh = 1 << (lth - 1);
  const int i2 = tx * hw + (t & (hw - 1)), j2 = ty * hh + (t >> (ltw - 1));
  const int W2 = layer_dim(c.W, 2), H2 = layer_dim(c.H, 2);
  const bool in2 = two && t < PT && i2 < W2 && j2 < H2;
  uint32_t b2 = 0, fc2 = 0;
  int t2 = 0;
  if (two && t < PT) {
    float G[D], dg[KEEP], tg[KEEP];
#pragma unroll
    for (int d = 0; d < D; ++d) G[d] = 0.0f;
#pragma unroll
    for (int m = 0; m < KEEP; ++m) { dg[m] = 0.0f; tg[m] = 0.0f; }
    if (in2) {
      texel_bin(P, v, 2, i2, j2, b2, t2);
      fc2 = fcnt[size_t(b2) * TP + t2];
      blended_adjoint<D, false>(src, b2, t2, fc2, size_t(c.lout[2]) + size_t(j2) * W2 + i2,
                                P.n > 0, desc, gpyr, X, G, dg, tg);
    }
#pragma unroll
    for (int m = 0; m < KEEP; ++m) {
      s_up[t][m][0] = dg[m];
#pragma unroll
      for (int d = 0; d < D; ++d) s_up[t][m][1 + d] = tg[m] * G[d];
    }
  }
  // layer 1 (and the four layer-0 texels of each of its texels)
  const size_t tb = size_t(b) * KEEP;
  uint32_t mask = 0, k = 0;
  float tot[KEEP][S];
  if (in) {
    const uint32_t fc = fcnt[size_t(b) * TP + t];
    mask = fc >> 16;
    {
      float G[D], dg[KEEP], tg[KEEP];
      k = blended_adjoint<D, false>(src, b, t, fc, size_t(c.lout[1]) + size_t(j) * W1 + i, P.n > 0,
                                    desc, gpyr, X, G, dg, tg);
#pragma unroll
      for (int m = 0; m < KEEP; ++m) {
        tot[m][0] = dg[m];
#pragma unroll
        for (int d = 0; d < D; ++d) tot[m][1 + d] = tg[m] * G[d];
      }
    }
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      const int ci = 2 * i + (q & 1), cj = 2 * j + (q >> 1);
      if (!(ci < W0 && cj < H0)) continue;
      uint32_t cb;
      int ct;
      texel_bin(P, v, 0, ci, cj, cb, ct);
      const uint32_t cfc = fcnt[size_t(cb) * TP + ct];
      const uint32_t cmask = cfc >> 16;
      float G[D], dg[KEEP], tg[KEEP];
      // layer 0's lists are rebuilt from their own lists and this texel's (b, t)
      const BlendedSrc csrc{fkey, fgam, kkey, kgam, b, t};
      const uint32_t ck = blended_adjoint<D, true>(csrc, cb, ct, cfc,
                                                   size_t(c.lout[0]) + size_t(cj) * W0 + ci,
                                                   P.n > 0, desc, gpyr, X, G, dg, tg);
      const size_t ctb = size_t(cb) * KEEP;
      uint32_t so = 0, sp = 0;
#pragma unroll
      for (int m = 0; m < KEEP; ++m) {
        if (uint32_t(m) < ck) {
          if ((cmask >> m) & 1u) {
            s_dg[sp][t] = dg[m];
            s_tg[sp][t] = tg[m];
            ++sp;
          } else {
            float* dst = itot + ((ctb + so) * S) * TP + ct;
            dst[0] = dg[m];
#pragma unroll
            for (int d = 0; d < D; ++d) dst[size_t(1 + d) * TP] = tg[m] * G[d];
            ++so;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < KEEP; ++m)
        if (uint32_t(m) < sp) {
          tot[m][0] += s_dg[m][t];
          const float w = s_tg[m][t];
#pragma unroll
          for (int d = 0; d < D; ++d) tot[m][1 + d] += w * G[d];
        }
    }
    // own items to their slots
    uint32_t so = 0;
#pragma unroll
    for (int m = 0; m < KEEP; ++m) {
      if (uint32_t(m) < k && !((mask >> m) & 1u)) {
        float* dst = itot + ((tb + so) * S) * TP + t;
#pragma unroll
        for (int r = 0; r < S; ++r) dst[size_t(r) * TP] = tot[m][r];
        ++so;
      }
    }
  }
  if (!two) return;  // uniform: layer 1 is the coarsest and takes nothing from above
  // items of the coarser list to the layer-2 totals, one child position at a time
  {
    const int il = t & ((1 << ltw) - 1), jl = t >> ltw;
    const int q = (jl & 1) * 2 + (il & 1);
    const int pq = (jl >> 1) * hw + (il >> 1);
#pragma unroll 1
    for (int qd = 0; qd < 4; ++qd) {
      __syncthreads();
      if (in && q == qd) {
        uint32_t sp = 0;
#pragma unroll
        for (int m = 0; m < KEEP; ++m) {
          if (uint32_t(m) < k && ((mask >> m) & 1u)) {
#pragma unroll
            for (int r = 0; r < S; ++r) s_up[pq][sp][r] += tot[m][r];
            ++sp;
          }
        }
      }
    }
    __syncthreads();
  }
  if (!in2) return;
  // layer 2: own items to their slots, items of the coarser list up to layer 3
  const uint32_t mask2 = fc2 >> 16;
  const uint32_t k2 = (fc2 & 31u) + ((fc2 >> 5) & 31u);
  const size_t tb2 = size_t(b2) * KEEP;
  uint32_t so = 0, sp = 0;
#pragma unroll
  for (int m = 0; m < KEEP; ++m) {
    if (uint32_t(m) < k2) {
      const bool up = (mask2 >> m) & 1u;
      float* dst = up ? iup + ((tb2 + sp) * S) * TP + t2 : itot + ((tb2 + so) * S) * TP + t2;
#pragma unroll
      for (int r = 0; r < S; ++r) dst[size_t(r) * TP] = s_up[t][m][r];
      sp += up ? 1u : 0u;
      so += up ? 0u : 1u;
    }
  }
}

// bwd_points: per point, every view: read the rows of its entries, apply the layer and
// footprint factors, then the chain rule through the projection; sum over views.  With CAM,
// the workgroup also sums, per view, the gradient of the camera over its 256 points:
// d/dR (row-major, X_c = R X_w + t), d/dt, d/dfx, d/dfy, d/dcx, d/dcy, written to
// campart[block][view][16] for k_cam_reduce.
template <int D, bool CAM>
__global__ __launch_bounds__(256) void k_bwd_points(
    const Params P, const float* __restrict__ X, const float* __restrict__ Y,
    const float* __restrict__ Z, const float* __restrict__ SW, const float* __restrict__ A,
    const float* __restrict__ rows, float* __restrict__ gX, float* __restrict__ gY,
    float* __restrict__ gZ, float* __restrict__ gSW, float* __restrict__ gA,
    float* __restrict__ gD, const uint32_t* __restrict__ epos, float* __restrict__ campart) {
  constexpr int RW = 4 + D;
  __shared__ float s_cam[CAM ? 4 : 1][16];
  // chunks of 256 points go to the dies in runs of PT_GROUP consecutive chunks (about one
  // scatter block, whose entries' rows share lines): workgroup g XCDS PT_GROUP + XCDS j + q
  // takes chunk (g XCDS + q) PT_GROUP + j; the grid is padded to a multiple of XCDS PT_GROUP
  const uint32_t span = XCDS * PT_GROUP;
  const uint32_t chunk = (blockIdx.x / span * XCDS + blockIdx.x % XCDS) * PT_GROUP +
                         blockIdx.x % span / XCDS;
  if (int64_t(chunk) * blockDim.x >= P.n) return;  // (uniform: a padding workgroup)
  const int64_t p = int64_t(chunk) * blockDim.x + threadIdx.x;
  const bool live = p < P.n;
  if (!CAM && !live) return;
  float x = 0.f, y = 0.f, z = 0.f, sw = 0.f, alpha = 0.f;
  if (live) { x = X[p]; y = Y[p]; z = Z[p]; sw = SW[p]; alpha = A[p]; }
  float ax = 0.f, ay = 0.f, az = 0.f, asw = 0.f, aal = 0.f;
  float at[D];
#pragma unroll
  for (int d = 0; d < D; ++d) at[d] = 0.0f;
  for (int v = 0; v < P.V; ++v) {
    const ViewP& c = P.view[v];
    Geo g;
    const bool vis = live && project(c, x, y, z, sw, P.nl, P.eps, g);
    float gxs = 0.f, gys = 0.f, gs = 0.f;
    float dXc = 0.f, dYc = 0.f, dZc = 0.f, iz = 0.f;
    if (vis) {
      float gal = 0.f;
      float gt[D];
#pragma unroll
      for (int d = 0; d < D; ++d) gt[d] = 0.0f;
      // both layer entries' footprints and the point's eight entry positions (one 32-byte
      // record), then all eight rows at once: a slot without an entry reads row 0 and is
      // dropped, so no load waits on another
      uint32_t tm[2][4];
      const uint32_t last = uint32_t(8 * P.n * P.V) - 1u;  // row capacity (guards memory only)
      const uint4* ep4 = reinterpret_cast<const uint4*>(epos + (size_t(v) * size_t(P.n) + size_t(p)) * NSLOT);
      const uint4 ea = ep4[0], eb = ep4[1];
      const uint32_t er[8] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
#pragma unroll
      for (int sel = 0; sel < 2; ++sel) {
        const int L = g.L0 + sel;
        Foot ft;
        const bool ok = sel < g.nl && footprint(g.x, g.y, L, layer_dim(c.W, L), layer_dim(c.H, L), ft);
        if (ok) touches(ft, P.ltw, tm[sel]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (!ok) tm[sel][q] = 0;
      }
      float4 rv[2][4][1 + D / 4];
#pragma unroll
      for (int sel = 0; sel < 2; ++sel)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t e = tm[sel][q] ? min(er[sel * 4 + q], last) : 0u;
          const float4* r4 = reinterpret_cast<const float4*>(rows + size_t(e) * RW);
#pragma unroll
          for (int qq = 0; qq < 1 + D / 4; ++qq) rv[sel][q][qq] = r4[qq];
        }
#pragma unroll
      for (int sel = 0; sel < 2; ++sel) {
        const int L = g.L0 + sel;
        float sA = 0.f, sBx = 0.f, sBy = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!tm[sel][q]) continue;
          const float4 h = rv[sel][q][0];
          sA += h.x; sBx += h.y; sBy += h.z;
#pragma unroll
          for (int qq = 0; qq < D / 4; ++qq) {
            const float4 tv = rv[sel][q][1 + qq];
            gt[4 * qq] += tv.x; gt[4 * qq + 1] += tv.y; gt[4 * qq + 2] += tv.z; gt[4 * qq + 3] += tv.w;
          }
        }
        if (sel >= g.nl) break;
        const float io = g.io[sel];
        const float sc = pow2i(-L);
        gal += sA * io;
        gs += sA * alpha * g.dio[sel];
        gxs += sBx * io * alpha * sc;
        gys += sBy * io * alpha * sc;
      }
      // chain rule: x = fx Xc/Zc + cx, y = fy Yc/Zc + cy, s = fx sw / Zc
      iz = 1.0f / g.zc;
      dXc = gxs * c.fx * iz;
      dYc = gys * c.fy * iz;
      dZc = -(gxs * c.fx * g.qx + gys * c.fy * g.qy + gs * g.s) * iz;
      ax += c.R[0] * dXc + c.R[3] * dYc + c.R[6] * dZc;
      ay += c.R[1] * dXc + c.R[4] * dYc + c.R[7] * dZc;
      az += c.R[2] * dXc + c.R[5] * dYc + c.R[8] * dZc;
      asw += gs * c.fx * iz;
      // per-view sums first, then across views, so a batched call equals the sum of
      // single-view calls bit for bit
      aal += gal;
#pragma unroll
      for (int d = 0; d < D; ++d) at[d] += gt[d];
    }
    if (CAM) {
      float cv[16];
      cv[0] = dXc * x; cv[1] = dXc * y; cv[2] = dXc * z;
      cv[3] = dYc * x; cv[4] = dYc * y; cv[5] = dYc * z;
      cv[6] = dZc * x; cv[7] = dZc * y; cv[8] = dZc * z;
      cv[9] = dXc; cv[10] = dYc; cv[11] = dZc;
      cv[12] = vis ? gxs * g.qx + gs * sw * iz : 0.0f;
      cv[13] = vis ? gys * g.qy : 0.0f;
      cv[14] = gxs; cv[15] = gys;
      const int w = threadIdx.x >> 6;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const float r = wave_sum(cv[k]);
        if ((threadIdx.x & 63) == 0) s_cam[w][k] = r;
      }
      __syncthreads();
      if (threadIdx.x < 16)
        campart[(size_t(chunk) * P.V + v) * 16 + threadIdx.x] =
            ((s_cam[0][threadIdx.x] + s_cam[1][threadIdx.x]) + s_cam[2][threadIdx.x]) + s_cam[3][threadIdx.x];
      __syncthreads();
    }
  }
  if (!live) return;
  gX[p] = ax; gY[p] = ay; gZ[p] = az; gSW[p] = asw; gA[p] = aal;
  float4* gd4 = reinterpret_cast<float4*>(gD + size_t(p) * D);
#pragma unroll
  for (int q = 0; q < D / 4; ++q) gd4[q] = make_float4(at[4 * q], at[4 * q + 1], at[4 * q + 2], at[4 * q + 3]);
}

// cam_reduce: one workgroup per view sums the per-block camera partials in a fixed order.
__global__ __launch_bounds__(256) void k_cam_reduce(const float* __restrict__ campart,
                                                    uint32_t nblk, int32_t V,
                                                    float* __restrict__ gcam) {
  __shared__ float s_cam[4][16];
  const int v = blockIdx.x;
  float acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0f;
  for (uint32_t bk = threadIdx.x; bk < nblk; bk += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] += campart[(size_t(bk) * V + v) * 16 + k];
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float r = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) s_cam[w][k] = r;
  }
  __syncthreads();
  if (threadIdx.x < 16)
    gcam[size_t(v) * 16 + threadIdx.x] =
        ((s_cam[0][threadIdx.x] + s_cam[1][threadIdx.x]) + s_cam[2][threadIdx.x]) + s_cam[3][threadIdx.x];
}

// ------------------------------------------------------------------------------------
// Host side.

thread_local int32_t g_last_hip = 0;

// Optional per-kernel timing (reports only): a start and an end event around every kernel
// launch, on the launch stream; read back and summed per stage by trips_timing_read.
enum Stage { ST_COUNT, ST_COLSCAN, ST_BINSCAN, ST_SCATTER, ST_FWD_ITEMS,
             ST_FWD_FINE, ST_FWD_MERGE, ST_BWD_PIXELS, ST_BWD_ITEMS, ST_BWD_FINE, ST_BWD_POINTS,
             ST_EXPORT, ST_INCL_FWD, ST_INCL_BWD, NUM_STAGES };
const char* const kStageNames[NUM_STAGES] = {
    "count", "colscan", "binscan", "scatter", "fwd_items", "fwd_fine", "fwd_merge",
    "bwd_pixels", "bwd_items", "bwd_fine", "bwd_points", "export", "incl_fwd", "incl_bwd"};
static_assert(NUM_STAGES == TRIPS_NUM_STAGES, "stage table");

struct TimingState {
  bool on = false;
  std::vector<hipEvent_t> pool;  // pairs: start, end
  std::vector<int> stage;        // stage of each recorded pair
  size_t used = 0;               // pairs recorded since the last read
};
thread_local TimingState g_timing;

// Wraps one kernel launch: records events around it when timing is enabled and the stream
// is not being captured into a graph.
struct StageTimer {
  hipStream_t st;
  int pair = -1;
  StageTimer(int stage, hipStream_t s) : st(s) {
    if (!g_timing.on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    TimingState& t = g_timing;
    if (t.used * 2 + 2 > t.pool.size()) {
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
      t.pool.push_back(a);
      t.pool.push_back(b);
      t.stage.push_back(0);
    }
    pair = int(t.used++);
    t.stage[pair] = stage;
    (void)hipEventRecord(t.pool[2 * pair], s);
  }
  ~StageTimer() {
    if (pair >= 0) (void)hipEventRecord(g_timing.pool[2 * pair + 1], st);
  }
};

struct Layout {
  Params P;
  uint32_t nbv_max;   // largest bin count of one view (LDS histogram size)
  uint64_t ecap;      // entry capacity
  uint64_t icap;      // work-item capacity
  uint64_t npyr;      // texels of all views and layers
  // saved buffer
  size_t s_info, s_bin_start, s_item_start, s_multi, s_fine, s_coarse, s_npix, s_kkey, s_kgam,
      s_fkey, s_fgam, s_fcnt, s_kslot, s_tables_end, s_work, s_ent, s_epos;
  size_t saved_bytes;
  // workspace
  size_t w_H16, w_H, w_tot, w_csum, w_coff, w_pcnt, w_pkey, w_pgam, w_bst, w_rows, w_cam, w_itot, w_iup,
      ws_bytes;
  size_t ws_fwd_bytes;  // the part of the workspace a forward call uses
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The binning passes keep a 16-bit counter per tile of one view in LDS (at most 64 KB);
// the scatter pass also stages a 32-bit base per tile when both tables fit in 150 KB.
constexpr uint32_t kMaxViewBins = 32768;
constexpr size_t kLdsLimit = 150 * 1024;
size_t count_lds(uint32_t nbins) { return size_t((nbins + 1) / 2) * 4; }
size_t staged_scatter_lds(uint32_t nbins) { return size_t((nbins + 1) / 2 + nbins) * 4; }

trips_status make_layout(const trips_config* cfg, const trips_camera* cams, int32_t views,
                         int64_t n, const trips_tuning* tun, Layout& lay) {
  if (!cfg || !cams) return TRIPS_ERR_INVALID_ARG;
  if (views < 1 || views > MAXV || n < 0) return TRIPS_ERR_INVALID_ARG;
  if (cfg->num_layers < 1 || cfg->num_layers > MAXL) return TRIPS_ERR_INVALID_ARG;
  if (!(cfg->eps >= 0.0f && cfg->eps <= 1.0f)) return TRIPS_ERR_INVALID_ARG;
  if (cfg->desc_dim < 1 || cfg->max_list < 1) return TRIPS_ERR_INVALID_ARG;
  if (cfg->max_list != KEEP) return TRIPS_ERR_UNSUPPORTED;
  if (cfg->desc_dim != 4 && cfg->desc_dim != 8) return TRIPS_ERR_UNSUPPORTED;
  int tile_w = 16, pb = 4096, item_e = 8192;
  {
    // default work-item size: 8192 entries up to one point per pixel of the largest view,
    // doubled for each doubling of that density, up to 32768 (denser clouds put more entries
    // in every tile, and smaller items then spend more on merges than they save)
    int64_t px = 0;
    for (int v = 0; v < views; ++v)
      px = std::max<int64_t>(px, int64_t(cams[v].width) * cams[v].height);
    while (item_e < 32768 && px > 0 && n > int64_t(item_e / 8192) * px) item_e *= 2;
  }
  if (tun) {
    if (tun->tile_w) tile_w = tun->tile_w;
    if (tun->points_per_block) pb = tun->points_per_block;
    if (tun->item_entries) item_e = tun->item_entries;
  }
  int ltw = 0;
  while ((1 << ltw) < tile_w) ++ltw;
  if ((1 << ltw) != tile_w || ltw < 3 || ltw > 6) return TRIPS_ERR_INVALID_ARG;
  if (pb < 256 || pb > 65535 || item_e < 256 || item_e > 65536) return TRIPS_ERR_INVALID_ARG;
  std::memset(&lay, 0, sizeof(lay));
  Params& P = lay.P;
  P.V = views; P.nl = cfg->num_layers; P.D = cfg->desc_dim; P.ltw = ltw; P.eps = cfg->eps;
  P.pb = uint32_t(pb); P.item_e = uint32_t(item_e); P.n = n;
  if (cfg->include_coarser != 0 && cfg->include_coarser != 1) return TRIPS_ERR_INVALID_ARG;
  P.coarser = cfg->include_coarser;
  P.fine_e = P.coarser ? 0u : FINE_E;
  P.nblk = uint32_t((n + pb - 1) / pb);
  const int lth = 8 - ltw;
  uint64_t bins = 0, texels = 0;
  lay.nbv_max = 0;
  for (int v = 0; v < views; ++v) {
    const trips_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > (1 << 16) || c.height > (1 << 16))
      return TRIPS_ERR_INVALID_ARG;
    if (!(c.znear > 0.0f) || !std::isfinite(c.znear)) return TRIPS_ERR_INVALID_ARG;
    for (int k = 0; k < 9; ++k) if (!std::isfinite(c.R[k])) return TRIPS_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k) if (!std::isfinite(c.t[k])) return TRIPS_ERR_INVALID_ARG;
    if (!std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
      return TRIPS_ERR_INVALID_ARG;
    ViewP& vp = P.view[v];
    std::memcpy(vp.R, c.R, sizeof(vp.R));
    std::memcpy(vp.t, c.t, sizeof(vp.t));
    vp.fx = c.fx; vp.fy = c.fy; vp.cx = c.cx; vp.cy = c.cy; vp.znear = c.znear;
    vp.W = c.width; vp.H = c.height;
    vp.bin_base = uint32_t(bins);
    uint64_t vb = 0;
    for (int L = 0; L < P.nl; ++L) {
      const uint64_t WL = (uint64_t(c.width) + (1ull << L) - 1) >> L;
      const uint64_t HL = (uint64_t(c.height) + (1ull << L) - 1) >> L;
      const uint64_t tx = (WL + (1ull << ltw) - 1) >> ltw;
      const uint64_t ty = (HL + (1ull << lth) - 1) >> lth;
      vp.lbin[L] = uint32_t(bins + vb);
      vp.lout[L] = uint32_t(texels);
      vb += tx * ty;
      texels += WL * HL;
    }
    vp.lbin[P.nl] = uint32_t(bins + vb);
    vp.nbins = uint32_t(vb);
    bins += vb;
    if (vb > kMaxViewBins) return TRIPS_ERR_UNSUPPORTED;  // LDS tables of one view
    lay.nbv_max = std::max<uint32_t>(lay.nbv_max, uint32_t(vb));
    if (bins >= (1ull << 31) / TP || texels >= (1ull << 32)) return TRIPS_ERR_CAPACITY;
  }
  P.NB = uint32_t(bins);
  lay.npyr = texels;
  lay.ecap = 8ull * uint64_t(n) * uint64_t(views);  // <= 2 layers x 4 tiles per point and view
  if (lay.ecap >= (1ull << 32) - 1) return TRIPS_ERR_CAPACITY;
  lay.icap = bins + (lay.ecap + item_e - 1) / item_e;
  lay.icap = (lay.icap + XCDS - 1) / XCDS * XCDS;
  if (lay.icap * BWD_SPLIT >= (1ull << 32) - 1) return TRIPS_ERR_CAPACITY;
  const size_t NB = bins;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  lay.s_info = take(64 * 4);
  lay.s_bin_start = take((NB + 1) * 4);
  lay.s_item_start = take((NB + 1) * 4);
  lay.s_multi = take(2 * NB * 4);
  lay.s_fine = take(NB * sizeof(uint4));
  lay.s_coarse = take(NB * 4);
  // texel tables: their offsets depend only on the cameras and config (export reads them)
  lay.s_npix = take(NB * TP * 4);
  lay.s_kkey = take(NB * TP * KEEP * 8);
  lay.s_kgam = take(NB * TP * KEEP * 4);
  // coarser-layer inclusion: every texel's blended list and its make-up
  const size_t inc = P.coarser ? 1 : 0;
  lay.s_fkey = take(inc * NB * TP * KEEP * 8);
  lay.s_fgam = take(inc * NB * TP * KEEP * 4);
  lay.s_fcnt = take(inc * NB * TP * 4);
  // kept slots of the entries of fine tiles (written by the forward, read by the backward)
  lay.s_kslot = take((P.fine_e ? NB : 0) * TP * 4);
  lay.s_tables_end = o;
  // point-count dependent parts
  lay.s_work = take(size_t(lay.icap) * sizeof(uint4));
  lay.s_ent = take(size_t(lay.ecap) * sizeof(Entry));
  lay.s_epos = take(size_t(views) * NSLOT * size_t(n) * 4);
  lay.saved_bytes = o;
  o = 0;
  const size_t scratch = o;
  // forward scratch
  lay.w_H16 = take(size_t(P.nblk) * NB * 2);  // per-block counts per tile
  lay.w_H = take(size_t(P.nblk) * NB * 4);    // their exclusive prefixes over blocks
  lay.w_tot = take(NB * 4);
  lay.w_csum = take(((NB + CHUNK - 1) / CHUNK) * CSUM * 4);
  lay.w_coff = take(((NB + CHUNK - 1) / CHUNK) * 4 * 4);
  // partial lists of the items of multi-item tiles only: such a tile has e > item_e entries
  // and ceil(e / item_e) < 2 e / item_e items, so they number fewer than 2 ecap / item_e
  const uint64_t pcap = std::min<uint64_t>(lay.icap, 2 * lay.ecap / item_e + 1);
  lay.w_pcnt = take(size_t(pcap) * TP * 4);
  lay.w_pkey = take(size_t(pcap) * TP * KEEP * 8);
  lay.w_pgam = take(size_t(pcap) * TP * KEEP * 4);
  const size_t fwd_end = o;
  // backward scratch reuses the same bytes
  o = scratch;
  lay.w_bst = take(NB * TP * KEEP * sizeof(float2));
  lay.w_rows = take(size_t(views) * NSLOT * size_t(n) * (4 + P.D) * 4);
  lay.w_cam = take(size_t((n + 255) / 256) * size_t(views) * 16 * 4);
  lay.w_itot = take(inc * NB * TP * KEEP * size_t(1 + P.D) * 4);
  lay.w_iup = take(inc * NB * TP * KEEP * size_t(1 + P.D) * 4);
  lay.ws_bytes = std::max(fwd_end, o);
  lay.ws_fwd_bytes = fwd_end;
  return TRIPS_OK;
}

#define TRIPS_HIP(call)                                        \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) { g_last_hip = int32_t(e_); return TRIPS_ERR_HIP; } \
  } while (0)

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// The optional arguments of one call; only the fields of its direction are taken.
trips_status take_extras(const trips_extras* e, bool forward, bool backward, Extras& X) {
  X = Extras{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (!e) return TRIPS_OK;
  if (e->background && !aligned16(e->background)) return TRIPS_ERR_INVALID_ARG;
  X.bg = e->background;
  if (forward) X.alpha = e->alpha_out;
  if (backward) {
    if (e->grad_background && !aligned16(e->grad_background)) return TRIPS_ERR_INVALID_ARG;
    X.galpha = e->grad_alpha;
    X.gbg = e->grad_background;
    X.gcam = e->grad_camera;
  }
  return TRIPS_OK;
}

trips_status check_points(const trips_points* pts, const Layout& lay) {
  if (!pts) return TRIPS_ERR_INVALID_ARG;
  if (pts->n != lay.P.n) return TRIPS_ERR_INVALID_ARG;
  if (pts->n > 0 && (!pts->x || !pts->y || !pts->z || !pts->size_w || !pts->opacity || !pts->desc))
    return TRIPS_ERR_INVALID_ARG;
  if (pts->n > 0 && !aligned16(pts->desc)) return TRIPS_ERR_INVALID_ARG;
  return TRIPS_OK;
}

// Forward scratch for callers that cannot allocate device memory (trips_forward_noalloc):
// a device array of the library, one copy per GPU, alive until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a stand-in for the
// symbol): each device's address is looked up once, with that device current, and kept.
constexpr size_t kStaticScratchBytes = size_t(TRIPS_STATIC_SCRATCH_MB) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_make;
void* g_scratch_ptr[64];

trips_status static_scratch(void*& out) {
  int dev = 0;
  TRIPS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return TRIPS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_make);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    TRIPS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || !aligned(p)) return TRIPS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  out = g_scratch_ptr[dev];
  return TRIPS_OK;
}

// A second stream per device for the fine-tile kernels, which touch other tiles than the
// work-item kernels and run beside them (a fork and a join on the caller's stream; in a
// captured plan these become two branches of the graph).  Created on first use with the
// default priority and kept until the process ends; g_side_launch serialises the calls that
// use it, so the fork and join events of one call are never interleaved with another's.
struct SideStream {
  hipStream_t s;
  hipEvent_t fork, join;
};
std::mutex g_side_make, g_side_launch;
constexpr int kMaxDevices = 64;
SideStream g_side[kMaxDevices];

trips_status side_stream(SideStream*& out) {
  int dev = 0;
  TRIPS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return TRIPS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_side_make);
  SideStream& sd = g_side[dev];
  if (!sd.s) {
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    TRIPS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    TRIPS_HIP(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    TRIPS_HIP(hipEventCreateWithFlags(&b, hipEventDisableTiming));
    sd.fork = a;
    sd.join = b;
    sd.s = s;
  }
  out = &sd;
  return TRIPS_OK;
}

// Largest tile count of layer L over the views (grid width of the per-layer passes).
uint32_t layer_tiles_max(const Params& P, int L) {
  uint32_t m = 0;
  for (int v = 0; v < P.V; ++v) m = std::max(m, P.view[v].lbin[L + 1] - P.view[v].lbin[L]);
  return m;
}
// grid of a pass laid out by quad_tile over layer L: every view's quads, 4 XCDS per XCDS quads
uint32_t layer_quad_grid(const Params& P, int L) {
  uint32_t m = 0;
  for (int v = 0; v < P.V; ++v) {
    const uint32_t WL = uint32_t(layer_dim(P.view[v].W, L)), HL = uint32_t(layer_dim(P.view[v].H, L));
    const uint32_t tx = (WL + (1u << P.ltw) - 1) >> P.ltw, ty = (HL + (1u << (8 - P.ltw)) - 1) >> (8 - P.ltw);
    m = std::max(m, ((tx + 1) / 2) * ((ty + 1) / 2));
  }
  return (m + XCDS - 1) / XCDS * (4 * XCDS);
}

template <int D>
trips_status launch_forward(const Layout& lay, const trips_points& pts, float* pyr, char* sv,
                            char* ws, const Extras& X, hipStream_t st) {
  const Params& P = lay.P;
  uint16_t* H16 = reinterpret_cast<uint16_t*>(ws + lay.w_H16);
  uint32_t* H = reinterpret_cast<uint32_t*>(ws + lay.w_H);
  uint32_t* tot = reinterpret_cast<uint32_t*>(ws + lay.w_tot);
  const uint32_t nch = (P.NB + CHUNK - 1) / CHUNK;
  uint32_t* csum = reinterpret_cast<uint32_t*>(ws + lay.w_csum);
  uint32_t* coff = reinterpret_cast<uint32_t*>(ws + lay.w_coff);
  uint32_t* pcnt = reinterpret_cast<uint32_t*>(ws + lay.w_pcnt);
  uint64_t* pkey = reinterpret_cast<uint64_t*>(ws + lay.w_pkey);
  float* pgam = reinterpret_cast<float*>(ws + lay.w_pgam);
  uint32_t* info = reinterpret_cast<uint32_t*>(sv + lay.s_info);
  uint32_t* bin_start = reinterpret_cast<uint32_t*>(sv + lay.s_bin_start);
  uint32_t* item_start = reinterpret_cast<uint32_t*>(sv + lay.s_item_start);
  uint4* work = reinterpret_cast<uint4*>(sv + lay.s_work);
  uint32_t* multi_bins = reinterpret_cast<uint32_t*>(sv + lay.s_multi);
  uint4* fine_work = reinterpret_cast<uint4*>(sv + lay.s_fine);
  uint32_t* coarse_bins = reinterpret_cast<uint32_t*>(sv + lay.s_coarse);
  uint32_t* npix = reinterpret_cast<uint32_t*>(sv + lay.s_npix);
  uint64_t* kkey = reinterpret_cast<uint64_t*>(sv + lay.s_kkey);
  float* kgam = reinterpret_cast<float*>(sv + lay.s_kgam);
  Entry* ent = reinterpret_cast<Entry*>(sv + lay.s_ent);
  uint32_t* epos = reinterpret_cast<uint32_t*>(sv + lay.s_epos);
  uint32_t* kslot = reinterpret_cast<uint32_t*>(sv + lay.s_kslot);

  if (P.nblk > 0) {
    StageTimer tm(ST_COUNT, st);
    hipLaunchKernelGGL(k_count, dim3(P.nblk * P.V), dim3(BIN_THREADS), count_lds(lay.nbv_max), st,
                       P, pts.x, pts.y, pts.z, pts.size_w, H16);
  }
  TRIPS_HIP(hipGetLastError());
  {
    StageTimer tm(ST_COLSCAN, st);
    if (P.nblk > 0) {  // also writes the chunk sums
      hipLaunchKernelGGL(k_colscan, dim3((P.NB + 63) / 64), dim3(64 * CS_SEG), 0, st, H16, H, tot,
                         P.NB, P.nblk, csum, P.item_e, P.fine_e);
    } else {
      hipLaunchKernelGGL(k_fill_u32, dim3((P.NB + 255) / 256), dim3(256), 0, st, tot, P.NB, 0u);
      hipLaunchKernelGGL(k_chunksum, dim3(nch), dim3(CHUNK), 0, st, tot, csum, P.NB, P.item_e,
                         P.fine_e);
    }
  }
  TRIPS_HIP(hipGetLastError());
  {
    StageTimer tm(ST_BINSCAN, st);
    if (nch <= FUSE_CHUNKS) {
      hipLaunchKernelGGL(k_binscan<true>, dim3(nch), dim3(CHUNK), 0, st, tot, csum, coff,
                         bin_start, item_start, multi_bins, fine_work, coarse_bins, info, work,
                         P.NB, nch, P.item_e, P.fine_e);
    } else {
      hipLaunchKernelGGL(k_chunkscan, dim3(1), dim3(1024), 0, st, csum, coff, bin_start,
                         item_start, info, P.NB, nch);
      hipLaunchKernelGGL(k_binscan<false>, dim3(nch), dim3(CHUNK), 0, st, tot, csum, coff,
                         bin_start, item_start, multi_bins, fine_work, coarse_bins, info, work,
                         P.NB, nch, P.item_e, P.fine_e);
    }
  }
  TRIPS_HIP(hipGetLastError());
  if (P.nblk > 0) {
    StageTimer tm(ST_SCATTER, st);
    if (staged_scatter_lds(lay.nbv_max) <= kLdsLimit)
      hipLaunchKernelGGL(k_scatter<true>, dim3(P.nblk * P.V), dim3(BIN_THREADS),
                         staged_scatter_lds(lay.nbv_max), st, P, pts.x, pts.y, pts.z, pts.size_w,
                         pts.opacity, H, bin_start, ent, epos, info);
    else
      hipLaunchKernelGGL(k_scatter<false>, dim3(P.nblk * P.V), dim3(BIN_THREADS),
                         count_lds(lay.nbv_max), st, P, pts.x, pts.y, pts.z, pts.size_w,
                         pts.opacity, H, bin_start, ent, epos, info);
  }
  TRIPS_HIP(hipGetLastError());
  {
    // the fine tiles on the side stream, beside the work items and their merge
    SideStream* sd = nullptr;
    trips_status ss = side_stream(sd);
    if (ss != TRIPS_OK) return ss;
    std::lock_guard<std::mutex> lk(g_side_launch);
    TRIPS_HIP(hipEventRecord(sd->fork, st));
    {  // one workgroup per work item (the longer path, enqueued first); workgroups beyond the
       // item count exit at once
      StageTimer tm(ST_FWD_ITEMS, st);
      hipLaunchKernelGGL(k_fwd_items<D>, dim3(uint32_t(lay.icap)), dim3(256), 0, st, P, info,
                         work, bin_start, item_start, ent, pts.desc, pyr, npix, kkey, kgam, pcnt,
                         pkey, pgam, X.bg, X.alpha);
    }
    hipError_t e3 = hipGetLastError();
    hipError_t e0 = hipStreamWaitEvent(sd->s, sd->fork, 0);
    {  // one workgroup per fine tile; workgroups beyond their count exit at once
      StageTimer tm(ST_FWD_FINE, sd->s);
      hipLaunchKernelGGL(k_fwd_fine<D>, dim3(P.NB), dim3(256), 0, sd->s, P, info, fine_work, ent,
                         kslot, pts.desc, pyr, npix, kkey, kgam, X.bg, X.alpha);
    }
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipEventRecord(sd->join, sd->s);
    {
      StageTimer tm(ST_FWD_MERGE, st);
      hipLaunchKernelGGL(k_fwd_merge<D>, dim3(1024), dim3(256), 0, st, P, item_start, multi_bins,
                         info, pcnt, pkey, pgam, pts.desc, pyr, npix, kkey, kgam, X.bg, X.alpha);
    }
    hipError_t e4 = hipGetLastError();
    // the join is enqueued whatever failed, so a captured graph has no dangling branch
    TRIPS_HIP(hipStreamWaitEvent(st, sd->join, 0));
    TRIPS_HIP(e0);
    TRIPS_HIP(e1);
    TRIPS_HIP(e2);
    TRIPS_HIP(e3);
    TRIPS_HIP(e4);
  }
  if (P.coarser) {  // coarsest layer first: each layer merges the blended lists above it
    StageTimer tm(ST_INCL_FWD, st);
    uint64_t* fkey = reinterpret_cast<uint64_t*>(sv + lay.s_fkey);
    float* fgam = reinterpret_cast<float*>(sv + lay.s_fgam);
    uint32_t* fcnt = reinterpret_cast<uint32_t*>(sv + lay.s_fcnt);
    // layers 2 and up in groups of up to 1 + log2(shorter tile side) layers counted from
    // layer 2, coarsest group first, each one launch over the tiles of its finest layer;
    // layers 0 and 1 (most of the texels) keep one launch each
    const int gmax = std::min(1 + std::min(P.ltw, 8 - P.ltw), 5);
    int L = P.nl - 1;
    while (L >= 2) {
      const int Lb = 2 + ((L - 2) / gmax) * gmax;  // the group's finest layer
      hipLaunchKernelGGL(k_incl_fwd_group<D>, dim3(layer_tiles_max(P, Lb), uint32_t(P.V)),
                         dim3(256), 0, st, P, Lb, L, npix, kkey, kgam, fkey, fgam, fcnt,
                         pts.desc, pyr, X.bg, X.alpha);
      TRIPS_HIP(hipGetLastError());
      L = Lb - 1;
    }
    for (; L >= 0; --L) {
      hipLaunchKernelGGL(k_incl_fwd<D>, dim3(layer_quad_grid(P, L), uint32_t(P.V)), dim3(256), 0,
                         st, P, L, npix, kkey, kgam, fkey, fgam, fcnt, pts.desc, pyr, X.bg,
                         X.alpha);
      TRIPS_HIP(hipGetLastError());
    }
  }
  return TRIPS_OK;
}

template <int D>
trips_status launch_backward(const Layout& lay, const trips_points& pts, const float* gpyr,
                             const char* sv, char* ws, float* gx, float* gy, float* gz, float* gsw,
                             float* ga, float* gd, const Extras& X, hipStream_t st) {
  const Params& P = lay.P;
  float2* bst = reinterpret_cast<float2*>(ws + lay.w_bst);
  float* rows = reinterpret_cast<float*>(ws + lay.w_rows);
  const uint32_t* info = reinterpret_cast<const uint32_t*>(sv + lay.s_info);
  const uint4* work = reinterpret_cast<const uint4*>(sv + lay.s_work);
  const uint4* fine_work = reinterpret_cast<const uint4*>(sv + lay.s_fine);
  const uint32_t* coarse_bins = reinterpret_cast<const uint32_t*>(sv + lay.s_coarse);
  const uint32_t* npix = reinterpret_cast<const uint32_t*>(sv + lay.s_npix);
  const uint64_t* kkey = reinterpret_cast<const uint64_t*>(sv + lay.s_kkey);
  const float* kgam = reinterpret_cast<const float*>(sv + lay.s_kgam);
  const Entry* ent = reinterpret_cast<const Entry*>(sv + lay.s_ent);
  const uint32_t* epos = reinterpret_cast<const uint32_t*>(sv + lay.s_epos);
  const uint32_t* kslot = reinterpret_cast<const uint32_t*>(sv + lay.s_kslot);

  if (P.coarser) {
    // finest layer first: every layer's items collect what the finer lists took from them
    // (with inclusion the fine path holds only empty tiles, so every entry is in an item)
    const uint64_t* fkey = reinterpret_cast<const uint64_t*>(sv + lay.s_fkey);
    const float* fgam = reinterpret_cast<const float*>(sv + lay.s_fgam);
    const uint32_t* fcnt = reinterpret_cast<const uint32_t*>(sv + lay.s_fcnt);
    float* itot = reinterpret_cast<float*>(ws + lay.w_itot);
    float* iup = reinterpret_cast<float*>(ws + lay.w_iup);
    {
      StageTimer tm(ST_INCL_BWD, st);
      // the three finest layers run as one launch (layers 0 and 1 pass nothing up through
      // memory)
      const bool fuse = P.nl > 1;
      if (fuse) {
        hipLaunchKernelGGL(k_incl_bwd012<D>, dim3(layer_quad_grid(P, 1), uint32_t(P.V)), dim3(256),
                           0, st, P, fkey, fgam, kkey, kgam, fcnt, pts.desc, gpyr, itot, iup, X);
        TRIPS_HIP(hipGetLastError());
      }
      // a single layer on its own; from layer 3 on, groups of up to 1 + log2(shorter tile
      // side) layers as one launch over their finest layer's tiles
      const int gmax = std::min(1 + std::min(P.ltw, 8 - P.ltw), 5);
      for (int L = fuse ? 3 : 0; L < P.nl;) {
        if (L < 3) {
          hipLaunchKernelGGL(k_incl_bwd<D>, dim3(layer_tiles_max(P, L) * INCL_LANES, uint32_t(P.V)),
                             dim3(256),
                             0, st, P, L, fkey, fgam, fcnt, pts.desc, gpyr, itot, iup, iup, X);
          ++L;
        } else {
          const int Lt = std::min(P.nl - 1, L + gmax - 1);
          hipLaunchKernelGGL(k_incl_bwd_group<D>, dim3(layer_tiles_max(P, L), uint32_t(P.V)),
                             dim3(256), 0, st, P, L, Lt, fkey, fgam, fcnt, pts.desc, gpyr, itot,
                             iup, X);
          L = Lt + 1;
        }
        TRIPS_HIP(hipGetLastError());
      }
    }
    {
      StageTimer tm(ST_BWD_ITEMS, st);
      hipLaunchKernelGGL((k_bwd_items<D, true>), dim3(uint32_t(lay.icap) * BWD_SPLIT), dim3(256),
                         0, st, P, info, work, ent, npix, kkey, bst, gpyr, rows, BWD_SPLIT, fcnt,
                         itot);
    }
    TRIPS_HIP(hipGetLastError());
  } else {
    // the fine tiles on the side stream, beside the blend adjoints and rows of the items
    SideStream* sd = nullptr;
    trips_status ss = side_stream(sd);
    if (ss != TRIPS_OK) return ss;
    std::lock_guard<std::mutex> lk(g_side_launch);
    TRIPS_HIP(hipEventRecord(sd->fork, st));
    {  // the longer path first
      StageTimer tm(ST_BWD_PIXELS, st);
      hipLaunchKernelGGL(k_bwd_pixels<D>, dim3(P.NB), dim3(256), 0, st, P, info, coarse_bins, npix,
                         kkey, kgam, pts.desc, gpyr, bst, X);
    }
    hipError_t e3 = hipGetLastError();
    hipError_t e0 = hipStreamWaitEvent(sd->s, sd->fork, 0);
    {
      StageTimer tm(ST_BWD_FINE, sd->s);
      hipLaunchKernelGGL(k_bwd_fine<D>, dim3(P.NB), dim3(256), 0, sd->s, P, info, fine_work, ent,
                         kslot, npix, pts.desc, gpyr, rows, X);
    }
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipEventRecord(sd->join, sd->s);
    {
      StageTimer tm(ST_BWD_ITEMS, st);
      hipLaunchKernelGGL((k_bwd_items<D, false>), dim3(uint32_t(lay.icap) * BWD_SPLIT), dim3(256),
                         0, st, P, info, work, ent, npix, kkey, bst, gpyr, rows, BWD_SPLIT,
                         nullptr, nullptr);
    }
    hipError_t e4 = hipGetLastError();
    TRIPS_HIP(hipStreamWaitEvent(st, sd->join, 0));
    TRIPS_HIP(e0);
    TRIPS_HIP(e1);
    TRIPS_HIP(e2);
    TRIPS_HIP(e3);
    TRIPS_HIP(e4);
  }
  if (P.n > 0) {
    StageTimer tm(ST_BWD_POINTS, st);
    const uint32_t nblk = uint32_t((P.n + 255) / 256);
    const uint32_t grid = (nblk + XCDS * PT_GROUP - 1) / (XCDS * PT_GROUP) * (XCDS * PT_GROUP);
    float* campart = reinterpret_cast<float*>(ws + lay.w_cam);
    if (X.gcam)
      hipLaunchKernelGGL((k_bwd_points<D, true>), dim3(grid), dim3(256), 0, st, P, pts.x, pts.y,
                         pts.z, pts.size_w, pts.opacity, rows, gx, gy, gz, gsw, ga, gd, epos,
                         campart);
    else
      hipLaunchKernelGGL((k_bwd_points<D, false>), dim3(grid), dim3(256), 0, st, P, pts.x, pts.y,
                         pts.z, pts.size_w, pts.opacity, rows, gx, gy, gz, gsw, ga, gd, epos,
                         campart);
  }
  TRIPS_HIP(hipGetLastError());
  if (X.gcam) {
    if (P.n > 0) {
      hipLaunchKernelGGL(k_cam_reduce, dim3(uint32_t(P.V)), dim3(256), 0, st,
                         reinterpret_cast<const float*>(ws + lay.w_cam),
                         uint32_t((P.n + 255) / 256), int32_t(P.V), X.gcam);
    } else {
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(X.gcam),
                         uint32_t(P.V * 16), 0u);
    }
    TRIPS_HIP(hipGetLastError());
  }
  return TRIPS_OK;
}

trips_status check_buffers(const Layout& lay, const void* saved, size_t saved_bytes,
                           const void* ws, size_t ws_bytes, bool need_ws) {
  if (!saved || !aligned(saved)) return TRIPS_ERR_INVALID_ARG;
  if (saved_bytes < lay.saved_bytes) return TRIPS_ERR_WORKSPACE;
  if (need_ws) {
    if (!ws || !aligned(ws)) return TRIPS_ERR_INVALID_ARG;
    if (ws_bytes < lay.ws_bytes) return TRIPS_ERR_WORKSPACE;
  }
  return TRIPS_OK;
}

}  // namespace

struct trips_plan {
  Layout lay;
  Extras xf, xb;  // optional arguments of the forward and the backward launches
  trips_points pts;
  float* pyr;
  void* saved;
  void* ws;
  const float* gpyr;
  float *gx, *gy, *gz, *gsw, *ga, *gd;
  hipGraphExec_t exec[3];  // forward, backward, both
};

extern "C" {

const char* trips_status_string(trips_status s) {
  switch (s) {
    case TRIPS_OK: return "ok";
    case TRIPS_ERR_INVALID_ARG: return "invalid argument";
    case TRIPS_ERR_WORKSPACE: return "workspace or saved buffer too small";
    case TRIPS_ERR_CAPACITY: return "problem exceeds 32-bit fragment indexing";
    case TRIPS_ERR_HIP: return "HIP error";
    case TRIPS_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

int32_t trips_last_hip_error(void) { return g_last_hip; }

trips_status trips_timing_enable(int32_t enable) {
  g_timing.on = enable != 0;
  g_timing.used = 0;
  return TRIPS_OK;
}

trips_status trips_timing_read(float* ms, int32_t* calls) {
  if (!ms || !calls) return TRIPS_ERR_INVALID_ARG;
  for (int k = 0; k < NUM_STAGES; ++k) { ms[k] = 0.0f; calls[k] = 0; }
  TimingState& t = g_timing;
  for (size_t i = 0; i < t.used; ++i) {
    TRIPS_HIP(hipEventSynchronize(t.pool[2 * i + 1]));
    float e = 0.0f;
    TRIPS_HIP(hipEventElapsedTime(&e, t.pool[2 * i], t.pool[2 * i + 1]));
    ms[t.stage[i]] += e;
    calls[t.stage[i]] += 1;
  }
  t.used = 0;
  return TRIPS_OK;
}

const char* trips_stage_name(int32_t stage) {
  return (stage >= 0 && stage < NUM_STAGES) ? kStageNames[stage] : "";
}

trips_status trips_layer_layout(const trips_camera* cam, const trips_config* cfg, int32_t* dims,
                                int64_t* offsets) {
  if (!cam || !cfg) return TRIPS_ERR_INVALID_ARG;
  if (cfg->num_layers < 1 || cfg->num_layers > MAXL) return TRIPS_ERR_INVALID_ARG;
  if (cam->width < 1 || cam->height < 1 || cam->width > (1 << 16) || cam->height > (1 << 16))
    return TRIPS_ERR_INVALID_ARG;
  int64_t off = 0;
  for (int L = 0; L < cfg->num_layers; ++L) {
    const int64_t WL = (int64_t(cam->width) + (int64_t(1) << L) - 1) >> L;
    const int64_t HL = (int64_t(cam->height) + (int64_t(1) << L) - 1) >> L;
    if (dims) { dims[2 * L] = int32_t(WL); dims[2 * L + 1] = int32_t(HL); }
    if (offsets) offsets[L] = off;
    off += WL * HL;
  }
  if (offsets) offsets[cfg->num_layers] = off;
  return TRIPS_OK;
}

trips_status trips_buffer_sizes(const trips_config* cfg, const trips_camera* cams, int32_t views,
                                int64_t n, const trips_tuning* tun, size_t* ws_bytes,
                                size_t* saved_bytes) {
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, n, tun, lay);
  if (s != TRIPS_OK) return s;
  if (ws_bytes) *ws_bytes = lay.ws_bytes;
  if (saved_bytes) *saved_bytes = lay.saved_bytes;
  return TRIPS_OK;
}

trips_status trips_forward(const trips_config* cfg, const trips_points* pts,
                           const trips_camera* cams, int32_t views, const trips_tuning* tun,
                           float* pyr, void* saved, size_t saved_bytes, void* ws, size_t ws_bytes,
                           const trips_extras* extras, hipStream_t st) {
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, pts ? pts->n : -1, tun, lay);
  if (s != TRIPS_OK) return s;
  if ((s = check_points(pts, lay)) != TRIPS_OK) return s;
  if ((s = check_buffers(lay, saved, saved_bytes, ws, ws_bytes, true)) != TRIPS_OK) return s;
  if (!pyr || !aligned16(pyr)) return TRIPS_ERR_INVALID_ARG;
  Extras X;
  if ((s = take_extras(extras, true, false, X)) != TRIPS_OK) return s;
  char* sv = static_cast<char*>(saved);
  char* w = static_cast<char*>(ws);
  return cfg->desc_dim == 4 ? launch_forward<4>(lay, *pts, pyr, sv, w, X, st)
                            : launch_forward<8>(lay, *pts, pyr, sv, w, X, st);
}

trips_status trips_forward_noalloc(const trips_config* cfg, const trips_points* pts,
                                   const trips_camera* cams, int32_t views,
                                   const trips_tuning* tun, float* pyr, void* saved,
                                   size_t saved_bytes, const trips_extras* extras,
                                   hipStream_t st) {
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, pts ? pts->n : -1, tun, lay);
  if (s != TRIPS_OK) return s;
  if ((s = check_points(pts, lay)) != TRIPS_OK) return s;
  if ((s = check_buffers(lay, saved, saved_bytes, nullptr, 0, false)) != TRIPS_OK) return s;
  if (lay.ws_fwd_bytes > kStaticScratchBytes) return TRIPS_ERR_WORKSPACE;
  if (!pyr || !aligned16(pyr)) return TRIPS_ERR_INVALID_ARG;
  Extras X;
  if ((s = take_extras(extras, true, false, X)) != TRIPS_OK) return s;
  void* ws = nullptr;
  if ((s = static_scratch(ws)) != TRIPS_OK) return s;
  // every forward scratch word is written before it is read, so nothing is cleared
  char* sv = static_cast<char*>(saved);
  char* w = static_cast<char*>(ws);
  return cfg->desc_dim == 4 ? launch_forward<4>(lay, *pts, pyr, sv, w, X, st)
                            : launch_forward<8>(lay, *pts, pyr, sv, w, X, st);
}

trips_status trips_backward(const trips_config* cfg, const trips_points* pts,
                            const trips_camera* cams, int32_t views, const trips_tuning* tun,
                            const float* gpyr, const void* saved, size_t saved_bytes, void* ws,
                            size_t ws_bytes, float* gx, float* gy, float* gz, float* gsw,
                            float* ga, float* gd, const trips_extras* extras, hipStream_t st) {
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, pts ? pts->n : -1, tun, lay);
  if (s != TRIPS_OK) return s;
  if ((s = check_points(pts, lay)) != TRIPS_OK) return s;
  if ((s = check_buffers(lay, saved, saved_bytes, ws, ws_bytes, true)) != TRIPS_OK) return s;
  if (!gpyr || !aligned16(gpyr)) return TRIPS_ERR_INVALID_ARG;
  if (lay.P.n > 0 && (!gx || !gy || !gz || !gsw || !ga || !gd || !aligned16(gd)))
    return TRIPS_ERR_INVALID_ARG;
  Extras X;
  if ((s = take_extras(extras, false, true, X)) != TRIPS_OK) return s;
  const char* sv = static_cast<const char*>(saved);
  char* w = static_cast<char*>(ws);
  return cfg->desc_dim == 4 ? launch_backward<4>(lay, *pts, gpyr, sv, w, gx, gy, gz, gsw, ga, gd, X, st)
                            : launch_backward<8>(lay, *pts, gpyr, sv, w, gx, gy, gz, gsw, ga, gd, X, st);
}

trips_status trips_export_fragments(const trips_config* cfg, const trips_camera* cams,
                                    int32_t views, const trips_tuning* tun, const void* saved,
                                    size_t saved_bytes, int32_t* counts, int32_t* ids,
                                    hipStream_t st) {
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, 0, tun, lay);
  if (s != TRIPS_OK) return s;
  if (!saved || !aligned(saved) || !counts || !ids) return TRIPS_ERR_INVALID_ARG;
  // the texel tables do not depend on n; only their part of `saved` is read
  if (saved_bytes < lay.s_tables_end) return TRIPS_ERR_WORKSPACE;
  const char* sv = static_cast<const char*>(saved);
  if (lay.P.NB > 0) {
    StageTimer tm(ST_EXPORT, st);
    hipLaunchKernelGGL(k_export, dim3(lay.P.NB), dim3(256), 0, st, lay.P,
                       reinterpret_cast<const uint32_t*>(sv + lay.s_npix),
                       reinterpret_cast<const uint64_t*>(sv + lay.s_kkey),
                       reinterpret_cast<const uint64_t*>(sv + lay.s_fkey),
                       reinterpret_cast<const uint32_t*>(sv + lay.s_fcnt), counts, ids);
    TRIPS_HIP(hipGetLastError());
  }
  return TRIPS_OK;
}

trips_status trips_forward_stats(const trips_config* cfg, const trips_camera* cams, int32_t views,
                                 const trips_tuning* tun, const void* saved, size_t saved_bytes,
                                 int64_t* stats, hipStream_t st) {
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, 0, tun, lay);
  if (s != TRIPS_OK) return s;
  if (!saved || !aligned(saved) || !stats) return TRIPS_ERR_INVALID_ARG;
  if (saved_bytes < lay.s_bin_start) return TRIPS_ERR_WORKSPACE;
  uint32_t info[5] = {0, 0, 0, 0, 0};
  TRIPS_HIP(hipMemcpyAsync(info, static_cast<const char*>(saved) + lay.s_info, sizeof(info),
                           hipMemcpyDeviceToHost, st));
  TRIPS_HIP(hipStreamSynchronize(st));
  stats[0] = info[0];
  stats[1] = int64_t(info[1]) + info[4];  // item workgroups + fine-tile workgroups
  stats[2] = lay.P.NB;
  stats[3] = info[2];
  return TRIPS_OK;
}

trips_status trips_tile_stats(const trips_config* cfg, const trips_camera* cams, int32_t views,
                              const trips_tuning* tun, const void* saved, size_t saved_bytes,
                              uint32_t* entries, uint32_t* kept, hipStream_t st) {
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, 0, tun, lay);
  if (s != TRIPS_OK) return s;
  if (!saved || !aligned(saved) || !entries || !kept) return TRIPS_ERR_INVALID_ARG;
  if (saved_bytes < lay.s_tables_end) return TRIPS_ERR_WORKSPACE;
  const size_t NB = lay.P.NB;
  std::vector<uint32_t> bs(NB + 1), np(NB * TP);
  const char* sv = static_cast<const char*>(saved);
  TRIPS_HIP(hipMemcpyAsync(bs.data(), sv + lay.s_bin_start, (NB + 1) * 4, hipMemcpyDeviceToHost, st));
  TRIPS_HIP(hipMemcpyAsync(np.data(), sv + lay.s_npix, NB * TP * 4, hipMemcpyDeviceToHost, st));
  TRIPS_HIP(hipStreamSynchronize(st));
  for (size_t b = 0; b < NB; ++b) {
    entries[b] = bs[b + 1] - bs[b];
    uint32_t k = 0;
    for (int t = 0; t < TP; ++t) k += std::min<uint32_t>(np[b * TP + t], KEEP);
    kept[b] = k;
  }
  return TRIPS_OK;
}

trips_status trips_autotune(const trips_config* cfg, const trips_points* pts,
                            const trips_camera* cams, int32_t views,
                            const trips_tuning* candidates, int32_t ncand, int32_t reps,
                            float* pyr, void* saved, size_t saved_bytes, void* ws,
                            size_t ws_bytes, const float* gpyr, float* gx, float* gy, float* gz,
                            float* gsw, float* ga, float* gd, trips_tuning* best,
                            float* ms_host, hipStream_t st) {
  if (!candidates || ncand < 1 || reps < 1 || !best || !ms_host) return TRIPS_ERR_INVALID_ARG;
  // validate every candidate before launching anything
  for (int c = 0; c < ncand; ++c) {
    Layout lay;
    trips_status s = make_layout(cfg, cams, views, pts ? pts->n : -1, &candidates[c], lay);
    if (s != TRIPS_OK) return s;
    if ((s = check_points(pts, lay)) != TRIPS_OK) return s;
    if ((s = check_buffers(lay, saved, saved_bytes, ws, ws_bytes, true)) != TRIPS_OK) return s;
  }
  if (!pyr || !aligned16(pyr) || !gpyr || !aligned16(gpyr)) return TRIPS_ERR_INVALID_ARG;
  if (pts->n > 0 && (!gx || !gy || !gz || !gsw || !ga || !gd || !aligned16(gd)))
    return TRIPS_ERR_INVALID_ARG;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TRIPS_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return TRIPS_ERR_HIP; }
  trips_status rs = TRIPS_OK;
  float best_ms = 0.0f;
  for (int c = 0; c < ncand && rs == TRIPS_OK; ++c) {
    float total = 0.0f;
    for (int r = -1; r < reps && rs == TRIPS_OK; ++r) {  // r = -1: warm-up
      hipError_t e = hipEventRecord(e0, st);
      if (e == hipSuccess) {
        rs = trips_forward(cfg, pts, cams, views, &candidates[c], pyr, saved, saved_bytes, ws,
                           ws_bytes, nullptr, st);
        if (rs == TRIPS_OK)
          rs = trips_backward(cfg, pts, cams, views, &candidates[c], gpyr, saved, saved_bytes, ws,
                              ws_bytes, gx, gy, gz, gsw, ga, gd, nullptr, st);
        if (rs == TRIPS_OK) e = hipEventRecord(e1, st);
        if (rs == TRIPS_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (rs == TRIPS_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (r >= 0) total += ms;
      }
      if (e != hipSuccess) { g_last_hip = int32_t(e); rs = TRIPS_ERR_HIP; }
    }
    if (rs != TRIPS_OK) break;
    ms_host[c] = total / float(reps);
    if (c == 0 || ms_host[c] < best_ms) { best_ms = ms_host[c]; *best = candidates[c]; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rs;
}

trips_status trips_plan_create(const trips_config* cfg, const trips_points* pts,
                               const trips_camera* cams, int32_t views, const trips_tuning* tun,
                               float* pyr, void* saved, size_t saved_bytes, void* ws,
                               size_t ws_bytes, const float* gpyr, float* gx, float* gy, float* gz,
                               float* gsw, float* ga, float* gd, const trips_extras* extras,
                               hipStream_t st, trips_plan** out) {
  if (!out || !st) return TRIPS_ERR_INVALID_ARG;  // the null stream cannot be captured
  *out = nullptr;
  Layout lay;
  trips_status s = make_layout(cfg, cams, views, pts ? pts->n : -1, tun, lay);
  if (s != TRIPS_OK) return s;
  if ((s = check_points(pts, lay)) != TRIPS_OK) return s;
  if ((s = check_buffers(lay, saved, saved_bytes, ws, ws_bytes, true)) != TRIPS_OK) return s;
  if (!pyr || !aligned16(pyr)) return TRIPS_ERR_INVALID_ARG;
  const bool bwd = gpyr != nullptr;
  if (bwd && (!aligned16(gpyr) ||
              (lay.P.n > 0 && (!gx || !gy || !gz || !gsw || !ga || !gd || !aligned16(gd)))))
    return TRIPS_ERR_INVALID_ARG;
  Extras xf, xb;
  if ((s = take_extras(extras, true, false, xf)) != TRIPS_OK) return s;
  if ((s = take_extras(extras, false, true, xb)) != TRIPS_OK) return s;
  trips_plan* pl = new (std::nothrow) trips_plan();
  if (!pl) return TRIPS_ERR_INVALID_ARG;
  pl->lay = lay;
  pl->xf = xf;
  pl->xb = xb;
  pl->pts = *pts;
  pl->pyr = pyr; pl->saved = saved; pl->ws = ws; pl->gpyr = gpyr;
  pl->gx = gx; pl->gy = gy; pl->gz = gz; pl->gsw = gsw; pl->ga = ga; pl->gd = gd;
  {  // the side stream is created before any capture begins
    SideStream* sd = nullptr;
    trips_status ss = side_stream(sd);
    if (ss != TRIPS_OK) { trips_plan_destroy(pl); return ss; }
  }
  for (int which = 1; which <= 3; ++which) {
    pl->exec[which - 1] = nullptr;
    if ((which & 2) && !bwd) continue;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { g_last_hip = e; trips_plan_destroy(pl); return TRIPS_ERR_HIP; }
    trips_status ls = TRIPS_OK;
    char* sv = static_cast<char*>(saved);
    char* w = static_cast<char*>(ws);
    if (which & 1)
      ls = lay.P.D == 4 ? launch_forward<4>(lay, pl->pts, pyr, sv, w, pl->xf, st)
                        : launch_forward<8>(lay, pl->pts, pyr, sv, w, pl->xf, st);
    if (ls == TRIPS_OK && (which & 2))
      ls = lay.P.D == 4 ? launch_backward<4>(lay, pl->pts, gpyr, sv, w, gx, gy, gz, gsw, ga, gd, pl->xb, st)
                        : launch_backward<8>(lay, pl->pts, gpyr, sv, w, gx, gy, gz, gsw, ga, gd, pl->xb, st);
    e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(st, &dead);
        if (dead) (void)hipGraphDestroy(dead);
      }
    }
    if (ls != TRIPS_OK || e != hipSuccess) {
      if (e != hipSuccess) g_last_hip = e;
      if (g) (void)hipGraphDestroy(g);
      trips_plan_destroy(pl);
      return ls != TRIPS_OK ? ls : TRIPS_ERR_HIP;
    }
    e = hipGraphInstantiate(&pl->exec[which - 1], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { g_last_hip = e; pl->exec[which - 1] = nullptr; trips_plan_destroy(pl); return TRIPS_ERR_HIP; }
  }
  *out = pl;
  return TRIPS_OK;
}

trips_status trips_plan_launch(trips_plan* pl, int32_t which, hipStream_t st) {
  if (!pl || which < 1 || which > 3 || !pl->exec[which - 1]) return TRIPS_ERR_INVALID_ARG;
  TRIPS_HIP(hipGraphLaunch(pl->exec[which - 1], st));
  return TRIPS_OK;
}

void trips_plan_destroy(trips_plan* pl) {
  if (!pl) return;
  for (auto& e : pl->exec)
    if (e) (void)hipGraphExecDestroy(e);
  delete pl;
}

}  // extern "C"
