/*
 * trips_oracle.c -- CPU oracle for trilinear point splatting (TRIPS, Franke et al. 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or table
 * with the GPU library, and the GPU library never calls it.
 *
 * What it computes (scatter form, one view):
 *   1. Project every point with a pinhole camera to continuous screen
 *      coordinates (x, y), camera depth z and screen size s = f * s_w / z
 *      (Sec. 3.1, Eq. 2).
 *   2. Choose the pyramid layers floor(log2 s) and ceil(log2 s) and the linear
 *      layer weight iota (Sec. 3.1, Eq. 5); points with s < 1 go to layer 0 only,
 *      with iota = eps + (1 - eps) s.
 *   3. Write a bilinear 2x2 footprint in each chosen layer with beta from Eq. 4;
 *      each fragment carries gamma = beta * iota * alpha (Eq. 3).
 *   4. Collect the fragments of every (layer, pixel), sort them by depth (ties by
 *      point index) and keep the front-most 16 (Sec. 3.2).  Optionally (coarser-layer
 *      inclusion, Sec. 3.6) the list of a texel also holds the fragments of the texels of
 *      all coarser layers that cover it.
 *   5. Blend front to back, C = sum_m T_m gamma_m tau_m with
 *      T_m = prod_{i<m} (1 - gamma_i) (Eq. 6-7).
 *   The backward pass is the analytic adjoint of steps 3-5 and of the projection,
 *   differentiated with respect to positions, world sizes, opacities and
 *   descriptors (the paper states the pipeline is differentiable in all four).
 *   The _ex entry points add the optional terms: a background composited behind the
 *   kept fragments (C += T_K bg, T_K the transmittance left after the kept list; the
 *   environment map E of Eq. 1 sampled per texel), the coverage 1 - T_K of every texel,
 *   and the gradients with respect to the background and to the camera (R, t, fx, fy,
 *   cx, cy of Eq. 2).
 *
 * Precision.  Two modes:
 *   fp32 = 1: the projection and every decision that picks an integer (culling,
 *     layer pair, texel indices, which corners exist, depth order) are taken in
 *     IEEE single precision with a fixed operation order (explicit fmaf,
 *     correctly rounded division).  That is the precision of the renderer, so the
 *     same decisions come out of any correct single-precision implementation.
 *     Weights, blending and gradients are then evaluated in double precision from
 *     those single-precision values.
 *   fp32 = 0: everything in double precision (used for finite differences).
 *
 * Readings of the paper that this file fixes (the paper is silent or garbled):
 *   - log is log2 (the layer texel size is 2^L); computed exactly with ilogb.
 *   - the second case of Eq. 5 (points smaller than a pixel) writes to layer index 0.
 *   - s an exact power of two 2^e: one layer e with iota = 1 (the Eq. 5
 *     denominator would be 0).  s >= 2^(n-1): the coarsest layer only, iota = 1.
 *   - texel (i, j) of layer L has its centre at ((i + 0.5) 2^L, (j + 0.5) 2^L)
 *     in full-resolution pixel units, so u = x / 2^L - 0.5; distances in Eq. 4
 *     are in layer-L texel units.
 *   - layer L has ceil(W / 2^L) x ceil(H / 2^L) texels.
 *   - a fragment exists iff its texel is inside the layer and both 1-D weights
 *     are non-zero; no renormalisation at borders.
 *   - depth is camera-space z, ascending; ties by point index ascending.
 *   - the alpha of Eq. 6 is the fragment's gamma; the colour is the descriptor.
 *   - without a background an empty list gives 0; with one, the background is seen
 *     through the transmittance the kept fragments leave (an empty list shows it whole).
 *   - the coverage output is 1 - T_K over the kept list (the blend of a constant 1).
 *   - f in Eq. 2 is f_x; points with z <= znear or non-finite x, y, s are culled.
 *   - coarser-layer inclusion (the paper names the usual way and no more): texel
 *     (i, j) of layer L takes in the fragments of texel (i >> k, j >> k) of layer L + k
 *     for every k >= 1, each with its own gamma; the union is ordered by depth, then point
 *     index, then layer (finer first: a point written to two layers appears twice), and
 *     clamped to 16.  The per-texel count output stays the number of the texel's own
 *     fragments.
 *
 * Compile with -O2 -ffp-contract=off and without -ffast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_MEM -2

typedef struct {
  int valid;
  double x, y, z, s;      /* screen x, y (pixels), camera depth, screen size */
  double Xc, Yc;          /* camera-space coordinates (for the chain rule) */
  int nl;                 /* number of layers the point is written to (0, 1, 2) */
  int L[2];
  double iota[2];         /* layer weight */
  double diota[2];        /* d iota / d s */
  /* footprint per layer entry (filled by footprint()) */
} proj_t;

typedef struct {
  int64_t pix;            /* pixel index over the concatenated layers of the view */
  double z;               /* depth key */
  int64_t idx;            /* point index */
  double gamma;
  int L, sel, di, dj;     /* layer, which layer entry, corner */
  double wx, wy;          /* 1-D bilinear weights of this corner */
} frag_t;

typedef struct {
  double R[9], t[3], fx, fy, cx, cy, znear;
  int W, H;
} cam_t;

static void unpack_cam(const double* cam, int W, int H, cam_t* c) {
  for (int k = 0; k < 9; ++k) c->R[k] = cam[k];
  for (int k = 0; k < 3; ++k) c->t[k] = cam[9 + k];
  c->fx = cam[12]; c->fy = cam[13]; c->cx = cam[14]; c->cy = cam[15]; c->znear = cam[16];
  c->W = W; c->H = H;
}

/* Layer L has ceil(W/2^L) x ceil(H/2^L) texels. */
static int layer_w(int W, int L) { return (int)(((int64_t)W + ((int64_t)1 << L) - 1) >> L); }

/* Step 2: layer pair and iota from the screen size s (Eq. 5). */
static void layers_from_size(double s, int nlayers, double eps, int fp32, proj_t* p) {
  double smax = ldexp(1.0, nlayers - 1);
  if (s < 1.0) {
    p->nl = 1; p->L[0] = 0;
    p->iota[0] = eps + (1.0 - eps) * s;
    p->diota[0] = 1.0 - eps;
  } else if (s >= smax) {
    p->nl = 1; p->L[0] = nlayers - 1; p->iota[0] = 1.0; p->diota[0] = 0.0;
  } else {
    int e;
    double t;
    if (fp32) { float sf = (float)s; e = ilogbf(sf); t = (double)ldexpf(sf, -e); }
    else { e = ilogb(s); t = ldexp(s, -e); }
    if (t == 1.0) {
      p->nl = 1; p->L[0] = e; p->iota[0] = 1.0; p->diota[0] = 0.0;
    } else {
      /* iota = 1 - |s - 2^L| / (2^(e+1) - 2^e): lower layer 2 - t, upper layer t - 1 */
      p->nl = 2;
      p->L[0] = e; p->iota[0] = 2.0 - t; p->diota[0] = -ldexp(1.0, -e);
      p->L[1] = e + 1; p->iota[1] = t - 1.0; p->diota[1] = ldexp(1.0, -e);
    }
  }
}

/* Step 1: pinhole projection (Sec. 3.1, Eq. 2). */
static void project(const cam_t* c, double X, double Y, double Z, double sw, int nlayers,
                    double eps, int fp32, proj_t* p) {
  memset(p, 0, sizeof(*p));
  if (fp32) {
    float R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = (float)c->R[k];
    for (int k = 0; k < 3; ++k) t[k] = (float)c->t[k];
    float fx = (float)c->fx, fy = (float)c->fy, cx = (float)c->cx, cy = (float)c->cy;
    float Xf = (float)X, Yf = (float)Y, Zf = (float)Z, swf = (float)sw;
    float Xc = fmaf(R[0], Xf, fmaf(R[1], Yf, fmaf(R[2], Zf, t[0])));
    float Yc = fmaf(R[3], Xf, fmaf(R[4], Yf, fmaf(R[5], Zf, t[1])));
    float Zc = fmaf(R[6], Xf, fmaf(R[7], Yf, fmaf(R[8], Zf, t[2])));
    if (!(Zc > (float)c->znear)) return;
    float qx = Xc / Zc, qy = Yc / Zc;
    float x = fmaf(fx, qx, cx);
    float y = fmaf(fy, qy, cy);
    float s = (fx * swf) / Zc;
    if (!isfinite(x) || !isfinite(y) || !isfinite(s) || !(s > 0.0f)) return;
    p->valid = 1;
    p->x = x; p->y = y; p->z = Zc; p->s = s; p->Xc = Xc; p->Yc = Yc;
  } else {
    const double* R = c->R;
    double Xc = fma(R[0], X, fma(R[1], Y, fma(R[2], Z, c->t[0])));
    double Yc = fma(R[3], X, fma(R[4], Y, fma(R[5], Z, c->t[1])));
    double Zc = fma(R[6], X, fma(R[7], Y, fma(R[8], Z, c->t[2])));
    if (!(Zc > c->znear)) return;
    double x = fma(c->fx, Xc / Zc, c->cx);
    double y = fma(c->fy, Yc / Zc, c->cy);
    double s = (c->fx * sw) / Zc;
    if (!isfinite(x) || !isfinite(y) || !isfinite(s) || !(s > 0.0)) return;
    p->valid = 1;
    p->x = x; p->y = y; p->z = Zc; p->s = s; p->Xc = Xc; p->Yc = Yc;
  }
  layers_from_size(p->s, nlayers, eps, fp32, p);
}

/* Step 3: the 2x2 footprint of one layer entry; appends fragments. */
static int64_t emit_layer(const cam_t* c, const proj_t* p, int sel, int64_t idx, double alpha,
                          int fp32, const int64_t* layer_base, const uint8_t* mask, frag_t* out,
                          int64_t nout) {
  int L = p->L[sel];
  int WL = layer_w(c->W, L), HL = layer_w(c->H, L);
  double u, v, fu, fv;
  int64_t i0, j0;
  if (fp32) {
    float uf = ldexpf((float)p->x, -L) - 0.5f;
    float vf = ldexpf((float)p->y, -L) - 0.5f;
    if (!(uf > -1.0f && uf < (float)WL && vf > -1.0f && vf < (float)HL)) return nout;
    float fl_u = floorf(uf), fl_v = floorf(vf);
    i0 = (int64_t)fl_u; j0 = (int64_t)fl_v;
    /* the fractional parts are taken exactly (in double) from the single-precision u, v */
    fu = (double)uf - (double)fl_u; fv = (double)vf - (double)fl_v;
    u = uf; v = vf;
  } else {
    u = ldexp(p->x, -L) - 0.5;
    v = ldexp(p->y, -L) - 0.5;
    if (!(u > -1.0 && u < (double)WL && v > -1.0 && v < (double)HL)) return nout;
    double fl_u = floor(u), fl_v = floor(v);
    i0 = (int64_t)fl_u; j0 = (int64_t)fl_v;
    fu = u - fl_u; fv = v - fl_v;
  }
  (void)u; (void)v;
  double wxs[2] = {1.0 - fu, fu};
  double wys[2] = {1.0 - fv, fv};
  for (int dj = 0; dj < 2; ++dj) {
    for (int di = 0; di < 2; ++di) {
      int64_t i = i0 + di, j = j0 + dj;
      if (i < 0 || i >= WL || j < 0 || j >= HL) continue;
      double wx = wxs[di], wy = wys[dj];
      if (wx == 0.0 || wy == 0.0) continue;
      int64_t pix = layer_base[L] + j * WL + i;
      if (mask && !mask[pix]) continue; /* texel not requested */
      frag_t* f = &out[nout++];
      f->pix = pix;
      f->z = p->z;
      f->idx = idx;
      f->gamma = ((wx * wy) * p->iota[sel]) * alpha;
      f->L = L; f->sel = sel; f->di = di; f->dj = dj;
      f->wx = wx; f->wy = wy;
    }
  }
  return nout;
}

/* Blend order inside one texel's list (Sec. 3.2): depth ascending, ties by point index;
   with coarser-layer inclusion a point can appear twice (its two layers), and then the
   fragment of the finer layer comes first. */
static int order_cmp(const void* a, const void* b) {
  const frag_t* x = (const frag_t*)a;
  const frag_t* y = (const frag_t*)b;
  if (x->z != y->z) return x->z < y->z ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  if (x->L != y->L) return x->L < y->L ? -1 : 1;
  return 0;
}

static int frag_cmp(const void* a, const void* b) {
  const frag_t* x = (const frag_t*)a;
  const frag_t* y = (const frag_t*)b;
  if (x->pix != y->pix) return x->pix < y->pix ? -1 : 1;
  return order_cmp(a, b);
}

static void layer_bases(int W, int H, int nlayers, int64_t* base) {
  base[0] = 0;
  for (int L = 0; L < nlayers; ++L)
    base[L + 1] = base[L] + (int64_t)layer_w(W, L) * layer_w(H, L);
}

/* Steps 1-4 for one view: every fragment, sorted by (pixel, depth, index). */
static frag_t* collect(int64_t n, const double* X, const double* Y, const double* Z,
                       const double* SW, const double* A, const cam_t* c, int nlayers,
                       double eps, int fp32, const uint8_t* mask, int64_t* nfrag_out,
                       proj_t** proj_out) {
  int64_t base[33];
  layer_bases(c->W, c->H, nlayers, base);
  proj_t* pr = (proj_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(proj_t));
  frag_t* fr = (frag_t*)malloc((size_t)(n > 0 ? 8 * n : 1) * sizeof(frag_t));
  if (!pr || !fr) { free(pr); free(fr); return NULL; }
  int64_t nf = 0;
  for (int64_t p = 0; p < n; ++p) {
    project(c, X[p], Y[p], Z[p], SW[p], nlayers, eps, fp32, &pr[p]);
    if (!pr[p].valid) continue;
    double alpha = fp32 ? (double)(float)A[p] : A[p];
    for (int sel = 0; sel < pr[p].nl; ++sel)
      nf = emit_layer(c, &pr[p], sel, p, alpha, fp32, base, mask, fr, nf);
  }
  qsort(fr, (size_t)nf, sizeof(frag_t), frag_cmp);
  *nfrag_out = nf;
  if (proj_out) *proj_out = pr; else free(pr);
  return fr;
}

static int check_args(int64_t n, int D, int W, int H, int nlayers, int maxlist) {
  if (D > 64) return 0;
  if (n < 0 || D < 1 || W < 1 || H < 1 || nlayers < 1 || nlayers > 30 || maxlist < 1) return 0;
  return 1;
}

/* Start of every texel's run in the (pixel, depth, index)-sorted fragments: run[pix] ..
   run[pix + 1]. */
static int64_t* texel_runs(const frag_t* fr, int64_t nf, int64_t P) {
  int64_t* run = (int64_t*)calloc((size_t)P + 1, sizeof(int64_t));
  if (!run) return NULL;
  for (int64_t k = 0; k < nf; ++k) run[fr[k].pix + 1]++;
  for (int64_t pix = 0; pix < P; ++pix) run[pix + 1] += run[pix];
  return run;
}

/* Coarser-layer inclusion (Sec. 3.6): texel (i, j) of layer L also blends
   the fragments of the texel (i >> k, j >> k) of every coarser layer L + k, the texel of
   that layer that covers it.  Returns the list of texel pix in blend order (own fragments
   alone without inclusion); buf has room for every fragment. */
static const frag_t* texel_list(const frag_t* fr, const int64_t* run, const int64_t* base,
                                int W, int nlayers, int64_t pix, int coarser, frag_t* buf,
                                int64_t* len) {
  if (!coarser) {
    *len = run[pix + 1] - run[pix];
    return fr + run[pix];
  }
  int L = 0;
  while (pix >= base[L + 1]) ++L;
  int64_t local = pix - base[L];
  int64_t WL = layer_w(W, L);
  int64_t i = local % WL, j = local / WL;
  int64_t m = 0;
  for (int k = 0; L + k < nlayers; ++k) {
    int64_t q = base[L + k] + (j >> k) * layer_w(W, L + k) + (i >> k);
    for (int64_t a = run[q]; a < run[q + 1]; ++a) buf[m++] = fr[a];
  }
  qsort(buf, (size_t)m, sizeof(frag_t), order_cmp);
  *len = m;
  return buf;
}

/* With inclusion, the fragments a masked texel needs lie in it and in its ancestors. */
static uint8_t* ancestor_mask(const uint8_t* mask, int W, int H, int nlayers) {
  int64_t base[33];
  layer_bases(W, H, nlayers, base);
  uint8_t* m = (uint8_t*)malloc((size_t)base[nlayers]);
  if (!m) return NULL;
  memcpy(m, mask, (size_t)base[nlayers]);
  for (int L = 0; L + 1 < nlayers; ++L) {
    int64_t WL = layer_w(W, L), HL = layer_w(H, L), WP = layer_w(W, L + 1);
    for (int64_t j = 0; j < HL; ++j)
      for (int64_t i = 0; i < WL; ++i)
        if (m[base[L] + j * WL + i]) m[base[L + 1] + (j >> 1) * WP + (i >> 1)] = 1;
  }
  return m;
}

/* Number of texels of all layers of a W x H view. */
int64_t oracle_num_pixels(int W, int H, int nlayers) {
  if (W < 1 || H < 1 || nlayers < 1 || nlayers > 30) return -1;
  int64_t base[33];
  layer_bases(W, H, nlayers, base);
  return base[nlayers];
}

/* Step 1 alone, for tests: valid flag, x, y, z, s per point. */
int oracle_project(int64_t n, const double* X, const double* Y, const double* Z, const double* SW,
                   const double* cam, int W, int H, int nlayers, double eps, int fp32,
                   int32_t* valid, double* xyzs /* [n][4] */) {
  if (n < 0 || W < 1 || H < 1 || nlayers < 1) return OR_ERR_ARG;
  cam_t c;
  unpack_cam(cam, W, H, &c);
  for (int64_t p = 0; p < n; ++p) {
    proj_t pr;
    project(&c, X[p], Y[p], Z[p], SW[p], nlayers, eps, fp32, &pr);
    valid[p] = pr.valid;
    xyzs[4 * p + 0] = pr.x; xyzs[4 * p + 1] = pr.y; xyzs[4 * p + 2] = pr.z; xyzs[4 * p + 3] = pr.s;
  }
  return OR_OK;
}

/* Steps 1-4, for tests: every fragment in (pixel, depth, index) order.
   Returns the fragment count (or a negative error); writes at most cap rows:
   idx, layer, texel i, texel j, and per fragment gamma, beta (= wx*wy), iota, depth. */
int64_t oracle_fragments(int64_t n, const double* X, const double* Y, const double* Z,
                         const double* SW, const double* A, const double* cam, int W, int H,
                         int nlayers, double eps, int fp32, int64_t cap, int64_t* ints /* [cap][4] */,
                         double* reals /* [cap][4] */) {
  if (!check_args(n, 1, W, H, nlayers, 1)) return OR_ERR_ARG;
  cam_t c;
  unpack_cam(cam, W, H, &c);
  int64_t nf = 0;
  proj_t* pr = NULL;
  frag_t* fr = collect(n, X, Y, Z, SW, A, &c, nlayers, eps, fp32, NULL, &nf, &pr);
  if (!fr) return OR_ERR_MEM;
  for (int64_t k = 0; k < nf && k < cap; ++k) {
    const frag_t* f = &fr[k];
    int WL = layer_w(W, f->L);
    int64_t base[33];
    layer_bases(W, H, nlayers, base);
    int64_t local = f->pix - base[f->L];
    ints[4 * k + 0] = f->idx; ints[4 * k + 1] = f->L;
    ints[4 * k + 2] = local % WL; ints[4 * k + 3] = local / WL;
    reals[4 * k + 0] = f->gamma; reals[4 * k + 1] = f->wx * f->wy;
    reals[4 * k + 2] = pr[f->idx].iota[f->sel]; reals[4 * k + 3] = f->z;
  }
  free(fr); free(pr);
  return nf;
}

/* Forward, one view.  pyr: [sum_L H_L W_L][D] (layers concatenated, each row-major);
   counts: untruncated number of the texel's own fragments; ids: [P][maxlist] kept point
   indices in blend order, -1 padded.  mask (optional, [P] bytes): only texels with a
   non-zero mask byte are evaluated; the others are left at 0 / -1.  bg (optional, [P][D]):
   background composited behind the kept list; alpha (optional, [P]): coverage 1 - T_K.
   Texels outside the mask keep bg = 0 and alpha = 0 too.  coarser: blend each texel's
   fragments together with those of the texels of coarser layers that cover it. */
int oracle_forward_ex(int64_t n, const double* X, const double* Y, const double* Z,
                      const double* SW, const double* A, const double* DESC, int D,
                      const double* cam, int W, int H, int nlayers, int maxlist, double eps,
                      int fp32, int coarser, const uint8_t* mask, const double* bg, double* pyr,
                      int32_t* counts, int64_t* ids, double* alpha) {
  if (!check_args(n, D, W, H, nlayers, maxlist)) return OR_ERR_ARG;
  cam_t c;
  unpack_cam(cam, W, H, &c);
  int64_t P = oracle_num_pixels(W, H, nlayers);
  int64_t base[33];
  layer_bases(W, H, nlayers, base);
  memset(pyr, 0, (size_t)P * D * sizeof(double));
  memset(counts, 0, (size_t)P * sizeof(int32_t));
  if (alpha) memset(alpha, 0, (size_t)P * sizeof(double));
  for (int64_t k = 0; k < P * maxlist; ++k) ids[k] = -1;
  uint8_t* cmask = (coarser && mask) ? ancestor_mask(mask, W, H, nlayers) : NULL;
  if (coarser && mask && !cmask) return OR_ERR_MEM;
  int64_t nf = 0;
  frag_t* fr = collect(n, X, Y, Z, SW, A, &c, nlayers, eps, fp32, cmask ? cmask : mask, &nf, NULL);
  free(cmask);
  if (!fr) return OR_ERR_MEM;
  int64_t* run = texel_runs(fr, nf, P);
  frag_t* buf = (frag_t*)malloc((size_t)(nf > 0 ? nf : 1) * sizeof(frag_t));
  if (!run || !buf) { free(fr); free(run); free(buf); return OR_ERR_MEM; }
  for (int64_t pix = 0; pix < P; ++pix) {
    if (mask && !mask[pix]) continue;
    int64_t len = 0;
    const frag_t* list = texel_list(fr, run, base, W, nlayers, pix, coarser, buf, &len);
    counts[pix] = (int32_t)(run[pix + 1] - run[pix]);
    int64_t keep = len < maxlist ? len : maxlist;
    double T = 1.0;
    double col[64];
    for (int d = 0; d < D; ++d) col[d] = 0.0;
    for (int64_t m = 0; m < keep; ++m) {
      const frag_t* f = &list[m];
      ids[pix * maxlist + m] = f->idx;
      double w = T * f->gamma;
      for (int d = 0; d < D; ++d) {
        double tau = fp32 ? (double)(float)DESC[f->idx * D + d] : DESC[f->idx * D + d];
        col[d] += w * tau;
      }
      T = T * (1.0 - f->gamma);
    }
    /* an empty list shows the whole background */
    for (int d = 0; d < D; ++d) pyr[pix * D + d] = col[d] + (bg ? T * bg[pix * D + d] : 0.0);
    if (alpha) alpha[pix] = 1.0 - T;
  }
  free(fr); free(run); free(buf);
  return OR_OK;
}

int oracle_forward(int64_t n, const double* X, const double* Y, const double* Z, const double* SW,
                   const double* A, const double* DESC, int D, const double* cam, int W, int H,
                   int nlayers, int maxlist, double eps, int fp32, const uint8_t* mask,
                   double* pyr, int32_t* counts, int64_t* ids) {
  return oracle_forward_ex(n, X, Y, Z, SW, A, DESC, D, cam, W, H, nlayers, maxlist, eps, fp32,
                           0, mask, NULL, pyr, counts, ids, NULL);
}

/* Backward, one view: gradients of sum(G * pyr) (+ sum(Galpha * alpha) when Galpha is
   given) with respect to X, Y, Z, SW, A and DESC; with bg, the background the forward
   composited; gbg (optional, [P][D]) receives dL/dbg = T_K G and gcam (optional, [16])
   the camera gradient: dL/dR (row-major), dL/dt, dL/dfx, dL/dfy, dL/dcx, dL/dcy.
   Outputs are overwritten.  The depth order, culling and the 16-element clamp are
   piecewise constant and carry no gradient; fragments beyond the clamp get none.
   mask (optional): only texels with a non-zero mask byte contribute, so a point's
   gradient is exact when every texel it writes is in the mask (with inclusion: every
   texel whose list can hold its fragments).  coarser: as in oracle_forward_ex; a
   fragment included in finer texels' lists collects the adjoint of every list it is
   kept in. */
int oracle_backward_ex(int64_t n, const double* X, const double* Y, const double* Z,
                       const double* SW, const double* A, const double* DESC, int D,
                       const double* cam, int W, int H, int nlayers, int maxlist, double eps,
                       int fp32, int coarser, const uint8_t* mask, const double* bg,
                       const double* G, const double* Galpha, double* gX, double* gY, double* gZ,
                       double* gSW, double* gA, double* gDESC, double* gbg, double* gcam) {
  if (!check_args(n, D, W, H, nlayers, maxlist)) return OR_ERR_ARG;
  cam_t c;
  unpack_cam(cam, W, H, &c);
  int64_t P = oracle_num_pixels(W, H, nlayers);
  int64_t base[33];
  layer_bases(W, H, nlayers, base);
  uint8_t* cmask = (coarser && mask) ? ancestor_mask(mask, W, H, nlayers) : NULL;
  if (coarser && mask && !cmask) return OR_ERR_MEM;
  int64_t nf = 0;
  proj_t* pr = NULL;
  frag_t* fr = collect(n, X, Y, Z, SW, A, &c, nlayers, eps, fp32, cmask ? cmask : mask, &nf, &pr);
  free(cmask);
  if (!fr) return OR_ERR_MEM;
  double* gxs = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* gys = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* gss = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* Tm = (double*)malloc((size_t)maxlist * sizeof(double));
  int64_t* run = texel_runs(fr, nf, P);
  frag_t* buf = (frag_t*)malloc((size_t)(nf > 0 ? nf : 1) * sizeof(frag_t));
  if (!gxs || !gys || !gss || !Tm || !run || !buf) {
    free(fr); free(pr); free(gxs); free(gys); free(gss); free(Tm); free(run); free(buf);
    return OR_ERR_MEM;
  }
  memset(gA, 0, (size_t)n * sizeof(double));
  memset(gDESC, 0, (size_t)n * D * sizeof(double));
  if (gcam) memset(gcam, 0, 16 * sizeof(double));
  if (gbg) memset(gbg, 0, (size_t)P * D * sizeof(double));
  for (int64_t pix = 0; pix < P; ++pix) {
    if (mask && !mask[pix]) continue;
    int64_t len = 0;
    const frag_t* list = texel_list(fr, run, base, W, nlayers, pix, coarser, buf, &len);
    int64_t keep = len < maxlist ? len : maxlist;
    const double* g = &G[pix * D];
    double T = 1.0;
    for (int64_t m = 0; m < keep; ++m) { Tm[m] = T; T = T * (1.0 - list[m].gamma); }
    if (gbg)
      for (int d = 0; d < D; ++d) gbg[pix * D + d] = T * g[d];
    /* Reverse sweep.  With g_m = G . tau_m (+ Galpha: the coverage blends a constant 1),
       the output is C.G = sum_m T_m gamma_m g_m + T_K (G . bg);
       B_m = sum_{i>m} (T_i / T_{m+1}) gamma_i g_i + (T_K / T_{m+1}) G . bg is the
       normalised tail behind m, built back to front: B_last = G . bg,
       B_{m-1} = gamma_m g_m + (1 - gamma_m) B_m.  Then dC.G/dgamma_m = T_m (g_m - B_m),
       with no division by (1 - gamma). */
    double B = 0.0;
    if (bg)
      for (int d = 0; d < D; ++d) B += g[d] * bg[pix * D + d];
    for (int64_t m = keep - 1; m >= 0; --m) {
      const frag_t* f = &list[m];
      int64_t p = f->idx;
      double gm = 0.0;
      for (int d = 0; d < D; ++d) {
        double tau = fp32 ? (double)(float)DESC[p * D + d] : DESC[p * D + d];
        gm += g[d] * tau;
      }
      if (Galpha) gm += Galpha[pix];
      double w = Tm[m] * f->gamma;
      for (int d = 0; d < D; ++d) gDESC[p * D + d] += w * g[d];
      double dgam = Tm[m] * (gm - B);
      B = f->gamma * gm + (1.0 - f->gamma) * B;
      const proj_t* q = &pr[p];
      double alpha = fp32 ? (double)(float)A[p] : A[p];
      double iota = q->iota[f->sel];
      double scale = ldexp(1.0, -f->L);
      double sx = f->di ? 1.0 : -1.0;
      double sy = f->dj ? 1.0 : -1.0;
      gA[p] += dgam * f->wx * f->wy * iota;
      gxs[p] += dgam * iota * alpha * sx * f->wy * scale;
      gys[p] += dgam * iota * alpha * f->wx * sy * scale;
      gss[p] += dgam * f->wx * f->wy * alpha * q->diota[f->sel];
    }
  }
  for (int64_t p = 0; p < n; ++p) {
    gX[p] = gY[p] = gZ[p] = gSW[p] = 0.0;
    const proj_t* q = &pr[p];
    if (!q->valid) continue;
    double fx = fp32 ? (double)(float)c.fx : c.fx;
    double fy = fp32 ? (double)(float)c.fy : c.fy;
    double R[9];
    for (int k = 0; k < 9; ++k) R[k] = fp32 ? (double)(float)c.R[k] : c.R[k];
    double Zc = q->z;
    double dXc = gxs[p] * fx / Zc;
    double dYc = gys[p] * fy / Zc;
    double dZc = -(gxs[p] * fx * q->Xc / Zc + gys[p] * fy * q->Yc / Zc + gss[p] * q->s) / Zc;
    gX[p] = R[0] * dXc + R[3] * dYc + R[6] * dZc;
    gY[p] = R[1] * dXc + R[4] * dYc + R[7] * dZc;
    gZ[p] = R[2] * dXc + R[5] * dYc + R[8] * dZc;
    gSW[p] = gss[p] * fx / Zc;
    if (gcam) {
      /* X_c = R X_w + t: dL/dR_rc = dL/dX_c[r] X_w[c], dL/dt = dL/dX_c;
         x = fx X_c/Z_c + cx, y = fy Y_c/Z_c + cy, s = fx s_w / Z_c */
      double Xw[3], dX[3] = {dXc, dYc, dZc};
      Xw[0] = fp32 ? (double)(float)X[p] : X[p];
      Xw[1] = fp32 ? (double)(float)Y[p] : Y[p];
      Xw[2] = fp32 ? (double)(float)Z[p] : Z[p];
      double sw = fp32 ? (double)(float)SW[p] : SW[p];
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) gcam[3 * r + k] += dX[r] * Xw[k];
      for (int r = 0; r < 3; ++r) gcam[9 + r] += dX[r];
      gcam[12] += gxs[p] * q->Xc / Zc + gss[p] * sw / Zc;
      gcam[13] += gys[p] * q->Yc / Zc;
      gcam[14] += gxs[p];
      gcam[15] += gys[p];
    }
  }
  free(fr); free(pr); free(gxs); free(gys); free(gss); free(Tm); free(run); free(buf);
  return OR_OK;
}

int oracle_backward(int64_t n, const double* X, const double* Y, const double* Z, const double* SW,
                    const double* A, const double* DESC, int D, const double* cam, int W, int H,
                    int nlayers, int maxlist, double eps, int fp32, const uint8_t* mask,
                    const double* G, double* gX, double* gY, double* gZ, double* gSW, double* gA,
                    double* gDESC) {
  return oracle_backward_ex(n, X, Y, Z, SW, A, DESC, D, cam, W, H, nlayers, maxlist, eps, fp32,
                            0, mask, NULL, G, NULL, gX, gY, gZ, gSW, gA, gDESC, NULL, NULL);
}
