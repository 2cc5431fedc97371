/*
 * gs_oracle.c -- FP64 CPU reference renderer for tile-based 3D Gaussian Splatting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library calls, links or
 * includes this file; only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * What it computes (the plain definition of the rendered image):
 *   - per Gaussian (paper, Background: frustum culling and feature
 *     computation): camera transform, near-plane cull, covariance from scale
 *     and rotation, first-order (EWA) projection of the covariance with a
 *     0.3 px^2 screen-space dilation, conic = inverse 2D covariance, projected
 *     mean, 3-sigma square footprint, 16x16 tile rectangle, view-dependent
 *     colour from real spherical harmonics, depth = camera-space z;
 *   - per tile (Background: Gaussian sorting): the Gaussians whose rectangle
 *     covers the tile, ordered by (depth, index);
 *   - per pixel (Background: rasterization, eq. power_d and eq. power, the
 *     alpha and transmittance definitions): d = x - mu', power = -1/2 d^T
 *     Sigma'^-1 d, alpha = min(0.99, o exp(power)), contributions with
 *     alpha < 1/255 skipped, front-to-back C += alpha T c, stop before the
 *     Gaussian that would take T below 1e-4;
 *   - grouped lists (Cross-tile grouping, Algorithm 1): one entry per
 *     overlapped group of GxG tiles with a tile-membership bit mask, ordered
 *     by (depth, index).
 * Everything is double precision, single-threaded per tile; the composite
 * step can spread tiles over threads with identical per-tile arithmetic.
 *
 * Pinned by the CPU tests: closed-form single-Gaussian projection and image,
 * finite-difference Jacobian, clamp invariance, SH against a library
 * spherical-harmonics routine and by quadrature, brute-force tile overlap,
 * Porter-Duff over for two co-centred Gaussians, the telescoping identity
 * sum(alpha T) + T_final = 1, permutation invariance and an independent
 * numpy brute-force renderer on tiny images.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TILE 16
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_ALPHA_MAX 0.99
#define OR_T_MIN 1e-4
#define OR_DILATE 0.3
#define OR_CLAMP 1.3
/* guard bands of decisions that FP32 arithmetic may take either way */
#define OR_GUARD_LNA 1e-4 /* relative, on alpha against the 1/255 cut */
#define OR_GUARD_LNT 2e-3 /* relative, on T against the 1e-4 stop (1 - alpha near 0.01 amplifies alpha error) */
#define OR_GUARD_PX 1e-3  /* pixels, on footprint edges */
#define OR_GUARD_Z 1e-6   /* near plane (absolute) and depth ties (relative) */

/* record flags */
#define OR_VISIBLE 1u
#define OR_AMB_ZNEAR 2u
#define OR_AMB_X0 4u
#define OR_AMB_X1 8u
#define OR_AMB_Y0 16u
#define OR_AMB_Y1 32u

/* per-pixel ambiguity flags */
#define OR_PIX_ALPHA 1u
#define OR_PIX_T 2u
#define OR_PIX_TIE 4u
#define OR_PIX_MEMBER 8u

/* ------------------------------------------------------------------------ */
/* Real orthonormal spherical harmonics.                                     */
/* Y_{l,m}, index l*l + l + m.  With the Condon-Shortley phase in P_l^m:     */
/*   m > 0: sqrt(2) K_l^m P_l^m(cos t) cos(m p)                              */
/*   m < 0: sqrt(2) K_l^|m| P_l^|m|(cos t) sin(|m| p)                        */
/*   m = 0: K_l^0 P_l^0(cos t)                                               */
/*   K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)                               */
/* ------------------------------------------------------------------------ */
static double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

/* associated Legendre P_l^m(x), 0 <= m <= l, with the (-1)^m phase */
static double assoc_legendre(int l, int m, double x) {
  double pmm = 1.0;
  double s = sqrt(fmax(0.0, 1.0 - x * x));
  for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
  if (l == m) return pmm;
  double pm1 = x * (2.0 * m + 1.0) * pmm;
  if (l == m + 1) return pm1;
  double pl = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
    pmm = pm1;
    pm1 = pl;
  }
  return pl;
}

void oracle_sh_basis(int deg, const double *dir, double *out) {
  double ct = dir[2];
  double phi = atan2(dir[1], dir[0]);
  for (int l = 0; l <= deg; ++l) {
    for (int m = -l; m <= l; ++m) {
      int am = m < 0 ? -m : m;
      double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
      double P = assoc_legendre(l, am, ct);
      double y;
      if (m > 0)
        y = sqrt(2.0) * K * P * cos(am * phi);
      else if (m < 0)
        y = sqrt(2.0) * K * P * sin(am * phi);
      else
        y = K * P;
      out[l * l + l + m] = y;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Per-Gaussian preprocessing.                                               */
/* cam: R[9] (row-major world->camera), t[3], fx, fy, cx, cy, znear (float)  */
/* ------------------------------------------------------------------------ */
static double near_int_dist(double v) { return fabs(v - floor(v + 0.5)); }

void oracle_preprocess(int64_t n, int deg, const float *mean, const float *log_scale,
                       const float *quat, const float *sh,
                       const float *cam, int W, int H,
                       double *xy, double *depth, double *cov2d, double *conic,
                       double *rgb, double *radius, int32_t *rect, uint8_t *flags) {
  double R[9], T[3];
  for (int i = 0; i < 9; ++i) R[i] = cam[i];
  for (int i = 0; i < 3; ++i) T[i] = cam[9 + i];
  double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15], znear = cam[16];
  int TX = (W + OR_TILE - 1) / OR_TILE, TY = (H + OR_TILE - 1) / OR_TILE;
  /* camera centre in world space: -R^T t */
  double campos[3];
  for (int i = 0; i < 3; ++i) campos[i] = -(R[0 * 3 + i] * T[0] + R[1 * 3 + i] * T[1] + R[2 * 3 + i] * T[2]);
  int nb = (deg + 1) * (deg + 1);
  double limx = OR_CLAMP * (0.5 * W) / fx, limy = OR_CLAMP * (0.5 * H) / fy;

  for (int64_t g = 0; g < n; ++g) {
    uint8_t fl = 0;
    xy[2 * g] = xy[2 * g + 1] = 0.0;
    depth[g] = 0.0;
    for (int k = 0; k < 3; ++k) { cov2d[3 * g + k] = 0.0; conic[3 * g + k] = 0.0; rgb[3 * g + k] = 0.0; }
    radius[g] = 0.0;
    for (int k = 0; k < 4; ++k) rect[4 * g + k] = 0;

    double p[3] = {mean[g], mean[n + g], mean[2 * n + g]};
    double tc[3];
    for (int i = 0; i < 3; ++i) tc[i] = R[3 * i] * p[0] + R[3 * i + 1] * p[1] + R[3 * i + 2] * p[2] + T[i];
    double tz = tc[2];
    int near_amb = fabs(tz - znear) < OR_GUARD_Z;
    if (tz <= znear && !near_amb) { flags[g] = 0; continue; }
    if (near_amb) fl |= OR_AMB_ZNEAR;

    /* 3D covariance Sigma = M S S^T M^T */
    double s[3];
    for (int i = 0; i < 3; ++i) s[i] = exp((double)log_scale[i * n + g]);
    double qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
    double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    double M[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                   2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                   2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    double Sig[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += M[3 * i + k] * s[k] * s[k] * M[3 * j + k];
        Sig[3 * i + j] = acc;
      }
    /* camera-space covariance V = R Sigma R^T */
    double RS[9], V[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += R[3 * i + k] * Sig[3 * k + j];
        RS[3 * i + j] = acc;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += RS[3 * i + k] * R[3 * j + k];
        V[3 * i + j] = acc;
      }
    /* Jacobian of the perspective map at the (laterally clamped) centre */
    double ux = tc[0] / tz, uy = tc[1] / tz;
    ux = fmin(fmax(ux, -limx), limx);
    uy = fmin(fmax(uy, -limy), limy);
    double txc = ux * tz, tyc = uy * tz;
    double J[6] = {fx / tz, 0.0, -fx * txc / (tz * tz), 0.0, fy / tz, -fy * tyc / (tz * tz)};
    double JV[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += J[3 * i + k] * V[3 * k + j];
        JV[3 * i + j] = acc;
      }
    double C2[4];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += JV[3 * i + k] * J[3 * j + k];
        C2[2 * i + j] = acc;
      }
    double sxx = C2[0] + OR_DILATE, sxy = 0.5 * (C2[1] + C2[2]), syy = C2[3] + OR_DILATE;
    double det = sxx * syy - sxy * sxy;
    if (!(det > 0.0)) { flags[g] = 0; continue; }
    double a = syy / det, b = -sxy / det, c = sxx / det;
    double mx = fx * tc[0] / tz + cx, my = fy * tc[1] / tz + cy;
    double mid = 0.5 * (sxx + syy);
    double lmax = mid + sqrt(fmax(mid * mid - det, 0.0));
    double r = 3.0 * sqrt(lmax);

    double lox = (mx - r) / OR_TILE, hix = (mx + r) / OR_TILE;
    double loy = (my - r) / OR_TILE, hiy = (my + r) / OR_TILE;
    if (near_int_dist(lox) < OR_GUARD_PX / OR_TILE) fl |= OR_AMB_X0;
    if (near_int_dist(hix) < OR_GUARD_PX / OR_TILE) fl |= OR_AMB_X1;
    if (near_int_dist(loy) < OR_GUARD_PX / OR_TILE) fl |= OR_AMB_Y0;
    if (near_int_dist(hiy) < OR_GUARD_PX / OR_TILE) fl |= OR_AMB_Y1;
    double fx0 = floor(lox), fx1 = floor(hix), fy0 = floor(loy), fy1 = floor(hiy);
    int x0 = (int)fmax(fx0, 0.0), x1 = (int)fmin(fx1, TX - 1.0);
    int y0 = (int)fmax(fy0, 0.0), y1 = (int)fmin(fy1, TY - 1.0);

    xy[2 * g] = mx;
    xy[2 * g + 1] = my;
    depth[g] = tz;
    cov2d[3 * g] = sxx; cov2d[3 * g + 1] = sxy; cov2d[3 * g + 2] = syy;
    conic[3 * g] = a; conic[3 * g + 1] = b; conic[3 * g + 2] = c;
    radius[g] = r;

    /* colour */
    double d[3] = {p[0] - campos[0], p[1] - campos[1], p[2] - campos[2]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; ++i) d[i] /= dn;
    double Y[16];
    oracle_sh_basis(deg, d, Y);
    for (int ch = 0; ch < 3; ++ch) {
      double acc = 0.0;
      for (int k = 0; k < nb; ++k) acc += (double)sh[((int64_t)k * 3 + ch) * n + g] * Y[k];
      acc += 0.5;
      rgb[3 * g + ch] = acc < 0.0 ? 0.0 : acc;
    }

    int empty = (x0 > x1) || (y0 > y1);
    /* the rectangle is stored half-open even when empty-but-ambiguous */
    rect[4 * g] = x0; rect[4 * g + 1] = y0; rect[4 * g + 2] = x1 + 1; rect[4 * g + 3] = y1 + 1;
    if (!empty && !(tz <= znear)) fl |= OR_VISIBLE;
    if (empty) {
      rect[4 * g] = rect[4 * g + 1] = rect[4 * g + 2] = rect[4 * g + 3] = 0;
    }
    flags[g] = fl;
  }
}

/* ------------------------------------------------------------------------ */
/* Lists per bin (tile when G == 1, group of GxG tiles otherwise).           */
/* ------------------------------------------------------------------------ */
typedef struct { double z; int64_t id; uint64_t mask; } or_entry;

static int cmp_entry(const void *pa, const void *pb) {
  const or_entry *a = (const or_entry *)pa, *b = (const or_entry *)pb;
  if (a->z < b->z) return -1;
  if (a->z > b->z) return 1;
  return (a->id > b->id) - (a->id < b->id);
}

/* Returns the total entry count.  With start == NULL only counts.
 * start[nbins+1], ids[count], masks[count] (bit (ty%G)*G + (tx%G) per member tile). */
int64_t oracle_lists(int64_t n, const int32_t *rect, const double *depth, const uint8_t *flags,
                     int W, int H, int G, int64_t *start, int64_t *ids, uint64_t *masks) {
  int TX = (W + OR_TILE - 1) / OR_TILE, TY = (H + OR_TILE - 1) / OR_TILE;
  int GX = (TX + G - 1) / G, GY = (TY + G - 1) / G;
  int64_t nbins = (int64_t)GX * GY;
  int64_t *cnt = (int64_t *)calloc((size_t)nbins, sizeof(int64_t));
  int64_t total = 0;
  for (int64_t g = 0; g < n; ++g) {
    if (!(flags[g] & OR_VISIBLE)) continue;
    int gx0 = rect[4 * g] / G, gx1 = (rect[4 * g + 2] - 1) / G;
    int gy0 = rect[4 * g + 1] / G, gy1 = (rect[4 * g + 3] - 1) / G;
    for (int gy = gy0; gy <= gy1; ++gy)
      for (int gx = gx0; gx <= gx1; ++gx) { cnt[(int64_t)gy * GX + gx]++; total++; }
  }
  if (!start) { free(cnt); return total; }
  start[0] = 0;
  for (int64_t b = 0; b < nbins; ++b) start[b + 1] = start[b] + cnt[b];
  or_entry *tmp = (or_entry *)malloc(sizeof(or_entry) * (size_t)(total ? total : 1));
  int64_t *fill = (int64_t *)calloc((size_t)nbins, sizeof(int64_t));
  for (int64_t g = 0; g < n; ++g) {
    if (!(flags[g] & OR_VISIBLE)) continue;
    int x0 = rect[4 * g], y0 = rect[4 * g + 1], x1 = rect[4 * g + 2], y1 = rect[4 * g + 3];
    int gx0 = x0 / G, gx1 = (x1 - 1) / G, gy0 = y0 / G, gy1 = (y1 - 1) / G;
    for (int gy = gy0; gy <= gy1; ++gy)
      for (int gx = gx0; gx <= gx1; ++gx) {
        uint64_t m = 0;
        for (int ty = gy * G; ty < gy * G + G; ++ty)
          for (int tx = gx * G; tx < gx * G + G; ++tx)
            if (tx >= x0 && tx < x1 && ty >= y0 && ty < y1) m |= (uint64_t)1 << ((ty % G) * G + (tx % G));
        int64_t b = (int64_t)gy * GX + gx;
        or_entry *e = &tmp[start[b] + fill[b]++];
        e->z = depth[g]; e->id = g; e->mask = m;
      }
  }
  for (int64_t b = 0; b < nbins; ++b)
    if (cnt[b] > 1) qsort(tmp + start[b], (size_t)cnt[b], sizeof(or_entry), cmp_entry);
  for (int64_t i = 0; i < total; ++i) {
    ids[i] = tmp[i].id;
    if (masks) masks[i] = tmp[i].mask;
  }
  free(tmp); free(fill); free(cnt);
  return total;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel front-to-back compositing.                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int W, H, TX, TY;
  const double *xy, *depth, *conic, *rgb, *opacity;
  const int64_t *start, *ids;          /* tile lists */
  const int64_t *astart, *aids;        /* per-tile Gaussians of ambiguous membership */
  const double *bg;
  double *image, *tfinal, *wsum;
  int64_t *neval;
  uint8_t *amb;
  const int64_t *tiles;                /* selected tiles, NULL = all */
  int64_t ntiles;
  int nthreads, tid;
} or_job;

static void composite_tile(const or_job *J, int64_t tile) {
  int tx = (int)(tile % J->TX), ty = (int)(tile / J->TX);
  int64_t s = J->start[tile], e = J->start[tile + 1];
  const double lnamin = log(OR_ALPHA_MIN), lntmin = log(OR_T_MIN);
  int64_t HW = (int64_t)J->W * J->H;
  for (int j = 0; j < OR_TILE; ++j) {
    int py_i = ty * OR_TILE + j;
    if (py_i >= J->H) break;
    for (int i = 0; i < OR_TILE; ++i) {
      int px_i = tx * OR_TILE + i;
      if (px_i >= J->W) break;
      double px = px_i + 0.5, py = py_i + 0.5;
      double T = 1.0, C[3] = {0.0, 0.0, 0.0}, Wt = 0.0;
      int64_t cnt = 0;
      uint8_t am = 0;
      double zprev = -1.0;
      int64_t k;
      for (k = s; k < e; ++k) {
        int64_t g = J->ids[k];
        cnt++;
        double dx = px - J->xy[2 * g], dy = py - J->xy[2 * g + 1];
        double a = J->conic[3 * g], b = J->conic[3 * g + 1], c = J->conic[3 * g + 2];
        double power = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
        double o = J->opacity[g];
        double lnal = log(o) + power;
        if (fabs(lnal - lnamin) < OR_GUARD_LNA) am |= OR_PIX_ALPHA;
        double alpha = fmin(OR_ALPHA_MAX, o * exp(power));
        if (alpha < OR_ALPHA_MIN) continue;
        double z = J->depth[g];
        if (zprev > 0.0 && z - zprev < OR_GUARD_Z * z) am |= OR_PIX_TIE;
        zprev = z;
        double Tn = T * (1.0 - alpha);
        if (fabs(log(Tn) - lntmin) < OR_GUARD_LNT) am |= OR_PIX_T;
        if (Tn < OR_T_MIN) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += alpha * T * J->rgb[3 * g + ch];
        Wt += alpha * T;
        T = Tn;
      }
      if (k < e) {
        /* terminated at k: a Gaussian at nearly the same depth could be ordered first */
        double zt = J->depth[J->ids[k]];
        for (int64_t q = k + 1; q < e; ++q) {
          int64_t g = J->ids[q];
          double z = J->depth[g];
          if (z - zt >= OR_GUARD_Z * zt) break;
          double dx = px - J->xy[2 * g], dy = py - J->xy[2 * g + 1];
          double a = J->conic[3 * g], b = J->conic[3 * g + 1], c = J->conic[3 * g + 2];
          double power = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
          if (log(J->opacity[g]) + power >= lnamin - OR_GUARD_LNA) am |= OR_PIX_TIE;
        }
      }
      for (int64_t q = J->astart[tile]; q < J->astart[tile + 1]; ++q) {
        int64_t g = J->aids[q];
        double dx = px - J->xy[2 * g], dy = py - J->xy[2 * g + 1];
        double a = J->conic[3 * g], b = J->conic[3 * g + 1], c = J->conic[3 * g + 2];
        double power = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
        if (log(J->opacity[g]) + power >= lnamin - OR_GUARD_LNA) am |= OR_PIX_MEMBER;
      }
      int64_t pix = (int64_t)py_i * J->W + px_i;
      for (int ch = 0; ch < 3; ++ch) J->image[ch * HW + pix] = C[ch] + T * J->bg[ch];
      J->tfinal[pix] = T;
      J->wsum[pix] = Wt;
      J->neval[pix] = cnt;
      J->amb[pix] = am;
    }
  }
}

static void *composite_worker(void *arg) {
  const or_job *J = (const or_job *)arg;
  for (int64_t q = J->tid; q < J->ntiles; q += J->nthreads)
    composite_tile(J, J->tiles ? J->tiles[q] : q);
  return NULL;
}

/* tiles: list of tile ids to composite (NULL = all).  Threads split tiles
 * round-robin; every tile's arithmetic is the same for any thread count. */
void oracle_composite(int W, int H, const double *xy, const double *depth, const double *conic,
                      const double *rgb, const double *opacity, const int64_t *start,
                      const int64_t *ids, const int64_t *astart, const int64_t *aids,
                      const double *bg, int nthreads, const int64_t *tiles, int64_t ntiles_sel,
                      double *image, double *tfinal, double *wsum, int64_t *neval, uint8_t *amb) {
  or_job base;
  memset(&base, 0, sizeof(base));
  base.W = W; base.H = H;
  base.TX = (W + OR_TILE - 1) / OR_TILE; base.TY = (H + OR_TILE - 1) / OR_TILE;
  base.xy = xy; base.depth = depth; base.conic = conic; base.rgb = rgb; base.opacity = opacity;
  base.start = start; base.ids = ids; base.astart = astart; base.aids = aids; base.bg = bg;
  base.image = image; base.tfinal = tfinal; base.wsum = wsum; base.neval = neval; base.amb = amb;
  base.tiles = tiles;
  base.ntiles = tiles ? ntiles_sel : (int64_t)base.TX * base.TY;
  if (nthreads < 1) nthreads = 1;
  if (nthreads == 1) {
    base.nthreads = 1; base.tid = 0;
    composite_worker(&base);
    return;
  }
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  or_job *jobs = (or_job *)malloc(sizeof(or_job) * (size_t)nthreads);
  for (int i = 0; i < nthreads; ++i) {
    jobs[i] = base; jobs[i].nthreads = nthreads; jobs[i].tid = i;
    pthread_create(&th[i], NULL, composite_worker, &jobs[i]);
  }
  for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
  free(th); free(jobs);
}

/* ------------------------------------------------------------------------ */
/* Admissible results of a pixel whose decisions fall in a guard band.       */
/* ------------------------------------------------------------------------ */
/* A decision inside a guard band is one that exact arithmetic takes one way and FP32
 * arithmetic may take the other, so several images are correct there (each is the plain
 * definition applied to inputs within rounding of the true ones).  For one pixel this
 * enumerates them: every combination of
 *   - tile membership of a Gaussian whose footprint edge or near-plane distance lies in its
 *     guard band (the tile's ambiguous-membership set): listed or not;
 *   - the 1/255 cut when |ln alpha - ln(1/255)| is inside its band: skipped or blended;
 *   - the 1e-4 stop when |ln T' - ln 1e-4| is inside its band: stop or blend;
 *   - the depth order: by (depth, index), the definition, or by (depth rounded to FP32, index),
 *     the order of 32-bit depth keys (FP32 rounding is monotone, so the two differ only where
 *     Gaussians whose depths round to the same FP32 value are not in index order; the pixel is
 *     flagged by the wider OR_GUARD_Z band);
 * each composited front to back exactly as composite_tile does.  Only Gaussians whose
 * ln alpha reaches the cut's band at this pixel take part: the others contribute nothing
 * under any reading. */
typedef struct {
  int64_t id;
  double z, lnal, alpha;
  float z32;
  int optional;
} or_cand;

typedef struct {
  double px, py;
  const double *rgb, *bg;
  double *out;       /* max_alt x 4: colour with background, T_final */
  int max_alt, n_out, overflow;
} or_alt_ctx;

static int cmp_cand(const void *pa, const void *pb) {
  const or_cand *a = (const or_cand *)pa, *b = (const or_cand *)pb;
  if (a->z < b->z) return -1;
  if (a->z > b->z) return 1;
  return (a->id > b->id) - (a->id < b->id);
}

static int cmp_cand32(const void *pa, const void *pb) {
  const or_cand *a = (const or_cand *)pa, *b = (const or_cand *)pb;
  if (a->z32 < b->z32) return -1;
  if (a->z32 > b->z32) return 1;
  return (a->id > b->id) - (a->id < b->id);
}

static void alt_emit(or_alt_ctx *X, double T, const double *C) {
  if (X->n_out >= X->max_alt) { X->overflow = 1; return; }
  double *o = X->out + 4 * (size_t)X->n_out++;
  for (int ch = 0; ch < 3; ++ch) o[ch] = C[ch] + T * X->bg[ch];
  o[3] = T;
}

/* walks seq[i..m) from (T, C) */
static void alt_walk(or_alt_ctx *X, const or_cand *seq, int m, int i, double T, const double *Cin) {
  const double lnamin = log(OR_ALPHA_MIN), lntmin = log(OR_T_MIN);
  double C[3] = {Cin[0], Cin[1], Cin[2]};
  for (; i < m; ++i) {
    if (X->overflow) return;
    const or_cand *a = &seq[i];
    /* membership */
    if (a->optional) {
      alt_walk(X, seq, m, i + 1, T, C);   /* not listed */
      if (X->overflow) return;
    }
    /* the 1/255 cut */
    int blend;
    if (fabs(a->lnal - lnamin) < OR_GUARD_LNA) {
      alt_walk(X, seq, m, i + 1, T, C);   /* skipped */
      if (X->overflow) return;
      blend = 1;
    } else {
      blend = a->alpha >= OR_ALPHA_MIN;
    }
    if (!blend) continue;
    double Tn = T * (1.0 - a->alpha);
    int stop;
    if (fabs(log(Tn) - lntmin) < OR_GUARD_LNT) {
      alt_emit(X, T, C);                      /* stopped here */
      if (X->overflow) return;
      stop = 0;
    } else {
      stop = Tn < OR_T_MIN;
    }
    if (stop) { alt_emit(X, T, C); return; }
    for (int ch = 0; ch < 3; ++ch) C[ch] += a->alpha * T * X->rgb[3 * a->id + ch];
    T = Tn;
  }
  alt_emit(X, T, C);
}

/* For each pixel pix[q] (row-major index), writes up to max_alt results to
 * out[(q * max_alt + k) * 4 + (0..2: colour with background, 3: T_final)] and their number to
 * nout[q], or -1 when there are more than max_alt. */
void oracle_alternatives(int W, int H, const double *xy, const double *depth, const double *conic,
                         const double *rgb, const double *opacity, const int64_t *start, const int64_t *ids,
                         const int64_t *astart, const int64_t *aids, const double *bg, int64_t npix,
                         const int64_t *pix, int max_alt, double *out, int32_t *nout) {
  const double lnamin = log(OR_ALPHA_MIN);
  int TX = (W + OR_TILE - 1) / OR_TILE;
  for (int64_t q = 0; q < npix; ++q) {
    int px_i = (int)(pix[q] % W), py_i = (int)(pix[q] / W);
    int64_t tile = (int64_t)(py_i / OR_TILE) * TX + px_i / OR_TILE;
    int64_t s = start[tile], e = start[tile + 1], as = astart[tile], ae = astart[tile + 1];
    or_cand *seq = (or_cand *)malloc(sizeof(or_cand) * (size_t)(e - s + ae - as + 1));
    int m = 0;
    double px = px_i + 0.5, py = py_i + 0.5;
    for (int64_t k = s; k < e + (ae - as); ++k) {
      int64_t g;
      int optional = 0;
      if (k < e) {
        g = ids[k];
        for (int64_t u = as; u < ae; ++u) if (aids[u] == g) optional = 1;
      } else {
        g = aids[as + (k - e)];
        int listed = 0;
        for (int64_t u = s; u < e; ++u) if (ids[u] == g) { listed = 1; break; }
        if (listed) continue;
        optional = 1;
      }
      double dx = px - xy[2 * g], dy = py - xy[2 * g + 1];
      double a = conic[3 * g], b = conic[3 * g + 1], c = conic[3 * g + 2];
      double power = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
      double lnal = log(opacity[g]) + power;
      if (lnal < lnamin - OR_GUARD_LNA) continue;   /* never contributes here */
      or_cand *cd = &seq[m++];
      cd->id = g; cd->z = depth[g]; cd->z32 = (float)depth[g]; cd->lnal = lnal; cd->optional = optional;
      cd->alpha = fmin(OR_ALPHA_MAX, opacity[g] * exp(power));
    }
    qsort(seq, (size_t)m, sizeof(or_cand), cmp_cand);
    or_alt_ctx X;
    X.px = px; X.py = py; X.rgb = rgb; X.bg = bg;
    X.out = out + (size_t)q * (size_t)max_alt * 4;
    X.max_alt = max_alt; X.n_out = 0; X.overflow = 0;
    const double C0[3] = {0.0, 0.0, 0.0};
    alt_walk(&X, seq, m, 0, 1.0, C0);
    /* the order of 32-bit depth keys, where it differs */
    or_cand *seq32 = (or_cand *)malloc(sizeof(or_cand) * (size_t)(m ? m : 1));
    memcpy(seq32, seq, sizeof(or_cand) * (size_t)m);
    qsort(seq32, (size_t)m, sizeof(or_cand), cmp_cand32);
    int same = 1;
    for (int k = 0; k < m && same; ++k) same = seq32[k].id == seq[k].id;
    if (!same) alt_walk(&X, seq32, m, 0, 1.0, C0);
    free(seq32);
    nout[q] = X.overflow ? -1 : X.n_out;
    free(seq);
  }
}
