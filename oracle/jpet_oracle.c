/*
 * Oracle for the two-strip J-PET list-mode MLEM reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded
 * double-precision CPU implementation written from the paper (Bialas et al.,
 * "GPU accelerated image reconstruction in a two-strip J-PET tomograph",
 * arXiv:1502.07478).  Only the test-suite, the smoke check and the bench's CPU
 * baseline may load it.  It shares no code, header or constant with the GPU
 * library; the two only read the same synthetic event arrays.
 *
 * What it computes, step by step, in the paper's order:
 *   - sensitivity s(y,z) at each pixel centre            (Setup, Eq. 4)
 *   - direct reconstruction (tan theta, y~, z~) per event (Setup, Eq. 2)
 *   - bounding box of the 3-sigma ellipse                 (Appendix B)
 *   - ellipse test b C^-1 b <= 9 at each pixel centre     (Sec. 3, last paragraph;
 *                                                          Sec. 4 on the pixel loops)
 *   - the kernel P(e|i) from the vectors o, a, b          (Sec. 3, Eq. 7-12)
 *   - one MLEM iteration in the two-pass form of the
 *     implementation listing: denominator, then
 *     back-projection rho*P/denominator                   (Sec. 4, listing; Eq. 3/5)
 *   - the Poisson list-mode log-likelihood whose EM step
 *     is Eq. 3, and its gradient w.r.t. rho, sigma_z,
 *     sigma_dl (derived; the paper cites it for Eq. 3)
 *
 * Readings of points the paper leaves open or prints garbled (each is listed
 * with its reason in the design notes of the repository):
 *   R1  Eq. 2: the first printed forms are used (y~ = -dl/(2 sqrt(1+tan^2)),
 *       z~ = (z_u + z_d + 2 y~ tan)/2); the alternative printed forms do not
 *       invert Eq. 1.
 *   R2  Eq. 7 prefactor: det^(1/2) of C^-1 (the inverse covariance), which makes
 *       P the angular integral of a normalised 3-D Gaussian.
 *   R3  Eq. 9, third component of a: printed as -(dy+y~) tan/cos; variant 1
 *       doubles it (the exact derivative of dl(theta)).  Selected by
 *       kernel_variant.
 *   R4  Appendix B: the bounding box of A y^2 + C y z + B z^2 = r^2 has half
 *       sizes r/sqrt(A - C^2/(4B)) and r/sqrt(B - C^2/(4A)), with r^2 = 9.
 *   R5  The ellipse is the closed set b C^-1 b <= 9, tested at pixel centres.
 *   R6  Eq. 3 is read as sensitivity-normalised list-mode MLEM:
 *       D_j = sum_i P_ji rho_i, rho'_l = rho_l * B_l / s_l with
 *       B_l = sum_j P_jl / D_j, and rho' = 0 where s = 0.  With no
 *       sensitivity the update is Eq. 5 (s = 1 everywhere).
 *   R7  An event is valid when its three numbers are finite, both strip
 *       positions lie within the strips (|z| <= L/2) and at least one grid pixel
 *       centre lies in its ellipse.  Valid events with D = 0 are skipped in the
 *       update and counted.
 *   R8  Kernel values with a non-positive kappa = a C^-1 a + 2 o C^-1 b are
 *       taken as 0 and counted.
 *   R9  The log-likelihood is sum_j log(D_j / pi) - sum_l s_l rho_l over valid
 *       events (P is pi times a probability density, as its integral over all
 *       detectable events is pi s).  Its sigma-gradient holds the ellipse
 *       mask fixed (the mask may be evaluated at separate sigmas).
 *   R13 sigma_z depending on the measured hit positions (Sec. 3, after Eq. 12:
 *       weak, about 10% from the strip centre, lowest, to its ends, highest; no
 *       functional form is given).  Read as one sigma_z per event, entering both
 *       z slots of C^-1 as in the printed matrix:
 *         sigma_z(e) = sigma_z (1 + sigma_z_edge * zeta),
 *         zeta = ((2 z_u / L)^2 + (2 z_d / L)^2) / 2  in [0, 1] for valid events,
 *       i.e. the mean of a quadratic profile over the two hits.  The event's
 *       3-sigma ellipse and kernel both use it; sigma_z_edge = 0 is the
 *       constant-resolution method.  The log-likelihood is defined here for
 *       sigma_z_edge = 0 only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
  double R;        /* strip half-separation (mm) */
  double L;        /* strip length (mm) */
  double sigma_z;  /* resolution of z_u, z_d (mm) */
  double sigma_dl; /* resolution of dl (mm) */
  double gamma;    /* off-diagonal element of C^-1 (Eq. 12) */
  double pixel;    /* square pixel pitch (mm) */
  int32_t n_y;     /* rows (y) */
  int32_t n_z;     /* columns (z) */
  int32_t kernel_variant; /* R3: 0 as printed, 1 doubled a_3 */
  int32_t reserved;
  double sigma_z_edge;     /* R13: relative rise of sigma_z at the strip ends, in [0, 1] */
} orc_geometry;

typedef struct {
  int64_t n_events;
  int64_t n_valid;
  int64_t n_dropped;
  int64_t n_zero_denominator;
  int64_t n_pairs;           /* (valid event, in-ellipse pixel) pairs */
  int64_t n_kappa_nonpositive;
} orc_stats;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EDOMAIN = -2, ORC_ENOMEM = -5 };

/* ------------------------------------------------------------------ */
/* geometry                                                            */

static void pixel_centre(const orc_geometry* g, int i, int k, double* y, double* z) {
  *y = ((double)i + 0.5 - 0.5 * (double)g->n_y) * g->pixel;
  *z = ((double)k + 0.5 - 0.5 * (double)g->n_z) * g->pixel;
}

int orc_check_geometry(const orc_geometry* g) {
  if (!g) return ORC_EINVAL;
  if (!(g->R > 0) || !(g->L > 0) || !(g->sigma_z > 0) || !(g->sigma_dl > 0) || !(g->pixel > 0))
    return ORC_EDOMAIN;
  if (g->n_y <= 0 || g->n_z <= 0) return ORC_EDOMAIN;
  if (0.5 * g->n_y * g->pixel >= g->R) return ORC_EDOMAIN;
  if (g->kernel_variant != 0 && g->kernel_variant != 1) return ORC_EDOMAIN;
  if (!(g->sigma_z_edge >= 0.0 && g->sigma_z_edge <= 1.0)) return ORC_EDOMAIN;
  return ORC_OK;
}

/* Eq. 4: fraction of in-plane directions from (y, z) that hit both strips.  The
 * upper hit z + (R - y) tan(theta) and the lower hit z - (R + y) tan(theta) must both lie
 * in [-L/2, L/2]; theta is uniform on (-pi/2, pi/2). */
double orc_sensitivity_point(const orc_geometry* g, double y, double z) {
  const double R = g->R, hl = 0.5 * g->L;
  double hi = fmin((hl - z) / (R - y), (hl + z) / (R + y));
  double lo = fmax(-(hl + z) / (R - y), (-hl + z) / (R + y));
  double s = (atan(hi) - atan(lo)) / M_PI;
  return s > 0.0 ? s : 0.0;
}

int orc_sensitivity(const orc_geometry* g, double* s_out) {
  int rc = orc_check_geometry(g);
  if (rc) return rc;
  for (int i = 0; i < g->n_y; ++i)
    for (int k = 0; k < g->n_z; ++k) {
      double y, z;
      pixel_centre(g, i, k, &y, &z);
      s_out[(int64_t)i * g->n_z + k] = orc_sensitivity_point(g, y, z);
    }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* per-event quantities                                                */

typedef struct {
  double tan_t;  /* tan(theta~) */
  double sec_t;  /* 1/cos(theta~) = sqrt(1 + tan^2) */
  double y;      /* y~ */
  double z;      /* z~ */
} orc_estimate;

/* Eq. 2 (first forms, reading R1). */
void orc_direct(const orc_geometry* g, double zu, double zd, double dl, double out[4]) {
  double t = (zu - zd) / (2.0 * g->R);
  double c = sqrt(1.0 + t * t);
  double y = -0.5 * dl / c;
  double z = 0.5 * (zu + zd + 2.0 * y * t);
  out[0] = t; out[1] = c; out[2] = y; out[3] = z;
}

/* Direct-reconstruction image: each valid event (finite, both hits on the strips) counted at the
 * pixel containing its point (y~, z~) of Eq. 2 (first forms); points outside the grid are not
 * counted.  The pixel of a coordinate x on a grid of n pixels is floor(x / pixel + n / 2).
 * out: n_y * n_z doubles, overwritten; returns the number of events counted. */
int64_t orc_direct_image(const orc_geometry* g, const float* events, int64_t n, double* out) {
  for (int64_t q = 0; q < (int64_t)g->n_y * g->n_z; ++q) out[q] = 0.0;
  int64_t counted = 0;
  for (int64_t j = 0; j < n; ++j) {
    const float* e = events + 3 * j;
    if (!isfinite(e[0]) || !isfinite(e[1]) || !isfinite(e[2])) continue;
    if (fabs((double)e[0]) > 0.5 * g->L || fabs((double)e[1]) > 0.5 * g->L) continue;
    double o[4];
    orc_direct(g, (double)e[0], (double)e[1], (double)e[2], o);
    const double fi = floor(o[2] / g->pixel + 0.5 * g->n_y);
    const double fk = floor(o[3] / g->pixel + 0.5 * g->n_z);
    if (fi < 0.0 || fi >= (double)g->n_y || fk < 0.0 || fk >= (double)g->n_z) continue;
    out[(int64_t)fi * g->n_z + (int64_t)fk] += 1.0;
    ++counted;
  }
  return counted;
}

static void estimate(const orc_geometry* g, const float* e, orc_estimate* ev) {
  double o[4];
  orc_direct(g, (double)e[0], (double)e[1], (double)e[2], o);
  ev->tan_t = o[0]; ev->sec_t = o[1]; ev->y = o[2]; ev->z = o[3];
}

/* Reading R13: the event's sigma_z over the geometry's, 1 + sigma_z_edge * zeta with zeta the
 * mean over the two measured hits of (z / (L/2))^2. */
double orc_sigma_z_factor(const orc_geometry* g, double zu, double zd) {
  const double xu = zu / (0.5 * g->L), xd = zd / (0.5 * g->L);
  const double zeta = 0.5 * (xu * xu + xd * xd);
  return 1.0 + g->sigma_z_edge * zeta;
}

/* Appendix B (reading R4).  b C^-1 b written as a quadratic form in (dy, dz) is
 *   A dy^2 + C dy dz + B dz^2 with
 *   A = 2 tan^2/sz^2 + 4/(sdl^2 cos^2), C = -4 tan/sz^2, B = 2/sz^2
 * and the 3-sigma ellipse is that form <= 9. */
void orc_box_halfsize(double sigma_z, double sigma_dl, double tan_t, double sec_t, double out[2]) {
  double sz2 = sigma_z * sigma_z, sd2 = sigma_dl * sigma_dl;
  double A = 2.0 * tan_t * tan_t / sz2 + 4.0 * sec_t * sec_t / sd2;
  double B = 2.0 / sz2;
  double C = -4.0 * tan_t / sz2;
  out[0] = 3.0 / sqrt(A - C * C / (4.0 * B)); /* half size in y */
  out[1] = 3.0 / sqrt(B - C * C / (4.0 * A)); /* half size in z */
}

/* pixel index range [lo, hi] whose centres lie in [c - h, c + h], clipped to [0, n) */
static void index_range(double c, double h, double pixel, int n, int* lo, int* hi) {
  double a = (c - h) / pixel + 0.5 * n - 0.5;
  double b = (c + h) / pixel + 0.5 * n - 0.5;
  double fa = ceil(a), fb = floor(b);
  if (fa < 0) fa = 0;
  if (fb > n - 1) fb = n - 1;
  if (fa > fb) { *lo = 0; *hi = -1; return; }
  *lo = (int)fa; *hi = (int)fb;
}

/* ------------------------------------------------------------------ */
/* the kernel, Eq. 7-12                                                */

typedef struct {
  double u, w, gamma; /* C^-1 = [[u,0,g],[0,u,-g],[g,-g,w]] with u = 1/sz^2, w = 1/sdl^2 */
  int variant;
} orc_resolution;

static double form(const orc_resolution* r, const double x[3], const double y[3]) {
  /* x^T C^-1 y */
  return r->u * (x[0] * y[0] + x[1] * y[1]) + r->w * x[2] * y[2] +
         r->gamma * (x[0] * y[2] + x[2] * y[0]) - r->gamma * (x[1] * y[2] + x[2] * y[1]);
}
static double form_du(const double x[3], const double y[3]) { return x[0] * y[0] + x[1] * y[1]; }
static double form_dw(const double x[3], const double y[3]) { return x[2] * y[2]; }

static double det_cinv(const orc_resolution* r) {
  /* determinant of [[u,0,g],[0,u,-g],[g,-g,w]] expanded along the first row */
  return r->u * (r->u * r->w - r->gamma * r->gamma) + r->gamma * (0.0 * (-r->gamma) - r->u * r->gamma);
}

typedef struct {
  double P;       /* kernel value (0 when kappa <= 0) */
  double q;       /* b C^-1 b */
  double kappa;   /* a C^-1 a + 2 o C^-1 b */
  double dlogP_du, dlogP_dw;
  int kappa_ok;
} orc_kernel_value;

/* P(e|i) for pixel centre (y, z) and the event estimate ev (Eq. 7 with o, a, b of Eq. 8-10,
 * dy, dz of Eq. 11 and C^-1 of Eq. 12). */
static void kernel(const orc_geometry* g, const orc_resolution* r, const orc_estimate* ev, double y, double z,
                   orc_kernel_value* kv) {
  const double R = g->R;
  const double t = ev->tan_t, c = ev->sec_t;
  const double dy = y - ev->y, dz = z - ev->z;
  const double fa = r->variant ? 2.0 : 1.0;
  double o[3] = { -(dy + ev->y - R) * t * c * c,
                  -(dy + ev->y + R) * t * c * c,
                  -(dy + ev->y) * c * (1.0 + 2.0 * t * t) };
  double a[3] = { -(dy + ev->y - R) * c * c,
                  -(dy + ev->y + R) * c * c,
                  -fa * (dy + ev->y) * c * t };
  double b[3] = { dz - dy * t, dz - dy * t, -2.0 * dy * c };
  double aCa = form(r, a, a), oCb = form(r, o, b), bCb = form(r, b, b), bCa = form(r, b, a);
  double kappa = aCa + 2.0 * oCb;
  kv->q = bCb;
  kv->kappa = kappa;
  if (!(kappa > 0.0)) {
    kv->P = 0.0; kv->dlogP_du = 0.0; kv->dlogP_dw = 0.0; kv->kappa_ok = 0;
    return;
  }
  kv->kappa_ok = 1;
  double det = det_cinv(r);
  double expo = -0.5 * (bCb - bCa * bCa / kappa);
  kv->P = sqrt(det) / (2.0 * M_PI * sqrt(kappa)) * exp(expo);
  /* d log P / d u and d w: every quadratic form is linear in (u, w). */
  double k_u = form_du(a, a) + 2.0 * form_du(o, b), k_w = form_dw(a, a) + 2.0 * form_dw(o, b);
  double q_u = form_du(b, b), q_w = form_dw(b, b);
  double g_u = form_du(b, a), g_w = form_dw(b, a);
  double det_u = 2.0 * r->u * r->w - 2.0 * r->gamma * r->gamma;
  double det_w = r->u * r->u;
  double gk = bCa / kappa;
  kv->dlogP_du = 0.5 * det_u / det - 0.5 * k_u / kappa - 0.5 * (q_u - 2.0 * gk * g_u + gk * gk * k_u);
  kv->dlogP_dw = 0.5 * det_w / det - 0.5 * k_w / kappa - 0.5 * (q_w - 2.0 * gk * g_w + gk * gk * k_w);
}

static void resolution(const orc_geometry* g, double sigma_z, double sigma_dl, orc_resolution* r) {
  r->u = 1.0 / (sigma_z * sigma_z);
  r->w = 1.0 / (sigma_dl * sigma_dl);
  r->gamma = g->gamma;
  r->variant = g->kernel_variant;
}

/* Unmasked kernel for events given as double triples at one pixel centre (quadrature pins). */
int orc_kernel_points(const orc_geometry* g, const double* events, int64_t n, double y, double z,
                      double* P_out, double* q_out) {
  int rc = orc_check_geometry(g);
  if (rc) return rc;
  for (int64_t j = 0; j < n; ++j) {
    double o[4];
    orc_direct(g, events[3 * j], events[3 * j + 1], events[3 * j + 2], o);
    orc_estimate ev = { o[0], o[1], o[2], o[3] };
    orc_resolution r;
    resolution(g, g->sigma_z * orc_sigma_z_factor(g, events[3 * j], events[3 * j + 1]), g->sigma_dl, &r);
    orc_kernel_value kv;
    kernel(g, &r, &ev, y, z, &kv);
    if (P_out) P_out[j] = kv.P;
    if (q_out) q_out[j] = kv.q;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* the pixels of one event                                             */

typedef struct {
  int64_t* pix;   /* row-major pixel index */
  double* P;      /* kernel value */
  double* dlu;    /* d log P / du */
  double* dlw;    /* d log P / dw */
  int64_t count;
  int64_t cap;
  int64_t kappa_bad;
} orc_pixel_list;

static int list_push(orc_pixel_list* l, int64_t pix, const orc_kernel_value* kv) {
  if (l->count == l->cap) {
    int64_t cap = l->cap ? 2 * l->cap : 4096;
    int64_t* p = (int64_t*)realloc(l->pix, cap * sizeof(int64_t));
    if (!p) return ORC_ENOMEM;
    l->pix = p;
    double* q = (double*)realloc(l->P, cap * sizeof(double));
    if (!q) return ORC_ENOMEM;
    l->P = q;
    q = (double*)realloc(l->dlu, cap * sizeof(double));
    if (!q) return ORC_ENOMEM;
    l->dlu = q;
    q = (double*)realloc(l->dlw, cap * sizeof(double));
    if (!q) return ORC_ENOMEM;
    l->dlw = q;
    l->cap = cap;
  }
  l->pix[l->count] = pix;
  l->P[l->count] = kv->P;
  l->dlu[l->count] = kv->dlogP_du;
  l->dlw[l->count] = kv->dlogP_dw;
  l->count++;
  return ORC_OK;
}

static void list_free(orc_pixel_list* l) {
  free(l->pix); free(l->P); free(l->dlu); free(l->dlw);
  memset(l, 0, sizeof(*l));
}

/* Pixels of the event's 3-sigma ellipse (mask at (msz, mdl)) with the kernel r, in row-major
 * order inside the bounding box.  Both sigma_z's are scaled by the event's factor (reading R13;
 * 1 when sigma_z_edge = 0).  Returns 0 and count = 0 for an invalid event (reading R7). */
static int event_pixels(const orc_geometry* g, double msz, double mdl, const orc_resolution* r0,
                        const float* e, orc_pixel_list* l) {
  l->count = 0;
  l->kappa_bad = 0;
  if (!isfinite(e[0]) || !isfinite(e[1]) || !isfinite(e[2])) return ORC_OK;
  if (fabs((double)e[0]) > 0.5 * g->L || fabs((double)e[1]) > 0.5 * g->L) return ORC_OK;
  orc_estimate ev;
  estimate(g, e, &ev);
  const double f = orc_sigma_z_factor(g, (double)e[0], (double)e[1]);
  msz *= f;
  orc_resolution rr = *r0;
  rr.u = r0->u / (f * f);  /* u = sigma_z^-2 */
  const orc_resolution* r = &rr;
  double h[2];
  orc_box_halfsize(msz, mdl, ev.tan_t, ev.sec_t, h);
  int i0, i1, k0, k1;
  index_range(ev.y, h[0], g->pixel, g->n_y, &i0, &i1);
  index_range(ev.z, h[1], g->pixel, g->n_z, &k0, &k1);
  orc_resolution mask;
  mask.u = 1.0 / (msz * msz);
  mask.w = 1.0 / (mdl * mdl);
  mask.gamma = 0.0;
  mask.variant = r->variant;
  for (int i = i0; i <= i1; ++i)
    for (int k = k0; k <= k1; ++k) {
      double y, z;
      pixel_centre(g, i, k, &y, &z);
      double dy = y - ev.y, dz = z - ev.z;
      double b[3] = { dz - dy * ev.tan_t, dz - dy * ev.tan_t, -2.0 * dy * ev.sec_t };
      if (form(&mask, b, b) > 9.0) continue; /* reading R5 */
      orc_kernel_value kv;
      kernel(g, r, &ev, y, z, &kv);
      if (!kv.kappa_ok) l->kappa_bad++;
      int rc = list_push(l, (int64_t)i * g->n_z + k, &kv);
      if (rc) return rc;
    }
  return ORC_OK;
}

/* Pixel list and kernel values of one event (tests build dense matrices from it). */
int64_t orc_event_pixels(const orc_geometry* g, const double* sigma_mask, const float* e, int64_t cap,
                         int64_t* pix_out, double* P_out) {
  if (orc_check_geometry(g)) return -1;
  orc_resolution r;
  resolution(g, g->sigma_z, g->sigma_dl, &r);
  double msz = sigma_mask ? sigma_mask[0] : g->sigma_z, mdl = sigma_mask ? sigma_mask[1] : g->sigma_dl;
  orc_pixel_list l;
  memset(&l, 0, sizeof(l));
  if (event_pixels(g, msz, mdl, &r, e, &l)) { list_free(&l); return -1; }
  int64_t n = l.count;
  for (int64_t m = 0; m < n && m < cap; ++m) {
    if (pix_out) pix_out[m] = l.pix[m];
    if (P_out) P_out[m] = l.P[m];
  }
  list_free(&l);
  return n;
}

/* ------------------------------------------------------------------ */
/* MLEM                                                                */

/* One or more iterations of the implementation listing (Sec. 4) with the update of Eq. 3/5
 * (reading R6).  rho is read and overwritten in place; s may be NULL (Eq. 5).  D_out, when
 * given, receives the denominators of the LAST iteration (0 for invalid events). */
int orc_mlem(const orc_geometry* g, const float* events, int64_t n, const double* s, double* rho,
             int n_iter, double* D_out, orc_stats* st) {
  int rc = orc_check_geometry(g);
  if (rc) return rc;
  if (!events || !rho || n < 0 || n_iter < 0) return ORC_EINVAL;
  const int64_t npix = (int64_t)g->n_y * g->n_z;
  double* rho_new = (double*)calloc((size_t)npix, sizeof(double));
  if (!rho_new) return ORC_ENOMEM;
  orc_resolution r;
  resolution(g, g->sigma_z, g->sigma_dl, &r);
  orc_pixel_list l;
  memset(&l, 0, sizeof(l));
  orc_stats acc;
  memset(&acc, 0, sizeof(acc));
  for (int it = 0; it < n_iter; ++it) {
    memset(&acc, 0, sizeof(acc));
    acc.n_events = n;
    for (int64_t p = 0; p < npix; ++p) rho_new[p] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      rc = event_pixels(g, g->sigma_z, g->sigma_dl, &r, events + 3 * j, &l);
      if (rc) goto done;
      if (l.count == 0) {
        acc.n_dropped++;
        if (D_out && it == n_iter - 1) D_out[j] = 0.0;
        continue;
      }
      acc.n_valid++;
      acc.n_pairs += l.count;
      acc.n_kappa_nonpositive += l.kappa_bad;
      double denominator = 0.0;
      for (int64_t m = 0; m < l.count; ++m) denominator += l.P[m] * rho[l.pix[m]];
      if (D_out && it == n_iter - 1) D_out[j] = denominator;
      if (!(denominator > 0.0)) { acc.n_zero_denominator++; continue; }
      for (int64_t m = 0; m < l.count; ++m)
        rho_new[l.pix[m]] += rho[l.pix[m]] * l.P[m] / denominator;
    }
    for (int64_t p = 0; p < npix; ++p) {
      if (s) rho[p] = s[p] > 0.0 ? rho_new[p] / s[p] : 0.0;
      else rho[p] = rho_new[p];
    }
  }
done:
  list_free(&l);
  free(rho_new);
  if (st) *st = acc;
  return rc;
}

/* ------------------------------------------------------------------ */
/* log-likelihood and gradient                                         */

/* out3 = { l, dl/dsigma_z, dl/dsigma_dl } with l = sum_valid log(D_j/pi) - sum_l s_l rho_l
 * (reading R9).  grad_rho (nullable) = B - s.  sigma_mask (nullable) = sigmas of the ellipse
 * mask; the kernel uses the geometry's sigmas.  Returns ORC_EDOMAIN (and l = -inf) when a
 * valid event has D = 0. */
int orc_loglik_grad(const orc_geometry* g, const double* sigma_mask, const float* events, int64_t n,
                    const double* s, const double* rho, double* out3, double* grad_rho, double* D_out,
                    orc_stats* st) {
  int rc = orc_check_geometry(g);
  if (rc) return rc;
  if (!events || !rho || !out3 || n < 0) return ORC_EINVAL;
  if (g->sigma_z_edge != 0.0) return ORC_EINVAL; /* reading R13: constant resolution only */
  const int64_t npix = (int64_t)g->n_y * g->n_z;
  double msz = sigma_mask ? sigma_mask[0] : g->sigma_z, mdl = sigma_mask ? sigma_mask[1] : g->sigma_dl;
  orc_resolution r;
  resolution(g, g->sigma_z, g->sigma_dl, &r);
  double* B = NULL;
  if (grad_rho) {
    B = (double*)calloc((size_t)npix, sizeof(double));
    if (!B) return ORC_ENOMEM;
  }
  orc_pixel_list l;
  memset(&l, 0, sizeof(l));
  orc_stats acc;
  memset(&acc, 0, sizeof(acc));
  acc.n_events = n;
  double sum_log = 0.0, sum_du = 0.0, sum_dw = 0.0;
  int zero = 0;
  for (int64_t j = 0; j < n; ++j) {
    rc = event_pixels(g, msz, mdl, &r, events + 3 * j, &l);
    if (rc) goto done;
    if (l.count == 0) {
      acc.n_dropped++;
      if (D_out) D_out[j] = 0.0;
      continue;
    }
    acc.n_valid++;
    acc.n_pairs += l.count;
    acc.n_kappa_nonpositive += l.kappa_bad;
    double D = 0.0, Du = 0.0, Dw = 0.0;
    for (int64_t m = 0; m < l.count; ++m) {
      double pr = l.P[m] * rho[l.pix[m]];
      D += pr;
      Du += pr * l.dlu[m];
      Dw += pr * l.dlw[m];
    }
    if (D_out) D_out[j] = D;
    if (!(D > 0.0)) { acc.n_zero_denominator++; zero = 1; continue; }
    sum_log += log(D / M_PI);
    sum_du += Du / D;
    sum_dw += Dw / D;
    if (B)
      for (int64_t m = 0; m < l.count; ++m) B[l.pix[m]] += l.P[m] / D;
  }
  {
    double srho = 0.0;
    for (int64_t p = 0; p < npix; ++p) srho += (s ? s[p] : 1.0) * rho[p];
    out3[0] = zero ? -INFINITY : sum_log - srho;
    /* u = sigma_z^-2, du/dsigma_z = -2 u / sigma_z; likewise for w and sigma_dl */
    out3[1] = sum_du * (-2.0 * r.u / g->sigma_z);
    out3[2] = sum_dw * (-2.0 * r.w / g->sigma_dl);
  }
  if (grad_rho)
    for (int64_t p = 0; p < npix; ++p) grad_rho[p] = B[p] - (s ? s[p] : 1.0);
  rc = zero ? ORC_EDOMAIN : ORC_OK;
done:
  list_free(&l);
  free(B);
  if (st) *st = acc;
  return rc;
}

/* ------------------------------------------------------------------ */
/* sampled outputs for large workloads                                 */

/* rho_new (the listing's accumulator, sum_j rho_l P_jl / D_j) at selected pixels only.  Every
 * event whose ellipse covers a selected pixel gets its full denominator computed; other events
 * are skipped after the cheap box test. */
int orc_backprojection_at(const orc_geometry* g, const float* events, int64_t n, const double* rho,
                          int64_t n_sel, const int64_t* sel, double* out) {
  int rc = orc_check_geometry(g);
  if (rc) return rc;
  orc_resolution r;
  resolution(g, g->sigma_z, g->sigma_dl, &r);
  for (int64_t m = 0; m < n_sel; ++m) out[m] = 0.0;
  orc_pixel_list l;
  memset(&l, 0, sizeof(l));
  for (int64_t j = 0; j < n; ++j) {
    const float* e = events + 3 * j;
    if (!isfinite(e[0]) || !isfinite(e[1]) || !isfinite(e[2])) continue;
    if (fabs((double)e[0]) > 0.5 * g->L || fabs((double)e[1]) > 0.5 * g->L) continue;
    orc_estimate ev;
    estimate(g, e, &ev);
    double h[2];
    orc_box_halfsize(g->sigma_z * orc_sigma_z_factor(g, (double)e[0], (double)e[1]), g->sigma_dl, ev.tan_t,
                     ev.sec_t, h);
    int i0, i1, k0, k1;
    index_range(ev.y, h[0], g->pixel, g->n_y, &i0, &i1);
    index_range(ev.z, h[1], g->pixel, g->n_z, &k0, &k1);
    int touches = 0;
    for (int64_t m = 0; m < n_sel && !touches; ++m) {
      int i = (int)(sel[m] / g->n_z), k = (int)(sel[m] % g->n_z);
      touches = i >= i0 && i <= i1 && k >= k0 && k <= k1;
    }
    if (!touches) continue;
    rc = event_pixels(g, g->sigma_z, g->sigma_dl, &r, e, &l);
    if (rc) break;
    double D = 0.0;
    for (int64_t q = 0; q < l.count; ++q) D += l.P[q] * rho[l.pix[q]];
    if (!(D > 0.0)) continue;
    for (int64_t q = 0; q < l.count; ++q)
      for (int64_t m = 0; m < n_sel; ++m)
        if (l.pix[q] == sel[m]) out[m] += rho[l.pix[q]] * l.P[q] / D;
  }
  list_free(&l);
  return rc;
}

/* Denominators of selected events only. */
int orc_denominators_at(const orc_geometry* g, const float* events, int64_t n_sel, const int64_t* sel,
                        const double* rho, double* D_out, int64_t* count_out) {
  int rc = orc_check_geometry(g);
  if (rc) return rc;
  orc_resolution r;
  resolution(g, g->sigma_z, g->sigma_dl, &r);
  orc_pixel_list l;
  memset(&l, 0, sizeof(l));
  for (int64_t m = 0; m < n_sel; ++m) {
    rc = event_pixels(g, g->sigma_z, g->sigma_dl, &r, events + 3 * sel[m], &l);
    if (rc) break;
    double D = 0.0;
    for (int64_t q = 0; q < l.count; ++q) D += l.P[q] * rho[l.pix[q]];
    D_out[m] = D;
    if (count_out) count_out[m] = l.count;
  }
  list_free(&l);
  return rc;
}
