// C-ABI of libjpet: argument validation, workspace layout and the launch sequence of each
// entry point declared in include/jpet.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include "jpet_internal.h"

namespace jpet {

namespace {

thread_local int g_last_hip_error = 0;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  return JPET_EHIP;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// Full validation of the geometry (before anything is enqueued).
int check_geometry(const jpet_geometry* g) {
  if (!g) return JPET_EINVAL;
  if (!finite_pos(g->R) || !finite_pos(g->L) || !finite_pos(g->sigma_z) || !finite_pos(g->sigma_dl) ||
      !finite_pos(g->pixel))
    return JPET_EDOMAIN;
  if (g->n_y <= 0 || g->n_z <= 0 || g->n_y > 32768 || g->n_z > 32768) return JPET_EDOMAIN;
  if (!(0.5 * (double)g->n_y * g->pixel < g->R)) return JPET_EDOMAIN;
  if (g->kernel_variant != 0 && g->kernel_variant != 1) return JPET_EDOMAIN;
  if (!isfinite(g->gamma)) return JPET_EDOMAIN;
  if (g->gamma != 0.0) return JPET_ENOTSUP;
  if (g->reserved != 0) return JPET_EINVAL;
  return JPET_OK;
}

Geo make_geo(const jpet_geometry* g, double mask_sz, double mask_sdl) {
  Geo o;
  o.R = g->R;
  o.L = g->L;
  o.sigma_z = g->sigma_z;
  o.sigma_dl = g->sigma_dl;
  o.pixel = g->pixel;
  o.u = 1.0 / (g->sigma_z * g->sigma_z);
  o.w = 1.0 / (g->sigma_dl * g->sigma_dl);
  o.um = 1.0 / (mask_sz * mask_sz);
  o.wm = 1.0 / (mask_sdl * mask_sdl);
  o.fa = g->kernel_variant ? 2.0 : 1.0;
  o.y0 = (0.5 - 0.5 * (double)g->n_y) * g->pixel;
  o.z0 = (0.5 - 0.5 * (double)g->n_z) * g->pixel;
  o.n_y = g->n_y;
  o.n_z = g->n_z;
  return o;
}

int64_t npix_of(const jpet_geometry* g) { return (int64_t)g->n_y * (int64_t)g->n_z; }

int carve(const jpet_geometry* g, int64_t n, void* ws, size_t ws_bytes, Workspace* out) {
  if (!ws) return JPET_EWORKSPACE;
  if (((uintptr_t)ws & 255) != 0) return JPET_EWORKSPACE;
  size_t need = workspace_layout(n, npix_of(g), ws, out);
  if (ws_bytes < need) return JPET_EWORKSPACE;
  return JPET_OK;
}

int read_stats(const Workspace& ws, int64_t n, jpet_stats* stats, hipStream_t st) {
  unsigned long long c[C_COUNT];
  hipError_t e = hipMemcpyAsync(c, ws.cnt, sizeof(c), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e);
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  stats->n_events = n;
  stats->n_valid = (int64_t)c[C_VALID];
  stats->n_dropped = (int64_t)c[C_DROPPED];
  stats->n_zero_denominator = (int64_t)c[C_ZERO_DEN];
  stats->n_pairs = (int64_t)c[C_PAIRS];
  stats->n_kappa_nonpositive = (int64_t)c[C_KAPPA_BAD];
  return JPET_OK;
}

int do_prepare(const Geo& geo, const float* events, int64_t n, const Workspace& w, hipStream_t st) {
  hipError_t e = launch_fill_u64(w.cnt, C_COUNT, st);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_prepare(geo, events, n, w, st);
  if (e != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

}  // namespace

size_t workspace_layout(int64_t n, int64_t npix, void* base, Workspace* out) {
  size_t off = 0;
  char* b = (char*)base;
  Workspace w;
  w.ev = (EventRec*)(b + off);
  off = align_up(off + sizeof(EventRec) * (size_t)(n > 0 ? n : 0), 256);
  w.cnt = (unsigned long long*)(b + off);
  off = align_up(off + sizeof(unsigned long long) * C_COUNT, 256);
  w.acc = (float*)(b + off);
  off = align_up(off + sizeof(float) * (size_t)npix, 256);
  w.red = (double*)(b + off);
  off = align_up(off + sizeof(double) * RED_SLOTS, 256);
  w.bytes = off;
  if (out) *out = w;
  return off;
}

}  // namespace jpet

using namespace jpet;

extern "C" {

const char* jpet_strerror(int status) {
  switch (status) {
    case JPET_OK: return "success";
    case JPET_EINVAL: return "invalid argument (NULL pointer, negative count or unknown flag)";
    case JPET_EDOMAIN: return "argument out of domain (geometry, resolution or grid) or log-likelihood is -inf";
    case JPET_EWORKSPACE: return "workspace missing, misaligned or smaller than jpet_mlem_workspace_size";
    case JPET_EHIP: return "HIP runtime error (see jpet_last_hip_error)";
    case JPET_ENOTSUP: return "not supported by this build (gamma != 0)";
    default: return "unknown status";
  }
}

int jpet_last_hip_error(void) { return g_last_hip_error; }

int jpet_abi_version(void) { return JPET_ABI_VERSION; }

int jpet_sensitivity(const jpet_geometry* g, float* s_out, void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (!s_out) return JPET_EINVAL;
  const Geo geo = make_geo(g, g->sigma_z, g->sigma_dl);
  hipError_t e = launch_sensitivity(geo, s_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

int jpet_mlem_workspace_size(const jpet_geometry* g, int64_t n_events, size_t* bytes) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (!bytes || n_events < 0) return JPET_EINVAL;
  *bytes = workspace_layout(n_events, npix_of(g), nullptr, nullptr);
  return JPET_OK;
}

int jpet_mlem_prepare(const jpet_geometry* g, const float* events, int64_t n, void* ws, size_t ws_bytes,
                      void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || (n > 0 && !events)) return JPET_EINVAL;
  Workspace w;
  rc = carve(g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  return do_prepare(make_geo(g, g->sigma_z, g->sigma_dl), events, n, w, (hipStream_t)stream);
}

int jpet_mlem_iterate(const jpet_geometry* g, const float* events, int64_t n, const float* s, float* rho,
                      int32_t n_iter, void* ws, size_t ws_bytes, uint32_t flags, jpet_stats* stats,
                      void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || (n > 0 && !events) || !rho || n_iter < 0) return JPET_EINVAL;
  if (flags & ~JPET_WS_PREPARED) return JPET_EINVAL;
  Workspace w;
  rc = carve(g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geo geo = make_geo(g, g->sigma_z, g->sigma_dl);
  if (!(flags & JPET_WS_PREPARED)) {
    rc = do_prepare(geo, events, n, w, st);
    if (rc) return rc;
  }
  hipError_t e = launch_fill_f32(w.acc, npix_of(g), st);
  if (e != hipSuccess) return hip_fail(e);
  for (int it = 0; it < n_iter; ++it) {
    // per-iteration counters: zero-denominator events and non-positive kappa pairs
    e = launch_fill_u64(w.cnt + C_ZERO_DEN, 2, st);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_event_pass(geo, n, w, rho, st);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_update(geo, s, rho, w, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (stats) return read_stats(w, n, stats, st);
  return JPET_OK;
}

int jpet_loglik_grad(const jpet_geometry* g, const double* sigma_mask, const float* events, int64_t n,
                     const float* s, const float* rho, double* out3, float* grad_rho, float* D_out, void* ws,
                     size_t ws_bytes, uint32_t flags, jpet_stats* stats, void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || (n > 0 && !events) || !rho || !out3) return JPET_EINVAL;
  if (flags & ~JPET_WS_PREPARED) return JPET_EINVAL;
  double msz = g->sigma_z, mdl = g->sigma_dl;
  if (sigma_mask) {
    msz = sigma_mask[0];
    mdl = sigma_mask[1];
    if (!finite_pos(msz) || !finite_pos(mdl)) return JPET_EDOMAIN;
  }
  Workspace w;
  rc = carve(g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geo geo = make_geo(g, msz, mdl);
  if (!(flags & JPET_WS_PREPARED)) {
    rc = do_prepare(geo, events, n, w, st);
    if (rc) return rc;
  }
  hipError_t e = launch_fill_u64(w.cnt + C_ZERO_DEN, 2, st);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_loglik(geo, n, w, rho, s, D_out, grad_rho, out3, st);
  if (e != hipSuccess) return hip_fail(e);
  if (stats) {
    rc = read_stats(w, n, stats, st);
    if (rc) return rc;
    if (stats->n_zero_denominator > 0) return JPET_EDOMAIN;
  }
  return JPET_OK;
}

}  // extern "C"
