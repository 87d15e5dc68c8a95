// C-ABI of libjpet: argument validation, workspace layout and the launch sequence of each
// entry point declared in include/jpet.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "jpet_internal.h"

namespace jpet {

namespace {

thread_local int g_last_hip_error = 0;

// event-pass timing (jpet_profile_enable / jpet_profile_read)
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;

void prof_forget_locked() {
  for (auto& pr : g_prof_events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  g_prof_events.clear();
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  return JPET_EHIP;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// Events per call: event positions and bin offsets are 32-bit on the device.  Longer lists go
// through jpet_mlem_backproject in pieces.
constexpr int64_t kMaxEvents = 2147483647;

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
  if (!(g->sigma_z_edge >= 0.0 && g->sigma_z_edge <= 1.0)) return JPET_EDOMAIN;
  // C^-1 (Eq. 12) must be positive definite for every event: u > 0, w > 0 and
  // u^2 w - 2 u gamma^2 > 0 down to the smallest u, that of the largest sigma_z
  {
    const double szm = g->sigma_z * (1.0 + g->sigma_z_edge);
    const double u = 1.0 / (szm * szm), w = 1.0 / (g->sigma_dl * g->sigma_dl);
    if (!(2.0 * g->gamma * g->gamma < u * w)) return JPET_EDOMAIN;
  }
  if (!plan_code_valid(g->plan)) return JPET_EINVAL;
  return JPET_OK;
}

Geo make_geo(const jpet_geometry* g, double mask_sz, double mask_sdl) {
  Geo o;
  o.R = g->R;
  o.L = g->L;
  o.sigma_z = g->sigma_z;
  o.sigma_dl = g->sigma_dl;
  o.pixel = g->pixel;
  o.ipix = 1.0 / g->pixel;
  o.u = 1.0 / (g->sigma_z * g->sigma_z);
  o.w = 1.0 / (g->sigma_dl * g->sigma_dl);
  o.um = 1.0 / (mask_sz * mask_sz);
  o.wm = 1.0 / (mask_sdl * mask_sdl);
  o.fa = g->kernel_variant ? 2.0 : 1.0;
  o.gamma = g->gamma;
  o.zedge = g->sigma_z_edge;
  {
    const double det = o.u * o.u * o.w - 2.0 * o.u * o.gamma * o.gamma;
    o.cnorm = sqrt(det) / (2.0 * 3.14159265358979323846);
    o.cu = (2.0 * o.u * o.w - 2.0 * o.gamma * o.gamma) / (2.0 * det);
    o.cw = o.u * o.u / (2.0 * det);
  }
  o.y0 = (0.5 - 0.5 * (double)g->n_y) * g->pixel;
  o.z0 = (0.5 - 0.5 * (double)g->n_z) * g->pixel;
  o.n_y = g->n_y;
  o.n_z = g->n_z;
  return o;
}

int64_t npix_of(const jpet_geometry* g) { return (int64_t)g->n_y * (int64_t)g->n_z; }

int carve(const Plan& p, const jpet_geometry* g, int64_t n, void* ws, size_t ws_bytes, Workspace* out) {
  if (!ws) return JPET_EWORKSPACE;
  if (((uintptr_t)ws & 255) != 0) return JPET_EWORKSPACE;
  size_t need = workspace_layout(p, n, npix_of(g), ws, out);
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
  stats->n_unplaced_rows = (int64_t)c[C_OUTSIDE];
  return JPET_OK;
}

int do_prepare(const Geo& geo, const Plan& p, const float* events, int64_t n, const Workspace& w, hipStream_t st) {
  hipError_t e = launch_fill_u64(w.cnt, C_COUNT, st);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_prepare(geo, p, events, n, w, st);
  if (e != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

}  // namespace

int record_hip_failure(hipError_t e) { return hip_fail(e); }

// LDS row-pitch alignment of the binned pass's column-major region
static const int kBankAlign = 64;

// Events per batch: as many as the row segments of the largest ellipses allow on the workgroup's
// threads.
static int events_per_batch(int waves, int units_max) {
  const int epb = (64 * waves) / units_max;
  return epb < 32 ? epb : 32;
}

// Dynamic LDS of the tiled pass for a region of RY x W pixels (row pitch `pitch`): the image and the
// accumulators, the double buffer of per-event constants, the per-row column shifts.
static size_t tiled_lds_layout(int pitch, int W, int RY, int acc32, int epb, bool loglik, int* ev_at, int* off_at) {
  const size_t region = (size_t)pitch * (size_t)W * (acc32 ? 8u : 12u);
  const size_t ev = align_up(region, 16);
  const size_t off = ev + 2u * (size_t)epb * (size_t)event_const_bytes(loglik);
  if (ev_at) *ev_at = (int)ev;
  if (off_at) *off_at = (int)off;
  return align_up(off + 4u * (size_t)RY, 16);
}

// Derived fields of a binned plan whose region (waves, acc32, tile, halo, t bins) is set.
static void finish_plan(const jpet_geometry* g, int rows_max, int64_t n, Plan& p) {
  const double pix = g->pixel;
  p.ev_per_batch = events_per_batch(p.waves, rows_max * p.segs);
  p.cbytes = p.ev_per_batch * event_const_bytes(p.loglik != 0);
  p.lds_bytes = tiled_lds_layout(p.pitch, p.W, p.RY, p.acc32, p.ev_per_batch, p.loglik != 0, &p.lds_ev, &p.lds_off);
  p.batch_bytes = (int)(((unsigned)p.cbytes + 4u * (64u + kBlockTailWords) * (unsigned)p.waves + 255u) / 256u * 256u);
  p.nty = (g->n_y + p.TY - 1) / p.TY;
  // sheared column span: the widest over the t bins
  int span = g->n_z;
  for (int b = 0; b < p.ntb; ++b) {
    const double tc = p.ntb > 1 ? p.tmin + (b + 0.5) * p.dt : 0.0;
    const double y0 = (0.5 - 0.5 * (double)g->n_y) * pix, y1 = y0 + (g->n_y - 1) * pix;
    const int o0 = (int)rint(tc * y0 / pix), o1 = (int)rint(tc * y1 / pix);
    const int lo = o0 < o1 ? o0 : o1, hi = o0 < o1 ? o1 : o0;
    const int sp = g->n_z + (hi - lo);
    if (sp > span) span = sp;
  }
  p.ntz = (span + p.TZ - 1) / p.TZ;
  p.nbins = p.ntb * p.nty * p.ntz;
  // events per workgroup item: enough items to fill the chip, at most 128 batches (the region's
  // staging and flush are amortised over the item)
  int64_t per = n / 1024;
  if (per < p.ev_per_batch) per = p.ev_per_batch;
  if (per > 128 * p.ev_per_batch) per = 128 * p.ev_per_batch;
  // 32-bit accumulators hold 2^-s units: one event adds at most 2^s to a pixel, so an item of up
  // to 2^(32-s) - 1 events cannot overflow before the flush.  Items of at most 511 events keep
  // s = 23 (a rounding step of 2^-23 of a count per pair).
  if (p.acc32 && per > 511) per = 511;
  p.ev_per_wg = (int)((per / p.ev_per_batch) * p.ev_per_batch);
  if (p.acc32) {
    int bits = 0;
    while ((1 << bits) <= p.ev_per_wg) ++bits;  // ev_per_wg < 2^bits
    p.acc_shift = 32 - bits;
  }
  const int64_t nonempty = n < p.nbins ? n : p.nbins;
  p.max_items = (n + p.ev_per_wg - 1) / p.ev_per_wg + nonempty;
  if (p.max_items < 1) p.max_items = 1;
  p.max_batches = (n + p.ev_per_batch - 1) / p.ev_per_batch + nonempty;
  if (p.max_batches < 1) p.max_batches = 1;
  p.tiled = 1;
}

void plan_candidates(const jpet_geometry* g, double msz, double mdl, int64_t n, bool loglik,
                     std::vector<PlanCand>* out) {
  out->clear();
  const bool allow_acc32 = !loglik;
  msz *= 1.0 + g->sigma_z_edge;  // the largest ellipse: sigma_z at the strip ends
  Plan none;
  memset(&none, 0, sizeof(none));
  none.ntb = 1;
  none.segs = 1;
  none.dt = 1.0;
  none.code = kPlanGeneric;
  const double pix = g->pixel;
  const double hy_px = 1.5 * mdl / pix;                 // largest half height of an ellipse (rows)
  const double chord_px = 2.0 * 3.0 * msz / sqrt(2.0) / pix;  // longest chord along z (columns)
  const int maxrow = (int)floor(chord_px) + 1;
  const int rows_max = (int)floor(2.0 * hy_px) + 1;
  const double tmax = 0.5 * g->L / g->R;               // |tan| of any valid event
  int natural = 0;  // the smallest register cache that holds the longest row
  for (int c : {16, 32, 48, 64})
    if (maxrow <= c) {
      natural = c;
      break;
    }
  if (natural == 0 || rows_max > 64 * 16) {  // generic pass only
    out->push_back({none, 0.0});
    return;
  }
  const int HY = (int)ceil(hy_px + 0.5) + 1;
  // Candidate regions: workgroups of 8 or 16 wavefronts, 1 to 4 of them resident per CU (their
  // LDS regions share the CU's 160 KB with the static batch buffers), 64-bit or 32-bit
  // accumulators (12 or 8 bytes per region pixel); for each, no shear or t bins of a given width,
  // and square tiles of a given size.  Residency is also bounded by registers: the event pass
  // compiled for a register cache of 16/32/48/64 pixels keeps at most 8/6/5/4 wavefronts per SIMD
  // (its launch bounds guarantee that many).
  //
  // Each candidate's cost-model figure, in units of (event, pixel) pairs:
  //   pairs of all events (an ellipse's area at theta = 0)
  //     x (4 / wavefronts per SIMD)^0.58  (measured: 6 resident wavefronts per SIMD run the pass
  //                                        in 0.79 of the time of 4)
  //     x 1.1 for 16-wave workgroups (more wavefronts meet at every barrier)
  //     x 0.82 for 32-bit accumulators (the back-projection's LDS atomics, about 30% of the pass
  //            with 64-bit ones, run 2.7 times faster on 32-bit words)
  //   + 1.6 x region pixels x workgroup items,
  // the second term being the staging of the image region and the flush of its accumulators
  // (about 1.6 pair evaluations per region pixel); items are the events over the events per item
  // plus, at most, one partial item per bin.
  // (the log-likelihood pass, with its derivative terms, keeps 6 / 4 / 4 / 4).  Rows longer than
  // a cache of 16 or 32 may also be split into two segments, one thread each (x 1.3: the second
  // row setups, the shorter segments and the lanes they leave idle; a prior, not a measurement,
  // that keeps whole rows the model's choice wherever they fit and leaves split plans to timing).
  for (int cache = 0; cache <= 2; ++cache) {
    int maxlen = natural, segs = 1;
    if (cache > 0) {
      maxlen = cache == 1 ? 16 : 32;
      if (!(maxrow > maxlen && maxrow <= 2 * maxlen)) continue;  // not needed, or too long to split in two
      segs = 2;
    }
    const int simd_waves = loglik ? (maxlen <= 16 ? 6 : 4) : maxlen <= 16 ? 8 : maxlen <= 32 ? 6 : maxlen <= 48 ? 5 : 4;
    // LDS per CU, the passes' static LDS (per-event denominators; the log-likelihood pass also its
    // derivative sums), and the allocation granule: measured on gfx950, three workgroups of 51,984
    // bytes each run on one CU but three of 54,032 bytes do not (the pass then runs 27% slower), so
    // a workgroup's LDS is counted in whole 2 KB granules.
    const size_t kLdsPerCU = 160 * 1024, kStatic = loglik ? 3 * 1024 : 1024, kGranule = 2048;
    const double pairs_per_event = 3.14159265358979323846 * hy_px * (3.0 * msz / sqrt(2.0) / pix);
    const double nn = (double)(n > 0 ? n : 1);
    for (int waves : {8, 16}) {
      if (rows_max * segs > 64 * waves) continue;
      for (int wgs = 1; wgs <= 4; ++wgs) {
        const int occ = wgs * waves / 4;  // resident wavefronts per SIMD
        if (occ > simd_waves) continue;
        const size_t budget = kLdsPerCU / (size_t)wgs / kGranule * kGranule - kStatic;
        const double occ_factor = pow(4.0 / (double)occ, 0.58) * (waves == 16 ? 1.1 : 1.0) * (segs > 1 ? 1.3 : 1.0);
        for (int acc32 = 0; acc32 <= 1; ++acc32) {
          if (acc32 && !allow_acc32) continue;
          for (int dti = 0; dti < kPlanDtCount; ++dti) {
            const double dt = kPlanDt[dti];
            // largest |t - t_c| / c inside a bin (no shear: |t| / c <= sin(atan(tmax)))
            const double tau = dt == 0.0 ? tmax / sqrt(1.0 + tmax * tmax) : 0.5 * dt;
            const double hz = 3.0 * sqrt(0.5 * msz * msz + 0.25 * mdl * mdl * tau * tau);
            const int HZ = (int)ceil(hz / pix + 1.0) + 1;
            for (int ti = 0; ti < kPlanTileCount; ++ti) {
              const int T = kPlanTile[ti];
              // LDS: float image, then the accumulators, column-major with the row pitch rounded
              // up to the bank alignment; masked reads up to maxlen columns past the image must stay
              // in the accumulator array (W columns of 4 or 8 bytes)
              const int RY = T + 2 * HY, W = T + 2 * HZ;
              const int pitch = (RY + kBankAlign - 1) / kBankAlign * kBankAlign;
              const size_t bytes = tiled_lds_layout(pitch, W, RY, acc32, events_per_batch(waves, rows_max * segs),
                                                    loglik, nullptr, nullptr);
              const int reach = acc32 ? W : 2 * W;
              // thread words address columns with 8 bits and rows with 9 bits
              if (bytes > budget || reach < maxlen || W > 256 || RY > 512) continue;
              Plan p = none;
              p.maxlen = maxlen;
              p.segs = segs;
              p.HY = HY;
              p.pitch = pitch;
              p.waves = waves;
              p.acc32 = acc32;
              p.TY = T;
              p.TZ = T;
              p.HZ = HZ;
              p.RY = RY;
              p.W = W;
              p.wgs = wgs;
              p.loglik = loglik ? 1 : 0;
              p.code = plan_code(waves, acc32, wgs, dti, ti, cache);
              if (dt != 0.0) {
                p.ntb = (int)ceil(2.0 * tmax / dt);
                if (p.ntb < 1) p.ntb = 1;
                p.dt = dt;
                p.tmin = -0.5 * dt * p.ntb;
              }
              finish_plan(g, rows_max, n, p);
              const double items = nn / p.ev_per_wg + (nn < p.nbins ? nn : (double)p.nbins);
              const double cost = nn * pairs_per_event * occ_factor * (acc32 ? 0.82 : 1.0) +
                                  1.6 * items * (double)pitch * (double)W;
              out->push_back({p, cost});
            }
          }
        }
      }
    }
  }
  if (out->empty()) {
    out->push_back({none, 0.0});
    return;
  }
  std::stable_sort(out->begin(), out->end(), [](const PlanCand& a, const PlanCand& b) { return a.cost < b.cost; });
}

Plan make_plan(const jpet_geometry* g, double msz, double mdl, int64_t n, bool loglik) {
  std::vector<PlanCand> c;
  plan_candidates(g, msz, mdl, n, loglik, &c);
  const int32_t want = g->plan;
  if (want == 0) return c[0].p;
  if (want == kPlanGeneric) {
    Plan p;
    memset(&p, 0, sizeof(p));
    p.ntb = 1;
    p.segs = 1;
    p.dt = 1.0;
    p.code = kPlanGeneric;
    return p;
  }
  for (const PlanCand& x : c)
    if (x.p.code == want) return x.p;
  Plan bad = c[0].p;
  bad.invalid = 1;
  bad.code = want;
  return bad;
}

size_t workspace_layout(const Plan& p, int64_t n, int64_t npix, void* base, Workspace* out) {
  size_t off = 0;
  // offsets from base; a size query (base NULL) forms no pointers
  auto take = [&](size_t bytes) {
    char* q = base ? (char*)base + off : nullptr;
    off = align_up(off + bytes, 256);
    return q;
  };
  const size_t nn = (size_t)(n > 0 ? n : 0);
  const size_t nb = (size_t)(p.tiled ? p.nbins : 0);
  Workspace w;
  // buffers every entry point uses come first, so their offsets do not depend on the binning
  w.cnt = (unsigned long long*)take(sizeof(unsigned long long) * C_COUNT);
  w.red = (double*)take(sizeof(double) * RED_SLOTS);
  w.acc = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)npix);
  w.B = (double*)take(sizeof(double) * (size_t)npix);
  w.ev = (EventRec*)take(sizeof(EventRec) * nn);
  w.key = (uint32_t*)take(sizeof(uint32_t) * nn);
  // binning (tiled pass only)
  w.evs = (EventRec*)take(p.tiled ? sizeof(EventRec) * nn : 0);
  w.batches = (unsigned char*)take(p.tiled ? (size_t)p.batch_bytes * (size_t)p.max_batches : 0);
  w.bin_count = (uint32_t*)take(sizeof(uint32_t) * nb);
  w.bin_start = (uint32_t*)take(sizeof(uint32_t) * (nb + 1));
  w.bin_fill = (uint32_t*)take(sizeof(uint32_t) * nb);
  w.item_start = (uint32_t*)take(sizeof(uint32_t) * (nb + 1));
  w.batch_start = (uint32_t*)take(sizeof(uint32_t) * (nb + 1));
  w.items = (BinItem*)take(p.tiled ? sizeof(BinItem) * (size_t)p.max_items : 0);
  w.bytes = off;
  if (out) *out = w;
  return off;
}

// Layout of a batched workspace: the instance table, then one ordinary workspace per instance.
// Every instance that fits the binned pass takes the plan its geometry names or the cost model's
// cheapest plan with 32-bit accumulators.  Instances whose plans share the register cache, the
// wavefronts per workgroup, the workgroups resident per CU and the region's row pitch (64, 128,
// 256 or any other) form a class, served by one batched launch per iteration with the class's
// largest LDS region; a batch of like instances is one class.  Within a class the table lists the instances heaviest workgroup
// item first, so that the longest items are pulled earliest.  Instances that fit only the generic
// pass follow the classes, with their own launches.
struct BatchClass {
  int first = 0, count = 0;  // table positions
  int maxlen = 0, waves = 0, wgs = 0;
  int pitch = 0;             // region row pitch the class is compiled for (0: a runtime value)
  size_t lds = 0;
  int64_t items = 0;         // workgroup items of the class's instances (set once they are prepared)
  double cost = 0.0;         // estimated pairs of those items (set with items)
  int stream = 0;            // 0: the caller's stream, k > 0: the batch's k-th side stream
};

// Streams that share a batch's class launches: the caller's and kBatchStreams - 1 of the library's.
constexpr int kBatchStreams = 2;

struct BatchLayout {
  std::vector<Plan> plan;       // per instance
  std::vector<size_t> off;      // per instance: byte offset of its workspace
  std::vector<int> order;       // table position -> instance
  std::vector<double> work;     // per instance: estimated pairs of one full workgroup item
  std::vector<BatchClass> cls;  // the batched launches
  std::vector<int> launch;      // class indices in launch order: heaviest first
  int streams = 1;              // streams the classes are spread over
  int64_t max_npix = 0;
  size_t total = 0;
  bool invalid = false;         // a named plan does not fit its geometry or the batched pass
};

static bool batchable(const Plan& p) { return p.tiled && p.acc32 && !p.loglik; }

BatchLayout batch_layout(const jpet_instance* inst, int count) {
  BatchLayout L;
  L.plan.resize(count);
  L.off.resize(count);
  std::vector<double>& work = L.work;
  work.assign(count, 0.0);
  std::vector<int> key(count, 1 << 30);  // class key; generic instances last
  std::vector<PlanCand> cand;
  for (int k = 0; k < count; ++k) {
    const jpet_geometry& g = inst[k].g;
    Plan p;
    if (g.plan != 0) {
      p = make_plan(&g, g.sigma_z, g.sigma_dl, inst[k].n);
      if (p.invalid || (p.tiled && !batchable(p))) {
        L.invalid = true;
        return L;
      }
    } else {
      plan_candidates(&g, g.sigma_z, g.sigma_dl, inst[k].n, false, &cand);
      p = cand[0].p;  // the generic pass when no binned plan fits
      for (const PlanCand& x : cand)  // sorted by cost: the first batchable one
        if (batchable(x.p)) {
          p = x.p;
          break;
        }
      if (p.tiled && !batchable(p)) {  // binned plans fit, none with a cache of 32 or less
        L.invalid = true;
        return L;
      }
    }
    L.plan[k] = p;
    if (p.tiled) {
      key[k] = ((batched_pitch_class(p.pitch) * 128 + p.maxlen) * 32 + p.waves) * 8 + p.wgs;
      // pixels of a typical ellipse (App. B half sizes at theta = 0) times events per workgroup
      work[k] = (1.5 * g.sigma_dl / g.pixel) * (3.0 * g.sigma_z / sqrt(2.0) / g.pixel) * p.ev_per_wg;
    }
    const int64_t np = npix_of(&g);
    if (np > L.max_npix) L.max_npix = np;
  }
  L.order.resize(count);
  for (int k = 0; k < count; ++k) L.order[k] = k;
  std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) {
    if (key[a] != key[b]) return key[a] < key[b];
    return work[a] > work[b];
  });
  for (int t = 0; t < count; ++t) {
    const int k = L.order[t];
    const Plan& p = L.plan[k];
    if (!p.tiled) break;
    if (L.cls.empty() || key[L.order[L.cls.back().first]] != key[k]) {
      BatchClass c;
      c.first = t;
      c.waves = p.waves;
      c.wgs = p.wgs;
      c.pitch = batched_pitch_class(p.pitch);
      L.cls.push_back(c);
    }
    BatchClass& c = L.cls.back();
    ++c.count;
    c.maxlen = p.maxlen > c.maxlen ? p.maxlen : c.maxlen;
    if (p.lds_bytes > c.lds) c.lds = p.lds_bytes;
  }
  size_t off = align_up(sizeof(BatchInst) * (size_t)count, 256);
  for (int k = 0; k < count; ++k) {
    L.off[k] = off;
    off = align_up(off + workspace_layout(L.plan[k], inst[k].n, npix_of(&inst[k].g), nullptr, nullptr), 256);
  }
  L.total = off;
  return L;
}

int check_instances(const jpet_instance* inst, int32_t count) {
  if (count < 0 || count > 65535 || (count > 0 && !inst)) return JPET_EINVAL;
  for (int k = 0; k < count; ++k) {
    const int rc = check_geometry(&inst[k].g);
    if (rc) return rc;
    if (inst[k].n < 0 || inst[k].n > kMaxEvents || (inst[k].n > 0 && !inst[k].events) || !inst[k].rho)
      return JPET_EINVAL;
  }
  return JPET_OK;
}

}  // namespace jpet

using namespace jpet;

// One event pass (per-iteration counters reset first), bracketed by timing events when profiling
// is on.
// Runs launch() bracketed by timing events when profiling is on.
template <class F>
static int timed(F launch, hipStream_t st) {
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool on = false;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    on = g_prof_on;
  }
  hipError_t e;
  if (on) {
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return hip_fail(e);
    if ((e = hipEventCreate(&ev1)) != hipSuccess) return hip_fail(e);
    if ((e = hipEventRecord(ev0, st)) != hipSuccess) return hip_fail(e);
  }
  e = launch();
  if (e != hipSuccess) return hip_fail(e);
  if (on) {
    if ((e = hipEventRecord(ev1, st)) != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_events.emplace_back(ev0, ev1);
  }
  return JPET_OK;
}

static int timed_event_pass(const Geo& geo, const Plan& p, int64_t n, const Workspace& w, const float* rho,
                            hipStream_t st, int granularity = kPassPlanned, float* D_out = nullptr) {
  // per-pass counters: zero-denominator events, non-positive kappa pairs, unplaced rows
  hipError_t e = launch_fill_u64(w.cnt + C_ZERO_DEN, 2, st);
  if (e != hipSuccess) return hip_fail(e);
  return timed([&] { return launch_event_pass(geo, p, n, w, rho, st, granularity, D_out); }, st);
}

// The pass granularity a flag word asks for; -1 for unknown flags or both comparison flags.
static int pass_granularity(uint32_t flags) {
  if (flags & ~(JPET_WS_PREPARED | JPET_PASS_WAVE_PER_EVENT | JPET_PASS_THREAD_PER_EVENT)) return -1;
  const bool wv = (flags & JPET_PASS_WAVE_PER_EVENT) != 0, th = (flags & JPET_PASS_THREAD_PER_EVENT) != 0;
  if (wv && th) return -1;
  return wv ? kPassWavePerEvent : th ? kPassThreadPerEvent : kPassPlanned;
}

extern "C" {

const char* jpet_strerror(int status) {
  switch (status) {
    case JPET_OK: return "success";
    case JPET_EINVAL: return "invalid argument (NULL pointer, negative count or unknown flag)";
    case JPET_EDOMAIN:
      return "argument out of domain (geometry, resolution, grid, or a plan that does not fit them) or "
             "log-likelihood is -inf";
    case JPET_EWORKSPACE: return "workspace missing, misaligned or smaller than jpet_mlem_workspace_size";
    case JPET_EHIP: return "HIP runtime error (see jpet_last_hip_error)";
    case JPET_ENOTSUP: return "not supported by this build";
    default: return "unknown status";
  }
}

int jpet_last_hip_error(void) { return g_last_hip_error; }

int jpet_abi_version(void) { return JPET_ABI_VERSION; }

int jpet_profile_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = enable != 0;
  if (!g_prof_on) prof_forget_locked();
  return JPET_OK;
}

int jpet_profile_read(int64_t* launches, double* total_ms) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  int rc = JPET_OK;
  for (auto& pr : g_prof_events) {
    hipError_t e = hipEventSynchronize(pr.second);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess && rc == JPET_OK) rc = hip_fail(e);
    tot += ms;
  }
  if (launches) *launches = (int64_t)g_prof_events.size();
  if (total_ms) *total_ms = tot;
  prof_forget_locked();
  return rc;
}

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
  if (!bytes || n_events < 0 || n_events > kMaxEvents) return JPET_EINVAL;
  const Plan p = make_plan(g, g->sigma_z, g->sigma_dl, n_events);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  *bytes = workspace_layout(p, n_events, npix_of(g), nullptr, nullptr);
  return JPET_OK;
}

int jpet_direct_image(const jpet_geometry* g, const float* events, int64_t n, float* img, void* stream) {
  const int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || (n > 0 && !events) || !img) return JPET_EINVAL;
  const hipError_t e =
      launch_direct_image(make_geo(g, g->sigma_z, g->sigma_dl), g->L, events, n, img, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

int jpet_loglik_workspace_size(const jpet_geometry* g, const double* sigma_mask, int64_t n_events, size_t* bytes) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (!bytes || n_events < 0 || n_events > kMaxEvents) return JPET_EINVAL;
  if (g->sigma_z_edge != 0.0) return JPET_ENOTSUP;  // defined for one sigma_z for all events
  double msz = g->sigma_z, mdl = g->sigma_dl;
  if (sigma_mask) {
    msz = sigma_mask[0];
    mdl = sigma_mask[1];
    if (!finite_pos(msz) || !finite_pos(mdl)) return JPET_EDOMAIN;
  }
  const Plan p = make_plan(g, msz, mdl, n_events, true);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  *bytes = workspace_layout(p, n_events, npix_of(g), nullptr, nullptr);
  return JPET_OK;
}

int jpet_mlem_launch_info(const jpet_geometry* g, int64_t n_events, jpet_launch_info* info) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (!info || n_events < 0 || n_events > kMaxEvents) return JPET_EINVAL;
  const Plan p = make_plan(g, g->sigma_z, g->sigma_dl, n_events);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  memset(info, 0, sizeof(*info));
  info->binned = p.tiled;
  info->tile_rows = p.TY;
  info->tile_cols = p.TZ;
  info->halo_rows = p.HY;
  info->halo_cols = p.HZ;
  info->t_bins = p.ntb;
  info->bins = p.nbins;
  info->waves = p.waves;
  info->row_cache = p.maxlen;
  info->events_per_batch = p.ev_per_batch;
  info->events_per_workgroup = p.ev_per_wg;
  info->t_bin_width = p.ntb > 1 ? p.dt : 0.0;
  info->lds_bytes = (int64_t)p.lds_bytes;
  info->max_workgroups = p.max_items;
  info->accumulator_bits = p.tiled ? (p.acc32 ? 32 : 64) : 64;
  info->plan = p.code;
  info->workgroups_per_cu = p.tiled ? p.wgs : 0;
  info->accumulator_shift = p.tiled && p.acc32 ? p.acc_shift : 0;
  info->row_segments = p.tiled ? p.segs : 1;
  return JPET_OK;
}

int jpet_mlem_plan_candidates(const jpet_geometry* g, int32_t pass, const double* sigma_mask, int64_t n_events,
                              int32_t* codes, double* model_cost, int32_t cap, int32_t* count) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (!count || cap < 0 || (cap > 0 && !codes) || n_events < 0 || n_events > kMaxEvents) return JPET_EINVAL;
  if (pass != 0 && pass != 1) return JPET_EINVAL;
  if (pass == 0 && sigma_mask) return JPET_EINVAL;
  double msz = g->sigma_z, mdl = g->sigma_dl;
  if (sigma_mask) {
    msz = sigma_mask[0];
    mdl = sigma_mask[1];
    if (!finite_pos(msz) || !finite_pos(mdl)) return JPET_EDOMAIN;
  }
  std::vector<PlanCand> c;
  plan_candidates(g, msz, mdl, n_events, pass == 1, &c);
  *count = (int32_t)c.size();
  for (int32_t k = 0; k < cap && k < (int32_t)c.size(); ++k) {
    codes[k] = c[k].p.code;
    if (model_cost) model_cost[k] = c[k].cost;
  }
  return JPET_OK;
}

int jpet_mlem_prepare(const jpet_geometry* g, const float* events, int64_t n, void* ws, size_t ws_bytes,
                      void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || n > kMaxEvents || (n > 0 && !events)) return JPET_EINVAL;
  const Plan p = make_plan(g, g->sigma_z, g->sigma_dl, n);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  Workspace w;
  rc = carve(p, g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  return do_prepare(make_geo(g, g->sigma_z, g->sigma_dl), p, events, n, w, (hipStream_t)stream);
}

int jpet_mlem_iterate(const jpet_geometry* g, const float* events, int64_t n, const float* s, float* rho,
                      int32_t n_iter, void* ws, size_t ws_bytes, uint32_t flags, jpet_stats* stats,
                      void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || n > kMaxEvents || (n > 0 && !events) || !rho || n_iter < 0) return JPET_EINVAL;
  const int gran = pass_granularity(flags);
  if (gran < 0) return JPET_EINVAL;
  const Plan p = make_plan(g, g->sigma_z, g->sigma_dl, n);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  Workspace w;
  rc = carve(p, g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geo geo = make_geo(g, g->sigma_z, g->sigma_dl);
  if (!(flags & JPET_WS_PREPARED)) {
    rc = do_prepare(geo, p, events, n, w, st);
    if (rc) return rc;
  }
  hipError_t e = launch_fill_u64(w.acc, npix_of(g), st);
  if (e != hipSuccess) return hip_fail(e);
  for (int it = 0; it < n_iter; ++it) {
    rc = timed_event_pass(geo, p, n, w, rho, st, gran);
    if (rc) return rc;
    e = launch_update(geo, s, rho, w, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (stats) return read_stats(w, n, stats, st);
  return JPET_OK;
}

int jpet_mlem_backproject(const jpet_geometry* g, const float* events, int64_t n, const float* rho, uint64_t* acc,
                          void* ws, size_t ws_bytes, uint32_t flags, jpet_stats* stats, void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || n > kMaxEvents || (n > 0 && !events) || !rho || !acc) return JPET_EINVAL;
  const int gran = pass_granularity(flags);
  if (gran < 0) return JPET_EINVAL;
  const Plan p = make_plan(g, g->sigma_z, g->sigma_dl, n);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  Workspace w;
  rc = carve(p, g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geo geo = make_geo(g, g->sigma_z, g->sigma_dl);
  if (!(flags & JPET_WS_PREPARED)) {
    rc = do_prepare(geo, p, events, n, w, st);
    if (rc) return rc;
  }
  w.acc = reinterpret_cast<unsigned long long*>(acc);
  rc = timed_event_pass(geo, p, n, w, rho, st, gran);
  if (rc) return rc;
  if (stats) return read_stats(w, n, stats, st);
  return JPET_OK;
}

int jpet_mlem_denominators(const jpet_geometry* g, const float* events, int64_t n, const float* rho, float* D_out,
                           void* ws, size_t ws_bytes, uint32_t flags, jpet_stats* stats, void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || n > kMaxEvents || (n > 0 && !events) || !rho || (n > 0 && !D_out)) return JPET_EINVAL;
  const int gran = pass_granularity(flags);
  if (gran < 0) return JPET_EINVAL;
  const Plan p = make_plan(g, g->sigma_z, g->sigma_dl, n);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  Workspace w;
  rc = carve(p, g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geo geo = make_geo(g, g->sigma_z, g->sigma_dl);
  if (!(flags & JPET_WS_PREPARED)) {
    rc = do_prepare(geo, p, events, n, w, st);
    if (rc) return rc;
  }
  hipError_t e = launch_fill_f32(D_out, n, st);
  if (e != hipSuccess) return hip_fail(e);
  rc = timed_event_pass(geo, p, n, w, rho, st, gran, D_out);
  if (rc) return rc;
  if ((e = launch_fill_u64(w.acc, npix_of(g), st)) != hipSuccess) return hip_fail(e);
  if (stats) return read_stats(w, n, stats, st);
  return JPET_OK;
}

int jpet_mlem_tune_workspace_size(const jpet_geometry* g, int64_t n_events, const int32_t* codes, int32_t ncodes,
                                  size_t* bytes) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (!bytes || n_events < 0 || n_events > kMaxEvents || ncodes < 0 || (ncodes > 0 && !codes)) return JPET_EINVAL;
  size_t most = 0;
  for (int32_t k = 0; k < ncodes; ++k) {
    if (!plan_code_valid(codes[k])) return JPET_EINVAL;
    jpet_geometry gk = *g;
    gk.plan = codes[k];
    const Plan p = make_plan(&gk, gk.sigma_z, gk.sigma_dl, n_events);
    if (p.invalid) continue;  // timed as not fitting
    const size_t b = workspace_layout(p, n_events, npix_of(g), nullptr, nullptr);
    if (b > most) most = b;
  }
  *bytes = most;
  return JPET_OK;
}

int jpet_mlem_tune(const jpet_geometry* g, const float* events, int64_t n, const float* rho, const int32_t* codes,
                   int32_t ncodes, int32_t reps, void* ws, size_t ws_bytes, double* ms_out, void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || n > kMaxEvents || (n > 0 && !events) || !rho || ncodes < 0 || (ncodes > 0 && (!codes || !ms_out)) ||
      reps < 1)
    return JPET_EINVAL;
  for (int32_t k = 0; k < ncodes; ++k)
    if (!plan_code_valid(codes[k])) return JPET_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e);
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e);
  }
  struct Guard {
    hipEvent_t a, b;
    ~Guard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  for (int32_t k = 0; k < ncodes; ++k) {
    ms_out[k] = -1.0;  // does not fit
    jpet_geometry gk = *g;
    gk.plan = codes[k];
    const Plan p = make_plan(&gk, gk.sigma_z, gk.sigma_dl, n);
    if (p.invalid) continue;
    Workspace w;
    rc = carve(p, &gk, n, ws, ws_bytes, &w);
    if (rc) return rc;
    const Geo geo = make_geo(&gk, gk.sigma_z, gk.sigma_dl);
    if ((rc = do_prepare(geo, p, events, n, w, st))) return rc;
    if ((e = launch_fill_u64(w.acc, npix_of(g), st)) != hipSuccess) return hip_fail(e);
    // one pass untimed (first-launch costs), then reps passes; rho is only read
    if ((e = launch_event_pass(geo, p, n, w, rho, st)) != hipSuccess) return hip_fail(e);
    if ((e = hipEventRecord(e0, st)) != hipSuccess) return hip_fail(e);
    for (int32_t r = 0; r < reps; ++r)
      if ((e = launch_event_pass(geo, p, n, w, rho, st)) != hipSuccess) return hip_fail(e);
    if ((e = hipEventRecord(e1, st)) != hipSuccess) return hip_fail(e);
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e);
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return hip_fail(e);
    ms_out[k] = (double)ms / reps;
  }
  return JPET_OK;
}

int jpet_mlem_update(const jpet_geometry* g, const float* s, uint64_t* acc, float* rho, void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (!acc || !rho) return JPET_EINVAL;
  Workspace w;
  memset(&w, 0, sizeof(w));
  w.acc = reinterpret_cast<unsigned long long*>(acc);
  const hipError_t e = launch_update(make_geo(g, g->sigma_z, g->sigma_dl), s, rho, w, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

int jpet_loglik_grad(const jpet_geometry* g, const double* sigma_mask, const float* events, int64_t n,
                     const float* s, const float* rho, double* out3, float* grad_rho, float* D_out, void* ws,
                     size_t ws_bytes, uint32_t flags, jpet_stats* stats, void* stream) {
  int rc = check_geometry(g);
  if (rc) return rc;
  if (n < 0 || n > kMaxEvents || (n > 0 && !events) || !rho || !out3) return JPET_EINVAL;
  if (flags & ~(JPET_WS_PREPARED | JPET_LOGLIK_VALUE_ONLY)) return JPET_EINVAL;
  const bool value_only = (flags & JPET_LOGLIK_VALUE_ONLY) != 0;
  if (value_only && grad_rho) return JPET_EINVAL;
  if (g->sigma_z_edge != 0.0) return JPET_ENOTSUP;  // defined for one sigma_z for all events
  double msz = g->sigma_z, mdl = g->sigma_dl;
  if (sigma_mask) {
    msz = sigma_mask[0];
    mdl = sigma_mask[1];
    if (!finite_pos(msz) || !finite_pos(mdl)) return JPET_EDOMAIN;
  }
  // a prepared workspace carries the kernel constants of the sigmas it was prepared with
  if ((flags & JPET_WS_PREPARED) && (msz != g->sigma_z || mdl != g->sigma_dl)) return JPET_EINVAL;
  // the binned log-likelihood pass accumulates doubles: plans with 64-bit region slots only
  const Plan p = make_plan(g, msz, mdl, n, true);
  if (p.invalid) return JPET_EDOMAIN;  // the named plan does not fit this geometry
  Workspace w;
  rc = carve(p, g, n, ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geo geo = make_geo(g, msz, mdl);
  if (!(flags & JPET_WS_PREPARED)) {
    rc = do_prepare(geo, p, events, n, w, st);
    if (rc) return rc;
  }
  hipError_t e = launch_fill_u64(w.cnt + C_ZERO_DEN, 2, st);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_loglik(geo, p, n, w, rho, s, D_out, grad_rho, out3, value_only, st);
  if (e != hipSuccess) return hip_fail(e);
  if (stats) {
    rc = read_stats(w, n, stats, st);
    if (rc) return rc;
    if (stats->n_zero_denominator > 0) return JPET_EDOMAIN;
  }
  return JPET_OK;
}

int jpet_mlem_batched_workspace_size(const jpet_instance* inst, int32_t count, size_t* bytes) {
  if (!bytes) return JPET_EINVAL;
  const int rc = check_instances(inst, count);
  if (rc) return rc;
  const BatchLayout L = batch_layout(inst, count);
  if (L.invalid) return JPET_EDOMAIN;
  *bytes = L.total;
  return JPET_OK;
}

static int batched_carve(const jpet_instance* inst, int32_t count, void* ws, size_t ws_bytes, BatchLayout* L,
                         std::vector<Workspace>* w) {
  int rc = check_instances(inst, count);
  if (rc) return rc;
  *L = batch_layout(inst, count);
  if (L->invalid) return JPET_EDOMAIN;
  if (!ws || ((uintptr_t)ws & 255) != 0 || ws_bytes < L->total) return JPET_EWORKSPACE;
  w->resize(count);
  for (int k = 0; k < count; ++k) {
    rc = carve(L->plan[k], &inst[k].g, inst[k].n, (char*)ws + L->off[k], ws_bytes - L->off[k], &(*w)[k]);
    if (rc) return rc;
  }
  return JPET_OK;
}

int jpet_mlem_batched_prepare(const jpet_instance* inst, int32_t count, void* ws, size_t ws_bytes, void* stream) {
  BatchLayout L;
  std::vector<Workspace> w;
  int rc = batched_carve(inst, count, ws, ws_bytes, &L, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  for (int k = 0; k < count; ++k) {
    const jpet_geometry& g = inst[k].g;
    rc = do_prepare(make_geo(&g, g.sigma_z, g.sigma_dl), L.plan[k], inst[k].events, inst[k].n, w[k], st);
    if (rc) return rc;
  }
  return JPET_OK;
}

}  // extern "C"

// Each class's workgroup items and each binned instance's first work index within its class, from
// the items the instances' preparation produced (read back once; the stream is synchronised).
static int batched_items(int32_t count, BatchLayout* L, const std::vector<Workspace>& w, hipStream_t st,
                         std::vector<int64_t>* item_begin) {
  std::vector<unsigned long long> items((size_t)count, 0ull);
  hipError_t e;
  for (int t = 0; t < count; ++t) {
    const int k = L->order[t];
    if (!L->plan[k].tiled) continue;
    if ((e = hipMemcpyAsync(&items[k], w[k].cnt + C_ITEMS, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
      return hip_fail(e);
  }
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e);
  item_begin->assign((size_t)count, 0);
  for (BatchClass& C : L->cls) {
    C.items = 0;
    C.cost = 0.0;
    for (int t = C.first; t < C.first + C.count; ++t) {
      const int k = L->order[t];
      (*item_begin)[k] = C.items;
      C.items += (int64_t)items[k];
      C.cost += (double)items[k] * L->work[k];
    }
    if (C.items > 0x7fffffffll) return JPET_EINVAL;  // the launch grid is 32-bit
  }
  // the streams share the classes, heaviest first to the least loaded one, so that one class's
  // tail overlaps another class's work; each stream launches its classes heaviest first, so that
  // the streams end on their lightest classes
  std::vector<int>& by_cost = L->launch;
  by_cost.resize(L->cls.size());
  for (size_t c = 0; c < by_cost.size(); ++c) by_cost[c] = (int)c;
  std::stable_sort(by_cost.begin(), by_cost.end(), [&](int a, int b) { return L->cls[a].cost > L->cls[b].cost; });
  L->streams = std::max(1, std::min(kBatchStreams, (int)L->cls.size()));
  double load[kBatchStreams] = {};
  for (int c : by_cost) {
    int s = 0;
    for (int q = 1; q < L->streams; ++q)
      if (load[q] < load[s]) s = q;
    L->cls[c].stream = s;
    load[s] += L->cls[c].cost;
  }
  return JPET_OK;
}

// The setup of a batch's iterations, in stream order: the instance table (with each binned
// instance's first work index) and cleared accumulators.
static int batched_setup(const jpet_instance* inst, int32_t count, const BatchLayout& L,
                         const std::vector<Workspace>& w, const std::vector<Geo>& geo,
                         const std::vector<int64_t>& item_begin, void* ws, hipStream_t st) {
  BatchInst* table = reinterpret_cast<BatchInst*>(ws);
  hipError_t e;
  // written by small launches (by-value arguments) so that it stays stream-ordered
  for (int t0 = 0; t0 < count; t0 += kInstPerWrite) {
    InstWrite iw;
    memset(&iw, 0, sizeof(iw));
    iw.first = t0;
    iw.count = count - t0 < kInstPerWrite ? count - t0 : kInstPerWrite;
    for (int j = 0; j < iw.count; ++j) {
      const int k = L.order[t0 + j];
      BatchInst& b = iw.v[j];
      b.g = geo[k];
      b.p = L.plan[k];
      b.tiled = L.plan[k].tiled;
      b.index = k;
      b.item_begin = item_begin[k];
      b.cls = -1;
      for (int c = 0; c < (int)L.cls.size(); ++c)
        if (t0 + j >= L.cls[c].first && t0 + j < L.cls[c].first + L.cls[c].count) b.cls = c;
      b.n = inst[k].n;
      b.blocks = w[k].batches;
      b.items = w[k].items;
      b.rho = inst[k].rho;
      b.s = inst[k].s;
      b.acc = w[k].acc;
      b.cnt = w[k].cnt;
    }
    if ((e = launch_write_insts(iw, table, st)) != hipSuccess) return hip_fail(e);
  }
  for (int k = 0; k < count; ++k)
    if ((e = launch_fill_u64(w[k].acc, npix_of(&inst[k].g), st)) != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

// The batched pass's side streams on the current device (default priority) with the fork event
// and one join event each: created on first use, outside any capture (batched_begin), kept until
// the process ends.
struct SideStream {
  hipStream_t s[kBatchStreams - 1] = {};
  hipEvent_t fork = nullptr, join[kBatchStreams - 1] = {};
};
static std::mutex g_side_mu;
static std::vector<SideStream> g_side;  // per device

static int side_stream(SideStream* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  std::lock_guard<std::mutex> lk(g_side_mu);
  if ((int)g_side.size() <= dev) g_side.resize((size_t)dev + 1);
  SideStream& S = g_side[(size_t)dev];
  if (!S.fork) {
    for (int q = 0; q < kBatchStreams - 1; ++q) {
      if ((e = hipStreamCreateWithFlags(&S.s[q], hipStreamNonBlocking)) != hipSuccess) return hip_fail(e);
      if ((e = hipEventCreateWithFlags(&S.join[q], hipEventDisableTiming)) != hipSuccess) return hip_fail(e);
    }
    if ((e = hipEventCreateWithFlags(&S.fork, hipEventDisableTiming)) != hipSuccess) return hip_fail(e);
  }
  *out = S;
  return JPET_OK;
}

// n_iter iterations of a set-up batch: per iteration the counters' reset, one batched pass per
// class over its instances' items (the classes shared by the caller's stream and the side
// streams, joined before the update), the generic instances' passes and the pixel update of all.
static int batched_iterations(const jpet_instance* inst, int32_t count, int32_t n_iter, const BatchLayout& L,
                              const std::vector<Workspace>& w, const std::vector<Geo>& geo, void* ws, bool timing,
                              hipStream_t st) {
  BatchInst* table = reinterpret_cast<BatchInst*>(ws);
  hipError_t e;
  SideStream side;
  const int ns = L.streams;
  if (ns > 1) {
    const int rc = side_stream(&side);
    if (rc) return rc;
  }
  for (int it = 0; it < n_iter; ++it) {
    if ((e = launch_batched_reset(table, count, st)) != hipSuccess) return hip_fail(e);
    if (!L.cls.empty()) {
      auto pass = [&] {
        hipError_t r = hipSuccess;
        if (ns > 1) r = hipEventRecord(side.fork, st);
        for (int q = 1; q < ns && r == hipSuccess; ++q) r = hipStreamWaitEvent(side.s[q - 1], side.fork, 0);
        for (size_t i = 0; i < L.launch.size() && r == hipSuccess; ++i) {
          const BatchClass& C = L.cls[(size_t)L.launch[i]];
          r = launch_event_pass_batched(table + C.first, C.count, C.maxlen, C.waves, C.pitch, C.lds, C.items,
                                        C.stream > 0 ? side.s[C.stream - 1] : st);
        }
        for (int q = 1; q < ns && r == hipSuccess; ++q) {
          r = hipEventRecord(side.join[q - 1], side.s[q - 1]);
          if (r == hipSuccess) r = hipStreamWaitEvent(st, side.join[q - 1], 0);
        }
        return r;
      };
      if (timing) {
        const int rc = timed(pass, st);
        if (rc) return rc;
      } else if ((e = pass()) != hipSuccess) {
        return hip_fail(e);
      }
    }
    for (int k = 0; k < count; ++k) {
      if (L.plan[k].tiled) continue;
      if ((e = launch_event_pass(geo[k], L.plan[k], inst[k].n, w[k], inst[k].rho, st)) != hipSuccess)
        return hip_fail(e);
    }
    if ((e = launch_update_batched(table, count, L.max_npix, st)) != hipSuccess) return hip_fail(e);
  }
  return JPET_OK;
}

// A batch, validated and carved, with its geometries; prepared (unless flagged as prepared) and set
// up for iterating on stream st.
static int batched_begin(const jpet_instance* inst, int32_t count, void* ws, size_t ws_bytes, uint32_t flags,
                         hipStream_t st, BatchLayout* L, std::vector<Workspace>* w, std::vector<Geo>* geo) {
  int rc = batched_carve(inst, count, ws, ws_bytes, L, w);
  if (rc) return rc;
  geo->resize(count);
  for (int k = 0; k < count; ++k) (*geo)[k] = make_geo(&inst[k].g, inst[k].g.sigma_z, inst[k].g.sigma_dl);
  if (!(flags & JPET_WS_PREPARED)) {
    for (int k = 0; k < count; ++k) {
      rc = do_prepare((*geo)[k], L->plan[k], inst[k].events, inst[k].n, (*w)[k], st);
      if (rc) return rc;
    }
  }
  // classes compiled alike share one kernel, whose LDS limit is their largest region
  for (size_t c = 0; c < L->cls.size(); ++c) {
    const BatchClass& C = L->cls[c];
    size_t lds = C.lds;
    for (const BatchClass& D : L->cls)
      if (D.maxlen == C.maxlen && D.waves == C.waves && D.pitch == C.pitch && D.lds > lds) lds = D.lds;
    const hipError_t e = set_batched_lds(C.maxlen, C.waves, C.pitch, lds);
    if (e != hipSuccess) return hip_fail(e);
  }
  std::vector<int64_t> item_begin;
  if ((rc = batched_items(count, L, *w, st, &item_begin))) return rc;
  if (L->streams > 1) {
    SideStream side;
    if ((rc = side_stream(&side))) return rc;
  }
  return batched_setup(inst, count, *L, *w, *geo, item_begin, ws, st);
}

struct jpet_batched_graph {
  hipGraphExec_t exec = nullptr;
  int device = 0;
  int32_t n_iter = 0;
};

extern "C" {

int jpet_mlem_batched_iterate(const jpet_instance* inst, int32_t count, int32_t n_iter, void* ws, size_t ws_bytes,
                              uint32_t flags, jpet_stats* stats, void* stream) {
  if (n_iter < 0 || (flags & ~JPET_WS_PREPARED)) return JPET_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  BatchLayout L;
  std::vector<Workspace> w;
  std::vector<Geo> geo;
  int rc = batched_begin(inst, count, ws, ws_bytes, flags, st, &L, &w, &geo);
  if (rc) return rc;
  rc = batched_iterations(inst, count, n_iter, L, w, geo, ws, true, st);
  if (rc) return rc;
  if (stats) {
    for (int k = 0; k < count; ++k) {
      rc = read_stats(w[k], inst[k].n, &stats[k], st);
      if (rc) return rc;
    }
  }
  return JPET_OK;
}

int jpet_mlem_batched_graph_create(const jpet_instance* inst, int32_t count, int32_t n_iter, void* ws,
                                   size_t ws_bytes, uint32_t flags, void* stream, jpet_batched_graph** out) {
  if (!out || n_iter < 1 || (flags & ~JPET_WS_PREPARED)) return JPET_EINVAL;
  *out = nullptr;
  hipStream_t st = (hipStream_t)stream;
  BatchLayout L;
  std::vector<Workspace> w;
  std::vector<Geo> geo;
  int rc = batched_begin(inst, count, ws, ws_bytes, flags, st, &L, &w, &geo);
  if (rc) return rc;
  // capture the iterations on a stream of the library's own, at the default priority
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e);
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = batched_iterations(inst, count, n_iter, L, w, geo, ws, false, cs);
    e = hipStreamEndCapture(cs, &graph);
  }
  (void)hipStreamDestroy(cs);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e);
  jpet_batched_graph* gr = new (std::nothrow) jpet_batched_graph;
  if (!gr) {
    (void)hipGraphExecDestroy(exec);
    return JPET_EINVAL;
  }
  gr->exec = exec;
  gr->n_iter = n_iter;
  (void)hipGetDevice(&gr->device);
  *out = gr;
  return JPET_OK;
}

int jpet_mlem_batched_graph_launch(jpet_batched_graph* gr, void* stream) {
  if (!gr || !gr->exec) return JPET_EINVAL;
  const hipError_t e = hipGraphLaunch(gr->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

int jpet_mlem_batched_graph_destroy(jpet_batched_graph* gr) {
  if (!gr) return JPET_OK;
  hipError_t e = hipSuccess;
  if (gr->exec) e = hipGraphExecDestroy(gr->exec);
  delete gr;
  if (e != hipSuccess) return hip_fail(e);
  return JPET_OK;
}

}  // extern "C"
