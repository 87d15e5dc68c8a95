// Internal declarations shared by the C-ABI layer and the gfx950 kernels of libjpet.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "jpet.h"

namespace jpet {

// Geometry constants in the form the kernels use (host-computed, passed by value).
struct Geo {
  double R, L, sigma_z, sigma_dl, pixel, ipix;
  double u, w;         // sigma_z^-2, sigma_dl^-2 (diagonal of C^-1, Eq. 12) used by the kernel
  double um, wm;       // the same for the 3-sigma ellipse mask (equal to u, w except for gradients)
  double fa;           // factor of the third component of a (Eq. 9): 1 as printed, 2 exact
  double y0, z0;       // centre of pixel (0, 0)
  double gamma;        // off-diagonal element of C^-1 (Eq. 12)
  double cnorm;        // sqrt(det C^-1) / (2 pi), det C^-1 = u^2 w - 2 u gamma^2: P = cnorm P'
  double cu, cw;       // (d det / du) / (2 det) and (d det / dw) / (2 det): the prefactor's share
                       // of d log P / du and d log P / dw
  double zedge;        // relative rise of sigma_z at the strip ends (per-event sigma_z; 0: none)
  int32_t n_y, n_z;
};

// Per-event iteration-invariant record written by the prepare step.  The reconstructed
// quantities are kept in double precision so that the ellipse's pixel set is decided in the
// same precision as a per-pixel double-precision test.
struct EventRec {
  double t;      // tan(theta~)                      (Eq. 2)
  double c;      // 1 / cos(theta~) = sqrt(1 + t^2)
  double y;      // y~
  double z;      // z~
  double su;     // this event's u over the geometry's: (sigma_z / sigma_z(e))^2, 1 for a constant
                 // sigma_z
  int32_t r0;    // first pixel row of the 3-sigma ellipse (App. B), clipped to the grid
  int32_t r1;    // last row; r1 < r0 marks an invalid (dropped) event
  int32_t npix;  // pixel centres inside the ellipse
  int32_t index; // position of the event in the caller's array
};

// Per-event constants of the binned event pass (64 bytes), written at prepare time.  With Y the
// row's y, dy = Y - y~ and b1 = z - z~ - dy tan (Eq. 8-12):
//   kappa = aC^-1a + 2 oC^-1b = A1 (R^2 + Y^2) + A2 Y^2 + A3 Y dy + KB Y b1
//   gamma = bC^-1a           = G1 Y dy + GB Y b1
//   S q   = S bC^-1b         = S2u b1^2 + Q3s dy^2             (S = log2(e) / 2)
// with u this event's sigma_z^-2.
struct EvConst {
  float yr, zr;         // y~ and z~ relative to the centre of the bin region's pixel (0, 0)
  int32_t index;        // position of the event in the caller's array
  float S2u;            // S 2u
  float t;              // tan(theta~)
  float A1, A2, A3, KB; // 2u c^4, w fa^2 c^2 t^2, 4 w c^2 (1 + 2t^2), -4 u t c^2
  float G1, GB, Q3s;    // 2 fa w c^2 t, -2 u c^2, S 4 w c^2
  float GK, GG;          // gamma terms: kappa += GK (fa y + 2 dy), gamma^ += GG dy (-4 g R c^3 t, -4 g R c^3)
  int32_t pad[2];
};

static_assert(sizeof(EvConst) == 64, "EvConst is copied to LDS in 16-byte units");

// Per-event constants of the binned MLEM pass (80 bytes): every row constant of the kernel along
// a pixel row as a polynomial in r, the row's index in its bin's region (Eq. 7-12, with Y the row's
// y, dy = Y - y~ and b1 = z - z~ - dy tan, all linear in r):
//   b1 at the row's first pixel = pix c + BT r + B0                (c: the pixel's region column)
//   kappa  = KR(r) + KB(r) b1,      KR = K0 + K1 r + K2 r^2,  KB = KB0 + KB1 r
//   sqrt(S) gamma^ = GR(r) + GB(r) b1,  GR = S0 + S1 r + S2 r^2,  GB = GB0 + GB1 r
//   S q    = s2u b1^2 + Q(r),       Q = Q0 + Q1 r + Q2 r^2
// so that along the row, at its j-th pixel, kappa = kappa_0 + j KB pix, sqrt(S) gamma^ =
// gs_0 + j GB pix and S q = qa j^2 + QB b1 j + S q_0 (qa = s2u pix^2, QB = 2 s2u pix).  The
// coefficients are formed in double precision at prepare time and rounded once.
struct EvRow {
  float B0, BT;
  float K0, K1, K2, KB0, KB1;
  float S0, S1, S2, GB0, GB1;
  float Q0, Q1, Q2;
  float qa, QB, s2u;
  int32_t index;  // position of the event in the caller's array
  int32_t pad;
};

static_assert(sizeof(EvRow) == 80, "EvRow is copied to LDS in 16-byte units");

// Thread word of the binned pass: the pixel row a thread owns in a batch, relative to its bin's
// region: bits 0-7 first column (sheared, region-local), 8-16 row (region-local), 17-23 pixel
// count (0: idle thread), 24-28 event within the batch.
constexpr uint32_t kWordCol = 0, kWordRow = 8, kWordLen = 17, kWordEv = 24;

// A batch block: ev_per_batch per-event constants (EvRow for the MLEM pass, EvConst for the
// log-likelihood pass), then one thread word per thread of the workgroup, then two words per
// wavefront:
//   its longest row (pixels; bit kGuardBit set when a row of the wavefront may reach kappa <= 0 and
//   needs the per-pixel test);
//   its shortest non-empty row (bits 0-7) and, with bit kHalfBit set, the one event of each
//   half-wavefront's rows: lanes 0-31 in bits 8-12, lanes 32-63 in bits 16-20 (a half with no rows
//   names the other half's event).
constexpr int kBlockTailWords = 2;
constexpr uint32_t kGuardBit = 31;
constexpr uint32_t kHalfBit = 31, kHalfLo = 8, kHalfHi = 16;

// Spatial binning of events and launch shape of the tiled event pass.
//
// Events are binned by the pixel row of y~ (tiles of TY rows), by a column in a frame sheared
// along the bin's central slope t_c (tiles of TZ columns) and by tan(theta~) (bins of width
// dt).  In row r the sheared column of pixel k is k - off(r), off(r) = rint(t_c y_r / pixel).
// A bin's region -- its tile widened by HY rows and HZ columns on each side -- contains every
// pixel of every ellipse in the bin, so one workgroup holds the region's image and
// back-projection accumulators in LDS.
struct Plan {
  int tiled;            // 0: generic pass (one wavefront per event, global accumulation)
  int TY, TZ;           // tile core (rows, sheared columns)
  int HY, HZ;           // halo (rows, columns)
  int RY, W;            // region rows and width
  int pitch;            // LDS row pitch of a region column (RY rounded up to the bank count)
  int batch_bytes;      // stride of a batch block (see kBlockTailWords)
  int ntb, nty, ntz;    // bins along t, y, z
  int nbins;
  double tmin, dt;      // t bin b spans [tmin + b dt, tmin + (b+1) dt); ntb == 1: no shear
  int maxlen;           // register cache length (16/32/48/64): the longest row segment a thread holds
  int segs;             // row segments per ellipse row, at most (1, or 2: longer rows are split)
  int waves;            // wavefronts per workgroup
  int acc32;            // 1: 32-bit LDS accumulators in 2^-acc_shift units
  int acc_shift;        // 32 - bits of the largest item size (events): no 32-bit slot overflows
  int ev_per_batch;     // events whose rows are processed together (rows <= 64 * waves)
  int ev_per_wg;        // events per workgroup item (a multiple of ev_per_batch)
  int64_t max_items;    // upper bound of workgroup items (the launch grid)
  int64_t max_batches;  // upper bound of batch blocks
  size_t lds_bytes;     // dynamic LDS of the tiled pass
  int wgs;              // workgroups resident per CU the region was sized for
  int32_t code;         // plan code (see plan_code_* below): what jpet_geometry.plan names
  int invalid;          // 1: the requested code does not fit this geometry (JPET_EDOMAIN)
  int loglik;           // 1: a plan of the log-likelihood pass (EvConst blocks, 64-bit slots)
  int cbytes;           // per-event constants of one batch (bytes)
  // dynamic LDS of the tiled pass: the region's image and accumulators from 0, then at lds_ev
  // two buffers of cbytes (the current and the next batch's constants), then at lds_off one
  // int per region row (its sheared column shift)
  int lds_ev, lds_off;
};

// Bytes of the per-event constants of one event in a batch block.
inline int event_const_bytes(bool loglik) { return loglik ? (int)sizeof(EvConst) : (int)sizeof(EvRow); }

// Plan codes, the value of jpet_geometry.plan that names one plan: 0 lets the cost model choose;
// otherwise bits 0-1 are the kind (1: binned pass with 8-wavefront workgroups, 2: with 16, 3: the
// generic one-wavefront-per-event pass, all other bits 0), bit 2 selects 32-bit LDS
// accumulators, bits 3-5 the workgroups resident per CU (1-4) the LDS region is sized for,
// bits 6-8 the tan(theta~) bin width (index into kPlanDt), bits 9-11 the square tile (index
// into kPlanTile) and bits 12-13 the register cache: 0 the smallest that holds the longest row,
// 1 (2) rows split into segments of at most 16 (32) pixels.
constexpr int kPlanDtCount = 6, kPlanTileCount = 5;
constexpr double kPlanDt[kPlanDtCount] = {0.0, 0.4, 0.2, 0.1, 0.05, 0.025};
constexpr int kPlanTile[kPlanTileCount] = {32, 24, 16, 12, 8};
constexpr int32_t kPlanGeneric = 3;
inline int32_t plan_code(int waves, int acc32, int wgs, int dt_index, int tile_index, int cache) {
  return (waves == 16 ? 2 : 1) | (acc32 ? 4 : 0) | (wgs << 3) | (dt_index << 6) | (tile_index << 9) | (cache << 12);
}
// 1 when the code is well formed (not whether it fits a geometry)
inline bool plan_code_valid(int32_t c) {
  if (c == 0 || c == kPlanGeneric) return true;
  const int kind = c & 3, wgs = (c >> 3) & 7, dti = (c >> 6) & 7, ti = (c >> 9) & 7, cache = (c >> 12) & 3;
  return kind >= 1 && kind <= 2 && wgs >= 1 && wgs <= 4 && dti < kPlanDtCount && ti < kPlanTileCount && cache <= 2 &&
         (c >> 14) == 0;
}

// Counters kept in the workspace (unsigned 64-bit).
enum Counter {
  C_VALID = 0,
  C_DROPPED = 1,
  C_PAIRS = 2,
  C_ZERO_DEN = 3,
  C_KAPPA_BAD = 4,
  C_ITEMS = 5,       // workgroup items produced by the binning
  C_OUTSIDE = 6,     // ellipse rows that fell outside their bin's region (stays 0)
  C_COUNT = 8
};

struct BinItem {
  int32_t bin;
  int32_t start;  // first event in the sorted record array
  int32_t count;
  int32_t batch;  // first batch block of the item
};

// Workspace carve-up.
struct Workspace {
  EventRec* ev;               // [n] records in input order
  EventRec* evs;              // [n] records sorted by bin
  unsigned char* batches;     // [max_batches * batch_bytes] batch blocks of the binned pass
  uint32_t* key;              // [n] bin of each event (0xffffffff: dropped)
  uint32_t* bin_count;        // [nbins]
  uint32_t* bin_start;        // [nbins + 1]
  uint32_t* bin_fill;         // [nbins]
  uint32_t* item_start;       // [nbins + 1]
  uint32_t* batch_start;      // [nbins + 1] first batch block of each bin
  BinItem* items;             // [max_items]
  unsigned long long* acc;    // [npix] back-projection accumulator, units of 2^-32
  double* B;                  // [npix] sum_j P_jl / D_j (log-likelihood gradient)
  double* red;                // [RED_SLOTS] double partial sums
  unsigned long long* cnt;    // [C_COUNT]
  size_t bytes;
};

// One reconstruction of a batch, as the batched kernels read it from the workspace's instance
// table (sorted by item_begin).
struct BatchInst {
  Geo g;
  Plan p;
  int32_t tiled;              // 1: binned pass inside the batched launch; 0: generic pass, launched apart
  int32_t index;              // position in the caller's instance array
  int32_t cls;                // the batched launch (class) serving it, -1: none
  int32_t pad;
  int64_t item_begin;         // its first work index within its class (item 0 of the instance)
  int64_t n;                  // events
  const unsigned char* blocks;
  const BinItem* items;
  float* rho;                 // current image: read by the event pass, rewritten by the update
  const float* s;             // sensitivity or null
  unsigned long long* acc;
  unsigned long long* cnt;
};


constexpr int kInstPerWrite = 6;  // instances written per table-writing launch (by-value kernel argument)
struct InstWrite {
  BatchInst v[kInstPerWrite];
  int first, count;
};
static_assert(sizeof(InstWrite) <= 4096, "InstWrite is passed by value as a kernel argument");

constexpr int RED_SLOTS = 4096;
constexpr uint32_t kNoBin = 0xffffffffu;

// The plan of a pass: the one g->plan names, or with g->plan = 0 the cheapest candidate under the
// cost model.  loglik: plan for the log-likelihood pass (64-bit region slots for its doubles, its
// own register budget) instead of the MLEM pass.  A named plan that does not fit the geometry
// comes back with invalid = 1.
Plan make_plan(const jpet_geometry* g, double mask_sz, double mask_sdl, int64_t n, bool loglik = false);

// Every binned plan that fits the geometry, with its cost-model figure (lower is faster), sorted
// by that figure; the generic pass is listed last when no binned plan fits.
struct PlanCand {
  Plan p;
  double cost;
};
void plan_candidates(const jpet_geometry* g, double mask_sz, double mask_sdl, int64_t n, bool loglik,
                     std::vector<PlanCand>* out);
size_t workspace_layout(const Plan& p, int64_t n, int64_t npix, void* base, Workspace* out);

// Records e as this thread's last HIP error (jpet_last_hip_error) and returns JPET_EHIP.
int record_hip_failure(hipError_t e);

// Kernel launchers (return the hipError_t of the launch).
hipError_t launch_sensitivity(const Geo& g, float* s, hipStream_t st);
hipError_t launch_direct_image(const Geo& g, double L, const float* events, int64_t n, float* img, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st);
hipError_t launch_prepare(const Geo& g, const Plan& p, const float* events, int64_t n, const Workspace& ws,
                          hipStream_t st);
// Work split of the event pass: the plan's (binned when tiled), or for comparison one wavefront
// per event (the generic pass) or one thread per event.
constexpr int kPassPlanned = 0, kPassWavePerEvent = 1, kPassThreadPerEvent = 2;
// D_out (nullable): each event's denominator, with P's constant factor, at its input position
// (events that are dropped are not written).
hipError_t launch_event_pass(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                             hipStream_t st, int granularity = kPassPlanned, float* D_out = nullptr);
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t st);
hipError_t launch_update(const Geo& g, const float* s, float* rho, const Workspace& ws, hipStream_t st);
// batched: table of count instances in device memory; grid = total workgroups of the tiled ones
hipError_t launch_write_insts(const InstWrite& w, BatchInst* table, hipStream_t st);
hipError_t launch_batched_reset(const BatchInst* table, int count, hipStream_t st);
// the batched pass over one class of a batch (table: the class's entries): 32-bit accumulators,
// register cache maxlen (16, 32, 48 or 64), waves (8 or 16) wavefronts per workgroup, region row pitch
// (64, 128, 192, 256, or 0 for any other), one workgroup per item of the class (items in total)
hipError_t launch_event_pass_batched(const BatchInst* table, int count, int maxlen, int waves, int pitch,
                                     size_t lds_bytes, int64_t items, hipStream_t st);
// the pitch a batched class is compiled for: 64, 128, 192 or 256, else 0 (a runtime value)
inline int batched_pitch_class(int pitch) {
  return pitch == 64 || pitch == 128 || pitch == 192 || pitch == 256 ? pitch : 0;
}
// raises a batched pass's dynamic LDS limit (call before launching or capturing it)
hipError_t set_batched_lds(int maxlen, int waves, int pitch, size_t lds_bytes);
hipError_t launch_update_batched(const BatchInst* table, int count, int64_t max_npix, hipStream_t st);
// value_only: l alone (out3[1], out3[2] are NaN, grad_rho must be null)
hipError_t launch_loglik(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                         const float* s, float* D_out, float* grad_rho, double* out3, bool value_only,
                         hipStream_t st);
// the binned log-likelihood pass (B and red[0..2] zeroed by the caller); value_only: the per-event
// log D' sums alone
hipError_t launch_loglik_tiled(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                               float* D_out, bool value_only, hipStream_t st);

}  // namespace jpet
