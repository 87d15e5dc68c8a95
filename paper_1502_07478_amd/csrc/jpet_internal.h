// Internal declarations shared by the C-ABI layer and the gfx950 kernels of libjpet.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jpet.h"

namespace jpet {

// Geometry constants in the form the kernels use (host-computed, passed by value).
struct Geo {
  double R, L, sigma_z, sigma_dl, pixel, ipix;
  double u, w;         // sigma_z^-2, sigma_dl^-2 (diagonal of C^-1, Eq. 12) used by the kernel
  double um, wm;       // the same for the 3-sigma ellipse mask (equal to u, w except for gradients)
  double fa;           // factor of the third component of a (Eq. 9): 1 as printed, 2 exact
  double y0, z0;       // centre of pixel (0, 0)
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
  int32_t r0;    // first pixel row of the 3-sigma ellipse (App. B), clipped to the grid
  int32_t r1;    // last row; r1 < r0 marks an invalid (dropped) event
  int32_t npix;  // pixel centres inside the ellipse
  int32_t index; // position of the event in the caller's array
};

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
  int ntb, nty, ntz;    // bins along t, y, z
  int nbins;
  double tmin, dt;      // t bin b spans [tmin + b dt, tmin + (b+1) dt); ntb == 1: no shear
  int maxlen;           // register cache length (16/32/48/64) >= longest ellipse row
  int waves;            // wavefronts per workgroup
  int ev_per_batch;     // events whose rows are processed together (rows <= 64 * waves)
  int ev_per_wg;        // events per workgroup item (a multiple of ev_per_batch)
  int64_t max_items;    // upper bound of workgroup items (the launch grid)
  size_t lds_bytes;     // dynamic LDS of the tiled pass
};

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
  int32_t pad;
};

// Workspace carve-up.
struct Workspace {
  EventRec* ev;               // [n] records in input order
  EventRec* evs;              // [n] records sorted by bin
  uint32_t* key;              // [n] bin of each event (0xffffffff: dropped)
  uint32_t* bin_count;        // [nbins]
  uint32_t* bin_start;        // [nbins + 1]
  uint32_t* bin_fill;         // [nbins]
  uint32_t* item_start;       // [nbins + 1]
  BinItem* items;             // [max_items]
  unsigned long long* acc;    // [npix] back-projection accumulator, units of 2^-32
  double* B;                  // [npix] sum_j P_jl / D_j (log-likelihood gradient)
  double* red;                // [RED_SLOTS] double partial sums
  unsigned long long* cnt;    // [C_COUNT]
  size_t bytes;
};

constexpr int RED_SLOTS = 4096;
constexpr uint32_t kNoBin = 0xffffffffu;

Plan make_plan(const jpet_geometry* g, double mask_sz, double mask_sdl, int64_t n);
size_t workspace_layout(const Plan& p, int64_t n, int64_t npix, void* base, Workspace* out);

// Kernel launchers (return the hipError_t of the launch).
hipError_t launch_sensitivity(const Geo& g, float* s, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st);
hipError_t launch_prepare(const Geo& g, const Plan& p, const float* events, int64_t n, const Workspace& ws,
                          hipStream_t st);
hipError_t launch_event_pass(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                             hipStream_t st);
hipError_t launch_update(const Geo& g, const float* s, float* rho, const Workspace& ws, hipStream_t st);
hipError_t launch_loglik(const Geo& g, int64_t n, const Workspace& ws, const float* rho, const float* s,
                         float* D_out, float* grad_rho, double* out3, hipStream_t st);

}  // namespace jpet
