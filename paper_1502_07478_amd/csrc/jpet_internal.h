// Internal declarations shared by the C-ABI layer and the gfx950 kernels of libjpet.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jpet.h"

namespace jpet {

// Geometry constants in the form the kernels use (host-computed, passed by value).
struct Geo {
  double R, L, sigma_z, sigma_dl, pixel;
  double u, w;         // sigma_z^-2, sigma_dl^-2 (diagonal of C^-1, Eq. 12) used by the kernel
  double um, wm;       // the same for the 3-sigma ellipse mask (equal to u, w except for gradients)
  double fa;           // factor of the third component of a (Eq. 9): 1 as printed, 2 exact
  double y0, z0;       // centre of pixel (0, 0)
  int32_t n_y, n_z;
};

// Per-event iteration-invariant record written by the prepare step.
// The reconstructed quantities are kept in double precision so that the ellipse's pixel set is
// decided in the same precision as a per-pixel double-precision test.
struct EventRec {
  double t;     // tan(theta~)                      (Eq. 2)
  double c;     // 1 / cos(theta~) = sqrt(1 + t^2)
  double y;     // y~
  double z;     // z~
  int32_t r0;   // first pixel row of the 3-sigma ellipse (App. B), clipped to the grid
  int32_t r1;   // last row; r1 < r0 marks an invalid (dropped) event
  int32_t npix; // pixel centres inside the ellipse
  int32_t pad;
};

// Counters kept in the workspace (unsigned 64-bit).
enum Counter {
  C_VALID = 0,
  C_DROPPED = 1,
  C_PAIRS = 2,
  C_ZERO_DEN = 3,
  C_KAPPA_BAD = 4,
  C_COUNT = 8
};

// Workspace carve-up for n events on a grid of npix pixels.
struct Workspace {
  EventRec* ev;              // [n]
  unsigned long long* cnt;   // [C_COUNT]
  float* acc;                // [npix] accumulator of rho_l P_jl / D_j
  double* red;               // [RED_SLOTS] double-precision partial sums (log-likelihood)
  size_t bytes;
};

constexpr int RED_SLOTS = 4096;

size_t workspace_layout(int64_t n, int64_t npix, void* base, Workspace* out);

// Kernel launchers (return the hipError_t of the launch).
hipError_t launch_sensitivity(const Geo& g, float* s, hipStream_t st);
hipError_t launch_prepare(const Geo& g, const float* events, int64_t n, const Workspace& ws, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int n, hipStream_t st);
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t st);
hipError_t launch_event_pass(const Geo& g, int64_t n, const Workspace& ws, const float* rho, hipStream_t st);
hipError_t launch_update(const Geo& g, const float* s, float* rho, const Workspace& ws, hipStream_t st);
hipError_t launch_loglik(const Geo& g, int64_t n, const Workspace& ws, const float* rho, const float* s,
                         float* D_out, float* grad_rho, double* out3, hipStream_t st);

}  // namespace jpet
