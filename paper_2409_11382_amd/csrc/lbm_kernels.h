// Kernel argument blocks and launcher declarations of the Biot LBM (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace biot {

enum SweepMode : int { kSmooth = 0, kRestrict = 1, kApply = 2 };

// Population planes: value (q, x, y) at q * plane + y * pitch + x.
template <typename T, typename Tc> struct SweepArgs {
  const T* g;          // input populations (ignored when zero_g)
  T* out;              // smoothing / apply destination
  const T* r;          // coarse right-hand side, or null (finest level)
  const T* Ft;         // explicit force planes (finest level), or null
  const Tc* e;         // coarse correction to prolongate into g first, or null
  Tc* rc;              // restriction output (coarse right-hand side)
  const T* eref;       // displacement reference planes (shifted storage), or null
  double* partials;    // per-wave sums of rho^2 and g^2, or null
  int nx, ny, pitch;
  int64_t plane;
  int cpitch;
  int64_t cplane;
  int el[4];           // elastic side types
  const double* bc[4]; // per side: 8 additive terms per boundary cell, or null
  ElConst<T> k;
  int H;               // rows per wave strip
  int zero_g;          // input populations are all zero
};

template <typename T> struct FlowArgs {
  T* fbuf[2];               // population buffers (9 planes each), ping-pong by step
  const T* g;               // elastic populations (finest level) for D^n
  double* Dbuf[3];          // divergence fields D^n, rotated by step
  const int* phase;         // step counter on the device
  double* p_out;            // lattice pressure p' of this step
  const double* src;        // dt * s, or null
  const double* omf;        // per-cell relaxation rate, or null (uniform omf_u)
  double omf_u;
  double alpha_h;           // alpha / h
  double r;                 // coupling ratio
  double kD;                // D = kD m_s
  T* pref;                  // pressure reference (shifted storage), or null
  int nx, ny, pitch;
  int64_t plane;
  const int8_t* ftype[4];   // per side: flow type per boundary cell
  const double* bc[4];      // per side: 9 additive terms per boundary cell
  int H;
};

template <typename T> struct ForceArgs {
  T* fbuf[2];
  double* Dbuf[3];
  const int* phase;
  const double* fbody;      // h^2 c0 f, 2 planes (lattice units), or null
  const double* src;        // dt * s, or null
  const double* omf;
  double omf_u;
  double alpha, alpha_h, h, r;
  T* Ft;
  int nx, ny, pitch;
  int64_t plane;
  int perx, pery;
};

template <typename T> struct InitArgs {
  T* fbuf[2];
  T* g;
  double* Dbuf[3];
  int* phase;
  const double* fbody;
  const double* src;
  T* eref;
  T* pref;
  double* p_out;
  int nx, ny, pitch;
  int64_t plane;
};

template <typename T> struct RebaseArgs {
  T* fbuf[2];
  const int* phase;
  T* g;
  T* eref;
  T* pref;
  int nx, ny, pitch;
  int64_t plane;
};

template <typename T> struct ExtractArgs {
  const T* g;
  const T* Ft;
  const T* eref;
  double kD, cstar, b_s, b_d, inv_c0h;
  double* eta;     // 2 planes (dense nx*ny)
  double* sigma;   // 3 planes (dense)
  int nx, ny, pitch;
  int64_t plane;
  int perx, pery;
};

template <typename T, typename Tc, int MODE, bool SHIFT>
hipError_t launch_sweep(const SweepArgs<T, Tc>& a, hipStream_t s);
int sweep_waves(int nx, int ny, int H);

template <typename T, bool SHIFT>
hipError_t launch_flow(const FlowArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_force(const ForceArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_init(const InitArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_rebase(const RebaseArgs<T>& a, hipStream_t s);
template <typename T, bool SHIFT>
hipError_t launch_extract(const ExtractArgs<T>& a, hipStream_t s);

hipError_t launch_finalize(const double* partials, int n, double* out2, int* flags, hipStream_t s);
hipError_t launch_advance(int* phase, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s);

}  // namespace biot
