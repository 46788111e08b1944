// Device descriptors, launch blocks and launcher declarations of the batched
// Biot LBM engine (gfx950).
//
// Every launch works on a list of tiles drawn from one or many problems: a
// tile entry is (problem index, tile index within the level that the launch
// addresses).  Levels are aligned from the finest: "depth" d addresses level
// L_p - d of problem p, so problems with different hierarchy depths share the
// launches of their common depths (Algorithm 4 recursion aligned top-down).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace biot {

constexpr int kMaxLevels = 16;
constexpr int kTileY = 12;              // output rows of a sweep tile (even: 2x2 restriction pairs)
constexpr int kCellBX = 64, kCellBY = 4;  // per-cell kernels: 64 x 4 cells per block

enum SweepMode : int { kSmooth = 0, kRestrict = 1, kApply = 2 };

struct LevelD {
  void* gA;          // population buffer A (8 planes)
  void* gB;          // population buffer B
  void* r;           // coarse right-hand side (8 planes), null on the finest level
  int nx, ny, pitch;
  int tiles_x;       // sweep tiles along x: ceil(nx / kTileX)
  int tiles_xn[6];   // multi-application sweep tiles along x, by applications per launch (2..5)
  int dbl;           // FP64 storage
  int64_t plane;
};

// one problem as the kernels see it (device memory, read with scalar loads)
struct ProbD {
  LevelD lv[kMaxLevels + 1];  // 1..L, L is the finest
  int L;
  int el[4];                  // elastic side types
  const double* elbc[4];      // finest level: 8 additive terms per boundary cell (or null)
  const int8_t* ftype[4];     // flow type per boundary cell
  const double* flbc[4];      // 9 additive terms per boundary cell
  void* f[2];                 // flow populations, ping-pong by step parity
  double* D[3];               // D^n rotated by step number mod 3
  double* pout;               // lattice pressure of the last completed step
  const double* fbody;        // h^2 c0 f (2 planes) or null
  const double* src;          // dt s or null
  const double* omf;          // per-cell flow relaxation rate or null
  void* Ft;                   // explicit force (2 planes)
  void* eref;                 // displacement reference (shifted storage) or null
  void* eref2;                // its second buffer, written by a re-basing sweep
  void* pref;                 // pressure reference (shifted storage) or null
  double* eta;                // extraction output (2 dense planes)
  double* sig;                // extraction output (3 dense planes)
  double* partials;           // per finest-level tile: sum rho^2, sum g^2
  double* partials2;          // the same per two-application tile
  double* norm2;              // finalized sums
  int* phase;                 // completed steps (device copy)
  int* flags;                 // [0] non-finite seen
  double om_s, om_d, beta22, kD, cstar, gamma;
  double omf_u, alpha, alpha_h, h, r, b_s, b_d, inv_c0h;
  int ntiles_fine;            // sweep tiles of the finest level
  int grad_central;           // explicit force: central difference of p instead of first moments
  int ntiles_fine2;           // two-application sweep tiles of the finest level
  uint32_t* ttab;             // coarse tail: per-cell gather tables of levels 1.. (8 words per cell)
};

struct SweepL {
  const ProbD* probs;
  const int2* tiles;
  int depth;
  int in_sel;     // 0: buffer A, 1: buffer B, 2: zero input
  int out_sel;    // 0: A, 1: B
  int prolong;    // add the coarse correction (coarser level's buffer A) to the input
  int partials;   // write norm partials (finest level)
  int eref_in;    // shifted storage: the displacement reference is eref (0) or eref2 (1)
  int rebase_out; // re-base the output on its displacement and write the new
                  // reference to the other buffer (finest level, smoothing)
};

struct CellL {    // per-cell kernels over the finest level
  const ProbD* probs;
  const int2* tiles;  // (problem, cell block)
};

struct ProbL {    // one block per problem
  const ProbD* probs;
  const int* pids;
  int fused;      // finalize: partials of the two-application sweep
};

// Coarse "tail" of the multigrid recursion: one 1024-thread workgroup per
// problem runs Algorithm 4 for every level from L - depth down to 1, with the
// level's collision results in LDS and only workgroup barriers between sweeps.
// One cell per thread: a level of more cells keeps one CU's SIMDs busy for
// longer than the tile kernels take to sweep it across many CUs.
constexpr int kTailThreads = 1024;
constexpr int kTailCellsF32 = 1024;   // largest tail level (cells) in FP32 storage
constexpr int kTailCellsF64 = 1024;   // and in FP64 storage
constexpr int kTailLdsBytes = 9 * kTailCellsF64 * 8;
struct TailL {
  const ProbD* probs;
  const int* pids;
  int depth;       // depth of the tail's top level
  int K;           // smoothing steps
};

template <typename T, typename Tc, int MODE, bool SHIFT>
hipError_t launch_tsweep(const SweepL& a, int ntiles, hipStream_t s);
// Multi-application sweeps, by applications per launch A: 2 (a pair of
// smoothing applications), 3 (a pair, then the residual of its result
// restricted to the coarser level), 4 (four smoothing applications) and 5
// (four, then the restricted residual).  A region is COLS x (WAVES NK 64/COLS)
// cells with NK row indices per wave, each covering 64/COLS rows of COLS
// cells; a tile has (COLS - 4 A) x (rows - 4 A) outputs.  Pairs take 64-cell
// rows.  Four applications are used only on depths of few cells, where the
// launch is bound by the dependent work of one block rather than by HBM: a
// 32 x 32 region (16 x 16 outputs) spreads such a depth over about four times
// as many compute units as a 64-column one, at twice its redundant halo work.
// With the restriction (A = 5, halo 10) a 32 x 32 region keeps only 12 x 12
// outputs; the WIDE form (64 x 32 region, 44 x 12 outputs) serves the larger
// of the depths that take four applications.
template <int A>
__host__ __device__ constexpr int sweepn_waves() { return A <= 3 ? 8 : 16; }
template <typename T, int A>
__host__ __device__ constexpr int sweepn_rows() {
  return A == 2 ? (sizeof(T) == 8 ? 2 : 3) : (A == 3 ? 3 : 1);
}
template <int A>
__host__ __device__ constexpr int sweepn_cols() { return A <= 3 ? kWave : 32; }
inline int sweepn_tile_x(int A, bool wide = false) {
  return ((A <= 3 || wide) ? sweepn_cols<2>() : sweepn_cols<4>()) - 4 * A;
}
inline int sweepn_tile_y(int A, bool dbl) {
  int rr = 0;
  switch (A) {
    case 2: rr = sweepn_waves<2>() * (dbl ? sweepn_rows<double, 2>() : sweepn_rows<float, 2>()); break;
    case 3: rr = sweepn_waves<3>() * sweepn_rows<float, 3>(); break;
    case 4: rr = sweepn_waves<4>() * sweepn_rows<float, 4>() * (kWave / sweepn_cols<4>()); break;
    default: rr = sweepn_waves<5>() * sweepn_rows<float, 5>() * (kWave / sweepn_cols<5>()); break;
  }
  return rr - 4 * A;
}
// WIDE (APPS = 4 with RES only): 64-column regions of 16 waves x 2 rows
template <typename T, typename Tc, bool FINE, bool SHIFT, int APPS, bool RES, bool WIDE = false>
hipError_t launch_tsweep2(const SweepL& a, int ntiles, hipStream_t s);
template <typename T, bool SHIFT>
hipError_t launch_tflow(const CellL& a, int ntiles, hipStream_t s);
template <typename T>
hipError_t launch_force(const CellL& a, int ntiles, hipStream_t s);
template <typename T>
hipError_t launch_init(const CellL& a, int ntiles, hipStream_t s);
template <typename T>
hipError_t launch_rebase(const CellL& a, int ntiles, bool flow, hipStream_t s);
template <typename T, bool SHIFT>
hipError_t launch_extract(const CellL& a, int ntiles, hipStream_t s);

// levels >= 2 stored in FP64 (dbl) or FP32; level 1 is FP64 in both
hipError_t launch_tail(const TailL& a, int nprobs, bool dbl, hipStream_t s);
// gather tables of one coarse-tail level (nx * ny <= kTailThreads) for the
// elastic side types el[4]
hipError_t launch_tail_tables(const int* el, int nx, int ny, uint32_t* out, hipStream_t s);
hipError_t launch_finalize(const ProbL& a, int nprobs, hipStream_t s);
hipError_t launch_advance(const ProbL& a, int nprobs, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s);

inline int sweep_tiles_x(int nx) { return (nx + kTileX - 1) / kTileX; }
inline int sweep_tiles(int nx, int ny) { return sweep_tiles_x(nx) * ((ny + kTileY - 1) / kTileY); }
inline int sweepn_tiles_x(int nx, int apps, bool wide = false) {
  return (nx + sweepn_tile_x(apps, wide) - 1) / sweepn_tile_x(apps, wide);
}
// the row count of a WIDE region equals the narrow one's: 16 x 2 = 16 x 1 x 2
inline int sweepn_tiles(int nx, int ny, bool dbl, int apps, bool wide = false) {
  const int ty = sweepn_tile_y(apps, dbl);
  return sweepn_tiles_x(nx, apps, wide) * ((ny + ty - 1) / ty);
}
inline int cell_blocks(int nx, int ny) { return ((nx + kCellBX - 1) / kCellBX) * ((ny + kCellBY - 1) / kCellBY); }

}  // namespace biot
