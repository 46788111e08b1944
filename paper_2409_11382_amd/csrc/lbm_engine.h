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
  int ref64;                  // references (eref, eref2, pref) in FP64, else FP32
  void* pref[2];              // pressure reference (shifted storage) or null: the populations
                              // f[n & 1] of step n are offsets from pref[n & 1]
  double* eta;                // extraction output (2 dense planes)
  double* sig;                // extraction output (3 dense planes)
  double* partials;           // per finest-level tile: sum rho^2, sum g^2
  double* partials2;          // the same per two-application tile
  double* norm2;              // finalized sums
  int* phase;                 // completed steps (device copy)
  int* flags;                 // [0] non-finite seen
  int* ad;                    // adaptive cycles: [0] stop (1 converged or at N_E,max, 2 non-finite), [1] cycles done
  double* ad_ratio;           // adaptive cycles: the last measured ||g - S(g)|| / ||g||
  double om_s, om_d, beta22, kD, cstar, gamma;
  double omf_u, alpha, alpha_h, h, r, b_s, b_d, inv_c0h;
  int ntiles_fine;            // sweep tiles of the finest level
  int grad_central;           // explicit force: central difference of p instead of first moments
  int ntiles_fine2;           // tiles of the finest level's last post-smoothing launch (multi-application)
  int ntiles_test;            // tiles of the finest level's first pre-smoothing launch (the adaptive test)
  uint32_t* ttab;             // coarse tail: per-cell gather tables of levels 1.. (8 words per cell)
  void* addt;                 // whole-problem tail: the finest level's wall terms, 8 planes
                              // in the population precision (or null)
  int csweeps;                // smoothing steps on the coarsest level of the hierarchy (2K
                              // unless set)
  void* dlag[2];              // Algorithm 1 with the lag: divergence of the previous
                              // pseudo-time step's iterate, two planes in the population
                              // precision (or null)
  double* gref;               // growth test: [0] the largest ||g||^2 of the finest level at
                              // the end of the first kGrowthWindow steps where it is non-zero,
                              // [1] how many of those steps have passed
};
// step-end norms that set the growth test's reference
constexpr double kGrowthWindow = 16.0;

struct SweepL {
  const ProbD* probs;
  const int2* tiles;
  int depth;
  int in_sel;     // 0: buffer A, 1: buffer B, 2: zero input
  int out_sel;    // 0: A, 1: B
  int prolong;    // add the coarse correction (coarser level's buffer A) to the input
  int partials;   // write norm partials (finest level): 1 of the last application's input,
                  // 2 (multi-application launches) of the first application's input
  const int* skip;  // when set and *skip != 0 the launch does nothing (adaptive cycles past their stop)
  const int* need;  // when set the launch runs only if *need == 1 (the adaptive step before it
                    // stopped normally: work enqueued ahead of the host's read of the test)
  int eref_in;    // shifted storage: the displacement reference is eref (0) or eref2 (1)
  int rebase_out; // re-base the output on its displacement and write the new
                  // reference to the other buffer (finest level, smoothing)
  int lag;        // lagged self-force (one-level problems, finest level, single
                  // applications): 0 none, 1 the step's first application (its own
                  // divergence, stored to dlag[0]), 2 the divergence of dlag[lag_rd],
                  // the input's stored to dlag[1 - lag_rd]
  int lag_rd;
};

struct CellL {    // per-cell kernels over the finest level
  const ProbD* probs;
  const int2* tiles;  // (problem, cell block)
  const int* skip;    // as in SweepL
  const int* need;    // as in SweepL
};

struct ProbL {    // one block per problem
  const ProbD* probs;
  const int* pids;
  const int* skip;  // as in SweepL
  const int* need;  // as in SweepL
  int fused;      // finalize: partials of a multi-application launch: 1 the last post-smoothing
                  // one (ntiles_fine2 tiles), 2 the first pre-smoothing one (ntiles_test)
  int advance;    // finalize: also count the completed step (after the flow step)
  int decide;     // finalize: then the adaptive stopping test (tol, ne_max)
  double tol;
  int ne_max;
  int* div;       // finalize: per problem index, set to 1 when the problem's state
                  // is non-finite or its norm grew above 1e8 times its first value
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
  const int* skip;  // as in SweepL
  const int* need;  // as in SweepL
  int depth;       // depth of the tail's top level (< 0: each entry's own, V-cycles from zero)
  int K;           // smoothing steps
  int shape;       // cycle shape of this visit of the top level: 0 V, 1 W, 2 F
  int from_zero;   // the top level's iterate starts at zero (else from its buffer A)
  int full;        // the whole problem from its finest level (depth 0), whose iterate
                   // is read from buffer fine_in (0 A, 1 B) and pre-smoothed fine_pre
                   // times; the cycle's result ends in A
  int fine_in, fine_pre;
  int loop;        // full: all adaptive cycles of the step, each after the first
                   // preceded by the measuring sweep and the stopping test
  int ne_max;      // loop: at most this many cycles
  double tol;      // loop: stop when ||g - S(g)|| <= tol ||g||
};
// deepest top level a cycle-shaped tail handles (levels 1..kTailMaxLevel)
constexpr int kTailMaxLevel = 15;

template <typename T, typename Tc, int MODE, bool SHIFT>
hipError_t launch_tsweep(const SweepL& a, int ntiles, hipStream_t s);
// Multi-application sweeps, by applications per launch A: 2 (a pair of
// smoothing applications), 3 (a pair, then the residual of its result
// restricted to the coarser level), 4 (four smoothing applications) and 5
// (four, then the restricted residual).  A region is COLS x (WAVES NK 64/COLS)
// cells with NK row indices per wave, each covering 64/COLS rows of COLS
// cells; a tile has (COLS - 4 A) x (rows - 4 A) outputs.  Each A has a
// default region and, chosen per depth by the cells it covers in all, an
// alternative (ALT):
// - pairs, with or without the restriction, take 64-cell rows.  By default 8
//   waves of 3 rows (FP32 without shifted storage: 4, whose LDS then still
//   fits two blocks; FP64: 2): two blocks share a CU and hide each other's
//   barrier waits, which is what bounds large grids.  ALT, for depths that
//   fill the chip about once: tall regions of 32 rows (16 waves x 2) and 36
//   rows (12 waves x 3), 24 output rows, one block per CU on a 512^2 level and
//   less halo work; FP64 shifted storage lacks the LDS and keeps 8 waves.
// - four applications are used only on depths of few cells, where the launch
//   is bound by the dependent work of one block: a 32 x 32 region (16 x 16
//   outputs) spreads such a depth over about four times as many compute units
//   as a 64-column one.  With the restriction (A = 5, halo 10) the narrow
//   region keeps only 12 x 12 outputs; ALT (64 x 32 region, 44 x 12 outputs)
//   serves the larger of those depths.
template <typename T, bool SHIFT, int A, bool ALT>
__host__ __device__ constexpr int sweepn_waves() {
  return A >= 4 ? 16 : ((!ALT || (sizeof(T) == 8 && SHIFT)) ? 8 : (A == 2 ? 16 : 12));
}
template <typename T, bool SHIFT, int A, bool ALT>
__host__ __device__ constexpr int sweepn_rows() {
  return A >= 4 ? ((A == 5 && ALT) ? 2 : 1)
                : ((sizeof(T) == 4 && !SHIFT && !ALT) ? 4
                                                      : (A == 3 ? 3 : ((ALT && !(sizeof(T) == 8 && SHIFT)) ? 2 : (sizeof(T) == 8 ? 2 : 3))));
}
template <int A, bool ALT>
__host__ __device__ constexpr int sweepn_cols() { return (A <= 3 || ALT) ? kWave : 32; }
template <typename T, bool SHIFT, int A, bool ALT>
__host__ __device__ constexpr int sweepn_region_rows() {
  return sweepn_waves<T, SHIFT, A, ALT>() * sweepn_rows<T, SHIFT, A, ALT>() * (kWave / sweepn_cols<A, ALT>());
}
inline int sweepn_tile_x(int A, bool alt) { return ((A <= 3 || alt) ? kWave : 32) - 4 * A; }
template <int A, bool ALT>
inline int sweepn_region_rows_rt(bool dbl, bool shift) {
  return dbl ? (shift ? sweepn_region_rows<double, true, A, ALT>() : sweepn_region_rows<double, false, A, ALT>())
             : (shift ? sweepn_region_rows<float, true, A, ALT>() : sweepn_region_rows<float, false, A, ALT>());
}
// output rows
inline int sweepn_tile_y(int A, bool dbl, bool shift, bool alt) {
  int rr = 0;
  switch (A) {
    case 2: rr = alt ? sweepn_region_rows_rt<2, true>(dbl, shift) : sweepn_region_rows_rt<2, false>(dbl, shift); break;
    case 3: rr = alt ? sweepn_region_rows_rt<3, true>(dbl, shift) : sweepn_region_rows_rt<3, false>(dbl, shift); break;
    case 4: rr = sweepn_region_rows_rt<4, false>(dbl, shift); break;
    default: rr = alt ? sweepn_region_rows_rt<5, true>(dbl, shift) : sweepn_region_rows_rt<5, false>(dbl, shift); break;
  }
  return rr - 4 * A;
}
// ALT: the alternative region of the applications per launch (not for four
// applications without the restriction); ref64: shifted FP32 storage where
// some problem of the launch keeps FP64 references (selects the kernel variant
// that reads either precision, per problem)
template <typename T, typename Tc, bool FINE, bool SHIFT, int APPS, bool RES, bool ALT = false>
hipError_t launch_tsweep2(const SweepL& a, int ntiles, bool ref64, hipStream_t s);
template <typename T, typename Tc, bool FINE, bool SHIFT, int APPS, bool RES, bool ALT = false>
inline hipError_t launch_tsweep2(const SweepL& a, int ntiles, hipStream_t s) {
  return launch_tsweep2<T, Tc, FINE, SHIFT, APPS, RES, ALT>(a, ntiles, false, s);
}
template <typename T, bool SHIFT>
hipError_t launch_tflow(const CellL& a, int ntiles, hipStream_t s);
template <typename T>
hipError_t launch_force(const CellL& a, int ntiles, hipStream_t s);
template <typename T>
hipError_t launch_init(const CellL& a, int ntiles, hipStream_t s);
template <typename T>
hipError_t launch_rebase(const CellL& a, int ntiles, hipStream_t s);
// the step-start displacement re-base and the step's explicit force (either
// pressure gradient), in one pass over the cells
template <typename T>
hipError_t launch_rebase_force(const CellL& a, int ntiles, hipStream_t s);
template <typename T, bool SHIFT>
hipError_t launch_extract(const CellL& a, int ntiles, hipStream_t s);

// levels >= 2 stored in FP64 (dbl) or FP32; level 1 is FP64 in both
hipError_t launch_tail(const TailL& a, int nprobs, bool dbl, hipStream_t s);
// gather tables of one coarse-tail level (nx * ny <= kTailThreads) for the
// elastic side types el[4]
hipError_t launch_tail_tables(const int* el, int nx, int ny, uint32_t* out, hipStream_t s);
hipError_t launch_finalize(const ProbL& a, int nprobs, hipStream_t s);
// adaptive cycles on the device: reset the stop flag and count for a step
// (the stopping test itself follows the norms in k_finalize)
hipError_t launch_ad_reset(const ProbL& a, hipStream_t s);
hipError_t launch_advance(const ProbL& a, int nprobs, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s);

inline int sweep_tiles_x(int nx) { return (nx + kTileX - 1) / kTileX; }
inline int sweep_tiles(int nx, int ny) { return sweep_tiles_x(nx) * ((ny + kTileY - 1) / kTileY); }
inline int sweepn_tiles_x(int nx, int apps, bool alt) {
  return (nx + sweepn_tile_x(apps, alt) - 1) / sweepn_tile_x(apps, alt);
}
// shift: the level is the finest one of shifted storage
inline int sweepn_tiles(int nx, int ny, bool dbl, int apps, bool shift, bool alt) {
  const int ty = sweepn_tile_y(apps, dbl, shift, alt);
  return sweepn_tiles_x(nx, apps, alt) * ((ny + ty - 1) / ty);
}
inline int cell_blocks(int nx, int ny) { return ((nx + kCellBX - 1) / kCellBX) * ((ny + kCellBY - 1) / kCellBY); }

}  // namespace biot
