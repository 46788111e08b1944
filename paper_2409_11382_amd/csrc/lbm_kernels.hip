// HIP kernels of the coupled Biot LBM for gfx950 (CDNA4, 64-wide wavefronts).
//
// The per-level elastic sweep is a "column march": one wavefront owns 64
// adjacent columns (60 output columns plus two halo columns on each side) and
// walks up a strip of H rows.  Rows are kept in small register rings:
//   L(j): populations of row j and D(g) there (D feeds the self-force),
//   C(j): post-collision populations of row j, with the x-neighbour values that
//         the pull-stream needs exchanged between lanes by shuffles,
//   O(j): pull-stream, boundary rules and the mode's output for row j.
// Each population value is read from HBM once per sweep (plus a two-row halo
// per strip that neighbouring strips also read) and written once; no LDS is
// used.  Boundary data are precomputed per boundary cell and link on the host.
#include <hip/hip_runtime.h>

#include "lbm_kernels.h"

namespace biot {

// Direction tables as compile-time functions: every caller indexes them with
// an unrolled loop counter, so all population indices fold to constants and the
// register rings never spill to scratch.
// D2Q8 (order in lbm_device.h)
__device__ constexpr int cx8(int q) { return q == 0 || q == 4 || q == 7 ? 1 : (q == 2 || q == 5 || q == 6 ? -1 : 0); }
__device__ constexpr int cy8(int q) { return q == 1 || q == 4 || q == 5 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0); }
__device__ constexpr int opp8(int q) { return q < 4 ? (q + 2) % 4 : 4 + (q - 2) % 4; }
__device__ constexpr int mx8(int q) {  // (-cx, cy)
  return q == 0 ? 2 : q == 2 ? 0 : q == 4 ? 5 : q == 5 ? 4 : q == 6 ? 7 : q == 7 ? 6 : q;
}
// D2Q9 (order in lbm_device.h)
__device__ constexpr int cx9(int i) { return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0); }
__device__ constexpr int cy9(int i) { return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0); }
__device__ constexpr int opp9(int i) { return i == 0 ? 0 : (i < 5 ? 1 + (i + 1) % 4 : 5 + (i - 3) % 4); }
__device__ constexpr int mx9(int i) {
  return i == 1 ? 3 : i == 3 ? 1 : i == 5 ? 6 : i == 6 ? 5 : i == 7 ? 8 : i == 8 ? 7 : i;
}
__device__ constexpr double w9(int i) { return i == 0 ? 4.0 / 9 : (i < 5 ? 1.0 / 9 : 1.0 / 36); }

// ======================================================================
// elastic sweep
// ======================================================================
template <typename T> struct LRow {
  T g[8];
  T D, DL, DR;
};
template <typename T> struct CRow {
  T s[8];                    // own post-collision populations
  T sh0, sh2, sh4, sh5, sh6, sh7;  // pops 0,4,7 from lane-1; pops 2,5,6 from lane+1
  T ex, ey, exL, eyL, exR, eyR;    // displacement reference (shifted storage)
};

template <typename T, typename Tc, bool SHIFT>
__device__ __forceinline__ void sweep_load(const SweepArgs<T, Tc>& a, int j, int gx, bool col_ok, bool pery,
                                           LRow<T>& L) {
  const bool ok = col_ok && j >= -kHalo && j < a.ny + kHalo;
  if (ok) {
    const int gy = ghost_map(j, a.ny, pery);
    const int64_t idx = (int64_t)gy * a.pitch + gx;
    if (a.zero_g) {
#pragma unroll
      for (int q = 0; q < 8; ++q) L.g[q] = T(0);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) L.g[q] = a.g[q * a.plane + idx];
    }
    if (a.e) {
      const int64_t cidx = (int64_t)(gy >> 1) * a.cpitch + (gx >> 1);
#pragma unroll
      for (int q = 0; q < 8; ++q) L.g[q] += T(a.e[q * a.cplane + cidx]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) L.g[q] = T(0);
  }
  L.D = a.k.kD * el_ms(L.g);
  L.DL = from_left(L.D);
  L.DR = from_right(L.D);
}

template <typename T, typename Tc, bool SHIFT>
__device__ __forceinline__ void sweep_collide(const SweepArgs<T, Tc>& a, int j, int gx, bool col_ok, bool pery,
                                              const LRow<T>& Lm, const LRow<T>& L0, const LRow<T>& Lp,
                                              CRow<T>& C) {
  T v[3][3] = {{Lm.DL, Lm.D, Lm.DR}, {L0.DL, L0.D, L0.DR}, {Lp.DL, Lp.D, Lp.DR}};
  T Fx, Fy;
  grad_c(v, Fx, Fy);
  Fx *= a.k.cstar;
  Fy *= a.k.cstar;
  T u[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) u[q] = L0.g[q];
  const bool ok = col_ok && j >= -kHalo && j < a.ny + kHalo;
  T ex = T(0), ey = T(0);
  if (ok) {
    const int gy = ghost_map(j, a.ny, pery);
    const int64_t idx = (int64_t)gy * a.pitch + gx;
    if (a.Ft) {
      Fx += a.Ft[idx];
      Fy += a.Ft[a.plane + idx];
    }
    if (a.r) {
#pragma unroll
      for (int q = 0; q < 8; ++q) u[q] -= a.r[q * a.plane + idx];
    }
    if (SHIFT) {
      ex = a.eref[idx];
      ey = a.eref[a.plane + idx];
    }
  }
  el_collide(u, Fx, Fy, a.k, C.s);
  C.sh0 = from_left(C.s[0]);
  C.sh4 = from_left(C.s[4]);
  C.sh7 = from_left(C.s[7]);
  C.sh2 = from_right(C.s[2]);
  C.sh5 = from_right(C.s[5]);
  C.sh6 = from_right(C.s[6]);
  if (SHIFT) {
    C.ex = ex;
    C.ey = ey;
    C.exL = from_left(ex);
    C.eyL = from_left(ey);
    C.exR = from_right(ex);
    C.eyR = from_right(ey);
  }
}

// Population q arriving at a wall cell (x, y) whose source lies outside the
// domain (outx: across the left/right wall, outy: across the bottom/top wall).
// q is a compile-time constant at every call site.
template <typename T, typename Tc, bool SHIFT>
__device__ __forceinline__ T wall_pop(const SweepArgs<T, Tc>& a, const int q, bool outx, bool outy, int x, int y,
                                      const CRow<T>& Cm, const CRow<T>& C0, const CRow<T>& Cp) {
  const int cx = cx8(q), cy = cy8(q);
  const int elx = cx > 0 ? a.el[kLeft] : a.el[kRight];
  const int ely = cy > 0 ? a.el[kBottom] : a.el[kTop];
  const double* bcx = cx > 0 ? a.bc[kLeft] : a.bc[kRight];
  const double* bcy = cy > 0 ? a.bc[kBottom] : a.bc[kTop];
  bool usex;
  if (outx && outy) {
    const bool symx = elx == kElSymmetry, symy = ely == kElSymmetry;
    if (symx && symy) {  // corner between two mirrors: diagonal bounce-back
      T v = C0.s[opp8(q)];
      if (SHIFT) v -= T(2) * el_geq<T>(q, C0.ex, C0.ey);
      return v;
    }
    usex = symy;
  } else if (outx) {
    usex = true;
    if (elx == kElSymmetry) {  // mirror image: own column, row y - cy
      const int m = mx8(q);
      T v, sx, sy;
      if (cy > 0) { v = Cm.s[m]; sx = Cm.ex; sy = Cm.ey; }
      else if (cy < 0) { v = Cp.s[m]; sx = Cp.ex; sy = Cp.ey; }
      else { v = C0.s[m]; sx = C0.ex; sy = C0.ey; }
      if (SHIFT) v += el_geq<T>(m, sx, sy) - el_geq<T>(q, C0.ex, C0.ey);
      return v;
    }
  } else {
    usex = false;
    if (ely == kElSymmetry) {  // mirror image: column x - cx, own row
      T v, sx = C0.ex, sy = C0.ey;
      int m;
      if (q == 1) { v = C0.s[3]; m = 3; }
      else if (q == 3) { v = C0.s[1]; m = 1; }
      else if (q == 4) { v = C0.sh7; m = 7; sx = C0.exL; sy = C0.eyL; }
      else if (q == 7) { v = C0.sh4; m = 4; sx = C0.exL; sy = C0.eyL; }
      else if (q == 5) { v = C0.sh6; m = 6; sx = C0.exR; sy = C0.eyR; }
      else { v = C0.sh5; m = 5; sx = C0.exR; sy = C0.eyR; }
      if (SHIFT) v += el_geq<T>(m, sx, sy) - el_geq<T>(q, C0.ex, C0.ey);
      return v;
    }
  }
  // halfway rules at the cell itself
  const int type = usex ? elx : ely;
  const double* bc = usex ? bcx : bcy;
  const int idx = usex ? y : x;
  const T add = bc ? T(bc[8 * idx + q]) : T(0);
  const T o = C0.s[opp8(q)];
  if (type == kElDirichlet) {
    T v = o + add;
    if (SHIFT) v -= T(2) * el_geq<T>(q, C0.ex, C0.ey);
    return v;
  }
  return -o + add;  // traction
}

template <typename T, typename Tc, int MODE, bool SHIFT>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs<T, Tc> a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int ntx = (a.nx + kTileX - 1) / kTileX;
  const int nty = (a.ny + a.H - 1) / a.H;
  if (wid >= ntx * nty) return;  // whole wavefront
  const int tx = wid % ntx, ty = wid / ntx;
  const int x = tx * kTileX - kHalo + lane;
  const int y0 = ty * a.H;
  const int y1 = min(y0 + a.H, a.ny);
  const bool perx = a.el[kLeft] == kElPeriodic, pery = a.el[kBottom] == kElPeriodic;
  const bool col_ok = x >= -kHalo && x < a.nx + kHalo;
  const int gx = col_ok ? ghost_map(x, a.nx, perx) : 0;
  const bool out_lane = lane >= kHalo && lane < kWave - kHalo && x < a.nx;
  const bool wl = out_lane && x == 0 && !perx;
  const bool wr = out_lane && x == a.nx - 1 && !perx;
  const T gam = a.k.gamma, omg = T(1) - a.k.gamma;

  LRow<T> La, Lb, Lc;
  CRow<T> Cm, C0, Cp;
  sweep_load<T, Tc, SHIFT>(a, y0 - 2, gx, col_ok, pery, La);
  sweep_load<T, Tc, SHIFT>(a, y0 - 1, gx, col_ok, pery, Lb);
  sweep_load<T, Tc, SHIFT>(a, y0, gx, col_ok, pery, Lc);
  sweep_collide<T, Tc, SHIFT>(a, y0 - 1, gx, col_ok, pery, La, Lb, Lc, Cm);
  La = Lb;
  Lb = Lc;
  sweep_load<T, Tc, SHIFT>(a, y0 + 1, gx, col_ok, pery, Lc);
  sweep_collide<T, Tc, SHIFT>(a, y0, gx, col_ok, pery, La, Lb, Lc, C0);
  La = Lb;
  Lb = Lc;

  double acc_r = 0.0, acc_g = 0.0;
  T racc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) racc[q] = T(0);

  for (int y = y0; y < y1; ++y) {
    sweep_load<T, Tc, SHIFT>(a, y + 2, gx, col_ok, pery, Lc);
    sweep_collide<T, Tc, SHIFT>(a, y + 1, gx, col_ok, pery, La, Lb, Lc, Cp);

    // ---- pull-stream into row y
    T gin[8];
    gin[0] = C0.sh0;
    gin[2] = C0.sh2;
    gin[1] = Cm.s[1];
    gin[3] = Cp.s[3];
    gin[4] = Cm.sh4;
    gin[5] = Cm.sh5;
    gin[6] = Cp.sh6;
    gin[7] = Cp.sh7;
    if (SHIFT) {
      const T ex = C0.ex, ey = C0.ey;
      gin[0] += el_geq<T>(0, C0.exL - ex, C0.eyL - ey);
      gin[2] += el_geq<T>(2, C0.exR - ex, C0.eyR - ey);
      gin[1] += el_geq<T>(1, Cm.ex - ex, Cm.ey - ey);
      gin[3] += el_geq<T>(3, Cp.ex - ex, Cp.ey - ey);
      gin[4] += el_geq<T>(4, Cm.exL - ex, Cm.eyL - ey);
      gin[5] += el_geq<T>(5, Cm.exR - ex, Cm.eyR - ey);
      gin[6] += el_geq<T>(6, Cp.exR - ex, Cp.eyR - ey);
      gin[7] += el_geq<T>(7, Cp.exL - ex, Cp.eyL - ey);
    }
    const bool wb = out_lane && y == 0 && !pery;
    const bool wt = out_lane && y == a.ny - 1 && !pery;
    if (wl || wr || wb || wt) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int cx = cx8(q), cy = cy8(q);
        const bool ox = (cx > 0 && wl) || (cx < 0 && wr);
        const bool oy = (cy > 0 && wb) || (cy < 0 && wt);
        if (ox || oy) gin[q] = wall_pop<T, Tc, SHIFT>(a, q, ox, oy, x, y, Cm, C0, Cp);
      }
    }

    // ---- mode output
    const int64_t idx = (int64_t)y * a.pitch + x;
    if (a.partials && out_lane) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double rho = double(La.g[q]) - double(gin[q]);
        double gf = double(La.g[q]);
        if (SHIFT) gf += double(el_geq<T>(q, C0.ex, C0.ey));
        acc_r += rho * rho;
        acc_g += gf * gf;
      }
    }
    if (MODE == kSmooth) {
      if (out_lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a.out[q * a.plane + idx] = omg * La.g[q] + gam * gin[q];
      }
    } else if (MODE == kApply) {
      if (out_lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a.out[q * a.plane + idx] = gin[q];
      }
    } else {  // restriction: full sum over 2x2 blocks of rho = g - S(g)
      T rx[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const T rho = La.g[q] - gin[q];
        rx[q] = rho + from_right(rho);
      }
      if (((y - y0) & 1) == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) racc[q] = rx[q];
      } else if (out_lane && (x & 1) == 0) {
        const int64_t cidx = (int64_t)(y >> 1) * a.cpitch + (x >> 1);
#pragma unroll
        for (int q = 0; q < 8; ++q) a.rc[q * a.cplane + cidx] = Tc(racc[q] + rx[q]);
      }
    }

    La = Lb;
    Lb = Lc;
    Cm = C0;
    C0 = Cp;
  }
  if (a.partials) {
    acc_r = wave_sum(acc_r);
    acc_g = wave_sum(acc_g);
    if (lane == 0) {
      a.partials[2 * wid] = acc_r;
      a.partials[2 * wid + 1] = acc_g;
    }
  }
}

int sweep_waves(int nx, int ny, int H) {
  return ((nx + kTileX - 1) / kTileX) * ((ny + H - 1) / H);
}

template <typename T, typename Tc, int MODE, bool SHIFT>
hipError_t launch_sweep(const SweepArgs<T, Tc>& a, hipStream_t s) {
  const int waves = sweep_waves(a.nx, a.ny, a.H);
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((k_sweep<T, Tc, MODE, SHIFT>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ======================================================================
// flow step (SRT reaction-diffusion LBM with the centred source)
// ======================================================================
template <typename T> struct FRow {
  T s[9];
  T sh1, sh3, sh5, sh6, sh7, sh8;  // 1,5,8 from lane-1; 3,6,7 from lane+1
  T pr, prL, prR;                  // pressure reference (shifted storage)
};

template <typename T, bool SHIFT>
__device__ __forceinline__ void flow_collide(const FlowArgs<T>& a, int j, int x, int gx, bool col_ok, bool pery,
                                             bool write, const T* fin, const double* D1, const double* D2,
                                             double* Dn, FRow<T>& R) {
  const bool ok = col_ok && j >= -1 && j < a.ny + 1;
  T f[9];
  T s = T(0), om = T(a.omf_u), pr = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = T(0);
  if (ok) {
    const int gy = ghost_map(j, a.ny, pery);
    const int64_t idx = (int64_t)gy * a.pitch + gx;
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = fin[i * a.plane + idx];
    T gg[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) gg[q] = a.g[q * a.plane + idx];
    const double dn = a.kD * double(el_ms(gg));
    const double d1 = D1[idx], d2 = D2[idx];
    // centred coupling source (explicit part with ratio 1 - r, implicit with r)
    double sv = -a.alpha_h * ((1.0 - a.r) * (d1 - d2) + a.r * (dn - d1));
    if (a.src) sv += a.src[idx];
    s = T(sv);
    if (a.omf) om = T(a.omf[idx]);
    if (SHIFT) pr = a.pref[idx];
    if (write) {
      Dn[idx] = dn;
      T sum = T(0);
#pragma unroll
      for (int i = 0; i < 9; ++i) sum += f[i];
      a.p_out[idx] = double(sum) + 0.5 * sv + double(pr);
    }
  }
  T p = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) p += f[i];
  p += T(0.5) * s;
  const T so = (T(1) - T(0.5) * om) * s;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T w = T(w9(i));
    R.s[i] = f[i] - om * (f[i] - w * p) + w * so;
  }
  R.sh1 = from_left(R.s[1]);
  R.sh5 = from_left(R.s[5]);
  R.sh8 = from_left(R.s[8]);
  R.sh3 = from_right(R.s[3]);
  R.sh6 = from_right(R.s[6]);
  R.sh7 = from_right(R.s[7]);
  if (SHIFT) {
    R.pr = pr;
    R.prL = from_left(pr);
    R.prR = from_right(pr);
  }
}

template <typename T, bool SHIFT>
__device__ __forceinline__ T flow_wall_pop(const FlowArgs<T>& a, const int i, bool outx, bool outy, int x, int y,
                                           int tx_, int ty_, const FRow<T>& Fm, const FRow<T>& F0,
                                           const FRow<T>& Fp) {
  const int cx = cx9(i), cy = cy9(i);
  const double* bcx = cx > 0 ? a.bc[kLeft] : a.bc[kRight];
  const double* bcy = cy > 0 ? a.bc[kBottom] : a.bc[kTop];
  bool usex;
  if (outx && outy) {
    const bool symx = tx_ == kFlSymmetry, symy = ty_ == kFlSymmetry;
    if (symx && symy) return F0.s[opp9(i)];
    usex = symy;
  } else if (outx) {
    usex = true;
    if (tx_ == kFlSymmetry) {
      const int m = mx9(i);
      T v, ps;
      if (cy > 0) { v = Fm.s[m]; ps = Fm.pr; }
      else if (cy < 0) { v = Fp.s[m]; ps = Fp.pr; }
      else { v = F0.s[m]; ps = F0.pr; }
      if (SHIFT) v += T(w9(i)) * (ps - F0.pr);
      return v;
    }
  } else {
    usex = false;
    if (ty_ == kFlSymmetry) {
      T v, ps = F0.pr;
      if (i == 2) v = F0.s[4];
      else if (i == 4) v = F0.s[2];
      else if (i == 5) { v = F0.sh8; ps = F0.prL; }
      else if (i == 8) { v = F0.sh5; ps = F0.prL; }
      else if (i == 6) { v = F0.sh7; ps = F0.prR; }
      else { v = F0.sh6; ps = F0.prR; }  // 7
      if (SHIFT) v += T(w9(i)) * (ps - F0.pr);
      return v;
    }
  }
  const int type = usex ? tx_ : ty_;
  const T o = F0.s[opp9(i)];
  if (type == kFlNoflow) return o;
  const double* bc = usex ? bcx : bcy;
  const int idx = usex ? y : x;
  T v = -o + (bc ? T(bc[9 * idx + i]) : T(0));
  if (SHIFT) v -= T(2.0 * w9(i)) * F0.pr;
  return v;
}

template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_flow(FlowArgs<T> a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int ntx = (a.nx + kTileX - 1) / kTileX;
  const int nty = (a.ny + a.H - 1) / a.H;
  if (wid >= ntx * nty) return;
  const int tx = wid % ntx, ty = wid / ntx;
  const int x = tx * kTileX - kHalo + lane;
  const int y0 = ty * a.H;
  const int y1 = min(y0 + a.H, a.ny);
  const int n = *a.phase;
  const T* fin = a.fbuf[n & 1];
  T* fout = a.fbuf[(n + 1) & 1];
  const double* D1 = a.Dbuf[(n + 2) % 3];
  const double* D2 = a.Dbuf[(n + 1) % 3];
  double* Dn = a.Dbuf[n % 3];
  const bool perx = a.ftype[kLeft][0] == kFlPeriodic;
  const bool pery = a.ftype[kBottom][0] == kFlPeriodic;
  const bool col_ok = x >= -1 && x < a.nx + 1;
  const int gx = col_ok ? ghost_map(x, a.nx, perx) : 0;
  const bool out_lane = lane >= kHalo && lane < kWave - kHalo && x < a.nx;

  FRow<T> Fm, F0, Fp;
  flow_collide<T, SHIFT>(a, y0 - 1, x, gx, col_ok, pery, false, fin, D1, D2, Dn, Fm);
  flow_collide<T, SHIFT>(a, y0, x, gx, col_ok, pery, out_lane && y0 < y1, fin, D1, D2, Dn, F0);
  for (int y = y0; y < y1; ++y) {
    flow_collide<T, SHIFT>(a, y + 1, x, gx, col_ok, pery, out_lane && y + 1 < y1, fin, D1, D2, Dn, Fp);
    T fo[9];
    fo[0] = F0.s[0];
    fo[1] = F0.sh1;
    fo[3] = F0.sh3;
    fo[2] = Fm.s[2];
    fo[4] = Fp.s[4];
    fo[5] = Fm.sh5;
    fo[6] = Fm.sh6;
    fo[7] = Fp.sh7;
    fo[8] = Fp.sh8;
    if (SHIFT) {
      const T p0 = F0.pr;
      fo[1] += T(w9(1)) * (F0.prL - p0);
      fo[3] += T(w9(3)) * (F0.prR - p0);
      fo[2] += T(w9(2)) * (Fm.pr - p0);
      fo[4] += T(w9(4)) * (Fp.pr - p0);
      fo[5] += T(w9(5)) * (Fm.prL - p0);
      fo[6] += T(w9(6)) * (Fm.prR - p0);
      fo[7] += T(w9(7)) * (Fp.prR - p0);
      fo[8] += T(w9(8)) * (Fp.prL - p0);
    }
    if (out_lane) {
      const int tLy = a.ftype[kLeft][y], tRy = a.ftype[kRight][y];
      const int tBx = a.ftype[kBottom][x], tTx = a.ftype[kTop][x];
      const bool wl = x == 0 && tLy != kFlPeriodic;
      const bool wr = x == a.nx - 1 && tRy != kFlPeriodic;
      const bool wb = y == 0 && tBx != kFlPeriodic;
      const bool wt = y == a.ny - 1 && tTx != kFlPeriodic;
      if (wl || wr || wb || wt) {
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          const int cx = cx9(i), cy = cy9(i);
          const bool ox = (cx > 0 && wl) || (cx < 0 && wr);
          const bool oy = (cy > 0 && wb) || (cy < 0 && wt);
          if (ox || oy) {
            const int tx_ = cx > 0 ? tLy : tRy;
            const int ty_ = cy > 0 ? tBx : tTx;
            fo[i] = flow_wall_pop<T, SHIFT>(a, i, ox, oy, x, y, tx_, ty_, Fm, F0, Fp);
          }
        }
      }
      const int64_t idx = (int64_t)y * a.pitch + x;
#pragma unroll
      for (int i = 0; i < 9; ++i) fout[i * a.plane + idx] = fo[i];
    }
    Fm = F0;
    F0 = Fp;
  }
}

template <typename T, bool SHIFT>
hipError_t launch_flow(const FlowArgs<T>& a, hipStream_t s) {
  const int waves = sweep_waves(a.nx, a.ny, a.H);
  hipLaunchKernelGGL((k_flow<T, SHIFT>), dim3((waves + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ======================================================================
// explicit force of the step: Ft = h^2 c0 f - alpha h grad p, with the
// first-moment gradient and the explicit part of the centred source
// ======================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_force(ForceArgs<T> a) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= a.nx || y >= a.ny) return;
  const int n = *a.phase;
  const T* f = a.fbuf[n & 1];
  const double* D1 = a.Dbuf[(n + 2) % 3];
  const double* D2 = a.Dbuf[(n + 1) % 3];
  double st[3][3];
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int xs = ghost_map(x + dx, a.nx, a.perx), ys = ghost_map(y + dy, a.ny, a.pery);
      const int64_t k = (int64_t)ys * a.pitch + xs;
      const double d1 = D1[k], d2 = D2[k];
      double v = -a.alpha_h * ((1.0 - a.r) * (d1 - d2) - a.r * d1);
      if (a.src) v += a.src[k];
      st[dy + 1][dx + 1] = v;
    }
  double gx, gy;
  grad_c(st, gx, gy);
  const int64_t idx = (int64_t)y * a.pitch + x;
  double jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const double v = double(f[i * a.plane + idx]);
    jx += v * cx9(i);
    jy += v * cy9(i);
  }
  const double om = a.omf ? a.omf[idx] : a.omf_u;
  const double gpx = -3.0 * om * jx + 0.5 * gx;
  const double gpy = -3.0 * om * jy + 0.5 * gy;
  double Fx = -a.alpha * a.h * gpx, Fy = -a.alpha * a.h * gpy;
  if (a.fbody) {
    Fx += a.fbody[idx];
    Fy += a.fbody[a.plane + idx];
  }
  a.Ft[idx] = T(Fx);
  a.Ft[a.plane + idx] = T(Fy);
}

template <typename T>
hipError_t launch_force(const ForceArgs<T>& a, hipStream_t s) {
  dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4);
  hipLaunchKernelGGL((k_force<T>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ======================================================================
// initial conditions (eqs. ICs, ICs:moments with p = 0, eta = 0 at t = 0)
// ======================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_init(InitArgs<T> a) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x == 0 && y == 0 && blockIdx.x == 0 && blockIdx.y == 0) *a.phase = 0;
  if (x >= a.nx || y >= a.ny) return;
  const int64_t idx = (int64_t)y * a.pitch + x;
  const double s = a.src ? a.src[idx] : 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    a.fbuf[0][i * a.plane + idx] = T(-0.5 * w9(i) * s);
    a.fbuf[1][i * a.plane + idx] = T(0);
  }
  const double Fx = a.fbody ? a.fbody[idx] : 0.0, Fy = a.fbody ? a.fbody[a.plane + idx] : 0.0;
  // moments m10 = -F/2, m12 = -F/6 (x), m01 = -F/2, m21 = -F/6 (y); others 0
  const double A = -0.5 * Fx, B = -0.5 * Fy, P = -Fx / 6.0, Q = -Fy / 6.0;
  double g[8];
  g[0] = 0.5 * (A - P);
  g[2] = -0.5 * (A - P);
  g[1] = 0.5 * (B - Q);
  g[3] = -0.5 * (B - Q);
  g[4] = 0.25 * (P + Q);
  g[5] = 0.25 * (Q - P);
  g[6] = -0.25 * (P + Q);
  g[7] = 0.25 * (P - Q);
#pragma unroll
  for (int q = 0; q < 8; ++q) a.g[q * a.plane + idx] = T(g[q]);
  for (int k = 0; k < 3; ++k) a.Dbuf[k][idx] = 0.0;
  if (a.eref) {
    a.eref[idx] = T(0);
    a.eref[a.plane + idx] = T(0);
  }
  if (a.pref) a.pref[idx] = T(0);
  a.p_out[idx] = 0.0;
}

template <typename T>
hipError_t launch_init(const InitArgs<T>& a, hipStream_t s) {
  dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4);
  hipLaunchKernelGGL((k_init<T>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ======================================================================
// re-basing of the shifted storage: move the per-cell reference to the
// current displacement / pressure so the stored offsets stay small
// ======================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_rebase(RebaseArgs<T> a) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= a.nx || y >= a.ny) return;
  const int64_t idx = (int64_t)y * a.pitch + x;
  T u[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) u[q] = a.g[q * a.plane + idx];
  const T m10 = (u[0] - u[2]) + (u[4] - u[5]) + (u[7] - u[6]);
  const T m01 = (u[1] - u[3]) + (u[4] + u[5]) - (u[6] + u[7]);
#pragma unroll
  for (int q = 0; q < 8; ++q) a.g[q * a.plane + idx] = u[q] - el_geq<T>(q, m10, m01);
  a.eref[idx] += m10;
  a.eref[a.plane + idx] += m01;
  T* f = a.fbuf[(*a.phase) & 1];
  T fv[9];
  T p = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    fv[i] = f[i * a.plane + idx];
    p += fv[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i * a.plane + idx] = fv[i] - T(w9(i)) * p;
  a.pref[idx] += p;
}

template <typename T>
hipError_t launch_rebase(const RebaseArgs<T>& a, hipStream_t s) {
  dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4);
  hipLaunchKernelGGL((k_rebase<T>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ======================================================================
// displacement and stress of the current populations (eqs. displacement,
// moments:bared); stress in physical units
// ======================================================================
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_extract(ExtractArgs<T> a) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= a.nx || y >= a.ny) return;
  double D[3][3];
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int xs = ghost_map(x + dx, a.nx, a.perx), ys = ghost_map(y + dy, a.ny, a.pery);
      const int64_t k = (int64_t)ys * a.pitch + xs;
      T u[8];
      for (int q = 0; q < 8; ++q) u[q] = a.g[q * a.plane + k];
      D[dy + 1][dx + 1] = a.kD * double(el_ms(u));
    }
  double gx, gy;
  grad_c(D, gx, gy);
  const int64_t idx = (int64_t)y * a.pitch + x;
  double u[8];
  for (int q = 0; q < 8; ++q) u[q] = double(a.g[q * a.plane + idx]);
  const double Fx = double(a.Ft[idx]) + a.cstar * gx, Fy = double(a.Ft[a.plane + idx]) + a.cstar * gy;
  double m10 = (u[0] - u[2]) + (u[4] - u[5]) + (u[7] - u[6]);
  double m01 = (u[1] - u[3]) + (u[4] + u[5]) - (u[6] + u[7]);
  const double m11 = (u[4] - u[5]) + (u[6] - u[7]);
  const double ms = ((u[0] + u[2]) + (u[1] + u[3])) + 2.0 * ((u[4] + u[5]) + (u[6] + u[7]));
  const double md = (u[0] + u[2]) - (u[1] + u[3]);
  if (SHIFT) {
    m10 += double(a.eref[idx]);
    m01 += double(a.eref[a.plane + idx]);
  }
  const int64_t o = (int64_t)y * a.nx + x, N = (int64_t)a.nx * a.ny;
  a.eta[o] = m10 + 0.5 * Fx;
  a.eta[N + o] = m01 + 0.5 * Fy;
  const double bs = a.b_s * ms, bd = a.b_d * md, b11 = a.b_d * m11;
  a.sigma[o] = -0.5 * (bs + bd) * a.inv_c0h;
  a.sigma[N + o] = -b11 * a.inv_c0h;
  a.sigma[2 * N + o] = -0.5 * (bs - bd) * a.inv_c0h;
}

template <typename T, bool SHIFT>
hipError_t launch_extract(const ExtractArgs<T>& a, hipStream_t s) {
  dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4);
  hipLaunchKernelGGL((k_extract<T, SHIFT>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ======================================================================
// small utility kernels
// ======================================================================
__global__ __launch_bounds__(256) void k_finalize(const double* partials, int n, double* out2, int* flags) {
  __shared__ double sr[256], sg[256];
  double r = 0.0, g = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    r += partials[2 * k];
    g += partials[2 * k + 1];
  }
  sr[threadIdx.x] = r;
  sg[threadIdx.x] = g;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      sg[threadIdx.x] += sg[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = sr[0];
    out2[1] = sg[0];
    if (!isfinite(sr[0]) || !isfinite(sg[0])) flags[0] = 1;
  }
}

__global__ void k_advance(int* phase) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *phase += 1;
}

__global__ __launch_bounds__(256) void k_copy(uint4* dst, const uint4* src, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride) dst[k] = src[k];
}

__global__ __launch_bounds__(256) void k_zero(uint4* dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride) dst[k] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_finalize(const double* partials, int n, double* out2, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, n, out2, flags);
  return hipGetLastError();
}

hipError_t launch_advance(int* phase, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, phase);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  int blocks = (int)((n16 + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n16);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  int blocks = (int)((n16 + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (uint4*)dst, n16);
  return hipGetLastError();
}

// ---------------------------------------------------------- instantiations
#define BIOT_SWEEP(T, Tc)                                                                       \
  template hipError_t launch_sweep<T, Tc, kSmooth, false>(const SweepArgs<T, Tc>&, hipStream_t);   \
  template hipError_t launch_sweep<T, Tc, kRestrict, false>(const SweepArgs<T, Tc>&, hipStream_t); \
  template hipError_t launch_sweep<T, Tc, kApply, false>(const SweepArgs<T, Tc>&, hipStream_t);    \
  template hipError_t launch_sweep<T, Tc, kSmooth, true>(const SweepArgs<T, Tc>&, hipStream_t);    \
  template hipError_t launch_sweep<T, Tc, kRestrict, true>(const SweepArgs<T, Tc>&, hipStream_t);  \
  template hipError_t launch_sweep<T, Tc, kApply, true>(const SweepArgs<T, Tc>&, hipStream_t);
BIOT_SWEEP(float, float)
BIOT_SWEEP(float, double)
BIOT_SWEEP(double, double)
#undef BIOT_SWEEP

template hipError_t launch_flow<float, false>(const FlowArgs<float>&, hipStream_t);
template hipError_t launch_flow<float, true>(const FlowArgs<float>&, hipStream_t);
template hipError_t launch_flow<double, false>(const FlowArgs<double>&, hipStream_t);
template hipError_t launch_flow<double, true>(const FlowArgs<double>&, hipStream_t);
template hipError_t launch_force<float>(const ForceArgs<float>&, hipStream_t);
template hipError_t launch_force<double>(const ForceArgs<double>&, hipStream_t);
template hipError_t launch_init<float>(const InitArgs<float>&, hipStream_t);
template hipError_t launch_init<double>(const InitArgs<double>&, hipStream_t);
template hipError_t launch_rebase<float>(const RebaseArgs<float>&, hipStream_t);
template hipError_t launch_rebase<double>(const RebaseArgs<double>&, hipStream_t);
template hipError_t launch_extract<float, false>(const ExtractArgs<float>&, hipStream_t);
template hipError_t launch_extract<float, true>(const ExtractArgs<float>&, hipStream_t);
template hipError_t launch_extract<double, false>(const ExtractArgs<double>&, hipStream_t);
template hipError_t launch_extract<double, true>(const ExtractArgs<double>&, hipStream_t);

}  // namespace biot
