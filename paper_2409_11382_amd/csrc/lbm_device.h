// Device-side building blocks of the coupled Biot LBM for gfx950 (CDNA4).
//
// Velocity sets (Table 1 and Fig. 1 of Lunowa & Wohlmuth, arXiv:2409.11382):
//   D2Q8 (elasticity), population index q:
//     0:(1,0) 1:(0,1) 2:(-1,0) 3:(0,-1) 4:(1,1) 5:(-1,1) 6:(-1,-1) 7:(1,-1)
//   D2Q9 (flow), population index i:
//     0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
// All quantities are in lattice units (spacing, time step 1; c_s^2 = 1/3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace biot {

enum : int { kLeft = 0, kRight = 1, kBottom = 2, kTop = 3 };
enum : int { kElPeriodic = 0, kElDirichlet = 1, kElTraction = 2, kElSymmetry = 3 };
enum : int { kFlPeriodic = 0, kFlDirichlet = 1, kFlNoflow = 2, kFlSymmetry = 3 };

// Column tile of one wavefront: 64 lanes, two halo columns on each side.
constexpr int kWave = 64;
constexpr int kHalo = 2;
constexpr int kTileX = kWave - 2 * kHalo;   // 60 output columns per wave

// ---------------------------------------------------------------- lane shifts
// value held by lane (l - 1) / (l + 1); edge lanes receive their own value,
// which is never consumed (edge lanes are halo lanes).
template <typename T> __device__ __forceinline__ T from_left(T v);
template <typename T> __device__ __forceinline__ T from_right(T v);

template <> __device__ __forceinline__ float from_left<float>(float v) { return __shfl_up(v, 1, kWave); }
template <> __device__ __forceinline__ float from_right<float>(float v) { return __shfl_down(v, 1, kWave); }
template <> __device__ __forceinline__ double from_left<double>(double v) { return __shfl_up(v, 1, kWave); }
template <> __device__ __forceinline__ double from_right<double>(double v) { return __shfl_down(v, 1, kWave); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// periodic wrap or even reflection at a wall (ghost -k equals cell k-1)
__device__ __forceinline__ int ghost_map(int i, int n, bool periodic) {
  if (i >= 0 && i < n) return i;
  if (periodic) {
    int m = i % n;
    return m < 0 ? m + n : m;
  }
  return i < 0 ? -i - 1 : 2 * n - 1 - i;
}

// --------------------------------------------------------------- constants
template <typename T> struct ElConst {
  T om_s, om_d;      // relaxation rates of m_s and of m_d, m_11 (Table 2)
  T beta22;          // m*_22 = -beta22 m_s  (eq. moments:collision:22)
  T kD;              // D = kD m_s = -b_s m_s / (2 (lambda + mu))  (eqs. LBM:divergence, moments:bared)
  T cstar;           // self-dependence force F_* = cstar grad^c D
  T gamma;           // under-relaxation of the smoother
};

// ---------------------------------------------------------------- collision
// Post-collision populations from pre-collision u and the force F of this
// application (Algorithm 2: moments, two half forces, Table 2 relaxation,
// Table 3 back-transformation).  The moments 12, 21, f relax with rate 1, so
// only m10, m01, m11, m_s, m_d of u enter.  The result is multiplied by sc,
// which the back-transformation's coefficients absorb (a smoother that blends
// with weight gamma passes sc = gamma).
template <typename T>
__device__ __forceinline__ void el_collide(const T u[8], T Fx, T Fy, const ElConst<T>& c, T out[8],
                                           T sc = T(1)) {
  const T m10 = (u[0] - u[2]) + (u[4] - u[5]) + (u[7] - u[6]);
  const T m01 = (u[1] - u[3]) + (u[4] + u[5]) - (u[6] + u[7]);
  const T m11 = (u[4] - u[5]) + (u[6] - u[7]);
  const T ax = (u[0] + u[2]), ay = (u[1] + u[3]);
  const T ms = (ax + ay) + T(2) * ((u[4] + u[5]) + (u[6] + u[7]));
  const T md = ax - ay;
  const T hx = T(0.5) * Fx, hy = T(0.5) * Fy;
  const T A = (m10 + hx) + hx;            // m*10
  const T B = (m01 + hy) + hy;            // m*01
  const T P = (m10 + hx) * T(1.0 / 3.0);  // m*12 = bar m10 / 3
  const T Q = (m01 + hy) * T(1.0 / 3.0);  // m*21 = bar m01 / 3
  const T S = (T(1) - c.om_s) * ms;       // m*s
  const T Dd = (T(1) - c.om_d) * md;      // m*d
  const T X = (T(1) - c.om_d) * m11;      // m*11
  const T Z = -c.beta22 * ms;             // m*22
  const T h2 = sc * T(0.5), h4 = sc * T(0.25);
  const T a = h2 * (A - P), b = h2 * (B - Q);
  const T cc = h4 * S - h2 * Z, dd = h4 * Dd;
  out[0] = (cc + dd) + a;
  out[2] = (cc + dd) - a;
  out[1] = (cc - dd) + b;
  out[3] = (cc - dd) - b;
  const T e = h4 * Z, p = h4 * P, q = h4 * Q, x = h4 * X;
  out[4] = (e + x) + (p + q);
  out[5] = (e - x) + (q - p);
  out[6] = (e + x) - (p + q);
  out[7] = (e - x) + (p - q);
}

template <typename T>
__device__ __forceinline__ T el_ms(const T g[8]) {
  return ((g[0] + g[2]) + (g[1] + g[3])) + T(2) * ((g[4] + g[5]) + (g[6] + g[7]));
}

// rest equilibrium carrying displacement (ex, ey): 3 w_q c_q . eta
template <typename T>
__device__ __forceinline__ T el_geq(int q, T ex, T ey) {
  switch (q) {
    case 0: return ex * T(1.0 / 3.0);
    case 1: return ey * T(1.0 / 3.0);
    case 2: return -ex * T(1.0 / 3.0);
    case 3: return -ey * T(1.0 / 3.0);
    case 4: return (ex + ey) * T(1.0 / 12.0);
    case 5: return (ey - ex) * T(1.0 / 12.0);
    case 6: return -(ex + ey) * T(1.0 / 12.0);
    default: return (ex - ey) * T(1.0 / 12.0);
  }
}

// central gradient of eq. pressure:gradient:alternative on a 3x3 stencil
// v[row][col], row 0 = y-1, col 0 = x-1
template <typename T>
__device__ __forceinline__ void grad_c(const T v[3][3], T& gx, T& gy) {
  gx = T(1.0 / 3.0) * (v[1][2] - v[1][0]) + T(1.0 / 12.0) * ((v[2][2] - v[2][0]) + (v[0][2] - v[0][0]));
  gy = T(1.0 / 3.0) * (v[2][1] - v[0][1]) + T(1.0 / 12.0) * ((v[2][2] - v[0][2]) + (v[2][0] - v[0][0]));
}

}  // namespace biot
