// lattice.hpp -- lattice tables and per-node physics of the two-level LBM
// hot path (device side, gfx950).
//
// Everything here is written for unrolled loops over the populations: the
// velocity components are constexpr functions of the population index, so
// after unrolling every Hermite polynomial value folds into an immediate.
//
// Populations are handled in "stored form": s_i = f_i - DEV * w_i.  With
// DEV = 0 the stored value is the population itself (FP64 path); with DEV = 1
// it is the deviation from the rest state (FP32 deviation path), which keeps
// the single-precision significand for the O(Ma) part of f.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace lbm {

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1.
template <int N, int I = 0, typename F>
__host__ __device__ inline void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, I + 1>(f);
  }
}

// ---------------------------------------------------------------------------
// Lattices.  D2Q9 in the order of Sec. 3.1 (eq xi_i, eq w_i).  D3Q19 is the
// standard 19-velocity lattice: rest, +-x, +-y, +-z, then (+-1,+-1,0),
// (+-1,0,+-1), (0,+-1,+-1) in the order (1,1), (-1,-1), (1,-1), (-1,1).
template <int LAT>
struct Lattice;

template <>
struct Lattice<0> {
  static constexpr int D = 2, Q = 9;
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <>
struct Lattice<1> {
  static constexpr int D = 3, Q = 19;
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
           : ((i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
           : ((i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
           : ((i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0);
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// Number of independent strain-rate components kept: xx, yy, xy (2D) or
// xx, yy, zz, xy, xz, yz (3D).
template <int D>
struct NS {
  static constexpr int value = D == 2 ? 3 : 6;
};

// Symmetric second-order tensor, components xx, yy, zz, xy, xz, yz.
template <typename T>
struct Sym {
  T xx, yy, zz, xy, xz, yz;
};

// Third-order Hermite polynomial H_abc(xi) - the c_s^2 = 1/3 terms - for the
// mixed components the lattices use: H_aab = xi_a^2 xi_b - xi_b / 3.
__host__ __device__ constexpr double h3aab(int a, int b) { return (double)(a * a * b) - b / 3.0; }

// ---------------------------------------------------------------------------
// Macroscopic moments (eqs moment_rho, moment_rhoU) of stored populations.
template <int LAT, bool DEV, typename T>
struct Node {
  using L = Lattice<LAT>;
  static constexpr int Q = L::Q;
  static constexpr int D = L::D;

  // r0: sum of stored values (rho for DEV = 0, rho - 1 for DEV = 1)
  __device__ __host__ static inline void moments(const T* s, T& rho, T& r0, T* u) {
    T m = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      m += s[i];
      if (L::cx(i) > 0) jx += s[i];
      if (L::cx(i) < 0) jx -= s[i];
      if (L::cy(i) > 0) jy += s[i];
      if (L::cy(i) < 0) jy -= s[i];
      if (D == 3) {
        if (L::cz(i) > 0) jz += s[i];
        if (L::cz(i) < 0) jz -= s[i];
      }
    }
    r0 = m;
    rho = DEV ? T(1) + m : m;
    const T ir = T(1) / rho;
    u[0] = jx * ir;
    u[1] = jy * ir;
    u[2] = (D == 3) ? jz * ir : T(0);
  }

  // Third-order part of the equilibrium per unit density, per population,
  // given the six (or two) products u_a^2 u_b.  D2Q9: eq fEqO3.  D3Q19: the
  // pairs (xxy, yzz), (xzz, xyy), (yyz, xxz) enter through their sum (lattice
  // norm 2 c_s^6) and difference (lattice norm 6 c_s^6).
  template <int i>
  __device__ __host__ static inline T third(T axxy, T axyy, T ayzz, T axzz, T ayyz, T axxz) {
    constexpr int x = L::cx(i), y = L::cy(i), z = L::cz(i);
    if (D == 2) {
      constexpr double Hxxy = h3aab(x, y), Hxyy = h3aab(y, x);
      return T(13.5) * (T(Hxxy) * axxy + T(Hxyy) * axyy);
    } else {
      constexpr double Hxxy = h3aab(x, y), Hyzz = h3aab(z, y);
      constexpr double Hxzz = h3aab(z, x), Hxyy = h3aab(y, x);
      constexpr double Hyyz = h3aab(y, z), Hxxz = h3aab(x, z);
      T t = T(0);
      if (Hxxy + Hyzz != 0.0) t += T(13.5 * (Hxxy + Hyzz)) * (axxy + ayzz);
      if (Hxzz + Hxyy != 0.0) t += T(13.5 * (Hxzz + Hxyy)) * (axzz + axyy);
      if (Hyyz + Hxxz != 0.0) t += T(13.5 * (Hyyz + Hxxz)) * (ayyz + axxz);
      if (Hxxy - Hyzz != 0.0) t += T(4.5 * (Hxxy - Hyzz)) * (axxy - ayzz);
      if (Hxzz - Hxyy != 0.0) t += T(4.5 * (Hxzz - Hxyy)) * (axzz - axyy);
      if (Hyyz - Hxxz != 0.0) t += T(4.5 * (Hyyz - Hxxz)) * (ayyz - axxz);
      return t;
    }
  }

  // Stored-form equilibrium s0_i = w_i (r0 + rho E_i(u)) with
  // E_i = 3 xi.u + 9/2 (xi.u)^2 - 3/2 u^2 + third-order terms.
  template <int i>
  __device__ __host__ static inline T feq_one(T rho, T r0, const T* u, T usq, T axxy, T axyy, T ayzz,
                                              T axzz, T ayyz, T axxz) {
    constexpr int x = L::cx(i), y = L::cy(i), z = L::cz(i);
    T cu = T(0);
    if (x) cu += T(x) * u[0];
    if (y) cu += T(y) * u[1];
    if (D == 3 && z) cu += T(z) * u[2];
    T e = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq + third<i>(axxy, axyy, ayzz, axzz, ayyz, axxz);
    return T(L::w(i)) * (r0 + rho * e);
  }

  __device__ __host__ static inline void feq(T rho, T r0, const T* u, T* out) {
    const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T axxy = u[0] * u[0] * u[1], axyy = u[0] * u[1] * u[1];
    const T ayzz = u[1] * u[2] * u[2], axzz = u[0] * u[2] * u[2];
    const T ayyz = u[1] * u[1] * u[2], axxz = u[0] * u[0] * u[2];
    static_for<Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      out[i] = feq_one<i>(rho, r0, u, usq, axxy, axyy, ayzz, axzz, ayyz, axxz);
    });
  }

  // Second-order non-equilibrium moments a1^(2) = sum_i H2_i (f_i - f0_i)
  // (eq a1Proj).  With the third-order equilibrium,
  // sum_i xi xi f0_i = rho (u u + c_s^2 I), so a1 = Pi - r0/3 I - rho u u in
  // stored form (the rest state carries Pi = I/3).
  __device__ __host__ static inline Sym<T> a1(const T* s, T rho, T r0, const T* u) {
    T pxx = T(0), pyy = T(0), pzz = T(0), pxy = T(0), pxz = T(0), pyz = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int x = L::cx(i), y = L::cy(i), z = L::cz(i);
      if (x) pxx += s[i];
      if (y) pyy += s[i];
      if (D == 3 && z) pzz += s[i];
      if (x * y > 0) pxy += s[i];
      if (x * y < 0) pxy -= s[i];
      if (D == 3) {
        if (x * z > 0) pxz += s[i];
        if (x * z < 0) pxz -= s[i];
        if (y * z > 0) pyz += s[i];
        if (y * z < 0) pyz -= s[i];
      }
    }
    const T third_r0 = r0 * T(1.0 / 3.0);
    Sym<T> a;
    a.xx = pxx - third_r0 - rho * u[0] * u[0];
    a.yy = pyy - third_r0 - rho * u[1] * u[1];
    a.zz = (D == 3) ? pzz - third_r0 - rho * u[2] * u[2] : T(0);
    a.xy = pxy - rho * u[0] * u[1];
    a.xz = (D == 3) ? pxz - rho * u[0] * u[2] : T(0);
    a.yz = (D == 3) ? pyz - rho * u[1] * u[2] : T(0);
    return a;
  }

  // Recursive regularised non-equilibrium part (eqs f1RR, a13RR) from a1^(2)
  // and u, written to f1[i]:
  // f1_i = w_i [ 9/2 H2_i : a + third-order terms with a1^(3) ].
  __device__ __host__ static inline void f1rr(const Sym<T>& a, const T* u, T* f1) {
    const T tr = a.xx + a.yy + a.zz;
    const T axxy = T(2) * u[0] * a.xy + u[1] * a.xx;
    const T axyy = T(2) * u[1] * a.xy + u[0] * a.yy;
    const T ayzz = T(2) * u[2] * a.yz + u[1] * a.zz;
    const T axzz = T(2) * u[2] * a.xz + u[0] * a.zz;
    const T ayyz = T(2) * u[1] * a.yz + u[2] * a.yy;
    const T axxz = T(2) * u[0] * a.xz + u[2] * a.xx;
    static_for<Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      constexpr int x = L::cx(i), y = L::cy(i), z = L::cz(i);
      T h = -tr * T(1.0 / 3.0);
      if (x) h += a.xx;
      if (y) h += a.yy;
      if (D == 3 && z) h += a.zz;
      if (x * y) h += T(2 * x * y) * a.xy;
      if (D == 3 && x * z) h += T(2 * x * z) * a.xz;
      if (D == 3 && y * z) h += T(2 * y * z) * a.yz;
      f1[i] = T(L::w(i)) * (T(4.5) * h + third<i>(axxy, axyy, ayzz, axzz, ayyz, axxz));
    });
  }

  // Collision of one node, in place on stored populations s[Q].
  //   model 0 (BGK, eq BGKmodel):   s* = s0 + om (s - s0)
  //   model 1 (RR,  eq LBMscheme_reg): s* = s0 + om f1RR(a1)
  //   model 2 (H-RR, eq a1ij_HRR): a1 <- sig a1 + (1 - sig)(-2 tau rho c_s^2 S)
  // om = 1 - 1/tau.
  __device__ __host__ static inline void collide(T* s, int model, T om, T tau, T sig, const Sym<T>* S) {
    T rho, r0, u[3];
    moments(s, rho, r0, u);
    T s0[Q];
    feq(rho, r0, u, s0);
    if (model == 0) {
#pragma unroll
      for (int i = 0; i < Q; ++i) s[i] = s0[i] + om * (s[i] - s0[i]);
      return;
    }
    Sym<T> a = a1(s, rho, r0, u);
    if (model == 2) {
      const T k = (T(1) - sig) * (T(-2.0 / 3.0) * tau * rho);
      a.xx = sig * a.xx + k * S->xx;
      a.yy = sig * a.yy + k * S->yy;
      a.zz = sig * a.zz + k * S->zz;
      a.xy = sig * a.xy + k * S->xy;
      a.xz = sig * a.xz + k * S->xz;
      a.yz = sig * a.yz + k * S->yz;
      if (D == 2) a.zz = a.xz = a.yz = T(0);
    }
    T f1[Q];
    f1rr(a, u, f1);
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = s0[i] + om * f1[i];
  }
};



}  // namespace lbm
