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
// Per-node physics in moment space.
//
// Every population the scheme produces (equilibrium, BGK or regularised
// post-collision state) is a polynomial in the lattice velocity,
//   s_i = w_i [ A + xi_i.J + xi_i xi_i : M + sum_P H_P(xi_i) K_P ],
// where the H_P are the third-order Hermite polynomials the lattice carries
// (D2Q9: H_xxy, H_xyy; D3Q19: the sums and differences of the pairs
// (H_xxy, H_yzz), (H_xzz, H_xyy), (H_yyz, H_xxz)).  The node computes the
// coefficients (A, J, M, K) once and evaluates opposite velocities together:
// the even part A + xi xi : M is shared, the odd part flips sign.
template <int LAT, bool DEV, typename T>
struct Node {
  using L = Lattice<LAT>;
  static constexpr int Q = L::Q;
  static constexpr int D = L::D;
  static constexpr int NP = D == 2 ? 2 : 6;

  // index of the opposite velocity
  __host__ __device__ static constexpr int opp(int i) {
    for (int j = 0; j < Q; ++j)
      if (L::cx(j) == -L::cx(i) && L::cy(j) == -L::cy(i) && L::cz(j) == -L::cz(i)) return j;
    return i;
  }
  // value of third-order basis polynomial p at velocity i
  __host__ __device__ static constexpr double hp(int p, int i) {
    const int x = L::cx(i), y = L::cy(i), z = L::cz(i);
    if (D == 2) return p == 0 ? h3aab(x, y) : h3aab(y, x);
    const double pa[3] = {h3aab(x, y), h3aab(z, x), h3aab(y, z)};  // xxy, xzz, yyz
    const double pb[3] = {h3aab(z, y), h3aab(y, x), h3aab(x, z)};  // yzz, xyy, xxz
    return p < 3 ? pa[p] + pb[p] : pa[p - 3] - pb[p - 3];
  }
  // 1 / (lattice norm of H_P), i.e. 1/(2 c_s^6) or 1/(6 c_s^6)
  __host__ __device__ static constexpr double cp(int p) { return (D == 2 || p < 3) ? 13.5 : 4.5; }

  struct Coef {
    T A;
    T J[3];
    Sym<T> M;
    T K[6];
  };

  // eqs moment_rho, moment_rhoU.  r0: sum of stored values (rho for DEV = 0,
  // rho - 1 for DEV = 1).  Opposite velocities enter as the pair sum (even
  // moments) and the pair difference (odd moments); sums start from -0, which
  // the compiler folds away (x + -0 = x exactly).
  __device__ __host__ static __forceinline__ void moments(const T* s, T& rho, T& r0, T* u) {
    T m = s[0], jx = T(-0.0), jy = T(-0.0), jz = T(-0.0);
    static_for<Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      constexpr int j = opp(i);
      if constexpr (i != 0 && i < j) {
        const T p = s[i] + s[j], d = s[i] - s[j];
        m += p;
        if constexpr (L::cx(i) > 0) jx += d;
        if constexpr (L::cx(i) < 0) jx -= d;
        if constexpr (L::cy(i) > 0) jy += d;
        if constexpr (L::cy(i) < 0) jy -= d;
        if constexpr (D == 3 && L::cz(i) > 0) jz += d;
        if constexpr (D == 3 && L::cz(i) < 0) jz -= d;
      }
    });
    r0 = m;
    rho = DEV ? T(1) + m : m;
    const T ir = T(1) / rho;
    u[0] = jx * ir;
    u[1] = jy * ir;
    u[2] = (D == 3) ? jz * ir : T(0);
  }

  // Second moments Pi_ab = sum_i xi_a xi_b s_i, from the pair sums (xi_a xi_b
  // is the same for opposite velocities).
  __device__ __host__ static __forceinline__ Sym<T> second(const T* s) {
    T pxx = T(-0.0), pyy = T(-0.0), pzz = T(-0.0), pxy = T(-0.0), pxz = T(-0.0), pyz = T(-0.0);
    static_for<Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      constexpr int j = opp(i);
      if constexpr (i != 0 && i < j) {
        constexpr int x = L::cx(i), y = L::cy(i), z = L::cz(i);
        const T p = s[i] + s[j];
        if constexpr (x != 0) pxx += p;
        if constexpr (y != 0) pyy += p;
        if constexpr (D == 3 && z != 0) pzz += p;
        if constexpr (x * y > 0) pxy += p;
        if constexpr (x * y < 0) pxy -= p;
        if constexpr (D == 3 && x * z > 0) pxz += p;
        if constexpr (D == 3 && x * z < 0) pxz -= p;
        if constexpr (D == 3 && y * z > 0) pyz += p;
        if constexpr (D == 3 && y * z < 0) pyz -= p;
      }
    });
    if constexpr (D == 2) pzz = pxz = pyz = T(0);
    return Sym<T>{pxx, pyy, pzz, pxy, pxz, pyz};
  }

  // Third-order coefficient combinations of a fully symmetric tensor given
  // by its components (xxy, xyy, yzz, xzz, yyz, xxz), in basis order.
  __device__ __host__ static __forceinline__ void third_combo(T xxy, T xyy, T yzz, T xzz, T yyz, T xxz, T* out) {
    if (D == 2) {
      out[0] = xxy;
      out[1] = xyy;
    } else {
      out[0] = xxy + yzz;
      out[1] = xzz + xyy;
      out[2] = yyz + xxz;
      out[3] = xxy - yzz;
      out[4] = xzz - xyy;
      out[5] = yyz - xxz;
    }
  }

  // Coefficients of om * f1^RR + f0 (eqs fEqO3, f1RR, a13RR), a = a1^(2):
  //   A = r0 - 3/2 rho u^2 - 3/2 om tr(a),  J = 3 rho u,
  //   M = 9/2 (rho u u + om a),            K_P = c_P (rho u^3 + om a1^(3))_P.
  // om = 0 gives the equilibrium alone.
  __device__ __host__ static __forceinline__ Coef coef(T rho, T r0, const T* u, T om, const Sym<T>& a) {
    Coef c;
    const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T tra = a.xx + a.yy + a.zz;
    c.A = r0 - T(1.5) * rho * usq - T(1.5) * om * tra;
    c.J[0] = T(3) * rho * u[0];
    c.J[1] = T(3) * rho * u[1];
    c.J[2] = T(3) * rho * u[2];
    c.M.xx = T(4.5) * (rho * u[0] * u[0] + om * a.xx);
    c.M.yy = T(4.5) * (rho * u[1] * u[1] + om * a.yy);
    c.M.zz = T(4.5) * (rho * u[2] * u[2] + om * a.zz);
    c.M.xy = T(4.5) * (rho * u[0] * u[1] + om * a.xy);
    c.M.xz = T(4.5) * (rho * u[0] * u[2] + om * a.xz);
    c.M.yz = T(4.5) * (rho * u[1] * u[2] + om * a.yz);
    // a1^(3)_abg = u_a a_bg + u_b a_ag + u_g a_ab (eq a13RR), mixed components
    const T b_xxy = T(2) * u[0] * a.xy + u[1] * a.xx;
    const T b_xyy = T(2) * u[1] * a.xy + u[0] * a.yy;
    const T b_yzz = T(2) * u[2] * a.yz + u[1] * a.zz;
    const T b_xzz = T(2) * u[2] * a.xz + u[0] * a.zz;
    const T b_yyz = T(2) * u[1] * a.yz + u[2] * a.yy;
    const T b_xxz = T(2) * u[0] * a.xz + u[2] * a.xx;
    const T ru0 = rho * u[0], ru1 = rho * u[1];
    T k[6];
    third_combo(ru0 * u[0] * u[1] + om * b_xxy, ru0 * u[1] * u[1] + om * b_xyy, ru1 * u[2] * u[2] + om * b_yzz,
                ru0 * u[2] * u[2] + om * b_xzz, ru1 * u[1] * u[2] + om * b_yyz, ru0 * u[0] * u[2] + om * b_xxz, k);
#pragma unroll
    for (int p = 0; p < NP; ++p) c.K[p] = T(cp(p)) * k[p];
    return c;
  }

  template <int i>
  __device__ __host__ static __forceinline__ T even(const Coef& c) {
    constexpr int x = L::cx(i), y = L::cy(i), z = L::cz(i);
    T e = c.A;
    if (x) e += c.M.xx;
    if (y) e += c.M.yy;
    if (D == 3 && z) e += c.M.zz;
    if (x * y) e += T(2 * x * y) * c.M.xy;
    if (D == 3 && x * z) e += T(2 * x * z) * c.M.xz;
    if (D == 3 && y * z) e += T(2 * y * z) * c.M.yz;
    return e;
  }
  template <int i>
  __device__ __host__ static __forceinline__ T odd(const Coef& c) {
    constexpr int x = L::cx(i), y = L::cy(i), z = L::cz(i);
    T o = T(-0.0);  // folded away by the first term
    if (x > 0) o += c.J[0];
    if (x < 0) o -= c.J[0];
    if (y > 0) o += c.J[1];
    if (y < 0) o -= c.J[1];
    if (D == 3 && z > 0) o += c.J[2];
    if (D == 3 && z < 0) o -= c.J[2];
    static_for<NP>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr double h = hp(p, i);
      if (h != 0.0) o += T(h) * c.K[p];
    });
    return o;
  }

  // All Q stored values from coefficients.
  __device__ __host__ static __forceinline__ void eval(const Coef& c, T* out) {
    out[0] = T(L::w(0)) * even<0>(c);
    static_for<Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      constexpr int j = opp(i);
      if constexpr (i != 0 && i < j) {
        const T e = even<i>(c), o = odd<i>(c);
        out[i] = T(L::w(i)) * (e + o);
        out[j] = T(L::w(j)) * (e - o);
      }
    });
  }

  // Stored-form equilibrium s0_i = f0_i - DEV w_i (eq fEqO3 and its D3Q19
  // counterpart).
  __device__ __host__ static __forceinline__ void feq(T rho, T r0, const T* u, T* out) {
    const Sym<T> z{T(0), T(0), T(0), T(0), T(0), T(0)};
    eval(coef(rho, r0, u, T(0), z), out);
  }

  // Collision of one node, in place on stored populations s[Q].
  //   model 0 (BGK, eq BGKmodel):      s* = s0 + om (s - s0)
  //   model 1 (RR,  eq LBMscheme_reg): s* = s0 + om f1RR(a1)
  //   model 2 (H-RR, eq a1ij_HRR):     a1 <- sig a1 + (1 - sig)(-2 tau rho c_s^2 S)
  // om = 1 - 1/tau.  With the third-order equilibrium,
  // sum_i xi xi f0_i = rho (u u + c_s^2 I), so a1 = Pi - r0/3 I - rho u u
  // in stored form (the rest state carries Pi = I/3).
  __device__ __host__ static __forceinline__ void collide(T* s, int model, T om, T tau, T sig, const Sym<T>* S) {
    T rho, r0, u[3];
    moments(s, rho, r0, u);
    if (model == 0) {
      T s0[Q];
      feq(rho, r0, u, s0);
#pragma unroll
      for (int i = 0; i < Q; ++i) s[i] = s0[i] + om * (s[i] - s0[i]);
      return;
    }
    const Sym<T> P = second(s);
    const T tr0 = r0 * T(1.0 / 3.0);
    Sym<T> a;
    a.xx = P.xx - tr0 - rho * u[0] * u[0];
    a.yy = P.yy - tr0 - rho * u[1] * u[1];
    a.zz = (D == 3) ? P.zz - tr0 - rho * u[2] * u[2] : T(0);
    a.xy = P.xy - rho * u[0] * u[1];
    a.xz = (D == 3) ? P.xz - rho * u[0] * u[2] : T(0);
    a.yz = (D == 3) ? P.yz - rho * u[1] * u[2] : T(0);
    if (model == 2) {
      const T k = (T(1) - sig) * (T(-2.0 / 3.0) * tau * rho);
      a.xx = sig * a.xx + k * S->xx;
      a.yy = sig * a.yy + k * S->yy;
      a.xy = sig * a.xy + k * S->xy;
      if (D == 3) {
        a.zz = sig * a.zz + k * S->zz;
        a.xz = sig * a.xz + k * S->xz;
        a.yz = sig * a.yz + k * S->yz;
      }
    }
    eval(coef(rho, r0, u, om, a), s);
  }
};

}  // namespace lbm
