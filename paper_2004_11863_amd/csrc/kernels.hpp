// kernels.hpp -- gfx950 kernels of the two-level LBM hot path.
//
// Layout in HBM: every level stores its populations structure-of-arrays,
// s[q][node] with node = x + nx (y + ny z), in a ping-pong pair of buffers
// (pull scheme: a step reads one buffer and writes the other).  The bulk
// kernels are one work-item per node, 64-wide along x so a wavefront reads
// and writes 64 consecutive nodes of one population per instruction.  Work
// groups cover TX x TY node tiles; the tile index is remapped so that each of
// the 8 XCDs (which receive work groups round-robin) gets one contiguous run
// of tiles, keeping the +-y / +-z neighbour rows of a tile in the same L2.
//
// Interface kernels (history capture, ring reconstruction, fine-to-coarse
// coalescence) run one work-item per interface node in double precision.
#pragma once
#include <hip/hip_runtime.h>

#include "geometry.hpp"
#include "lattice.hpp"

namespace lbm {

constexpr int kXCD = 8;

// Model codes: BGK and RR collide in the streaming kernel; H-RR needs the
// strain rate of neighbouring nodes and so streams first (kernel writes the
// pre-collision state and rho, u) and collides in a second kernel.
enum Model : int { M_BGK = 0, M_RR = 1, M_HRR = 2 };

struct Tiling {
  int nx, ny, nz;     // level extent
  int ntx, nty;       // tiles per axis
  int ntiles;         // ntx * nty * nz
  int per_xcd;        // tiles given to each XCD (launch = per_xcd * 8 groups)
};

template <int TX, int TY>
inline Tiling make_tiling(int nx, int ny, int nz) {
  Tiling t;
  t.nx = nx;
  t.ny = ny;
  t.nz = nz;
  t.ntx = (nx + TX - 1) / TX;
  t.nty = (ny + TY - 1) / TY;
  t.ntiles = t.ntx * t.nty * nz;
  t.per_xcd = (t.ntiles + kXCD - 1) / kXCD;
  return t;
}

// Node of this work-item; false when outside the level.
template <int TX, int TY>
__device__ inline bool tile_node(const Tiling& t, int& x, int& y, int& z) {
  const int b = blockIdx.x;
  const int tile = (b % kXCD) * t.per_xcd + b / kXCD;
  if (tile >= t.ntiles) return false;
  const int tx = tile % t.ntx;
  const int r = tile / t.ntx;
  const int ty = r % t.nty;
  z = r / t.nty;
  x = tx * TX + (int)(threadIdx.x % TX);
  y = ty * TY + (int)(threadIdx.x / TX);
  return x < t.nx && y < t.ny;
}

template <typename S, bool DEV, typename T>
__device__ inline T load_pop(const S* p) {
  return (T)(*p);
}

// ---------------------------------------------------------------------------
// Bulk stream (+ collide) of one level.
//   LEVEL 0: coarse, periodic, skips TN and covered nodes.
//   LEVEL 1: fine patch, skips the ring (reconstructed from the coarse level).
// MODEL BGK/RR: dst = collide(pull(src)).  MODEL HRR: dst = pull(src),
// mac = (rho, u) of the pulled state.
template <int LAT, bool DEV, typename S, typename T, int MODEL, int LEVEL, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_stream(const S* __restrict__ src, S* __restrict__ dst,
                                                    T* __restrict__ mac, const Geo g, const Tiling tl,
                                                    const T om) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, T>;
  constexpr int Q = L::Q;
  int x, y, z;
  if (!tile_node<TX, TY>(tl, x, y, z)) return;
  const int nx = tl.nx, ny = tl.ny, nz = tl.nz;
  if (LEVEL == 0) {
    const int c = coarse_class(g, x, y, z);
    if (c == CC_TN || c == CC_COVERED) return;
  } else {
    if (fine_is_ring(g, x, y, z)) return;
  }
  const size_t NN = (size_t)nx * ny * nz;
  const size_t idx = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
  T s[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int xs = x - L::cx(i), ys = y - L::cy(i), zs = z - L::cz(i);
    if (LEVEL == 0) {
      xs = wrap(xs, nx);
      ys = wrap(ys, ny);
      if (L::D == 3) zs = wrap(zs, nz);
    }
    const size_t sidx = (size_t)xs + (size_t)nx * ((size_t)ys + (size_t)ny * zs);
    s[i] = (T)src[(size_t)i * NN + sidx];
  }
  if (MODEL == M_HRR) {
    T rho, r0, u[3];
    N::moments(s, rho, r0, u);
    mac[idx] = rho;
    mac[NN + idx] = u[0];
    mac[2 * NN + idx] = u[1];
    if (L::D == 3) mac[3 * NN + idx] = u[2];
  } else {
    N::collide(s, MODEL, om, T(0), T(0), nullptr);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[(size_t)i * NN + idx] = (S)s[i];
}

// Centred differences of u (second order, level lattice units) -> strain.
template <int D, typename T, typename IdxFn>
__device__ inline Sym<T> strain_fd(const T* __restrict__ mac, size_t NN, IdxFn nb) {
  // nb(axis, sign) -> node index of x + sign e_axis
  T g[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const size_t ip = nb(a, +1), im = nb(a, -1);
#pragma unroll
    for (int b = 0; b < D; ++b) g[a][b] = (mac[(size_t)(1 + b) * NN + ip] - mac[(size_t)(1 + b) * NN + im]) * T(0.5);
  }
  Sym<T> S;
  S.xx = g[0][0];
  S.yy = g[1][1];
  S.zz = (D == 3) ? g[2][2] : T(0);
  S.xy = T(0.5) * (g[0][1] + g[1][0]);
  S.xz = (D == 3) ? T(0.5) * (g[0][2] + g[2][0]) : T(0);
  S.yz = (D == 3) ? T(0.5) * (g[1][2] + g[2][1]) : T(0);
  return S;
}

// H-RR collision in place on a level, with the strain rate from centred
// differences of the macroscopic velocity array (Sec. 3.3).
template <int LAT, bool DEV, typename S, typename T, int LEVEL, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_collide_hrr(S* __restrict__ buf, const T* __restrict__ mac,
                                                         const Geo g, const Tiling tl, const T om, const T tau,
                                                         const T sig) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, T>;
  constexpr int Q = L::Q;
  int x, y, z;
  if (!tile_node<TX, TY>(tl, x, y, z)) return;
  const int nx = tl.nx, ny = tl.ny, nz = tl.nz;
  if (LEVEL == 0) {
    const int c = coarse_class(g, x, y, z);
    if (c == CC_TN || c == CC_COVERED) return;
  } else {
    if (fine_is_ring(g, x, y, z)) return;
  }
  const size_t NN = (size_t)nx * ny * nz;
  const size_t idx = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
  auto nb = [&](int a, int sgn) -> size_t {
    int c[3] = {x, y, z};
    c[a] += sgn;
    if (LEVEL == 0) c[a] = wrap(c[a], a == 0 ? nx : (a == 1 ? ny : nz));
    return (size_t)c[0] + (size_t)nx * ((size_t)c[1] + (size_t)ny * c[2]);
  };
  const Sym<T> Sr = strain_fd<L::D, T>(mac, NN, nb);
  T s[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) s[i] = (T)buf[(size_t)i * NN + idx];
  N::collide(s, M_HRR, om, tau, sig, &Sr);
#pragma unroll
  for (int i = 0; i < Q; ++i) buf[(size_t)i * NN + idx] = (S)s[i];
}

// ---------------------------------------------------------------------------
// Interface data.  History fields per coarse history node, double precision:
// rho, u[D], f1[Q] (pre-collision non-equilibrium part), S[NS] (H-RR).
template <int LAT>
struct HF {
  static constexpr int D = Lattice<LAT>::D, Q = Lattice<LAT>::Q;
  static constexpr int RHO = 0, U = 1, F1 = 1 + D, S = 1 + D + Q;
  static constexpr int NSC = NS<D>::value;
  static constexpr int N = 1 + D + Q + NSC;
};

struct Iface {
  int64_t NH;
  const int64_t* hnode;   // [NH] coarse node of each history entry
  int64_t NR;
  const int64_t* rnode;   // [NR] fine node of each ring entry
  const int32_t* rnp;     // [NR] stencil points (1, 4, 16)
  const int32_t* rpt;     // [NR][16] history entries
  int64_t NT;
  const int64_t* tnf;     // [NT] fine TN nodes
  const int64_t* tnc;     // [NT] coarse TN nodes
};

template <typename S, bool DEV, int LAT>
__device__ inline double full_pop(S v, int i) {
  return (double)v + (DEV ? Lattice<LAT>::w(i) : 0.0);
}
template <typename S, bool DEV, int LAT>
__device__ inline S store_pop(double f, int i) {
  return (S)(f - (DEV ? Lattice<LAT>::w(i) : 0.0));
}

// Pre-collision state of coarse history nodes at t+1 (pulled from the
// post-collision coarse state at t): rho, u and f1 = f - f0(rho, u).
template <int LAT, bool DEV, typename S>
__global__ void k_hist_capture(const S* __restrict__ src, double* __restrict__ H, const Geo g, const Iface itf) {
  using L = Lattice<LAT>;
  using F = HF<LAT>;
  using N = Node<LAT, false, double>;
  constexpr int Q = L::Q;
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= itf.NH) return;
  const int64_t ci = itf.hnode[h];
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int x = (int)(ci % nx), y = (int)((ci / nx) % ny), z = (int)(ci / ((int64_t)nx * ny));
  const size_t NN = (size_t)g.Nc;
  double f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int xs = wrap(x - L::cx(i), nx), ys = wrap(y - L::cy(i), ny);
    const int zs = L::D == 3 ? wrap(z - L::cz(i), nz) : 0;
    f[i] = full_pop<S, DEV, LAT>(src[(size_t)i * NN + (size_t)xs + (size_t)nx * ((size_t)ys + (size_t)ny * zs)], i);
  }
  double rho, r0, u[3], f0[Q];
  N::moments(f, rho, r0, u);
  N::feq(rho, r0, u, f0);
  const int64_t NH = itf.NH;
  H[F::RHO * NH + h] = rho;
#pragma unroll
  for (int d = 0; d < L::D; ++d) H[(F::U + d) * NH + h] = u[d];
#pragma unroll
  for (int i = 0; i < Q; ++i) H[(F::F1 + i) * NH + h] = f[i] - f0[i];
}

// H-RR: coarse strain rate at t+1 on the history nodes, by centred
// differences of the coarse macroscopic velocity (TN entries come from the
// fictitious propagation on the fine level).
template <int LAT, typename T>
__global__ void k_hist_strain(const T* __restrict__ mac_c, double* __restrict__ H, const Geo g, const Iface itf) {
  using L = Lattice<LAT>;
  using F = HF<LAT>;
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= itf.NH) return;
  const int64_t ci = itf.hnode[h];
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int x = (int)(ci % nx), y = (int)((ci / nx) % ny), z = (int)(ci / ((int64_t)nx * ny));
  auto nb = [&](int a, int sgn) -> size_t {
    int c[3] = {x, y, z};
    c[a] = wrap(c[a] + sgn, a == 0 ? nx : (a == 1 ? ny : nz));
    return (size_t)c[0] + (size_t)nx * ((size_t)c[1] + (size_t)ny * c[2]);
  };
  const Sym<T> S = strain_fd<L::D, T>(mac_c, (size_t)g.Nc, nb);
  const int64_t NH = itf.NH;
  H[(F::S + 0) * NH + h] = (double)S.xx;
  H[(F::S + 1) * NH + h] = (double)S.yy;
  if (L::D == 2) {
    H[(F::S + 2) * NH + h] = (double)S.xy;
  } else {
    H[(F::S + 2) * NH + h] = (double)S.zz;
    H[(F::S + 3) * NH + h] = (double)S.xy;
    H[(F::S + 4) * NH + h] = (double)S.xz;
    H[(F::S + 5) * NH + h] = (double)S.yz;
  }
}

// Temporal interpolation of every history field (eq TempInt): G = c0 H(t-1)
// + c1 H(t) + c2 H(t+1), for all fields of all history nodes.
__global__ void k_hist_time(const double* __restrict__ Hm, const double* __restrict__ H0,
                            const double* __restrict__ Hp, double* __restrict__ G, int64_t n, double c0,
                            double c1, double c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  G[k] = c0 * Hm[k] + c1 * H0[k] + c2 * Hp[k];
}

__device__ inline double cubic_w(int s) { return (s == 1 || s == 2) ? 9.0 / 16.0 : -1.0 / 16.0; }

// Spatial weight of point s of a ring stencil (eq spaceInt; tensor product on
// 3D face centres, first odd axis fastest).
__device__ inline double ring_w(int np, int s) {
  if (np == 1) return 1.0;
  if (np == 4) return cubic_w(s);
  return cubic_w(s & 3) * cubic_w(s >> 2);
}

// Ring nodes, rho and u only (H-RR needs them before the fine collision).
// Temporal weights c applied inline to the three history levels.
template <int LAT, typename T>
__global__ void k_ring_macro(const double* __restrict__ Hm, const double* __restrict__ H0,
                             const double* __restrict__ Hp, double c0, double c1, double c2,
                             T* __restrict__ mac_f, const Geo g, const Iface itf) {
  using L = Lattice<LAT>;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= itf.NR) return;
  const int np = itf.rnp[r];
  const int32_t* pt = itf.rpt + 16 * r;
  const int64_t NH = itf.NH;
  double v[1 + L::D];
#pragma unroll
  for (int k = 0; k < 1 + L::D; ++k) v[k] = 0.0;
  for (int s = 0; s < np; ++s) {
    const int64_t h = pt[s];
    const double ws = ring_w(np, s);
#pragma unroll
    for (int k = 0; k < 1 + L::D; ++k) {
      const int64_t o = (int64_t)k * NH + h;
      v[k] += ws * (c0 * Hm[o] + c1 * H0[o] + c2 * Hp[o]);
    }
  }
  const size_t NN = (size_t)g.Nf;
  const size_t fi = (size_t)itf.rnode[r];
#pragma unroll
  for (int k = 0; k < 1 + L::D; ++k) mac_f[(size_t)k * NN + fi] = (T)v[k];
}

// Ring nodes: rho, u, f1 (and S) interpolated from the (time-interpolated)
// history G, populations rebuilt as f0(rho, u) + tau_f/(2 tau_c) f1 (eq
// rescff), S^f = S^c / 2 (eq PijResc), collided with tau_f and stored.
template <int LAT, bool DEV, typename S, int MODEL>
__global__ void k_ring(const double* __restrict__ G, S* __restrict__ dst, const Geo g, const Iface itf,
                       double kf, double om_f, double tau_f, double sig) {
  using L = Lattice<LAT>;
  using F = HF<LAT>;
  using N = Node<LAT, false, double>;
  constexpr int Q = L::Q;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= itf.NR) return;
  const int np = itf.rnp[r];
  const int32_t* pt = itf.rpt + 16 * r;
  const int64_t NH = itf.NH;
  constexpr int NF = (MODEL == M_HRR) ? F::N : F::S;
  double v[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) v[k] = 0.0;
  for (int s = 0; s < np; ++s) {
    const int64_t h = pt[s];
    const double ws = ring_w(np, s);
#pragma unroll
    for (int k = 0; k < NF; ++k) v[k] += ws * G[(int64_t)k * NH + h];
  }
  double u[3] = {v[F::U], v[F::U + 1], L::D == 3 ? v[F::U + 2] : 0.0};
  double f[Q];
  N::feq(v[F::RHO], v[F::RHO], u, f);
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] += kf * v[F::F1 + i];
  Sym<double> Sf{0, 0, 0, 0, 0, 0};
  if (MODEL == M_HRR) {
    if (L::D == 2) {
      Sf.xx = 0.5 * v[F::S];
      Sf.yy = 0.5 * v[F::S + 1];
      Sf.xy = 0.5 * v[F::S + 2];
    } else {
      Sf.xx = 0.5 * v[F::S];
      Sf.yy = 0.5 * v[F::S + 1];
      Sf.zz = 0.5 * v[F::S + 2];
      Sf.xy = 0.5 * v[F::S + 3];
      Sf.xz = 0.5 * v[F::S + 4];
      Sf.yz = 0.5 * v[F::S + 5];
    }
  }
  N::collide(f, MODEL, om_f, tau_f, sig, &Sf);
  const size_t NN = (size_t)g.Nf;
  const size_t fi = (size_t)itf.rnode[r];
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[(size_t)i * NN + fi] = store_pop<S, DEV, LAT>(f[i], i);
}

// Pull of Q populations into fine node (x, y, z) from a fine buffer.
template <int LAT, bool DEV, typename S>
__device__ inline void pull_fine(const S* __restrict__ src, const Geo& g, int x, int y, int z, double* f) {
  using L = Lattice<LAT>;
  const int nx = g.nf[0], ny = g.nf[1];
  const size_t NN = (size_t)g.Nf;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const size_t sidx = (size_t)(x - L::cx(i)) + (size_t)nx * ((size_t)(y - L::cy(i)) + (size_t)ny * (z - L::cz(i)));
    f[i] = full_pop<S, DEV, LAT>(src[(size_t)i * NN + sidx], i);
  }
}

// H-RR: fictitious propagation onto TN^f (Sec. 4.3, step e): u(TN, t+1) from
// the fine post-collision state at t+1/2, written to the coarse macro array.
template <int LAT, bool DEV, typename S, typename T>
__global__ void k_fict(const S* __restrict__ src_f, T* __restrict__ mac_c, const Geo g, const Iface itf) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= itf.NT) return;
  const int64_t fi = itf.tnf[t];
  const int nx = g.nf[0], ny = g.nf[1];
  const int x = (int)(fi % nx), y = (int)((fi / nx) % ny), z = (int)(fi / ((int64_t)nx * ny));
  double f[L::Q], rho, r0, u[3];
  pull_fine<LAT, DEV, S>(src_f, g, x, y, z, f);
  N::moments(f, rho, r0, u);
  const size_t NN = (size_t)g.Nc;
  const size_t ci = (size_t)itf.tnc[t];
  mac_c[ci] = (T)rho;
#pragma unroll
  for (int d = 0; d < L::D; ++d) mac_c[(size_t)(1 + d) * NN + ci] = (T)u[d];
}

// Fine-to-coarse transfer at TN (Sec. 4.3, synchronous step d): the fine
// pre-collision state at t+1 around TN^f is re-pulled from the fine
// post-collision state at t+1/2; its non-equilibrium part is filtered with
// the tensor product of (1/4, 1/2, 1/4) (eq filterFneq), rescaled by
// 2 tau_c / tau_f (eq rescfc) and added to f0 of the co-located fine node;
// H-RR takes S^c = 2 S^f (eq PijResc) with S^f by fine centred differences.
// The coarse node is then collided with tau_c and stored.
template <int LAT, bool DEV, typename S, int MODEL>
__global__ void k_coalesce(const S* __restrict__ src_f, S* __restrict__ dst_c, const Geo g, const Iface itf,
                           double kc, double om_c, double tau_c, double sig) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  constexpr int Q = L::Q, D = L::D;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= itf.NT) return;
  const int64_t fi = itf.tnf[t];
  const int nx = g.nf[0], ny = g.nf[1];
  const int x = (int)(fi % nx), y = (int)((fi / nx) % ny), z = (int)(fi / ((int64_t)nx * ny));
  double ft[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) ft[i] = 0.0;
  double rc = 0.0, uc[3] = {0.0, 0.0, 0.0};
  double up[3][3] = {{0}}, um[3][3] = {{0}};  // u at x +- e_a
  constexpr int NST = (D == 2) ? 9 : 27;
  for (int s = 0; s < NST; ++s) {
    const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = (D == 3) ? s / 9 - 1 : 0;
    double f[Q], rho, r0, u[3], f0[Q];
    pull_fine<LAT, DEV, S>(src_f, g, x + ox, y + oy, z + oz, f);
    N::moments(f, rho, r0, u);
    N::feq(rho, r0, u, f0);
    const int nz = (ox != 0) + (oy != 0) + (oz != 0);
    const double w = (nz == 0 ? 1.0 : 1.0) * (ox ? 0.25 : 0.5) * (oy ? 0.25 : 0.5) * (D == 3 ? (oz ? 0.25 : 0.5) : 1.0);
#pragma unroll
    for (int i = 0; i < Q; ++i) ft[i] += w * (f[i] - f0[i]);
    if (nz == 0) {
      rc = rho;
      uc[0] = u[0];
      uc[1] = u[1];
      uc[2] = u[2];
    } else if (nz == 1) {
      const int a = ox ? 0 : (oy ? 1 : 2);
      const int sg = ox + oy + oz;
      for (int b = 0; b < 3; ++b) {
        if (sg > 0) up[a][b] = u[b];
        else um[a][b] = u[b];
      }
    }
  }
  double f[Q];
  N::feq(rc, rc, uc, f);
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] += kc * ft[i];
  Sym<double> Sc{0, 0, 0, 0, 0, 0};
  if (MODEL == M_HRR) {
    double gr[3][3] = {{0}};
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) gr[a][b] = 0.5 * (up[a][b] - um[a][b]);
    Sc.xx = 2.0 * gr[0][0];
    Sc.yy = 2.0 * gr[1][1];
    Sc.zz = (D == 3) ? 2.0 * gr[2][2] : 0.0;
    Sc.xy = 2.0 * (0.5 * (gr[0][1] + gr[1][0]));
    Sc.xz = (D == 3) ? 2.0 * (0.5 * (gr[0][2] + gr[2][0])) : 0.0;
    Sc.yz = (D == 3) ? 2.0 * (0.5 * (gr[1][2] + gr[2][1])) : 0.0;
  }
  N::collide(f, MODEL, om_c, tau_c, sig, &Sc);
  const size_t NN = (size_t)g.Nc;
  const size_t ci = (size_t)itf.tnc[t];
#pragma unroll
  for (int i = 0; i < Q; ++i) dst_c[(size_t)i * NN + ci] = store_pop<S, DEV, LAT>(f[i], i);
}

// ---------------------------------------------------------------------------
// State transfer kernels.

// Equilibrium populations of given fields: s = f0(rho, u) - DEV w.
template <int LAT, bool DEV, typename S>
__global__ void k_set_state(const double* __restrict__ rho, const double* __restrict__ u, S* __restrict__ dst,
                            int64_t NN) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  double uu[3] = {u[k], u[NN + k], L::D == 3 ? u[2 * NN + k] : 0.0};
  double f[L::Q];
  N::feq(rho[k], rho[k], uu, f);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) dst[(size_t)i * NN + k] = store_pop<S, DEV, LAT>(f[i], i);
}

// History at t = 0 from coarse fields rho, u (full coarse arrays): all three
// levels get rho, u, f1 = 0 and S = centred differences of u.
template <int LAT>
__global__ void k_hist_init(const double* __restrict__ rho, const double* __restrict__ u, double* __restrict__ H0,
                            double* __restrict__ H1, double* __restrict__ H2, const Geo g, const Iface itf) {
  using L = Lattice<LAT>;
  using F = HF<LAT>;
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= itf.NH) return;
  const int64_t ci = itf.hnode[h];
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int x = (int)(ci % nx), y = (int)((ci / nx) % ny), z = (int)(ci / ((int64_t)nx * ny));
  const size_t NN = (size_t)g.Nc;
  double v[F::N];
  v[F::RHO] = rho[ci];
  for (int d = 0; d < L::D; ++d) v[F::U + d] = u[(size_t)d * NN + ci];
  for (int i = 0; i < L::Q; ++i) v[F::F1 + i] = 0.0;
  double gr[3][3] = {{0}};
  for (int a = 0; a < L::D; ++a) {
    int cp[3] = {x, y, z}, cm[3] = {x, y, z};
    const int na = a == 0 ? nx : (a == 1 ? ny : nz);
    cp[a] = wrap(cp[a] + 1, na);
    cm[a] = wrap(cm[a] - 1, na);
    const size_t ip = (size_t)cp[0] + (size_t)nx * ((size_t)cp[1] + (size_t)ny * cp[2]);
    const size_t im = (size_t)cm[0] + (size_t)nx * ((size_t)cm[1] + (size_t)ny * cm[2]);
    for (int b = 0; b < L::D; ++b) gr[a][b] = 0.5 * (u[(size_t)b * NN + ip] - u[(size_t)b * NN + im]);
  }
  if (L::D == 2) {
    v[F::S] = gr[0][0];
    v[F::S + 1] = gr[1][1];
    v[F::S + 2] = 0.5 * (gr[0][1] + gr[1][0]);
  } else {
    v[F::S] = gr[0][0];
    v[F::S + 1] = gr[1][1];
    v[F::S + 2] = gr[2][2];
    v[F::S + 3] = 0.5 * (gr[0][1] + gr[1][0]);
    v[F::S + 4] = 0.5 * (gr[0][2] + gr[2][0]);
    v[F::S + 5] = 0.5 * (gr[1][2] + gr[2][1]);
  }
  const int64_t NH = itf.NH;
  for (int k = 0; k < F::N; ++k) {
    H0[(int64_t)k * NH + h] = v[k];
    H1[(int64_t)k * NH + h] = v[k];
    H2[(int64_t)k * NH + h] = v[k];
  }
}

// Moments of the stored post-collision state (double).  On the coarse level
// covered nodes take the co-located fine node's values.
template <int LAT, bool DEV, typename S>
__global__ void k_macros(const S* __restrict__ src, const S* __restrict__ fine, double* __restrict__ rho,
                         double* __restrict__ u, const Geo g, int level) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  const int64_t NN = level == 0 ? g.Nc : g.Nf;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  const S* p = src;
  int64_t kk = k, MM = NN;
  if (level == 0 && g.has_fine) {
    const int nx = g.n[0], ny = g.n[1];
    const int x = (int)(k % nx), y = (int)((k / nx) % ny), z = (int)(k / ((int64_t)nx * ny));
    if (coarse_class(g, x, y, z) == CC_COVERED) {
      const int jx = 2 * (x - g.a[0]), jy = 2 * (y - g.a[1]), jz = L::D == 3 ? 2 * (z - g.a[2]) : 0;
      kk = (int64_t)jx + (int64_t)g.nf[0] * ((int64_t)jy + (int64_t)g.nf[1] * jz);
      p = fine;
      MM = g.Nf;
    }
  }
  double f[L::Q], r, r0, uu[3];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) f[i] = full_pop<S, DEV, LAT>(p[(size_t)i * MM + kk], i);
  N::moments(f, r, r0, uu);
  rho[k] = r;
#pragma unroll
  for (int d = 0; d < L::D; ++d) u[(size_t)d * NN + k] = uu[d];
}

template <int LAT, bool DEV, typename S>
__global__ void k_pops_out(const S* __restrict__ src, double* __restrict__ f, int64_t n, int64_t NN) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  f[k] = full_pop<S, DEV, LAT>(src[k], (int)(k / NN));
}
template <int LAT, bool DEV, typename S>
__global__ void k_pops_in(const double* __restrict__ f, S* __restrict__ dst, int64_t n, int64_t NN) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  dst[k] = store_pop<S, DEV, LAT>(f[k], (int)(k / NN));
}

// Global totals, pass 1: per-block sums of rho and rho u (double) over the
// evolving nodes of a level.  256 threads per block, fixed reduction tree.
template <int LAT, bool DEV, typename S>
__global__ __launch_bounds__(256) void k_totals(const S* __restrict__ src, double* __restrict__ part,
                                                const Geo g, int level) {
  using L = Lattice<LAT>;
  const int64_t NN = level == 0 ? g.Nc : g.Nf;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (k < NN) {
    bool use = true;
    if (level == 0 && g.has_fine) {
      const int nx = g.n[0], ny = g.n[1];
      const int x = (int)(k % nx), y = (int)((k / nx) % ny), z = (int)(k / ((int64_t)nx * ny));
      use = coarse_class(g, x, y, z) != CC_COVERED;
    }
    if (use) {
#pragma unroll
      for (int i = 0; i < L::Q; ++i) {
        const double f = full_pop<S, DEV, LAT>(src[(size_t)i * NN + k], i);
        v[0] += f;
        v[1] += L::cx(i) * f;
        v[2] += L::cy(i) * f;
        v[3] += L::cz(i) * f;
      }
    }
  }
  __shared__ double sh[4][256];
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 4; ++c) part[(int64_t)blockIdx.x * 4 + c] = sh[c][0];
}

// Pass 2: one block adds the partials in a fixed order.
__global__ __launch_bounds__(256) void k_totals_final(const double* __restrict__ part, int64_t nb,
                                                      double* __restrict__ out) {
  __shared__ double sh[4][256];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nb; b += 256)
    for (int c = 0; c < 4; ++c) v[c] += part[b * 4 + c];
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 4; ++c) out[c] = sh[c][0];
}

}  // namespace lbm
