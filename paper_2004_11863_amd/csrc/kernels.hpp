// kernels.hpp -- gfx950 kernels of the two-level LBM hot path.
//
// Layout in HBM: every level stores its populations array-of-SoA (pop_at in
// geometry.hpp) over padded node positions with a row pitch that is a
// multiple of 4 nodes, so rows start 16-byte aligned, in a ping-pong pair of
// buffers (pull scheme: a step reads one buffer and writes the other).
//
// Bulk kernels: one work-item updates V consecutive nodes of a row, so every
// population is moved with one 16-byte access per lane (V = 4 in FP32, V = 2
// in FP64); the streams shifted by +-1 along x use 4/8-byte-aligned 16-byte
// loads, stores are aligned and non-temporal.  The vectors of the processed
// rows are numbered row after row ("flat" order) and a work group takes 256
// consecutive ones; work groups are handed to the 8 XCDs round-robin by the
// hardware, so the chunk index is remapped to give each XCD one contiguous
// run, which keeps the +-y / +-z neighbour rows of a chunk in the same L2.
// Fewer resident work groups per CU let HBM serve the 2Q streams with fewer
// row switches; the launch variants cap the residency through unused dynamic
// LDS (kVarLds).
//
// Interface kernels (history capture, ring reconstruction, fine-to-coarse
// coalescence) work per interface node in double precision, with small work
// groups so the few thousand interface nodes spread over all CUs.
#pragma once
#include <hip/hip_runtime.h>

#include "geometry.hpp"
#include "lattice.hpp"

namespace lbm {

constexpr int kXCD = 8;
constexpr int kIfaceBlock = 64;
// Bulk-kernel launch variants: dynamic LDS per 256-lane work group (none,
// then caps of 3, 2 and 1 resident work groups per CU of 160 KB LDS).
constexpr int kNVar = 4;
constexpr int kVarLds[kNVar] = {0, 53 * 1024, 80 * 1024, 160 * 1024};

// Model codes: BGK and RR collide in the streaming kernel.  H-RR needs the
// velocities of the neighbours at the same time level: a first pass pulls
// and writes only rho, u; a second pass pulls again, takes the strain rate
// from the neighbouring velocities and collides.
enum Model : int { M_BGK = 0, M_RR = 1, M_HRR = 2 };

// A product rounded on its own (never fused into a following add).
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }

// 16-byte vectors: "a" is the aligned type, "u" the same vector with element
// alignment only (used for the x-shifted loads).
template <typename S, int V>
struct VT;
template <>
struct VT<float, 4> {
  typedef float a __attribute__((ext_vector_type(4)));
  typedef float u __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct VT<double, 2> {
  typedef double a __attribute__((ext_vector_type(2)));
  typedef double u __attribute__((ext_vector_type(2), aligned(8)));
};
// Nodes per lane of the bulk kernels.
template <typename S>
struct VecOf {
  static constexpr int V = 16 / sizeof(S);
};

template <bool NT, typename A>
__device__ __forceinline__ void vstore(A* p, const A& v) {
  if (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Flat numbering of the bulk vectors of a level: rows y0 .. y0+nyr-1 of planes
// z0 .. z0+nzr-1, nv vectors of V nodes per row starting at node xb (the
// fine level starts at its first middle node x = 1, which is 16-byte aligned
// in storage, and skips its ring rows and planes; the coarse level covers
// every row).  A chunk is 256 consecutive vectors, one per lane.
struct Flat {
  int nx, ny, nz;  // level extent (nodes)
  int xb;          // first node of the vector grid along x
  int nv;          // vectors per row
  int y0, nyr;     // first processed row, processed rows per plane
  int z0, nzr;     // first processed plane, processed planes
  int64_t nvec;    // nv * nyr * nzr
  int nchunks;     // ceil(nvec / 256)
  int per_xcd;     // chunks given to each XCD (launch = per_xcd * 8 groups)
};

inline Flat make_flat(int nx, int ny, int nz, int V, bool fine, int D) {
  Flat f;
  f.nx = nx;
  f.ny = ny;
  f.nz = nz;
  f.xb = fine ? 1 : 0;
  f.nv = (nx - f.xb + V - 1) / V;
  f.y0 = fine ? 1 : 0;
  f.nyr = fine ? ny - 2 : ny;
  f.z0 = (fine && D == 3) ? 1 : 0;
  f.nzr = (fine && D == 3) ? nz - 2 : nz;
  f.nvec = (int64_t)f.nv * f.nyr * f.nzr;
  f.nchunks = (int)((f.nvec + 255) / 256);
  f.per_xcd = (f.nchunks + kXCD - 1) / kXCD;
  return f;
}

// Chunk of this work group in a single-grid launch: each XCD gets one
// contiguous run of per_xcd chunks.
__device__ __forceinline__ int xcd_chunk(const Flat& f) {
  const int b = blockIdx.x;
  return (b % kXCD) * f.per_xcd + b / kXCD;
}

// Block index of an interface-node launch whose grid is a multiple of 8:
// each XCD serves one contiguous range, so spatially adjacent interface
// nodes (consecutive table entries) share one L2.
__device__ __forceinline__ int64_t xcd_block() {
  const int b = blockIdx.x, per = gridDim.x / kXCD;
  return (int64_t)(b % kXCD) * per + b / kXCD;
}

// First node x0 of this work-item's V-node vector in chunk `chunk`; false
// past the last vector.
// (The vector count of a level is below 2^31, checked on the host, so the
// index arithmetic is 32-bit.)
template <int V>
__device__ __forceinline__ bool flat_vec(const Flat& f, int chunk, int& x0, int& y, int& z) {
  if (chunk >= f.nchunks) return false;
  const uint32_t v = (uint32_t)chunk * 256u + threadIdx.x;
  if ((int64_t)v >= f.nvec) return false;
  const uint32_t r = v / (uint32_t)f.nv;
  x0 = f.xb + (int)(v - r * (uint32_t)f.nv) * V;
  const uint32_t zq = r / (uint32_t)f.nyr;
  y = f.y0 + (int)(r - zq * (uint32_t)f.nyr);
  z = f.z0 + (int)zq;
  return true;
}

// Loads the V values of one row of a plain array (the velocity planes)
// starting at x0 - cx.  Coarse rows are periodic: vectors that cross a row
// end are gathered element-wise.
template <typename S, int V, int LEVEL>
__device__ __forceinline__ typename VT<S, V>::a load_row(const S* __restrict__ row, int x0, int cx, int nx) {
  using VA = typename VT<S, V>::a;
  using VU = typename VT<S, V>::u;
  const int xs = x0 - cx;
  if (LEVEL == 0 && cx != 0 && (xs < 0 || xs + V > nx)) {
    VA v;
#pragma unroll
    for (int k = 0; k < V; ++k) v[k] = row[wrap(xs + k, nx)];
    return v;
  }
  if (cx == 0) return *(const VA*)(row + xs);
  return (VA)(*(const VU*)(row + xs));
}

// Addressing of the pull-stream of one V-node vector, computed once per lane:
// the position of x0 in each row of the (y, z) neighbourhood (periodic on the
// coarse level) and, per row, whether the +x / -x shifted load leaves the
// 16-byte vector path -- because it crosses a coarse row end (periodic wrap)
// or a storage block (the aligned vector of x0 starts or ends a block).
// All Q vector loads are issued first, without branches (a lane whose
// shifted load leaves the vector path reads its own aligned vector instead,
// which is always in bounds); the few such lanes then gather those
// populations element-wise.  Branching around each load instead makes the
// compiler wait for every outstanding load at each join, which leaves a wave
// with one load in flight.
template <typename S, int Q, int V, int LEVEL, int D>
struct Pull {
  static constexpr int NR = D == 3 ? 9 : 3;
  using VA = typename VT<S, V>::a;
  using VU = typename VT<S, V>::u;
  int64_t rb[NR];    // position of node x0 of row (dy, dz), r = (dy + 1) + 3 (dz + 1)
  uint32_t sm, sp;   // bit r: the load shifted by cx = +1 / -1 from row r is gathered
  int x0, nx;

  __device__ __forceinline__ Pull(int64_t P, int xo, int x0_, int y, int z, int nx_, int ny, int nz)
      : sm(0), sp(0), x0(x0_), nx(nx_) {
    constexpr int64_t BM = PopBlock<S>::B - 1;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      int ys = y + r % 3 - 1, zs = D == 3 ? z + r / 3 - 1 : z;
      if (LEVEL == 0) {
        ys = wrap(ys, ny);
        if (D == 3) zs = wrap(zs, nz);
      }
      rb[r] = P * ((int64_t)ys + (int64_t)ny * zs) + xo + x0;
      const int64_t o = rb[r] & BM;
      if ((LEVEL == 0 && x0 == 0) || o == 0) sm |= 1u << r;
      if ((LEVEL == 0 && x0 + V >= nx) || o == BM - V + 1) sp |= 1u << r;
    }
  }
  // row holding the node a population is pulled from (x - xi)
  template <int CY, int CZ>
  static constexpr int row() {
    return (1 - CY) + (D == 3 ? 3 * (1 - CZ) : 0);
  }
  template <int CX, int CY>
  __device__ __forceinline__ bool gathered(int r) const {
    return CX > 0 ? ((sm >> r) & 1u) : (CX < 0 ? ((sp >> r) & 1u) : false);
  }
  // Vector load of population q with velocity (cx, cy, cz); wrong for lanes
  // whose load is gathered (fixed by gather()).
  template <int CX, int CY, int CZ>
  __device__ __forceinline__ VA load(const S* __restrict__ src, int q) const {
    constexpr int r = row<CY, CZ>();
    const int64_t a = pop_at<S, Q>(rb[r], q);
    if (CX == 0) return *(const VA*)(src + a);
    // a lane that is not gathered stays inside the storage block of rb[r]
    return (VA)(*(const VU*)(src + (gathered<CX, CY>(r) ? a : a - CX)));
  }
  // Element-wise load for lanes whose shifted load is gathered.
  template <int CX, int CY, int CZ>
  __device__ __forceinline__ void gather(const S* __restrict__ src, int q, VA& v) const {
    if (CX == 0) return;
    constexpr int r = row<CY, CZ>();
    if (!gathered<CX, CY>(r)) return;
    const int64_t b = rb[r];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      int x = x0 + k - CX;
      if (LEVEL == 0) x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
      v[k] = src[pop_at<S, Q>(b - x0 + x, q)];
    }
  }
  // All Q populations of the V nodes.
  template <typename Lat>
  __device__ __forceinline__ void load_all(const S* __restrict__ src, VA* v) const {
    static_for<Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      v[i] = load<Lat::cx(i), Lat::cy(i), Lat::cz(i)>(src, i);
    });
    if (sm | sp) {
      static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        gather<Lat::cx(i), Lat::cy(i), Lat::cz(i)>(src, i, v[i]);
      });
    }
  }
};

// A stored population in double (adds back the weight when the storage holds
// deviations) and the reverse.
template <typename S, bool DEV, int LAT>
__device__ __forceinline__ double full_pop(S v, int i) {
  return (double)v + (DEV ? Lattice<LAT>::w(i) : 0.0);
}
template <typename S, bool DEV, int LAT>
__device__ __forceinline__ S store_pop(double f, int i) {
  return (S)(f - (DEV ? Lattice<LAT>::w(i) : 0.0));
}

// Coarse vectors lying wholly inside the covered box are not evolved.
template <int LEVEL>
__device__ __forceinline__ bool skip_vec(const Geo& g, int x0, int V, int y, int z, int nx) {
  if (LEVEL == 1 || !g.has_fine) return false;
  const int xl = min(x0 + V - 1, nx - 1);
  return coarse_class(g, x0, y, z) == CC_COVERED && coarse_class(g, xl, y, z) == CC_COVERED;
}

// ---------------------------------------------------------------------------
// Bulk pull-stream (+ collide) of one level.
//   LEVEL 0: coarse, periodic.  LEVEL 1: fine patch.
// MODEL BGK/RR: dst = collide(pull(src)).  MODEL HRR: only mac = (rho, u) of
// the pulled state (padded planes of the level); dst is not touched.
// Every node of a processed vector is written, including coarse TN/covered
// nodes and the fine ring column x = nx - 1: the schedule overwrites TN and
// ring nodes afterwards and never reads covered ones.
// With xb set (fine level, the first substep of the two-launch D3Q19 path)
// the results of middle nodes in the x-bands also go to the compact band copy
// (xband_at), which the fine-to-coarse transfer reads.
// SENS (BGK, RR): the NH sensors' velocity record of the state this call
// leaves, the moments of the stored post-collision values in double (as
// k_sens_vel takes them), into the planes su ([1 + D][padded positions]).
template <int LAT, bool DEV, typename S, int MODEL, int LEVEL, bool NT, bool SENS = false>
__device__ __forceinline__ void stream_body(const S* __restrict__ src, S* __restrict__ dst, S* __restrict__ mac, const Geo& g,
                                   const Flat& fl, const S om, int chunk, S* __restrict__ xb = nullptr,
                                   double* __restrict__ su = nullptr) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V;
  using VA = typename VT<S, V>::a;
  constexpr int Q = L::Q;
  int x0, y, z;
  if (!flat_vec<V>(fl, chunk, x0, y, z)) return;
  const int nx = fl.nx, ny = fl.ny, nz = fl.nz;
  if (skip_vec<LEVEL>(g, x0, V, y, z, nx)) return;
  const int64_t P = LEVEL == 0 ? g.pc : g.pf;
  const int64_t NP = LEVEL == 0 ? g.Ncp : g.Nfp;
  const int xo = LEVEL == 0 ? 0 : g.fxo;
  const Pull<S, Q, V, LEVEL, L::D> pl(P, xo, x0, y, z, nx, ny, nz);
  VA v[Q];
  pl.template load_all<L>(src, v);
  const int64_t own = pl.rb[Pull<S, Q, V, LEVEL, L::D>::template row<0, 0>()];
  if (MODEL == M_HRR) {
    VA r, ux, uy, uz;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      S s[Q], rho, r0, u[3];
#pragma unroll
      for (int i = 0; i < Q; ++i) s[i] = v[i][k];
      N::moments(s, rho, r0, u);
      r[k] = rho;
      ux[k] = u[0];
      uy[k] = u[1];
      uz[k] = u[2];
    }
    vstore<NT>((VA*)(mac + own), r);
    vstore<NT>((VA*)(mac + NP + own), ux);
    vstore<NT>((VA*)(mac + 2 * NP + own), uy);
    if (L::D == 3) vstore<NT>((VA*)(mac + 3 * NP + own), uz);
    return;
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      S s[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) s[i] = v[i][k];
      N::collide(s, MODEL, om, S(0), S(0), nullptr);
#pragma unroll
      for (int i = 0; i < Q; ++i) v[i][k] = s[i];
      if constexpr (SENS) {
        if (x0 + k <= nx - 1) {
          double f[Q], r, r0, u[3];
#pragma unroll
          for (int i = 0; i < Q; ++i) f[i] = full_pop<S, DEV, LAT>(s[i], i);
          Node<LAT, false, double>::moments(f, r, r0, u);
#pragma unroll
          for (int d = 0; d < L::D; ++d) su[(int64_t)(1 + d) * NP + own + k] = u[d];
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) vstore<NT>((VA*)(dst + pop_at<S, Q>(own, i)), v[i]);
  if (LEVEL == 1 && xb && (x0 <= 4 || x0 + V - 1 >= nx - 5)) {
    // A vector wholly inside a band goes out as one 16-byte store per
    // population (it may hold the ring column x = nx - 1: the ring
    // reconstruction, which runs next, rewrites every population of it that
    // is read); otherwise node by node, middle nodes only.
    using VU = typename VT<S, V>::u;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int xo0 = side == 0 ? x0 : x0 - (nx - 5);
      if (xo0 >= 0 && xo0 + V - 1 <= 4 && x0 + V - 1 <= nx - 1) {
#pragma unroll
        for (int i = 0; i < Q; ++i) *(VU*)(xb + xband_at(g, Q, side, i, y, z, xo0)) = (VU)v[i];
      } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const int xo = xo0 + k;
          if (xo < 0 || xo > 4 || x0 + k > nx - 2) continue;
#pragma unroll
          for (int i = 0; i < Q; ++i) xb[xband_at(g, Q, side, i, y, z, xo)] = v[i][k];
        }
      }
    }
  }
}

template <int LAT, bool DEV, typename S, int MODEL, int LEVEL, bool NT>
__global__ __launch_bounds__(256) void k_stream(const S* __restrict__ src, S* __restrict__ dst, S* __restrict__ mac,
                                                const Geo g, const Flat fl, const S om, S* __restrict__ xb) {
  stream_body<LAT, DEV, S, MODEL, LEVEL, NT>(src, dst, mac, g, fl, om, xcd_chunk(fl), xb);
}

// H-RR pull-stream and collision of a level: dst = collide(pull(src)) with
// the strain rate from centred differences (second order, level lattice
// units) of the velocity planes of mac (Sec. 3.3), which the first pass and
// the interface kernels filled.  Processes whole vectors like k_stream; the
// coarse pass runs before the fine-to-coarse transfer overwrites TN nodes.
//
// DYN: sigma per node from the non-hydrodynamic sensors (a variant Sec. 9.3
// and Sec. 11 suggest): the divergence and curl of this collision's velocity
// gradient are compared with those of the node's previous collision on the
// level, kept in dyn ([4][NP]: divergence, then the curl's 1 or 3
// components); a product below -dthr (the SpuriousAc / SpuriousS tests of
// Sec. 7, the 3D curl as a dot product) takes sig_dyn, otherwise sig.  The
// products are formed without contraction, as the tests define them.
template <int LAT, bool DEV, typename S, int LEVEL, bool NT, bool DYN = false>
__device__ __forceinline__ void collide_hrr_body(const S* __restrict__ src, S* __restrict__ dst, const S* __restrict__ mac,
                                        const Geo& g, const Flat& fl, const S om, const S tau, const S sig,
                                        int chunk, S* __restrict__ dyn = nullptr, const S sig_dyn = S(0),
                                        const S dthr = S(0)) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V;
  using VA = typename VT<S, V>::a;
  constexpr int Q = L::Q, D = L::D;
  int x0, y, z;
  if (!flat_vec<V>(fl, chunk, x0, y, z)) return;
  const int nx = fl.nx, ny = fl.ny, nz = fl.nz;
  if (skip_vec<LEVEL>(g, x0, V, y, z, nx)) return;
  const int64_t P = LEVEL == 0 ? g.pc : g.pf;
  const int64_t NP = LEVEL == 0 ? g.Ncp : g.Nfp;
  const int xo = LEVEL == 0 ? 0 : g.fxo;
  using PL = Pull<S, Q, V, LEVEL, D>;
  const PL pl(P, xo, x0, y, z, nx, ny, nz);
  const int64_t own = pl.rb[PL::template row<0, 0>()];
  // velocity gradient: gr[a][b] = (u_b(x + e_a) - u_b(x - e_a)) / 2; the
  // velocity planes are plain padded planes with the rows of pl
  // the x-neighbours cross a row end only on the coarse level's first and
  // last vectors (periodic): those lanes read their own vector, then gather
  const bool xlo = LEVEL == 0 && x0 == 0, xhi = LEVEL == 0 && x0 + V >= nx;
  VA gr[3][3];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const S* ub = mac + (int64_t)(1 + b) * NP;
    using VU = typename VT<S, V>::u;
    VA up = (VA)(*(const VU*)(ub + own + (xhi ? 0 : 1)));
    VA um = (VA)(*(const VU*)(ub + own - (xlo ? 0 : 1)));
    if (xlo || xhi) {
      const S* rowc = ub + own - x0;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        up[k] = rowc[wrap(x0 + k + 1, nx)];
        um[k] = rowc[wrap(x0 + k - 1, nx)];
      }
    }
    gr[0][b] = (up - um) * S(0.5);
    gr[1][b] = (*(const VA*)(ub + pl.rb[PL::template row<-1, 0>()]) - *(const VA*)(ub + pl.rb[PL::template row<1, 0>()])) *
               S(0.5);
    if (D == 3)
      gr[2][b] = (*(const VA*)(ub + pl.rb[PL::template row<0, -1>()]) -
                  *(const VA*)(ub + pl.rb[PL::template row<0, 1>()])) *
                 S(0.5);
  }
  VA v[Q];
  pl.template load_all<L>(src, v);
  // DYN: the node's previous divergence and curl, then this collision's
  constexpr int NC = D == 2 ? 1 : 3;
  VA pv[1 + NC], cv[1 + NC];
  if constexpr (DYN) {
#pragma unroll
    for (int c = 0; c <= NC; ++c) pv[c] = *(const VA*)(dyn + (int64_t)c * NP + own);
    cv[0] = gr[0][0] + gr[1][1];
    if constexpr (D == 3) {
      cv[0] = cv[0] + gr[2][2];
      cv[1] = gr[1][2] - gr[2][1];
      cv[2] = gr[2][0] - gr[0][2];
      cv[3] = gr[0][1] - gr[1][0];
    } else {
      cv[1] = gr[0][1] - gr[1][0];
    }
#pragma unroll
    for (int c = 0; c <= NC; ++c) *(VA*)(dyn + (int64_t)c * NP + own) = cv[c];
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {
    Sym<S> Sr;
    Sr.xx = gr[0][0][k];
    Sr.yy = gr[1][1][k];
    Sr.xy = S(0.5) * (gr[0][1][k] + gr[1][0][k]);
    if (D == 3) {
      Sr.zz = gr[2][2][k];
      Sr.xz = S(0.5) * (gr[0][2][k] + gr[2][0][k]);
      Sr.yz = S(0.5) * (gr[1][2][k] + gr[2][1][k]);
    } else {
      Sr.zz = Sr.xz = Sr.yz = S(0);
    }
    S sg = sig;
    if constexpr (DYN) {
      const S pd = mul_rn(pv[0][k], cv[0][k]);
      S pc = mul_rn(pv[1][k], cv[1][k]);
#pragma unroll
      for (int c = 2; c <= NC; ++c) pc = pc + mul_rn(pv[c][k], cv[c][k]);
      if (pd < -dthr || pc < -dthr) sg = sig_dyn;
    }
    S s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = v[i][k];
    N::collide(s, M_HRR, om, tau, sg, &Sr);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i][k] = s[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) vstore<NT>((VA*)(dst + pop_at<S, Q>(own, i)), v[i]);
}

template <int LAT, bool DEV, typename S, int LEVEL, bool NT, bool DYN = false>
__global__ __launch_bounds__(256) void k_collide_hrr(const S* __restrict__ src, S* __restrict__ dst,
                                                     const S* __restrict__ mac, const Geo g, const Flat fl, const S om,
                                                     const S tau, const S sig, S* __restrict__ dyn, const S sig_dyn,
                                                     const S dthr) {
  collide_hrr_body<LAT, DEV, S, LEVEL, NT, DYN>(src, dst, mac, g, fl, om, tau, sig, xcd_chunk(fl), dyn, sig_dyn, dthr);
}

// ---------------------------------------------------------------------------
// Interface data.  History fields per coarse history node, double precision:
// rho, u[D], the pre-collision non-equilibrium part, and (H-RR) S[NS].  The
// non-equilibrium part is kept in full (f1[Q]) for BGK, whose collision keeps
// every non-equilibrium moment.  RR and H-RR rebuild ring and TN nodes from
// rho, u and the second-order moment a1 = sum_i H2_i f1_i only: the
// interpolation, rescaling and filtering are linear and f1 carries no mass or
// momentum, so transferring a1 (NS components) gives the same populations as
// transferring f1 and projecting afterwards.
template <int LAT, int MODEL>
struct HF {
  static constexpr int D = Lattice<LAT>::D, Q = Lattice<LAT>::Q;
  static constexpr int NSC = NS<D>::value;
  static constexpr int NF1 = MODEL == M_BGK ? Q : NSC;
  static constexpr int RHO = 0, U = 1, F1 = 1 + D, S = 1 + D + NF1;
  static constexpr int N = 1 + D + NF1 + (MODEL == M_HRR ? NSC : 0);
};

// Symmetric tensor <-> its NS stored components (xx, yy, xy | xx, yy, zz, xy,
// xz, yz).
template <int D>
__device__ __forceinline__ void sym_put(const Sym<double>& a, double* out, double scale) {
  out[0] = scale * a.xx;
  out[1] = scale * a.yy;
  if (D == 2) {
    out[2] = scale * a.xy;
  } else {
    out[2] = scale * a.zz;
    out[3] = scale * a.xy;
    out[4] = scale * a.xz;
    out[5] = scale * a.yz;
  }
}
template <int D>
__device__ __forceinline__ Sym<double> sym_get(const double* v, double scale) {
  Sym<double> a{0, 0, 0, 0, 0, 0};
  a.xx = scale * v[0];
  a.yy = scale * v[1];
  if (D == 2) {
    a.xy = scale * v[2];
  } else {
    a.zz = scale * v[2];
    a.xy = scale * v[3];
    a.xz = scale * v[4];
    a.yz = scale * v[5];
  }
  return a;
}

// Second-order non-equilibrium moment of full populations f with moments
// rho, u (eq a1Proj with the third-order equilibrium).
template <int LAT>
__device__ __forceinline__ Sym<double> a1_of(const double* f, double rho, const double* u) {
  using N = Node<LAT, false, double>;
  const Sym<double> P = N::second(f);
  const double r3 = rho * (1.0 / 3.0);
  Sym<double> a;
  a.xx = P.xx - r3 - rho * u[0] * u[0];
  a.yy = P.yy - r3 - rho * u[1] * u[1];
  a.zz = Lattice<LAT>::D == 3 ? P.zz - r3 - rho * u[2] * u[2] : 0.0;
  a.xy = P.xy - rho * u[0] * u[1];
  a.xz = Lattice<LAT>::D == 3 ? P.xz - rho * u[0] * u[2] : 0.0;
  a.yz = Lattice<LAT>::D == 3 ? P.yz - rho * u[1] * u[2] : 0.0;
  return a;
}

// H-RR stress mix of eq a1ij_HRR: a <- sig a + (1 - sig)(-2 tau rho c_s^2 S).
__device__ __forceinline__ Sym<double> hrr_mix(const Sym<double>& a, const Sym<double>& S, double sig, double tau, double rho) {
  const double k = (1.0 - sig) * (-2.0 / 3.0) * tau * rho;
  return Sym<double>{sig * a.xx + k * S.xx, sig * a.yy + k * S.yy, sig * a.zz + k * S.zz,
                     sig * a.xy + k * S.xy, sig * a.xz + k * S.xz, sig * a.yz + k * S.yz};
}

struct Iface {
  int64_t NH;
  const int64_t* hnode;  // [NH] coarse node (logical index) of each history entry
  int64_t NR;
  const int64_t* rnode;  // [NR] fine node (logical index) of each ring entry
  const int32_t* rnp;    // [NR] stencil points (1, 4, 16)
  const int32_t* rpt;    // [NR][16] history entries
  int64_t NT;
  const int64_t* tnf;    // [NT] fine TN nodes (logical)
  const int64_t* tnc;    // [NT] coarse TN nodes (logical)
};

// Temporal interpolation of a history value to t+1/2 (eq TempInt):
// -1/8 H(t-1) + 3/4 H(t) + 3/8 H(t+1).
__device__ __forceinline__ double time_half(double hm, double h0, double hp) {
  return -0.125 * hm + 0.75 * h0 + 0.375 * hp;
}

// Pre-collision state of coarse history nodes at t+1 (pulled from the
// post-collision coarse state at t): rho, u and the non-equilibrium part.
// With G set (BGK, RR: every field is known here) each value is also
// interpolated to t+1/2 from the two older levels Hm, H0 into G.
template <int LAT, bool DEV, typename S, int MODEL>
__device__ __forceinline__ void hist_capture_body(const S* __restrict__ src, double* __restrict__ H, const Geo& g,
                                         const Iface& itf, int64_t h, double* __restrict__ G = nullptr,
                                         const double* __restrict__ Hm = nullptr,
                                         const double* __restrict__ H0 = nullptr) {
  using L = Lattice<LAT>;
  using F = HF<LAT, MODEL>;
  using N = Node<LAT, false, double>;
  constexpr int Q = L::Q;
  if (h >= itf.NH) return;
  int x, y, z;
  cdecode(g, itf.hnode[h], x, y, z);
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  double f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int xs = wrap(x - L::cx(i), nx), ys = wrap(y - L::cy(i), ny);
    const int zs = L::D == 3 ? wrap(z - L::cz(i), nz) : 0;
    f[i] = full_pop<S, DEV, LAT>(src[pop_at<S, Q>(cpos(g, xs, ys, zs), i)], i);
  }
  double rho, r0, u[3];
  N::moments(f, rho, r0, u);
  const int64_t NH = itf.NH;
  auto put = [&](int field, double v) {
    const int64_t k = (int64_t)field * NH + h;
    H[k] = v;
    if (G) G[k] = time_half(Hm[k], H0[k], v);
  };
  put(F::RHO, rho);
#pragma unroll
  for (int d = 0; d < L::D; ++d) put(F::U + d, u[d]);
  if (MODEL == M_BGK) {
    double f0[Q];
    N::feq(rho, r0, u, f0);
#pragma unroll
    for (int i = 0; i < Q; ++i) put(F::F1 + i, f[i] - f0[i]);
  } else {
    double a[NS<L::D>::value];
    sym_put<L::D>(a1_of<LAT>(f, rho, u), a, 1.0);
#pragma unroll
    for (int k = 0; k < NS<L::D>::value; ++k) put(F::F1 + k, a[k]);
  }
}
template <int LAT, bool DEV, typename S, int MODEL>
__global__ void k_hist_capture(const S* __restrict__ src, double* __restrict__ H, const Geo g, const Iface itf,
                               double* __restrict__ G, const double* __restrict__ Hm, const double* __restrict__ H0) {
  hist_capture_body<LAT, DEV, S, MODEL>(src, H, g, itf, xcd_block() * blockDim.x + threadIdx.x, G, Hm, H0);
}


// H-RR: coarse strain rate at t+1 on the history nodes, by centred
// differences of the coarse velocity planes (TN entries come from the
// fictitious propagation on the fine level).
// With PULL (the one-pass coarse H-RR path, which writes no velocity
// planes) the velocities of the neighbours are the moments of their pulled
// coarse state, computed here exactly as the velocity pass would (TN nodes:
// the planes, where the fictitious propagation stored them).
template <int LAT, bool DEV, typename T, bool PULL>
__device__ __forceinline__ T hist_u(const T* __restrict__ src, const T* __restrict__ mac_c, const Geo& g, int x, int y,
                                    int z, int b) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, T>;
  constexpr int Q = L::Q;
  const int64_t ip = cpos(g, x, y, z);
  if (!PULL || coarse_class(g, x, y, z) == CC_TN) return mac_c[(1 + b) * g.Ncp + ip];
  T f[Q], rho, r0, u[3];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int xs = wrap(x - L::cx(i), g.n[0]), ys = wrap(y - L::cy(i), g.n[1]);
    const int zs = L::D == 3 ? wrap(z - L::cz(i), g.n[2]) : 0;
    f[i] = src[pop_at<T, Q>(cpos(g, xs, ys, zs), i)];
  }
  N::moments(f, rho, r0, u);
  return u[b];
}
template <int LAT, bool DEV, typename T, bool PULL>
__device__ __forceinline__ void hist_strain_body(const T* __restrict__ src, const T* __restrict__ mac_c,
                                                 double* __restrict__ H, const Geo& g, const Iface& itf, int64_t h) {
  using L = Lattice<LAT>;
  using F = HF<LAT, M_HRR>;
  constexpr int D = L::D;
  if (h >= itf.NH) return;
  int x, y, z;
  cdecode(g, itf.hnode[h], x, y, z);
  const int n3[3] = {g.n[0], g.n[1], g.n[2]};
  double gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < D; ++a) {
    int cp[3] = {x, y, z}, cm[3] = {x, y, z};
    cp[a] = wrap(cp[a] + 1, n3[a]);
    cm[a] = wrap(cm[a] - 1, n3[a]);
    for (int b = 0; b < D; ++b)
      gr[a][b] = 0.5 * ((double)hist_u<LAT, DEV, T, PULL>(src, mac_c, g, cp[0], cp[1], cp[2], b) -
                        (double)hist_u<LAT, DEV, T, PULL>(src, mac_c, g, cm[0], cm[1], cm[2], b));
  }
  const Sym<double> S{gr[0][0], gr[1][1], gr[2][2], 0.5 * (gr[0][1] + gr[1][0]), 0.5 * (gr[0][2] + gr[2][0]),
                      0.5 * (gr[1][2] + gr[2][1])};
  double v[NS<D>::value];
  sym_put<D>(S, v, 1.0);
  const int64_t NH = itf.NH;
#pragma unroll
  for (int k = 0; k < NS<D>::value; ++k) H[(F::S + k) * NH + h] = v[k];
}


// H-RR: the coarse strain rate of history node h (hist_strain_body), then
// the temporal interpolation of all of that node's fields to t+1/2
// (time_half) -- one thread per history node, one launch for both.
template <int LAT, bool DEV, typename T, bool PULL>
__global__ void k_hist_strain_time(const T* __restrict__ src, const T* __restrict__ mac_c, const double* __restrict__ Hm,
                                   const double* __restrict__ H0, double* __restrict__ Hp, double* __restrict__ G,
                                   const Geo g, const Iface itf) {
  using F = HF<LAT, M_HRR>;
  const int64_t h = xcd_block() * blockDim.x + threadIdx.x;
  if (h >= itf.NH) return;
  hist_strain_body<LAT, DEV, T, PULL>(src, mac_c, Hp, g, itf, h);
#pragma unroll
  for (int f = 0; f < F::N; ++f) {
    const int64_t k = (int64_t)f * itf.NH + h;
    G[k] = time_half(Hm[k], H0[k], Hp[k]);
  }
}


__device__ __forceinline__ double cubic_w(int s) { return (s == 1 || s == 2) ? 9.0 / 16.0 : -1.0 / 16.0; }

// Spatial weight of point s of a ring stencil (eq spaceInt; tensor product on
// 3D face centres, first odd axis fastest).
__device__ __forceinline__ double ring_w(int np, int s) {
  if (np == 1) return 1.0;
  if (np == 4) return cubic_w(s);
  return cubic_w(s & 3) * cubic_w(s >> 2);
}

// Ring nodes, rho and u only (H-RR needs them before the fine collision).
// Temporal weights c applied inline to the three history levels.
template <int LAT, typename T>
__device__ __forceinline__ void ring_macro_body(const double* __restrict__ Hm, const double* __restrict__ H0,
                                       const double* __restrict__ Hp, double c0, double c1, double c2,
                                       T* __restrict__ mac_f, const Geo& g, const Iface& itf, int64_t r) {
  using L = Lattice<LAT>;
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
  int x, y, z;
  fdecode(g, itf.rnode[r], x, y, z);
  const int64_t fi = fpos(g, x, y, z);
#pragma unroll
  for (int k = 0; k < 1 + L::D; ++k) mac_f[(int64_t)k * g.Nfp + fi] = (T)v[k];
}
template <int LAT, typename T>
__global__ void k_ring_macro(const double* __restrict__ Hm, const double* __restrict__ H0,
                             const double* __restrict__ Hp, double c0, double c1, double c2,
                             T* __restrict__ mac_f, const Geo g, const Iface itf) {
  ring_macro_body<LAT, T>(Hm, H0, Hp, c0, c1, c2, mac_f, g, itf, xcd_block() * blockDim.x + threadIdx.x);
}


// Ring nodes: rho, u, the non-equilibrium part (and S) interpolated from the
// (time-interpolated) history G; populations rebuilt as f0(rho, u) +
// tau_f/(2 tau_c) f1 (eq rescff), S^f = S^c / 2 (eq PijResc), collided with
// tau_f and stored.  RR / H-RR evaluate the post-collision state directly
// from rho, u and the rescaled a1.
// PARTIAL: only the populations that stream into a middle node (x + xi
// inside [1, nf - 2] on every axis) are stored -- the only ones the stepping
// reads; on the x-normal faces each stored value is a lone write into its own
// cache line, so skipping the others saves most of this kernel's traffic.
// The full state is rebuilt from the same history level before it can be
// observed (ring completion), with bitwise the same values.
// With xb set (the t+1/2 ring of the two-launch D3Q19 path) ring nodes in
// the x-bands also store the same populations into the compact band copy.
template <int LAT, bool DEV, typename S, int MODEL, bool PARTIAL>
__device__ __forceinline__ void ring_body(const double* __restrict__ G, S* __restrict__ dst, const Geo& g, const Iface& itf,
                                 double kf, double om_f, double tau_f, double sig, int64_t r,
                                 S* __restrict__ xb = nullptr) {
  using L = Lattice<LAT>;
  using F = HF<LAT, MODEL>;
  using N = Node<LAT, false, double>;
  constexpr int Q = L::Q, D = L::D;
  if (r >= itf.NR) return;
  const int np = itf.rnp[r];
  const int32_t* pt = itf.rpt + 16 * r;
  const int64_t NH = itf.NH;
  double v[F::N];
#pragma unroll
  for (int k = 0; k < F::N; ++k) v[k] = 0.0;
  for (int s = 0; s < np; ++s) {
    const int64_t h = pt[s];
    const double ws = ring_w(np, s);
#pragma unroll
    for (int k = 0; k < F::N; ++k) v[k] += ws * G[(int64_t)k * NH + h];
  }
  const double rho = v[F::RHO];
  double u[3] = {v[F::U], v[F::U + 1], D == 3 ? v[F::U + 2] : 0.0};
  double f[Q];
  if (MODEL == M_BGK) {
    N::feq(rho, rho, u, f);
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] += kf * v[F::F1 + i];
    N::collide(f, M_BGK, om_f, tau_f, sig, nullptr);
  } else {
    Sym<double> a = sym_get<D>(v + F::F1, kf);
    if (MODEL == M_HRR) a = hrr_mix(a, sym_get<D>(v + F::S, 0.5), sig, tau_f, rho);
    N::eval(N::coef(rho, rho, u, om_f, a), f);
  }
  int x, y, z;
  fdecode(g, itf.rnode[r], x, y, z);
  const int64_t fi = fpos(g, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (PARTIAL) {
      const int xs = x + L::cx(i), ys = y + L::cy(i), zs = z + L::cz(i);
      bool in = xs >= 1 && xs <= g.nf[0] - 2 && ys >= 1 && ys <= g.nf[1] - 2;
      if (D == 3) in = in && zs >= 1 && zs <= g.nf[2] - 2;
      if (!in) continue;
    }
    const S sv = store_pop<S, DEV, LAT>(f[i], i);
    dst[pop_at<S, Q>(fi, i)] = sv;
    if (xb) {
      if (x <= 4) xb[xband_at(g, Q, 0, i, y, z, x)] = sv;
      if (x >= g.nf[0] - 5) xb[xband_at(g, Q, 1, i, y, z, x - (g.nf[0] - 5))] = sv;
    }
  }
}
template <int LAT, bool DEV, typename S, int MODEL, bool PARTIAL>
__global__ void k_ring(const double* __restrict__ G, S* __restrict__ dst, const Geo g, const Iface itf,
                       double kf, double om_f, double tau_f, double sig) {
  ring_body<LAT, DEV, S, MODEL, PARTIAL>(G, dst, g, itf, kf, om_f, tau_f, sig,
                                         xcd_block() * blockDim.x + threadIdx.x);
}

// H-RR: the t+1/2 ring populations (as k_ring, from G into dst) and the
// t+1 ring velocities (as k_ring_macro with weights (0, 0, 1), into mac_f)
// in one launch of two XCD-contiguous halves of `half` blocks each: they
// read the history and write disjoint buffers.
template <int LAT, bool DEV, typename S, int MODEL>
__global__ void k_ring_half_macro(const double* __restrict__ G, S* __restrict__ dst, const double* __restrict__ Hm,
                                  const double* __restrict__ H0, const double* __restrict__ Hp, S* __restrict__ mac_f,
                                  const Geo g, const Iface itf, double kf, double om_f, double tau_f, double sig,
                                  int half) {
  const int part = (int)blockIdx.x >= half;
  const int b = (int)blockIdx.x - part * half, per = half / kXCD;
  const int64_t r = ((int64_t)(b % kXCD) * per + b / kXCD) * blockDim.x + threadIdx.x;
  if (part == 0) ring_body<LAT, DEV, S, MODEL, true>(G, dst, g, itf, kf, om_f, tau_f, sig, r);
  else ring_macro_body<LAT, S>(Hm, H0, Hp, 0.0, 0.0, 1.0, mac_f, g, itf, r);
}


// Pull of Q populations into fine node (x, y, z) from a fine buffer.
template <int LAT, bool DEV, typename S>
__device__ __forceinline__ void pull_fine(const S* __restrict__ src, const Geo& g, int x, int y, int z, double* f,
                                          const S* __restrict__ xb = nullptr) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  // nodes whose pulls stay inside an x-band read the compact band copy
  const int side = !xb ? -1 : (x <= 3 ? 0 : (x >= g.nf[0] - 4 ? 1 : -1));
  const int xb0 = side == 1 ? g.nf[0] - 5 : 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int xs = x - L::cx(i), ys = y - L::cy(i), zs = z - L::cz(i);
    const S v = side >= 0 ? xb[xband_at(g, Q, side, i, ys, zs, xs - xb0)] : src[pop_at<S, Q>(fpos(g, xs, ys, zs), i)];
    f[i] = full_pop<S, DEV, LAT>(v, i);
  }
}

// H-RR: fictitious propagation onto TN^f (Sec. 4.3, step e): u(TN, t+1) from
// the fine post-collision state at t+1/2, written to the coarse macro planes.
template <int LAT, bool DEV, typename S, typename T>
__device__ __forceinline__ void fict_body(const S* __restrict__ src_f, T* __restrict__ mac_c, const Geo& g, const Iface& itf,
                                 int64_t t) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  if (t >= itf.NT) return;
  int x, y, z;
  fdecode(g, itf.tnf[t], x, y, z);
  double f[L::Q], rho, r0, u[3];
  pull_fine<LAT, DEV, S>(src_f, g, x, y, z, f);
  N::moments(f, rho, r0, u);
  int cx, cy, cz;
  cdecode(g, itf.tnc[t], cx, cy, cz);
  const int64_t ci = cpos(g, cx, cy, cz);
  mac_c[ci] = (T)rho;
#pragma unroll
  for (int d = 0; d < L::D; ++d) mac_c[(int64_t)(1 + d) * g.Ncp + ci] = (T)u[d];
}
template <int LAT, bool DEV, typename S, typename T>
__global__ void k_fict(const S* __restrict__ src_f, T* __restrict__ mac_c, const Geo g, const Iface itf) {
  fict_body<LAT, DEV, S, T>(src_f, mac_c, g, itf, xcd_block() * blockDim.x + threadIdx.x);
}


// Fine-to-coarse transfer at TN (Sec. 4.3, synchronous step d).  The fine
// pre-collision state at t+1 around TN^f is re-pulled from the fine
// post-collision state at t+1/2; its non-equilibrium part (full f1 for BGK,
// a1 for RR / H-RR) is filtered with the tensor product of (1/4, 1/2, 1/4)
// (eq filterFneq), rescaled by 2 tau_c / tau_f (eq rescfc) and added to f0
// of the co-located fine node; H-RR takes S^c = 2 S^f (eq PijResc) with S^f
// by fine centred differences.  The coarse node is then collided with tau_c.
// One work group handles PER TN nodes: lane (stencil point s, TN node t),
// t fastest so neighbouring lanes read neighbouring nodes, computes the
// weighted non-equilibrium part of one stencil node into LDS; lanes per
// (TN node, component) sum the stencil in a fixed order; one lane per TN node
// rebuilds and collides.  SENS: the node's record for the NH sensors, as in
// stream_body.
template <int LAT, bool DEV, typename S, int MODEL, bool SENS = false>
__device__ __forceinline__ void coalesce_body(const S* __restrict__ src_f, S* __restrict__ dst_c, const Geo& g, const Iface& itf,
                                     double kc, double om_c, double tau_c, double sig, int64_t blk,
                                     const S* __restrict__ xb = nullptr, double* __restrict__ su = nullptr) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  using F = HF<LAT, MODEL>;
  constexpr int Q = L::Q, D = L::D;
  constexpr int NST = (D == 2) ? 9 : 27;
  constexpr int PER = 256 / NST;
  constexpr int CEN = (D == 2) ? 4 : 13;
  constexpr int NC = F::NF1;  // components filtered per stencil node
  __shared__ double sf1[PER][NST][NC];
  __shared__ double sm[PER][NST][4];
  __shared__ double sacc[PER][NC];
  __syncthreads();  // the LDS may still be read by a previous call in this work group
  const int lt = threadIdx.x % PER, s = threadIdx.x / PER;
  const int64_t t = blk * PER + lt;
  if (s < NST && t < itf.NT) {
    int x, y, z;
    fdecode(g, itf.tnf[t], x, y, z);
    const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = (D == 3) ? s / 9 - 1 : 0;
    double f[Q], rho, r0, u[3];
    pull_fine<LAT, DEV, S>(src_f, g, x + ox, y + oy, z + oz, f, xb);
    N::moments(f, rho, r0, u);
    const double w = (ox ? 0.25 : 0.5) * (oy ? 0.25 : 0.5) * (D == 3 ? (oz ? 0.25 : 0.5) : 1.0);
    if (MODEL == M_BGK) {
      double f0[Q];
      N::feq(rho, r0, u, f0);
#pragma unroll
      for (int i = 0; i < Q; ++i) sf1[lt][s][i] = w * (f[i] - f0[i]);
    } else {
      double a[NS<D>::value];
      sym_put<D>(a1_of<LAT>(f, rho, u), a, w);
#pragma unroll
      for (int k = 0; k < NC; ++k) sf1[lt][s][k] = a[k];
    }
    sm[lt][s][0] = rho;
    sm[lt][s][1] = u[0];
    sm[lt][s][2] = u[1];
    sm[lt][s][3] = u[2];
  }
  __syncthreads();
  for (int p = threadIdx.x; p < PER * NC; p += blockDim.x) {
    const int l2 = p / NC, q = p % NC;
    double acc = 0.0;
    for (int k = 0; k < NST; ++k) acc += sf1[l2][k][q];
    sacc[l2][q] = acc;
  }
  __syncthreads();
  if ((int)threadIdx.x >= PER) return;
  const int l3 = threadIdx.x;
  const int64_t t3 = blk * PER + l3;
  if (t3 >= itf.NT) return;
  const double rc = sm[l3][CEN][0];
  double uc[3] = {sm[l3][CEN][1], sm[l3][CEN][2], sm[l3][CEN][3]};
  double f[Q];
  if (MODEL == M_BGK) {
    N::feq(rc, rc, uc, f);
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] += kc * sacc[l3][i];
    N::collide(f, M_BGK, om_c, tau_c, sig, nullptr);
  } else {
    Sym<double> a = sym_get<D>(sacc[l3], kc);
    if (MODEL == M_HRR) {
      // neighbours along +-x, +-y, +-z are stencil entries CEN +- 1, 3, 9
      const int st[3] = {1, 3, 9};
      double gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int aa = 0; aa < D; ++aa)
        for (int b = 0; b < D; ++b) gr[aa][b] = 0.5 * (sm[l3][CEN + st[aa]][1 + b] - sm[l3][CEN - st[aa]][1 + b]);
      const Sym<double> Sc{2.0 * gr[0][0],
                           2.0 * gr[1][1],
                           2.0 * gr[2][2],
                           2.0 * (0.5 * (gr[0][1] + gr[1][0])),
                           2.0 * (0.5 * (gr[0][2] + gr[2][0])),
                           2.0 * (0.5 * (gr[1][2] + gr[2][1]))};
      a = hrr_mix(a, Sc, sig, tau_c, rc);
    }
    N::eval(N::coef(rc, rc, uc, om_c, a), f);
  }
  int cx, cy, cz;
  cdecode(g, itf.tnc[t3], cx, cy, cz);
  const int64_t ci = cpos(g, cx, cy, cz);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const S st = store_pop<S, DEV, LAT>(f[i], i);
    dst_c[pop_at<S, Q>(ci, i)] = st;
    if constexpr (SENS) f[i] = full_pop<S, DEV, LAT>(st, i);
  }
  if constexpr (SENS) {
    double r, r0, u[3];
    N::moments(f, r, r0, u);
#pragma unroll
    for (int d = 0; d < D; ++d) su[(int64_t)(1 + d) * g.Ncp + ci] = u[d];
  }
}


// Coarse pull-stream + collide (BGK, RR) and the ring reconstruction at
// t+1/2 (G -> the fine buffer of half times) in one launch: independent work,
// the ring latency-bound and the stream bandwidth-bound, so the ring hides
// inside the stream.  Blocks [0, nrb) take 256 ring nodes each (dispatched
// first), the rest are the stream's chunks; both parts are XCD-contiguous.
// SENS: the stream also records the NH sensors' coarse velocities into su.
template <int LAT, bool DEV, typename S, int MODEL, bool NT, bool SENS = false>
__global__ __launch_bounds__(256) void k_stream_ring(const S* __restrict__ src, S* __restrict__ dst, const Geo g,
                                                     const Flat fl, const S om, const double* __restrict__ G,
                                                     S* __restrict__ fdst, const Iface itf, double kf, double om_f,
                                                     double tau_f, double sig, int nrb, S* __restrict__ xb,
                                                     double* __restrict__ su) {
  const int b = blockIdx.x;
  if (b < nrb) {
    const int per = nrb / kXCD;
    const int64_t blk = (int64_t)(b % kXCD) * per + b / kXCD;
    ring_body<LAT, DEV, S, MODEL, true>(G, fdst, g, itf, kf, om_f, tau_f, sig, blk * 256 + threadIdx.x, xb);
  } else {
    const int b2 = b - nrb;
    stream_body<LAT, DEV, S, MODEL, 0, NT, SENS>(src, dst, nullptr, g, fl, om, (b2 % kXCD) * fl.per_xcd + b2 / kXCD,
                                                 nullptr, su);
  }
}

// Ring reconstruction at t+1 (Hp -> the fine buffer of integer times,
// populations that stream inward) and the fine-to-coarse transfer (fine
// state at t+1/2 -> coarse TN) in one launch: they write disjoint buffers and
// read none of each other's outputs.  Blocks [0, nrb) take 256 ring nodes
// each, the rest PER TN nodes each; both parts are XCD-contiguous (nrb is a
// multiple of 8).  SENS: the transfer records the NH sensors' velocities of
// the TN nodes into su.
template <int LAT, bool DEV, typename S, int MODEL, bool SENS = false>
__global__ __launch_bounds__(256) void k_ring_coalesce(const double* __restrict__ Hp, S* __restrict__ fdst,
                                                       const S* __restrict__ src_f, S* __restrict__ dst_c,
                                                       const Geo g, const Iface itf, double kf, double om_f,
                                                       double tau_f, double kc, double om_c, double tau_c, double sig,
                                                       int nrb, const S* __restrict__ xb, double* __restrict__ su) {
  const int b = blockIdx.x;
  if (b < nrb) {
    const int per = nrb / kXCD;
    const int64_t blk = (int64_t)(b % kXCD) * per + b / kXCD;
    ring_body<LAT, DEV, S, MODEL, true>(Hp, fdst, g, itf, kf, om_f, tau_f, sig, blk * 256 + threadIdx.x);
  } else {
    const int b2 = b - nrb, per = ((int)gridDim.x - nrb) / kXCD;
    coalesce_body<LAT, DEV, S, MODEL, SENS>(src_f, dst_c, g, itf, kc, om_c, tau_c, sig,
                                            (int64_t)(b2 % kXCD) * per + b2 / kXCD, xb, su);
  }
}

// ---------------------------------------------------------------------------
// Both fine substeps of a coarse step in one kernel (D2Q9, BGK / RR).
// A work group owns a tile of TXV vectors x TY rows of middle nodes.  Substep
// 1 (t -> t+1/2) is computed into LDS for the tile and a one-node halo (one
// vector on each side, one row above and below): middle nodes pull from src
// and collide exactly as k_stream does; ring nodes take their t+1/2 values
// from `half`, where the ring reconstruction stored them.  Substep 2
// (t+1/2 -> t+1) then pulls from LDS and collides the tile, writing dst.  HBM
// sees one read and one write of the populations per fine node per coarse
// step instead of two of each; the arithmetic per node is that of two
// k_stream launches, so the results are bitwise the same.  The t+1/2 state of
// the middle nodes within 2 nodes of the TN line (where the fine-to-coarse
// transfer pulls) is also stored into `half`.
// Substep 1 of one vector (node x0 = 1 + V k of row y) into an LDS row
// (`row[i]` points at population i of that row, c0 the vector's first
// column).  Middle nodes pull from src and collide; ring nodes take their
// t+1/2 values from `half`; `band` asks to store the result of middle nodes
// within 2 nodes of the TN line into `half` as well.  SENS (the NH sensors'
// record of this iteration, for the lane that owns the vector, `band`):
// every middle node's result goes to `half` and the velocity of its pulled
// (pre-collision) populations to the double planes su ([1 + D][padded
// positions]), in the arithmetic of k_sens_vel.
template <int LAT, bool DEV, typename S, int MODEL, bool SENS = false>
__device__ __forceinline__ void fine2_s1(const S* __restrict__ src, S* __restrict__ half, const Geo& g, const S om,
                                         int k, int y, int nv, S* const* row, int c0, bool band,
                                         double* __restrict__ su = nullptr) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  using VA = typename VT<S, V>::a;
  const int nx = g.nf[0], ny = g.nf[1];
  const int x0 = 1 + V * k;
  if (y == 0 || y == ny - 1 || k == -1) {
    // ring row, or the vector ending at ring node x = 0
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int x = x0 + j;
      if (x < 0 || x > nx - 1) continue;
      const int64_t p = fpos(g, x, y, 0);
#pragma unroll
      for (int i = 0; i < Q; ++i) row[i][c0 + j] = half[pop_at<S, Q>(p, i)];
    }
    return;
  }
  const Pull<S, Q, V, 1, 2> pl(g.pf, g.fxo, x0, y, 0, nx, ny, 1);
  VA v[Q];
  pl.template load_all<L>(src, v);
  // a vector of middle nodes only (x0 .. x0 + V - 1 <= nx - 2): the SENS
  // records go out as whole vectors (positions of vector starts are
  // multiples of V)
  const bool whole = x0 + V - 1 <= nx - 2;
  if constexpr (SENS) {
    if (band) {
      typedef double DV __attribute__((ext_vector_type(V)));
      DV uv[2];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        double f[Q], r, r0, u[3];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = full_pop<S, DEV, LAT>(v[i][j], i);
        Node<LAT, false, double>::moments(f, r, r0, u);
        uv[0][j] = u[0];
        uv[1][j] = u[1];
      }
      const int64_t p0 = fpos(g, x0, y, 0);
      if (whole) {
#pragma unroll
        for (int d = 0; d < 2; ++d) *(DV*)(su + (int64_t)(1 + d) * g.Nfp + p0) = uv[d];
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
          if (x0 + j <= nx - 2)
#pragma unroll
            for (int d = 0; d < 2; ++d) su[(int64_t)(1 + d) * g.Nfp + p0 + j] = uv[d][j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) {
    S f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = v[i][j];
    N::collide(f, MODEL, om, S(0), S(0), nullptr);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i][j] = f[i];
  }
#pragma unroll
  for (int j = 0; j < V; ++j)
#pragma unroll
    for (int i = 0; i < Q; ++i) row[i][c0 + j] = v[i][j];
  if (k == nv - 1) {
    // the ring node x = nx - 1 inside the last vector of the row
    const int jr = nx - 1 - x0;
    const int64_t p = fpos(g, nx - 1, y, 0);
    if (jr >= 0 && jr < V)
#pragma unroll
      for (int i = 0; i < Q; ++i) row[i][c0 + jr] = half[pop_at<S, Q>(p, i)];
  }
  if (band) {
    if (SENS && whole) {
      const int64_t p0 = fpos(g, x0, y, 0);
#pragma unroll
      for (int i = 0; i < Q; ++i) vstore<false>((VA*)(half + pop_at<S, Q>(p0, i)), v[i]);
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int x = x0 + j;
        if (x > nx - 2 || (!SENS && !(x <= 4 || x >= nx - 5 || y <= 4 || y >= ny - 5))) continue;
        const int64_t p = fpos(g, x, y, 0);
#pragma unroll
        for (int i = 0; i < Q; ++i) half[pop_at<S, Q>(p, i)] = v[i][j];
      }
    }
  }
}

// Substep 2 of one vector (node x0 = 1 + V k of row y) from LDS: population i
// is read from the row holding y - cy_i (rows[1 - cy_i]) at column c0 + j -
// cx_i; the result is stored to dst.
template <int LAT, bool DEV, typename S, int MODEL, bool NT>
__device__ __forceinline__ void fine2_s2(S* __restrict__ dst, const Geo& g, const S om, int k, int y,
                                         S* const* rm, S* const* r0, S* const* rp, int c0) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  using VA = typename VT<S, V>::a;
  VA v[Q];
  static_for<Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    S* const* rows = L::cy(i) == 1 ? rm : (L::cy(i) == 0 ? r0 : rp);
#pragma unroll
    for (int j = 0; j < V; ++j) v[i][j] = rows[i][c0 + j - L::cx(i)];
  });
#pragma unroll
  for (int j = 0; j < V; ++j) {
    S f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = v[i][j];
    N::collide(f, MODEL, om, S(0), S(0), nullptr);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i][j] = f[i];
  }
  const int64_t own = fpos(g, 1 + V * k, y, 0);
#pragma unroll
  for (int i = 0; i < Q; ++i) vstore<NT>((VA*)(dst + pop_at<S, Q>(own, i)), v[i]);
}

// Tiles (k_fine2): a work group of HXV x HYR lanes owns the middle nodes of
// HXV - 2 vectors x HYR - 2 rows.  Each lane computes substep 1 of one
// vector of the tile or of its halo (one vector on each side, one row above
// and below) into LDS; after the barrier the inner lanes compute substep 2
// of their own vector.  One lane per vector: waves made only of halo lanes
// skip substep 2, and the halo costs (HXV HYR) / ((HXV - 2)(HYR - 2)) of the
// substep-1 work.  MINW asks the compiler to fit that many waves per SIMD.
// Tile `tile` (of ntx per row of tiles) of one grid; the whole work group
// calls it.
template <int LAT, bool DEV, typename S, int MODEL, bool NT, int HXV, int HYR, bool SENS = false>
__device__ __forceinline__ void fine2_tile(const S* __restrict__ src, S* __restrict__ dst, S* __restrict__ half,
                                           const Geo& g, const S om, int ntx, int tile,
                                           double* __restrict__ su = nullptr) {
  using L = Lattice<LAT>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  constexpr int TXV = HXV - 2, TY = HYR - 2, RW = HXV * V;
  static_assert(L::D == 2, "fused fine substeps are two-dimensional");
  static_assert((HXV * HYR) % 64 == 0 && HXV * HYR <= 1024, "whole waves");
  __shared__ S lds[Q][HYR][RW];
  const int tx = tile % ntx, ty = tile / ntx;
  const int ny = g.nf[1];
  const int nv = (g.nf[0] - 1 + V - 1) / V;
  const int t = threadIdx.x;
  const int rv = t % HXV, rr = t / HXV;
  const int k = tx * TXV - 1 + rv, y = ty * TY + rr;  // vector and row of this lane (k >= -1, y >= 0)
  const bool inner = rr >= 1 && rr <= TY && rv >= 1 && rv <= TXV;
  if (y <= ny - 1 && k < nv) {
    S* row[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) row[i] = &lds[i][rr][0];
    fine2_s1<LAT, DEV, S, MODEL, SENS>(src, half, g, om, k, y, nv, row, rv * V, inner, su);
  }
  __syncthreads();
  if (inner && k < nv && y <= ny - 2) {
    S *rm[Q], *r0[Q], *rp[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      rm[i] = &lds[i][rr - 1][0];
      r0[i] = &lds[i][rr][0];
      rp[i] = &lds[i][rr + 1][0];
    }
    fine2_s2<LAT, DEV, S, MODEL, NT>(dst, g, om, k, y, rm, r0, rp, rv * V);
  }
}

// Fine tiles per row of tiles and rows of tiles of a grid for HXV x HYR lanes.
template <typename S>
__host__ __device__ inline int fine2_ntx(const Geo& g, int HXV) {
  return ((g.nf[0] - 1 + VecOf<S>::V - 1) / VecOf<S>::V + HXV - 3) / (HXV - 2);
}
__host__ __device__ inline int fine2_nty(const Geo& g, int HYR) { return (g.nf[1] - 2 + HYR - 3) / (HYR - 2); }

// SENS: also the NH sensors' record of the t+1/2 iteration (fine2_s1) in su.
template <int LAT, bool DEV, typename S, int MODEL, bool NT, int HXV, int HYR, int MINW, bool SENS = false>
__global__ __launch_bounds__(HXV * HYR, MINW) void k_fine2(const S* __restrict__ src, S* __restrict__ dst,
                                                         S* __restrict__ half, const Geo g, const S om, int ntx,
                                                         int nty, int per_xcd, double* __restrict__ su) {
  const int b = blockIdx.x;
  const int tile = (b % kXCD) * per_xcd + b / kXCD;
  if (tile >= ntx * nty) return;  // whole work group, before any barrier
  fine2_tile<LAT, DEV, S, MODEL, NT, HXV, HYR, SENS>(src, dst, half, g, om, ntx, tile, su);
}

// The H-RR collision of one lane's vector in the D2Q9 one-pass kernels: the
// strain rate by centred differences of the LDS velocity rows (ux, uy rows
// rr - 1 .. rr + 1, the vector's columns c ..  c + V - 1), then the collision,
// in place on v.  DYN: sigma per node as collide_hrr_body takes it -- the
// node's previous divergence and curl from dyn ([4][np] in the storage
// type, at position own), this collision's stored back -- with the same
// arithmetic, so the one-pass and two-pass substeps agree bitwise.
template <int LAT, bool DEV, typename S, bool DYN, int RW>
__device__ __forceinline__ void dyn2_collide(typename VT<S, VecOf<S>::V>::a* v, const S (*ux)[RW], const S (*uy)[RW],
                                             int rr, int c, const S om, const S tau, const S sig,
                                             S* __restrict__ dyn, int64_t np, int64_t own, const S sig_dyn,
                                             const S dthr) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  using VA = typename VT<S, V>::a;
  VA pv[2], cv[2];
  if constexpr (DYN) {
#pragma unroll
    for (int k = 0; k < 2; ++k) pv[k] = *(const VA*)(dyn + (int64_t)k * np + own);
  }
#pragma unroll
  for (int j = 0; j < V; ++j) {
    // gr[a][b] = (u_b(x + e_a) - u_b(x - e_a)) / 2
    const S g00 = (ux[rr][c + j + 1] - ux[rr][c + j - 1]) * S(0.5);
    const S g01 = (uy[rr][c + j + 1] - uy[rr][c + j - 1]) * S(0.5);
    const S g10 = (ux[rr + 1][c + j] - ux[rr - 1][c + j]) * S(0.5);
    const S g11 = (uy[rr + 1][c + j] - uy[rr - 1][c + j]) * S(0.5);
    Sym<S> Sr;
    Sr.xx = g00;
    Sr.yy = g11;
    Sr.xy = S(0.5) * (g01 + g10);
    Sr.zz = Sr.xz = Sr.yz = S(0);
    S sg = sig;
    if constexpr (DYN) {
      cv[0][j] = g00 + g11;
      cv[1][j] = g01 - g10;
      const S pd = mul_rn(pv[0][j], cv[0][j]);
      const S pc = mul_rn(pv[1][j], cv[1][j]);
      if (pd < -dthr || pc < -dthr) sg = sig_dyn;
    }
    S f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = v[i][j];
    N::collide(f, M_HRR, om, tau, sg, &Sr);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i][j] = f[i];
  }
  if constexpr (DYN) {
#pragma unroll
    for (int k = 0; k < 2; ++k) *(VA*)(dyn + (int64_t)k * np + own) = cv[k];
  }
}

// ---------------------------------------------------------------------------
// One H-RR fine substep in one pass (D2Q9): a work group of HXV x HYR lanes,
// one lane per vector of a tile and its one-vector / one-row halo.  Every
// lane pulls its vector and takes the velocity of its nodes from the pulled
// moments (ring nodes: from the velocity planes, where the ring macro step
// stored them) into LDS; after the barrier the inner lanes take the strain
// rate by centred differences of the neighbouring velocities and collide
// their own pulled populations.  Same arithmetic as the velocity pass
// followed by k_collide_hrr, without the velocity planes' round trip through
// HBM and without pulling the populations twice.
template <int LAT, bool DEV, typename S, bool NT, int HXV, int HYR, bool DYN = false>
__device__ __forceinline__ void hrr2_tile(const S* __restrict__ src, S* __restrict__ dst, const S* __restrict__ mac,
                                          const Geo& g, const S om, const S tau, const S sig, int ntx, int tile,
                                          S* __restrict__ dyn = nullptr, const S sig_dyn = S(0),
                                          const S dthr = S(0)) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  using VA = typename VT<S, V>::a;
  constexpr int TXV = HXV - 2, TY = HYR - 2, RW = HXV * V;
  static_assert(L::D == 2, "the one-pass H-RR tile is two-dimensional");
  __shared__ S lu[2][HYR][RW];
  const int tx = tile % ntx, ty = tile / ntx;
  const int nx = g.nf[0], ny = g.nf[1];
  const int nv = (nx - 1 + V - 1) / V;
  const int64_t NP = g.Nfp;
  const int t = threadIdx.x;
  const int rv = t % HXV, rr = t / HXV;
  const int k = tx * TXV - 1 + rv, y = ty * TY + rr;  // vector and row of this lane (k >= -1, y >= 0)
  const int x0 = 1 + V * k;
  const bool inner = rr >= 1 && rr <= TY && rv >= 1 && rv <= TXV && k < nv && y <= ny - 2;
  const bool mid = y >= 1 && y <= ny - 2 && k >= 0 && k < nv;
  VA v[Q];
  if (mid) {
    const Pull<S, Q, V, 1, 2> pl(g.pf, g.fxo, x0, y, 0, nx, ny, 1);
    pl.template load_all<L>(src, v);
    VA ux, uy;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      S f[Q], rho, r0, u[3];
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = v[i][j];
      N::moments(f, rho, r0, u);
      ux[j] = u[0];
      uy[j] = u[1];
    }
    if (k == nv - 1) {
      // the ring node x = nx - 1 inside the last vector of the row
      const int jr = nx - 1 - x0;
      const int64_t p = fpos(g, nx - 1, y, 0);
      const S rx = mac[NP + p], ry = mac[2 * NP + p];
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (j == jr) {
          ux[j] = rx;
          uy[j] = ry;
        }
    }
    *(VA*)&lu[0][rr][rv * V] = ux;
    *(VA*)&lu[1][rr][rv * V] = uy;
  } else if (y <= ny - 1 && k < nv) {
    // ring row, or the vector ending at ring node x = 0
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int x = x0 + j;
      if (x < 0 || x > nx - 1) continue;
      const int64_t p = fpos(g, x, y, 0);
      lu[0][rr][rv * V + j] = mac[NP + p];
      lu[1][rr][rv * V + j] = mac[2 * NP + p];
    }
  }
  __syncthreads();
  if (!inner) return;
  const int c = rv * V;
  const int64_t own = fpos(g, x0, y, 0);
  dyn2_collide<LAT, DEV, S, DYN>(v, lu[0], lu[1], rr, c, om, tau, sig, dyn, g.Nfp, own, sig_dyn, dthr);
#pragma unroll
  for (int i = 0; i < Q; ++i) vstore<NT>((VA*)(dst + pop_at<S, Q>(own, i)), v[i]);
}

// The coarse level in one pass (D2Q9 H-RR; rows a whole number of vectors):
// as hrr2_tile, periodic -- halo lanes take the wrapped neighbour vector and
// row -- with the velocity of TN nodes from the velocity planes (the
// fictitious propagation stored it there) and vectors wholly inside the
// covered box skipped, as k_collide_hrr does.
template <int LAT, bool DEV, typename S, bool NT, int HXV, int HYR, bool DYN = false>
__device__ __forceinline__ void hrr2c_tile(const S* __restrict__ src, S* __restrict__ dst, const S* __restrict__ mac,
                                           const Geo& g, const S om, const S tau, const S sig, int ntx, int tile,
                                           S* __restrict__ dyn = nullptr, const S sig_dyn = S(0),
                                           const S dthr = S(0)) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  using VA = typename VT<S, V>::a;
  constexpr int TXV = HXV - 2, TY = HYR - 2, RW = HXV * V;
  static_assert(L::D == 2, "the one-pass H-RR tile is two-dimensional");
  __shared__ S lu[2][HYR][RW];
  const int tx = tile % ntx, ty = tile / ntx;
  const int nx = g.n[0], ny = g.n[1];
  const int nv = nx / V;
  const int64_t NP = g.Ncp;
  const int t = threadIdx.x;
  const int rv = t % HXV, rr = t / HXV;
  const int kr = tx * TXV - 1 + rv, yr = ty * TY - 1 + rr;  // unwrapped vector and row (>= -1)
  const int k = (kr + nv) % nv, y = (yr + ny) % ny;          // a tile may be wider than the period
  const int x0 = V * k;
  const bool skip = skip_vec<0>(g, x0, V, y, 0, nx);
  const bool inner = rr >= 1 && rr <= TY && rv >= 1 && rv <= TXV && kr < nv && yr < ny && !skip;
  VA v[Q];
  // a skipped (wholly covered) vector stores zero velocities: only its TN
  // and covered neighbours read them (TN is rewritten by the transfer,
  // covered nodes are not evolved), but every slot a lane reads is defined
  VA ux = VA(S(0)), uy = VA(S(0));
  if (!skip) {
    const Pull<S, Q, V, 0, 2> pl(g.pc, 0, x0, y, 0, nx, ny, 1);
    pl.template load_all<L>(src, v);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (coarse_class(g, x0 + j, y, 0) == CC_TN) {
        const int64_t p = cpos(g, x0 + j, y, 0);
        ux[j] = mac[NP + p];
        uy[j] = mac[2 * NP + p];
      } else {
        S f[Q], rho, r0, u[3];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = v[i][j];
        N::moments(f, rho, r0, u);
        ux[j] = u[0];
        uy[j] = u[1];
      }
    }
  }
  *(VA*)&lu[0][rr][rv * V] = ux;
  *(VA*)&lu[1][rr][rv * V] = uy;
  __syncthreads();
  if (!inner) return;
  const int c = rv * V;
  const int64_t own = cpos(g, x0, y, 0);
  dyn2_collide<LAT, DEV, S, DYN>(v, lu[0], lu[1], rr, c, om, tau, sig, dyn, g.Ncp, own, sig_dyn, dthr);
#pragma unroll
  for (int i = 0; i < Q; ++i) vstore<NT>((VA*)(dst + pop_at<S, Q>(own, i)), v[i]);
}

// DYN: dynamic sigma (dyn, sig_dyn, dthr as for k_collide_hrr).
template <int LAT, bool DEV, typename S, bool NT, int HXV, int HYR, bool DYN = false>
__global__ __launch_bounds__(HXV * HYR) void k_hrr2c(const S* __restrict__ src, S* __restrict__ dst,
                                                     const S* __restrict__ mac, const Geo g, const S om, const S tau,
                                                     const S sig, int ntx, int nty, int per_xcd, S* __restrict__ dyn,
                                                     const S sig_dyn, const S dthr) {
  const int b = blockIdx.x;
  const int tile = (b % kXCD) * per_xcd + b / kXCD;
  if (tile >= ntx * nty) return;  // whole work group, before any barrier
  hrr2c_tile<LAT, DEV, S, NT, HXV, HYR, DYN>(src, dst, mac, g, om, tau, sig, ntx, tile, dyn, sig_dyn, dthr);
}

template <int LAT, bool DEV, typename S, bool NT, int HXV, int HYR, bool DYN = false>
__global__ __launch_bounds__(HXV * HYR) void k_hrr2(const S* __restrict__ src, S* __restrict__ dst,
                                                    const S* __restrict__ mac, const Geo g, const S om, const S tau,
                                                    const S sig, int ntx, int nty, int per_xcd, S* __restrict__ dyn,
                                                    const S sig_dyn, const S dthr) {
  const int b = blockIdx.x;
  const int tile = (b % kXCD) * per_xcd + b / kXCD;
  if (tile >= ntx * nty) return;  // whole work group, before any barrier
  hrr2_tile<LAT, DEV, S, NT, HXV, HYR, DYN>(src, dst, mac, g, om, tau, sig, ntx, tile, dyn, sig_dyn, dthr);
}

// ---------------------------------------------------------------------------
// Both fine substeps of a coarse step in one kernel, one node per lane
// (D3Q19, BGK / RR: k_fine3s).  A work group of TXH x TYH lanes holds the
// columns of a tile of (TXH - 2) x (TYH - 2) middle nodes and its one-node
// halo in x and y, lane (hx, hy) at x = tx (TXH - 2) + hx, y = ty (TYH - 2) +
// hy, and walks a run of zlen planes along z.  The iteration for plane z:
//   * every lane takes substep 1 (t -> t+1/2) of its node in plane z+1:
//     middle nodes collide the populations they pulled one iteration earlier
//     (the pulls of plane z+2 are issued first, so their latency overlaps
//     this arithmetic); ring nodes take the t+1/2 values the ring
//     reconstruction stored in `half`;
//   * the 16 populations that move in x or y go to an LDS exchange plane,
//     each with the time offset its z velocity asks for (cz = -1: plane
//     z+1, just computed; cz = 0: plane z; cz = +1: plane z-1 -- every lane
//     keeps its own column's values in registers until their turn);
//   * after one barrier the inner lanes take substep 2 (t+1/2 -> t+1) of
//     plane z: moving populations from the neighbours' slots, the three that
//     move only along z (rest, +z, -z) from their own registers.
// Two exchange planes alternate, so one barrier per plane suffices.  Every
// node's arithmetic is that of k_stream, so the result is bitwise the
// two-launch one.  One node per lane keeps a lane's registers to the
// populations of one column (the four-node lanes of an earlier design needed
// 227 registers and ran at two waves per SIMD), and the x halo is one node
// wide.  The t+1/2 state of middle nodes within 4 nodes of a patch face (what
// the fine-to-coarse transfer pulls) is stored: in the x-bands into the
// compact band copy `xb` (xband_at, rows 5 values apart, so a tile's band
// fills whole cache lines instead of a partial line per row and
// population), in the y- and z-bands into `half`; the t+1/2 ring
// reconstruction fills both, and a ring column x = 0 / nx - 1 away from the
// z faces reads the populations it sends inward from `xb`.
template <int LAT>
struct ZSets {
  using L = Lattice<LAT>;
  __host__ __device__ static constexpr bool moving(int i) { return L::cx(i) != 0 || L::cy(i) != 0; }
  __host__ __device__ static constexpr int count(int i, int cz) {
    int s = 0;
    for (int k = 0; k < i; ++k) s += (moving(k) && (cz == 2 || L::cz(k) == cz)) ? 1 : 0;
    return s;
  }
  __host__ __device__ static constexpr int slot(int i) { return count(i, 2); }  // exchange slot of a moving population
  __host__ __device__ static constexpr int uidx(int i) { return count(i, 1); }  // among moving, cz = +1
  __host__ __device__ static constexpr int midx(int i) { return count(i, 0); }  // among moving, cz = 0
  static constexpr int NS = count(L::Q, 2), NU = count(L::Q, 1), NM = count(L::Q, 0);
};

// Addressing inside the storage window of a marching kernel's run.  The run
// touches planes [z0, z1] of the fine level; relative to the storage block
// holding the first position of plane z0, every population element of those
// planes lies below 2^32 bytes (the host sizes runs so that it does).  The
// window is addressed through a buffer resource: an access is one 32-bit
// byte offset per lane (the node's position) plus a per-population offset
// held in a scalar register, so it costs no vector arithmetic beyond the
// position's offset.  With the array-of-SoA layout, population i of position
// pb0 + d sits at byte  sizeof(S) ((Q B) (d >> SH) + (d & (B - 1)) + i B)
// past the window's first element, population 0 of position pb0.
template <typename S, int Q>
struct Window {
  static constexpr int SH = PopBlock<S>::SHIFT;
  static constexpr uint32_t B = (uint32_t)PopBlock<S>::B;
  int64_t pb0;  // first position of the window (block-aligned)
  __device__ __forceinline__ explicit Window(int64_t first) : pb0((first >> SH) << SH) {}
  // byte offset of population 0 of window position d
  __device__ __forceinline__ static uint32_t boff(uint32_t d) {
    return (uint32_t)sizeof(S) * d + (uint32_t)sizeof(S) * (uint32_t)(Q - 1) * B * (d >> SH);
  }
  // byte offset of population i relative to population 0
  __device__ __forceinline__ static constexpr int poff(int i) { return (int)(sizeof(S) * B) * i; }
  // Buffer resource over the window of a population buffer.  Its range is
  // 2^31 bytes (the host sizes runs so that the window fits): a lane whose
  // offset is moved past it by kOff reads 0 and writes nothing, which masks
  // a lane without a branch.
  static constexpr uint32_t kOff = 0x80000000u;
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const S* buf) const {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(buf + (int64_t)Q * pb0), (short)0, (int)kOff, 0x00020000);
  }
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __device__ __forceinline__ static S load(__amdgpu_buffer_rsrc_t r, uint32_t bo, int i) {
    if constexpr (sizeof(S) == 4)
      return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, (int)bo, poff(i), 0));
    else
      return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, (int)bo, poff(i), 0));
  }
  // NT: non-temporal store (the streamed state is not read again soon)
  template <bool NT>
  __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t bo, int i, S v) {
    if constexpr (sizeof(S) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)bo, poff(i), NT ? 2 : 0);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)bo, poff(i), NT ? 2 : 0);
  }
};

template <int LAT, bool DEV, typename S, int MODEL, bool NT, int TXH, int TYH, int MINW>
__global__ __launch_bounds__(TXH * TYH, MINW) void k_fine3s(const S* __restrict__ src, S* __restrict__ dst,
                                                            S* __restrict__ half, S* __restrict__ xb, const Geo g,
                                                            const S om, int ntx, int nty, int nzc, int zlen,
                                                            int per_xcd) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  using C = ZSets<LAT>;
  constexpr int Q = L::Q, NL = TXH * TYH;
  static_assert(L::D == 3, "the marching fused kernel is three-dimensional");
  static_assert(NL <= 1024 && 2 * C::NS * NL * sizeof(S) <= 160 * 1024, "one work group per CU at most");
  static_assert(C::NS == 16 && C::NU == 4 && C::NM == 8, "D3Q19 population classes");
  __shared__ S lds[2][C::NS][NL];
  const int b = blockIdx.x;
  const int item = (b % kXCD) * per_xcd + b / kXCD;
  const int ntile = ntx * nty;
  if (item >= ntile * nzc) return;  // whole work group, before any barrier
  const int zc = item / ntile, tile = item - zc * ntile;
  const int tx = tile % ntx, ty = tile / ntx;
  const int nx = g.nf[0], ny = g.nf[1], nz = g.nf[2];
  const int t = threadIdx.x;
  const int hx = t % TXH, hy = t / TXH;
  const int x = tx * (TXH - 2) + hx, y = ty * (TYH - 2) + hy;
  const bool live = x <= nx - 1 && y <= ny - 1;
  const bool inner = live && hx >= 1 && hx <= TXH - 2 && hy >= 1 && hy <= TYH - 2 && x <= nx - 2 && y <= ny - 2;
  const bool xyring = live && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  const bool near = x <= 4 || x >= nx - 5 || y <= 4 || y >= ny - 5;
  // Wave modes (wave-uniform bits): 1 full -- the ring values of every
  // population from `half` and the band there (ring rows, or both ring
  // columns, in the wave; planes within 5 of a z face); else 2 / 4 the ring
  // column x = 0 / nx - 1 reads the populations it sends inward from the
  // compact x-band copy, 32 the y-band goes to `half`; always 8 / 16 the
  // x-band goes to the compact copy (from which the transfer reads it).
  const bool xs0 = inner && x <= 4, xs1 = inner && x >= nx - 5;
  const bool w_r0 = __any(live && x == 0) != 0, w_r1 = __any(live && x == nx - 1) != 0;
  const bool w_full = __any(live && (y == 0 || y == ny - 1)) != 0 || (w_r0 && w_r1);
  const int wbits = __builtin_amdgcn_readfirstlane((w_full ? 1 : 0) | (w_r0 ? 2 : 0) | (w_r1 ? 4 : 0) |
                                                   (__any(xs0) != 0 ? 8 : 0) | (__any(xs1) != 0 ? 16 : 0) |
                                                   (__any(inner && (y <= 4 || y >= ny - 5)) != 0 ? 32 : 0));
  const int zs = 1 + zc * zlen, ze = min(zs + zlen - 1, nz - 2);
  // The run computes planes zs - 1 .. ze + 1, whose pulls reach planes
  // zs - 2 .. ze + 2: the window starts at row 0 of plane max(zs - 2, 0);
  // d0 = this lane's node in plane zs - 1.  Every load and store below is
  // issued by every lane (masked lanes get an offset past the window), so
  // the number of memory operations per plane is the same on every path and
  // the loads of the next plane stay in flight across the barrier and the
  // stores of this one.
  using Wn = Window<S, Q>;
  const Wn W(fpos(g, 0, 0, max(zs - 2, 0)));
  const __amdgpu_buffer_rsrc_t rs = W.rsrc(src), rh = W.rsrc(half), rd = W.rsrc(dst);
  const uint32_t py = (uint32_t)g.pf, pz = (uint32_t)g.pf * (uint32_t)ny;
  const uint32_t d0 = live ? (uint32_t)(fpos(g, x, y, zs - 1) - W.pb0) : 0u;
  const uint32_t mlive = live ? 0u : Wn::kOff;      // offset mask of dead lanes
  const uint32_t mpull = (live && !xyring) ? 0u : Wn::kOff;
  const uint32_t mring = xyring ? 0u : Wn::kOff;
  const uint32_t minner = inner ? 0u : Wn::kOff;
  // the compact x-band copy (xband_at: [side][population][z][y][x offset])
  // through a buffer resource with the same masking
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void*)xb, (short)0, (int)Wn::kOff, 0x00020000);
  const int xpop = (int)sizeof(S) * 5 * ny * nz;  // bytes between populations of one side
  const uint32_t xzb = (uint32_t)sizeof(S) * 5u * (uint32_t)ny;  // bytes per plane
  const uint32_t xside = (uint32_t)xpop * (uint32_t)Q;            // bytes between the sides
  const uint32_t xo0 = (uint32_t)sizeof(S) * (uint32_t)(5 * y + x);
  const uint32_t xo1 = xside + (uint32_t)sizeof(S) * (uint32_t)(5 * y + x - (nx - 5));
  const uint32_t mr0 = (live && x == 0) ? 0u : Wn::kOff, mr1 = (live && x == nx - 1) ? 0u : Wn::kOff;
  auto xload = [&](uint32_t bo, int i) __attribute__((always_inline)) -> S {
    if constexpr (sizeof(S) == 4)
      return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(rx, (int)bo, i * xpop, 0));
    else
      return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(rx, (int)bo, i * xpop, 0));
  };
  auto xstore = [&](uint32_t bo, int i, S v) __attribute__((always_inline)) {
    if constexpr (sizeof(S) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rx, (int)bo, i * xpop, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(typename Wn::u2, v), rx, (int)bo, i * xpop, 0);
  };
  S U0[C::NU], U1[C::NU], M[C::NM], R = S(0), Z0 = S(0), Z1 = S(0);
#pragma unroll
  for (int i = 0; i < C::NU; ++i) U0[i] = U1[i] = S(0);
#pragma unroll
  for (int i = 0; i < C::NM; ++i) M[i] = S(0);
  // Every memory operation below is issued by every lane, every plane, and
  // never under a branch (a lane that has nothing to load or store gets an
  // offset past the window): the compiler's count of outstanding operations
  // is then the same on every path, so it waits for the loads of a plane
  // without waiting for the stores issued after them.  The price is one
  // masked load of the ring values and one masked store of the band per
  // population and plane in every wave.
  S P[Q], PR[Q];
  // Loads of substep 1 for plane zp (window position d of this lane's node):
  // pulls of middle nodes from src into P, t+1/2 values of ring nodes (ring
  // planes, columns and rows) from `half` into PR.
  auto load = [&](int zp, uint32_t d, int mode) __attribute__((always_inline)) {
    const bool pring = zp == 0 || zp == nz - 1;
    const uint32_t mp = pring ? Wn::kOff : mpull;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      P[i] = Wn::load(rs, Wn::boff(d - L::cx(i) - py * L::cy(i) - pz * L::cz(i)) | mp, i);
    if (mode & 1) {
      const uint32_t bo = Wn::boff(d) | (pring ? mlive : mring);
#pragma unroll
      for (int i = 0; i < Q; ++i) PR[i] = Wn::load(rh, bo, i);
    } else {
      const uint32_t zb = (uint32_t)zp * xzb;
      if (mode & 2) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          if (L::cx(i) == 1) PR[i] = xload((zb + (uint32_t)sizeof(S) * (uint32_t)(5 * y)) | mr0, i);
      }
      if (mode & 4) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          if (L::cx(i) == -1) PR[i] = xload((xside + zb + (uint32_t)sizeof(S) * (uint32_t)(5 * y + 4)) | mr1, i);
      }
    }
  };
  // Substep 1 of plane zl (window position dl) into T from the loads issued
  // one plane earlier (ring nodes take PR by a bitwise blend: a select
  // became a select of array addresses, which kept the arrays in scratch
  // memory); the t+1/2 state of inner middle nodes within 4 nodes of a face
  // goes to `half`.
  using U = typename std::conditional<sizeof(S) == 4, uint32_t, uint64_t>::type;
  // (outside a full plane a ring lane takes only the populations it sends
  // inward; no inner lane reads its others)
  auto take = [&](int zl, S* T, int mode) __attribute__((always_inline)) {
    const bool pring = zl == 0 || zl == nz - 1;
    const U mk = (xyring || pring) ? ~U(0) : U(0);
    const U m0 = (mode & 1) ? mk : U(0), mp1 = (mode & 3) ? mk : U(0), mm1 = (mode & 5) ? mk : U(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const U mi = L::cx(i) == 1 ? mp1 : (L::cx(i) == -1 ? mm1 : m0);
      T[i] = __builtin_bit_cast(S, (__builtin_bit_cast(U, PR[i]) & mi) | (__builtin_bit_cast(U, P[i]) & ~mi));
    }
  };
  auto s1 = [&](int zl, uint32_t dl, S* T, int mode) __attribute__((always_inline)) {
    const bool pring = zl == 0 || zl == nz - 1;
    if (live && !xyring && !pring) N::collide(T, MODEL, om, S(0), S(0), nullptr);
    const bool own = inner && !pring && zl >= zs && zl <= ze;
    if (mode & 33) {
      const bool st = own && (near || zl <= 4 || zl >= nz - 5);
      const uint32_t bo = Wn::boff(dl) | (st ? 0u : Wn::kOff);
#pragma unroll
      for (int i = 0; i < Q; ++i) Wn::template store<false>(rh, bo, i, T[i]);
    }
    const uint32_t zb = (uint32_t)zl * xzb;
    if (mode & 8) {
      const uint32_t bo = (zb + xo0) | (own && xs0 ? 0u : Wn::kOff);
#pragma unroll
      for (int i = 0; i < Q; ++i) xstore(bo, i, T[i]);
    }
    if (mode & 16) {
      const uint32_t bo = (zb + xo1) | (own && xs1 ? 0u : Wn::kOff);
#pragma unroll
      for (int i = 0; i < Q; ++i) xstore(bo, i, T[i]);
    }
  };
  // the planes move up by one
  auto shift = [&](const S* T) __attribute__((always_inline)) {
    static_for<Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int mi = C::midx(i), ui = C::uidx(i), cz = L::cz(i);
      constexpr bool mv = C::moving(i);
      if constexpr (mv && cz == 1) {
        U1[ui] = U0[ui];
        U0[ui] = T[i];
      } else if constexpr (mv && cz == 0) {
        M[mi] = T[i];
      } else if constexpr (!mv && cz == 0) {
        R = T[i];
      } else if constexpr (!mv && cz == 1) {
        Z1 = Z0;
        Z0 = T[i];
      }
    });
  };
  // planes zs - 1 and zs: substep 1 only
  {
    S T[Q];
    load(zs - 1, d0, wbits | 1);
    take(zs - 1, T, wbits | 1);
    load(zs, d0 + pz, wbits | 1);
    s1(zs - 1, d0, T, wbits | 1);
    shift(T);
    take(zs, T, wbits | 1);
    load(zs + 1, d0 + 2 * pz, wbits | 1);
    s1(zs, d0 + pz, T, wbits | 1);
    shift(T);
  }
  int buf = 0;
  for (int z = zs; z <= ze; ++z) {
    const int zl = z + 1;
    // planes zl in [5, nz - 6] are not full (nor those their loads are for,
    // in [6, nz - 5]; the ring values of a plane are loaded by the mode of the
    // iteration before, which is full for zl <= 5 and zl >= nz - 4)
    const int mode = (z <= 3 || z >= nz - 6) ? (wbits | 1) : wbits;
    const uint32_t dl = d0 + (uint32_t)(zl - zs + 1) * pz;  // window position of (x, y, zl)
    // the loads of plane zl (issued one plane earlier) into T; the band
    // stores of plane zl, then the loads of plane zl + 1 out (plane zl again
    // past the run's last plane), so that only the stores of this plane's
    // substep 2 follow the loads a wave waits for
    S T[Q];
    take(zl, T, mode);
    s1(zl, dl, T, mode);
    const int zn = zl + 1 <= ze + 1 ? zl + 1 : zl;
    load(zn, dl + (uint32_t)(zn - zl) * pz, mode);
    // (slot and register indices are forced to compile-time constants:
    // used directly as array indices, the counting loops behind them were
    // left to run on the device)
    static_for<Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (C::moving(i)) {
        constexpr int sl = C::slot(i), mi = C::midx(i), ui = C::uidx(i), cz = L::cz(i);
        S w;
        if constexpr (cz == -1) w = T[i];
        else if constexpr (cz == 0) w = M[mi];
        else w = U1[ui];
        lds[buf][sl][t] = w;
      }
    });
    __syncthreads();
    S f[Q];
    if (inner) {
      static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cz = L::cz(i);
        if constexpr (C::moving(i)) {
          constexpr int sl = C::slot(i), off = L::cx(i) + TXH * L::cy(i);
          f[i] = lds[buf][sl][t - off];
        } else if constexpr (cz == 0) {
          f[i] = R;
        } else if constexpr (cz == 1) {
          f[i] = Z1;
        } else {
          f[i] = T[i];
        }
      });
      N::collide(f, MODEL, om, S(0), S(0), nullptr);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = S(0);
    }
    const uint32_t bo = Wn::boff(dl - pz) | minner;  // (x, y, z)
#pragma unroll
    for (int i = 0; i < Q; ++i) Wn::template store<NT>(rd, bo, i, f[i]);
    buf ^= 1;
    shift(T);
  }
}

// ---------------------------------------------------------------------------
// One H-RR fine substep in one pass with one node per lane (D3Q19, k_hrr3s).
// A work group of TXH x TYH lanes holds the columns of a tile of (TXH - 2) x
// (TYH - 2) middle nodes and its one-node halo and walks a run of zlen planes
// along z.  The iteration for plane z takes the populations of plane z+1,
// pulled two iterations earlier, computes their velocities (ring nodes: from
// the velocity planes, where the ring macro step stored them) into one of
// four LDS velocity planes and issues the pulls of plane z+3 into the
// registers they leave (two planes of pulls in flight: two register sets,
// the loop unrolled by two); after one barrier the inner lanes take the
// strain rate of plane z by centred
// differences from the planes of z-1, z and z+1 and collide the populations
// of plane z they kept from the previous iteration.  Four velocity planes
// rotate, so the plane written in one iteration is never one read in the
// iteration before, and one barrier per plane suffices.  Every memory
// operation is issued by every lane (masked lanes get offsets past the
// window), so the loads of a plane stay in flight across the stores of the
// one before.  Same arithmetic as the velocity pass followed by
// k_collide_hrr, so bitwise the same.
template <int LAT, bool DEV, typename S, bool NT, int TXH, int TYH, int MINW>
__global__ __launch_bounds__(TXH * TYH, MINW) void k_hrr3s(const S* __restrict__ src, S* __restrict__ dst,
                                                           const S* __restrict__ mac, const Geo g, const S om,
                                                           const S tau, const S sig, int ntx, int nty, int nzc,
                                                           int zlen, int per_xcd) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int Q = L::Q, NL = TXH * TYH;
  static_assert(L::D == 3, "the marching one-pass H-RR kernel is three-dimensional");
  static_assert(NL <= 1024, "one work group");
  __shared__ S lu[4][3][NL];  // [plane slot][component][lane]
  const int b = blockIdx.x;
  const int item = (b % kXCD) * per_xcd + b / kXCD;
  const int ntile = ntx * nty;
  if (item >= ntile * nzc) return;  // whole work group, before any barrier
  const int zc = item / ntile, tile = item - zc * ntile;
  const int tx = tile % ntx, ty = tile / ntx;
  const int nx = g.nf[0], ny = g.nf[1], nz = g.nf[2];
  const int t = threadIdx.x;
  const int hx = t % TXH, hy = t / TXH;
  const int x = tx * (TXH - 2) + hx, y = ty * (TYH - 2) + hy;
  const bool live = x <= nx - 1 && y <= ny - 1;
  const bool inner = live && hx >= 1 && hx <= TXH - 2 && hy >= 1 && hy <= TYH - 2 && x <= nx - 2 && y <= ny - 2;
  const bool xyring = live && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  const int zs = 1 + zc * zlen, ze = min(zs + zlen - 1, nz - 2);
  // storage window of the run (pulls reach planes zs - 2 .. ze + 2); the
  // velocity planes are addressed from the same first position
  using Wn = Window<S, Q>;
  const Wn W(fpos(g, 0, 0, max(zs - 2, 0)));
  const __amdgpu_buffer_rsrc_t rs = W.rsrc(src), rd = W.rsrc(dst);
  const __amdgpu_buffer_rsrc_t rm =
      __builtin_amdgcn_make_buffer_rsrc((void*)(mac + W.pb0), (short)0, (int)Wn::kOff, 0x00020000);
  const int mplane = (int)(g.Nfp * (int64_t)sizeof(S));  // bytes between velocity planes
  const uint32_t py = (uint32_t)g.pf, pz = (uint32_t)g.pf * (uint32_t)ny;
  const uint32_t d0 = live ? (uint32_t)(fpos(g, x, y, zs - 1) - W.pb0) : 0u;  // node in plane zs - 1
  const uint32_t mpull = (live && !xyring) ? 0u : Wn::kOff;
  const uint32_t minner = inner ? 0u : Wn::kOff;
  S H[Q], P0[Q], P1[Q], U0[3], U1[3];
  // pulls of plane zp (window position d) into P; velocities of ring nodes
  // (ring planes, columns and rows) from the velocity planes into UR
  auto load = [&](int zp, uint32_t d, S (&P)[Q], S (&UR)[3]) __attribute__((always_inline)) {
    const bool pring = zp == 0 || zp == nz - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      P[i] = Wn::load(rs, Wn::boff(d - L::cx(i) - py * L::cy(i) - pz * L::cz(i)) | (pring ? Wn::kOff : mpull), i);
    const uint32_t mo = (uint32_t)sizeof(S) * d | ((pring && live) || xyring ? 0u : Wn::kOff);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if constexpr (sizeof(S) == 4)
        UR[k] = __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(rm, (int)mo, (1 + k) * mplane, 0));
      else
        UR[k] = __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(rm, (int)mo, (1 + k) * mplane, 0));
    }
  };
  // velocity of the loaded plane zp into its LDS slot; its populations into H
  auto put = [&](int zp, const S (&P)[Q], const S (&UR)[3]) __attribute__((always_inline)) {
    const bool ring = xyring || zp == 0 || zp == nz - 1;
    S rho, r0, u[3];
    N::moments(P, rho, r0, u);
    using U = typename std::conditional<sizeof(S) == 4, uint32_t, uint64_t>::type;
    const U mk = ring ? ~U(0) : U(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const S v = __builtin_bit_cast(S, (__builtin_bit_cast(U, UR[k]) & mk) | (__builtin_bit_cast(U, u[k]) & ~mk));
      lu[zp & 3][k][t] = live ? v : S(0);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) H[i] = P[i];
  };
  // planes zs - 1 (velocities) and zs (velocities and populations), the
  // pulls of planes zs + 1 and zs + 2 out (two planes in flight)
  load(zs - 1, d0, P0, U0);
  put(zs - 1, P0, U0);
  load(zs, d0 + pz, P0, U0);
  put(zs, P0, U0);
  load(zs + 1, d0 + 2 * pz, P0, U0);
  {
    const int zn = zs + 2 <= ze + 1 ? zs + 2 : ze + 1;
    load(zn, d0 + (uint32_t)(zn - zs + 1) * pz, P1, U1);
  }
  auto iter = [&](int z, S (&Pu)[Q], S (&Uu)[3]) __attribute__((always_inline)) {
    const uint32_t dz = d0 + (uint32_t)(z - zs + 1) * pz;  // window position of (x, y, z)
    S Hc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) Hc[i] = H[i];
    put(z + 1, Pu, Uu);
    // pulls of plane z + 3 (plane ze + 1 again past the run's last plane)
    const int zn = z + 3 <= ze + 1 ? z + 3 : ze + 1;
    load(zn, d0 + (uint32_t)(zn - zs + 1) * pz, Pu, Uu);
    __syncthreads();
    if (inner) {
      const int sm = (z - 1) & 3, s0 = z & 3, sp = (z + 1) & 3;
      S gr[3][3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        gr[0][d] = (lu[s0][d][t + 1] - lu[s0][d][t - 1]) * S(0.5);
        gr[1][d] = (lu[s0][d][t + TXH] - lu[s0][d][t - TXH]) * S(0.5);
        gr[2][d] = (lu[sp][d][t] - lu[sm][d][t]) * S(0.5);
      }
      Sym<S> Sr;
      Sr.xx = gr[0][0];
      Sr.yy = gr[1][1];
      Sr.xy = S(0.5) * (gr[0][1] + gr[1][0]);
      Sr.zz = gr[2][2];
      Sr.xz = S(0.5) * (gr[0][2] + gr[2][0]);
      Sr.yz = S(0.5) * (gr[1][2] + gr[2][1]);
      N::collide(Hc, M_HRR, om, tau, sig, &Sr);
    }
    const uint32_t bo = Wn::boff(dz) | minner;
#pragma unroll
    for (int i = 0; i < Q; ++i) Wn::template store<NT>(rd, bo, i, Hc[i]);
  };
  for (int z = zs; z <= ze; z += 2) {
    iter(z, P0, U0);
    if (z + 1 <= ze) iter(z + 1, P1, U1);
  }
}

// ---------------------------------------------------------------------------
// One H-RR fine substep in one pass (D3Q19, k_hrr3): a work group owns TXV
// vectors x TY rows of a run of zlen planes and walks it along z, one lane per
// vector of the tile and its x/y halo.  The iteration for plane z pulls plane
// z+1 into registers and writes its velocities into one of three LDS plane
// slots (ring nodes: from the velocity planes, where the ring macro step
// stored them); after the barrier the inner lanes take the strain rate of
// plane z from the three slots and collide the populations they pulled one
// iteration earlier.  Same arithmetic as the velocity pass followed by
// k_collide_hrr.
template <int LAT, bool DEV, typename S>
__device__ __forceinline__ void hrr3_pull(const S* __restrict__ src, const S* __restrict__ mac, const Geo& g, int k,
                                          int y, int z, int nv, typename VT<S, VecOf<S>::V>::a* P,
                                          typename VT<S, VecOf<S>::V>::a* u) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  const int nx = g.nf[0], ny = g.nf[1], nz = g.nf[2];
  const int64_t NP = g.Nfp;
  const int x0 = 1 + V * k;
  if (y == 0 || y == ny - 1 || z == 0 || z == nz - 1 || k == -1) {
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int x = x0 + j;
      const bool in = x >= 0 && x <= nx - 1;
      const int64_t p = fpos(g, in ? x : 0, y, z);
#pragma unroll
      for (int d = 0; d < 3; ++d) u[d][j] = in ? mac[(int64_t)(1 + d) * NP + p] : S(0);
    }
    return;
  }
  const Pull<S, Q, V, 1, 3> pl(g.pf, g.fxo, x0, y, z, nx, ny, nz);
  pl.template load_all<L>(src, P);
#pragma unroll
  for (int j = 0; j < V; ++j) {
    S f[Q], rho, r0, uu[3];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = P[i][j];
    N::moments(f, rho, r0, uu);
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d][j] = uu[d];
  }
  if (k == nv - 1) {
    const int jr = nx - 1 - x0;
    const int64_t p = fpos(g, nx - 1, y, z);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const S r = mac[(int64_t)(1 + d) * NP + p];
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (j == jr) u[d][j] = r;
    }
  }
}

template <int LAT, bool DEV, typename S, bool NT, int TXV, int TY, int MINW>
__global__ __launch_bounds__(256, MINW) void k_hrr3(const S* __restrict__ src, S* __restrict__ dst,
                                                    const S* __restrict__ mac, const Geo g, const S om, const S tau,
                                                    const S sig, int ntx, int nty, int nzc, int zlen, int per_xcd) {
  using L = Lattice<LAT>;
  using N = Node<LAT, DEV, S>;
  constexpr int V = VecOf<S>::V, Q = L::Q;
  using VA = typename VT<S, V>::a;
  constexpr int HX = TXV + 2, HY = TY + 2, RW = HX * V;
  static_assert(L::D == 3, "the marching one-pass H-RR kernel is three-dimensional");
  static_assert(HX * HY <= 256, "one lane per tile-and-halo vector");
  __shared__ S lu[3][3][HY][RW];  // [plane slot][component][row][node]
  const int b = blockIdx.x;
  const int item = (b % kXCD) * per_xcd + b / kXCD;
  const int ntile = ntx * nty;
  if (item >= ntile * nzc) return;  // whole work group, before any barrier
  const int zc = item / ntile, tile = item - zc * ntile;
  const int tx = tile % ntx, ty = tile / ntx;
  const int ny = g.nf[1], nz = g.nf[2];
  const int nv = (g.nf[0] - 1 + V - 1) / V;
  const int t = threadIdx.x;
  const int hv = t % HX, hr = t / HX;
  const int k = tx * TXV - 1 + hv, y = ty * TY + hr;
  const bool lane = t < HX * HY;
  const bool live = lane && y <= ny - 1 && k <= nv - 1;
  const bool inner = live && hv >= 1 && hv <= TXV && hr >= 1 && hr <= TY && y <= ny - 2;
  const int zs = 1 + zc * zlen, ze = min(zs + zlen - 1, nz - 2);
  const VA zero = VA(S(0));
  VA T[Q], P[Q], u[3];
#pragma unroll
  for (int i = 0; i < Q; ++i) T[i] = P[i] = zero;
  auto put = [&](int zp) {
    const int sl = zp % 3;
#pragma unroll
    for (int d = 0; d < 3; ++d) *(VA*)&lu[sl][d][hr][hv * V] = u[d];
  };
  // planes zs - 1 (velocities) and zs (velocities and populations)
  if (live) {
    hrr3_pull<LAT, DEV, S>(src, mac, g, k, y, zs - 1, nv, P, u);
    put(zs - 1);
    hrr3_pull<LAT, DEV, S>(src, mac, g, k, y, zs, nv, T, u);
    put(zs);
  }
  for (int z = zs; z <= ze; ++z) {
    if (live) {
      hrr3_pull<LAT, DEV, S>(src, mac, g, k, y, z + 1, nv, P, u);
      put(z + 1);
    }
    __syncthreads();
    if (inner) {
      const int sm = (z + 2) % 3, s0 = z % 3, sp = (z + 1) % 3;
      const int c = hv * V;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        S gr[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          gr[0][d] = (lu[s0][d][hr][c + j + 1] - lu[s0][d][hr][c + j - 1]) * S(0.5);
          gr[1][d] = (lu[s0][d][hr + 1][c + j] - lu[s0][d][hr - 1][c + j]) * S(0.5);
          gr[2][d] = (lu[sp][d][hr][c + j] - lu[sm][d][hr][c + j]) * S(0.5);
        }
        Sym<S> Sr;
        Sr.xx = gr[0][0];
        Sr.yy = gr[1][1];
        Sr.xy = S(0.5) * (gr[0][1] + gr[1][0]);
        Sr.zz = gr[2][2];
        Sr.xz = S(0.5) * (gr[0][2] + gr[2][0]);
        Sr.yz = S(0.5) * (gr[1][2] + gr[2][1]);
        S f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = T[i][j];
        N::collide(f, M_HRR, om, tau, sig, &Sr);
#pragma unroll
        for (int i = 0; i < Q; ++i) T[i][j] = f[i];
      }
      const int64_t own = fpos(g, 1 + V * k, y, z);
#pragma unroll
      for (int i = 0; i < Q; ++i) vstore<NT>((VA*)(dst + pop_at<S, Q>(own, i)), T[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) T[i] = P[i];
  }
}

// ---------------------------------------------------------------------------
// State transfer kernels (logical x-fastest arrays <-> device storage).

template <int LAT, bool DEV, typename S>
__global__ void k_set_state(const double* __restrict__ rho, const double* __restrict__ u, S* __restrict__ dst,
                            const Geo g, int level) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  const int64_t NN = level == 0 ? g.Nc : g.Nf;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  int x, y, z;
  int64_t pos;
  if (level == 0) {
    cdecode(g, k, x, y, z);
    pos = cpos(g, x, y, z);
  } else {
    fdecode(g, k, x, y, z);
    pos = fpos(g, x, y, z);
  }
  double uu[3] = {u[k], u[NN + k], L::D == 3 ? u[2 * NN + k] : 0.0};
  double f[L::Q];
  N::feq(rho[k], rho[k], uu, f);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) dst[pop_at<S, L::Q>(pos, i)] = store_pop<S, DEV, LAT>(f[i], i);
}

// History at t = 0 from coarse fields rho, u (logical coarse arrays): all
// three levels get rho, u, f1 = 0 and S = centred differences of u.
template <int LAT, int MODEL>
__global__ void k_hist_init(const double* __restrict__ rho, const double* __restrict__ u, double* __restrict__ H0,
                            double* __restrict__ H1, double* __restrict__ H2, const Geo g, const Iface itf) {
  using L = Lattice<LAT>;
  using F = HF<LAT, MODEL>;
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= itf.NH) return;
  const int64_t ci = itf.hnode[h];
  int x, y, z;
  cdecode(g, ci, x, y, z);
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int64_t NN = g.Nc;
  double v[HF<LAT, M_HRR>::N + L::Q];
  v[F::RHO] = rho[ci];
  for (int d = 0; d < L::D; ++d) v[F::U + d] = u[d * NN + ci];
  for (int i = 0; i < F::NF1; ++i) v[F::F1 + i] = 0.0;
  double gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < L::D; ++a) {
    int cp[3] = {x, y, z}, cm[3] = {x, y, z};
    const int na = a == 0 ? nx : (a == 1 ? ny : nz);
    cp[a] = wrap(cp[a] + 1, na);
    cm[a] = wrap(cm[a] - 1, na);
    const int64_t ip = (int64_t)cp[0] + (int64_t)nx * ((int64_t)cp[1] + (int64_t)ny * cp[2]);
    const int64_t im = (int64_t)cm[0] + (int64_t)nx * ((int64_t)cm[1] + (int64_t)ny * cm[2]);
    for (int b = 0; b < L::D; ++b) gr[a][b] = 0.5 * (u[b * NN + ip] - u[b * NN + im]);
  }
  if (MODEL == M_HRR) {
    const Sym<double> S{gr[0][0], gr[1][1], gr[2][2], 0.5 * (gr[0][1] + gr[1][0]), 0.5 * (gr[0][2] + gr[2][0]),
                        0.5 * (gr[1][2] + gr[2][1])};
    sym_put<L::D>(S, v + F::S, 1.0);
  }
  const int64_t NH = itf.NH;
  for (int k = 0; k < F::N; ++k) {
    H0[(int64_t)k * NH + h] = v[k];
    H1[(int64_t)k * NH + h] = v[k];
    H2[(int64_t)k * NH + h] = v[k];
  }
}

// Moments of the stored post-collision state (double, logical order).  On the
// coarse level covered nodes take the co-located fine node's values.
template <int LAT, bool DEV, typename S>
__global__ void k_macros(const S* __restrict__ src, const S* __restrict__ fine, double* __restrict__ rho,
                         double* __restrict__ u, const Geo g, int level) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  const int64_t NN = level == 0 ? g.Nc : g.Nf;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  int x, y, z;
  const S* p = src;
  int64_t pos;
  if (level == 0) {
    cdecode(g, k, x, y, z);
    pos = cpos(g, x, y, z);
    if (g.has_fine && coarse_class(g, x, y, z) == CC_COVERED) {
      p = fine;
      pos = fpos(g, 2 * (x - g.a[0]), 2 * (y - g.a[1]), L::D == 3 ? 2 * (z - g.a[2]) : 0);
    }
  } else {
    fdecode(g, k, x, y, z);
    pos = fpos(g, x, y, z);
  }
  double f[L::Q], r, r0, uu[3];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) f[i] = full_pop<S, DEV, LAT>(p[pop_at<S, L::Q>(pos, i)], i);
  N::moments(f, r, r0, uu);
  rho[k] = r;
#pragma unroll
  for (int d = 0; d < L::D; ++d) u[d * NN + k] = uu[d];
}

// ---------------------------------------------------------------------------
// Non-hydrodynamic-mode sensors (Sec. 7).  Diagnostics, in double precision,
// one thread per node.
//
// Velocities of a level into plain planes U[1 + d][pos] (plane 0 unused
// here; the layout is that of the velocity planes, so the ring macro kernel
// can fill ring entries): PULL = false takes the moments of src at the node,
// PULL = true the moments of the populations the node pulls from src (the
// pre-collision state one iteration later) -- fine level, non-ring nodes.
template <int LAT, bool DEV, typename S, int LEVEL, bool PULL>
__global__ void k_sens_vel(const S* __restrict__ src, double* __restrict__ U, const Geo g) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  constexpr int Q = L::Q;
  const int64_t NN = LEVEL == 0 ? g.Nc : g.Nf;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  int x, y, z;
  if (LEVEL == 0) cdecode(g, k, x, y, z);
  else fdecode(g, k, x, y, z);
  const int64_t pos = LEVEL == 0 ? cpos(g, x, y, z) : fpos(g, x, y, z);
  const int64_t NP = LEVEL == 0 ? g.Ncp : g.Nfp;
  if (PULL && LEVEL == 1 && fine_is_ring(g, x, y, z)) return;
  double f[Q], r, r0, u[3];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int64_t ps = pos;
    if (PULL) ps = fpos(g, x - L::cx(i), y - L::cy(i), z - L::cz(i));
    f[i] = full_pop<S, DEV, LAT>(src[pop_at<S, Q>(ps, i)], i);
  }
  N::moments(f, r, r0, u);
#pragma unroll
  for (int d = 0; d < L::D; ++d) U[(int64_t)(1 + d) * NP + pos] = u[d];
}

// Sensor flags of one node of a level after a step: bit 0 SpuriousAc (the
// velocity divergence changes sign between the two iterations, eq
// sensorSpuriousAc), bit 1 SpuriousS (the curl changes sign, eq
// sensorSpuriousS; in 3D the dot product of the two curl vectors), bit 2
// SpuriousG (eqs fneqSplit, reguProceduref1S, sensorSpuriousG: the norm of
// the non-equilibrium part of the pre-collision populations left after the
// second-order Hermite projection exceeds thr, and neither flag above is
// set).  A product of exactly zero gives 0.  Up: velocities of the previous
// iteration (planes, as k_sens_vel); cur: the post-collision state of the
// last iteration (its moments are the pre-collision ones); pre: the state
// the last iteration's pre-collision populations are pulled from.  Nodes the
// level does not evolve by streaming get 0: coarse TN and covered nodes,
// the fine ring.  flags and the optional diagnostics prod[3][N] (divergence
// product, curl product, ghost norm) are in logical node order.
template <int LAT, bool DEV, typename S, int LEVEL>
__global__ void k_sensors(const double* __restrict__ Up, const S* __restrict__ cur, const S* __restrict__ pre,
                          uint8_t* __restrict__ flags, double* __restrict__ prod, const Geo g, double thr) {
  using L = Lattice<LAT>;
  using N = Node<LAT, false, double>;
  constexpr int Q = L::Q, D = L::D;
  const int64_t NN = LEVEL == 0 ? g.Nc : g.Nf;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  int x, y, z;
  if (LEVEL == 0) cdecode(g, k, x, y, z);
  else fdecode(g, k, x, y, z);
  const int nx = LEVEL == 0 ? g.n[0] : g.nf[0], ny = LEVEL == 0 ? g.n[1] : g.nf[1],
            nz = LEVEL == 0 ? g.n[2] : g.nf[2];
  const int64_t NP = LEVEL == 0 ? g.Ncp : g.Nfp;
  bool ok;
  if (LEVEL == 0) {
    const int c = coarse_class(g, x, y, z);
    ok = c == CC_MIDDLE || c == CC_TF;
  } else {
    ok = !fine_is_ring(g, x, y, z);
  }
  uint8_t fl = 0;
  double pd = 0.0, pc = 0.0, gn = 0.0;
  if (ok) {
    auto at = [&](int xs, int ys, int zs) -> int64_t {
      if (LEVEL == 0) return cpos(g, wrap(xs, nx), wrap(ys, ny), D == 3 ? wrap(zs, nz) : 0);
      return fpos(g, xs, ys, zs);
    };
    auto ucur = [&](int64_t p, double* u) {
      double f[Q], r, r0;
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = full_pop<S, DEV, LAT>(cur[pop_at<S, Q>(p, i)], i);
      N::moments(f, r, r0, u);
    };
    // velocity gradients of both iterations, centred differences
    double gp[3][3], gc[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int e[3] = {a == 0, a == 1, a == 2};
      const int64_t pp = at(x + e[0], y + e[1], z + e[2]), pm = at(x - e[0], y - e[1], z - e[2]);
      double up[3], um[3];
      ucur(pp, up);
      ucur(pm, um);
#pragma unroll
      for (int b = 0; b < D; ++b) {
        gc[a][b] = (up[b] - um[b]) / 2.0;
        gp[a][b] = (Up[(int64_t)(1 + b) * NP + pp] - Up[(int64_t)(1 + b) * NP + pm]) / 2.0;
      }
    }
    double dp = 0.0, dc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dp += gp[a][a];
      dc += gc[a][a];
    }
    double cp[3], cc[3];
    if (D == 2) {
      cp[0] = gp[0][1] - gp[1][0];
      cc[0] = gc[0][1] - gc[1][0];
      cp[1] = cp[2] = cc[1] = cc[2] = 0.0;
    } else {
      cp[0] = gp[1][2] - gp[2][1];
      cp[1] = gp[2][0] - gp[0][2];
      cp[2] = gp[0][1] - gp[1][0];
      cc[0] = gc[1][2] - gc[2][1];
      cc[1] = gc[2][0] - gc[0][2];
      cc[2] = gc[0][1] - gc[1][0];
    }
    pd = dp * dc;
    pc = cp[0] * cc[0] + cp[1] * cc[1] + cp[2] * cc[2];
    const bool ac = pd < 0.0, sp = pc < 0.0;
    // pre-collision populations of the last iteration
    double f[Q], f0[Q], r, r0, u[3];
#pragma unroll
    for (int i = 0; i < Q; ++i)
      f[i] = full_pop<S, DEV, LAT>(pre[pop_at<S, Q>(at(x - L::cx(i), y - L::cy(i), z - L::cz(i)), i)], i);
    N::moments(f, r, r0, u);
    N::feq(r, r0, u, f0);
    double f1[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f1[i] = f[i] - f0[i];
    const Sym<double> P = N::second(f1);  // a1 = sum_i H_i f1_i (f1 carries no mass or momentum)
    double a[3][3] = {{P.xx, P.xy, P.xz}, {P.xy, P.yy, P.yz}, {P.xz, P.yz, P.zz}};
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double c[3] = {(double)L::cx(i), (double)L::cy(i), (double)L::cz(i)};
      double hs = 0.0;
#pragma unroll
      for (int p = 0; p < D; ++p)
#pragma unroll
        for (int q = 0; q < D; ++q) hs += (c[p] * c[q] - (p == q ? 1.0 / 3.0 : 0.0)) * a[p][q];
      const double gq = f1[i] - L::w(i) * 4.5 * hs;  // f1 - w / (2 c_s^4) H : a1
      nrm += gq * gq;
    }
    gn = sqrt(nrm);
    const bool gs = gn > thr && !ac && !sp;
    fl = (uint8_t)((ac ? 1 : 0) | (sp ? 2 : 0) | (gs ? 4 : 0));
  }
  flags[k] = fl;
  if (prod) {
    prod[k] = pd;
    prod[NN + k] = pc;
    prod[2 * NN + k] = gn;
  }
}

// Density at one node of a level, appended to a series (probe recording):
// series[*count] = rho, ++*count while below capacity.  One thread.
template <int LAT, bool DEV, typename S>
__global__ void k_probe(const S* __restrict__ src, int64_t pos, double* __restrict__ series,
                        int64_t* __restrict__ count, int64_t capacity) {
  using L = Lattice<LAT>;
  if (threadIdx.x != 0) return;
  const int64_t c = *count;
  if (c >= capacity) return;
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) r += full_pop<S, DEV, LAT>(src[pop_at<S, L::Q>(pos, i)], i);
  series[c] = r;
  *count = c + 1;
}

// Populations out / in: f[q][logical node] (double, full values).
template <int LAT, bool DEV, typename S>
__global__ void k_pops_out(const S* __restrict__ src, double* __restrict__ f, const Geo g, int level) {
  const int64_t NN = level == 0 ? g.Nc : g.Nf;
  const int64_t n = NN * Lattice<LAT>::Q;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = (int)(k / NN);
  const int64_t node = k % NN;
  int x, y, z;
  int64_t pos;
  if (level == 0) {
    cdecode(g, node, x, y, z);
    pos = pop_at<S, Lattice<LAT>::Q>(cpos(g, x, y, z), i);
  } else {
    fdecode(g, node, x, y, z);
    pos = pop_at<S, Lattice<LAT>::Q>(fpos(g, x, y, z), i);
  }
  f[k] = full_pop<S, DEV, LAT>(src[pos], i);
}
template <int LAT, bool DEV, typename S>
__global__ void k_pops_in(const double* __restrict__ f, S* __restrict__ dst, const Geo g, int level) {
  const int64_t NN = level == 0 ? g.Nc : g.Nf;
  const int64_t n = NN * Lattice<LAT>::Q;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = (int)(k / NN);
  const int64_t node = k % NN;
  int x, y, z;
  int64_t pos;
  if (level == 0) {
    cdecode(g, node, x, y, z);
    pos = pop_at<S, Lattice<LAT>::Q>(cpos(g, x, y, z), i);
  } else {
    fdecode(g, node, x, y, z);
    pos = pop_at<S, Lattice<LAT>::Q>(fpos(g, x, y, z), i);
  }
  dst[pos] = store_pop<S, DEV, LAT>(f[k], i);
}

// Global totals, pass 1: per-block sums of rho and rho u (double) over the
// evolving nodes of a level, in logical node order.  256 lanes per block,
// fixed reduction tree.
template <int LAT, bool DEV, typename S>
__global__ __launch_bounds__(256) void k_totals(const S* __restrict__ src, double* __restrict__ part,
                                                const Geo g, int level) {
  using L = Lattice<LAT>;
  const int64_t NN = level == 0 ? g.Nc : g.Nf;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (k < NN) {
    int x, y, z;
    int64_t pos;
    bool use = true;
    if (level == 0) {
      cdecode(g, k, x, y, z);
      pos = cpos(g, x, y, z);
      use = !g.has_fine || coarse_class(g, x, y, z) != CC_COVERED;
    } else {
      fdecode(g, k, x, y, z);
      pos = fpos(g, x, y, z);
    }
    if (use) {
#pragma unroll
      for (int i = 0; i < L::Q; ++i) {
        const double f = full_pop<S, DEV, LAT>(src[pop_at<S, L::Q>(pos, i)], i);
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
