// geometry.hpp -- two-level grid geometry and node classes (host and device).
//
// The fine patch is the box [a, a+m] of coarse vertices; fine node j sits at
// coarse coordinate a + j/2, so the fine level has 2m+1 nodes per axis and
// its outer layer (j = 0 or 2m) is the overlap ring of Fig. Overlap.  The
// classes follow that figure, written for a closed patch:
//   coarse TF  : coarse vertices on the boundary of [a, a+m]      (c -> f)
//   coarse TN  : coarse vertices on the boundary of [a+1, a+m-1]  (f -> c)
//   covered    : coarse vertices inside [a+1, a+m-1] (not evolved)
//   fine TF    : ring nodes co-located with a coarse vertex
//   fine IE    : other ring nodes (one half-integer coordinate)
//   fine IEFACE: 3D ring nodes with two half-integer coordinates
//   fine TN    : fine nodes co-located with coarse TN nodes
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

enum CoarseClass : int { CC_MIDDLE = 0, CC_TF = 1, CC_TN = 2, CC_COVERED = 3 };
enum FineClass : int { FC_MIDDLE = 0, FC_TF = 1, FC_IE = 2, FC_IEFACE = 3, FC_TN = 4 };

// Device arrays use a padded row pitch (pc, pf: nodes per row rounded up to
// a multiple of 4) so every row starts 16-byte aligned; Ncp, Nfp are the
// padded node counts of a level (the positions of pop_at below, and the plane
// size of the velocity planes).  Nc, Nf count logical nodes (the x-fastest
// order of the C ABI and of the interface tables).  (A power-of-two fine
// pitch, which keeps rows inside one storage block, was measured slower: rows
// a power of two apart share HBM channels.)
struct Geo {
  int D;
  int n[3];   // coarse nodes per axis (1 on unused axes)
  int a[3];   // patch lower corner (coarse vertex)
  int m[3];   // patch size in coarse cells
  int nf[3];  // fine nodes per axis (2m+1; 1 on unused axes or without patch)
  int has_fine;
  int64_t Nc, Nf;
  int pc, pf;        // row pitch of coarse / fine device arrays
  int fxo;           // offset of fine node x = 0 inside its row: the first
                     // middle node (x = 1) starts a 16-byte boundary
  int64_t Ncp, Nfp;  // padded plane sizes
};

constexpr int kPitchAlign = 4;
__host__ __device__ inline int pitch_of(int nx) { return (nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign; }

// Padded device offset of a coarse / fine node.
__host__ __device__ inline int64_t cpos(const Geo& g, int x, int y, int z) {
  return (int64_t)x + (int64_t)g.pc * ((int64_t)y + (int64_t)g.n[1] * z);
}
__host__ __device__ inline int64_t fpos(const Geo& g, int x, int y, int z) {
  return (int64_t)(x + g.fxo) + (int64_t)g.pf * ((int64_t)y + (int64_t)g.nf[1] * z);
}
// Logical node index -> coordinates.
__host__ __device__ inline void cdecode(const Geo& g, int64_t i, int& x, int& y, int& z) {
  x = (int)(i % g.n[0]);
  const int64_t r = i / g.n[0];
  y = (int)(r % g.n[1]);
  z = (int)(r / g.n[1]);
}
__host__ __device__ inline void fdecode(const Geo& g, int64_t i, int& x, int& y, int& z) {
  x = (int)(i % g.nf[0]);
  const int64_t r = i / g.nf[0];
  y = (int)(r % g.nf[1]);
  z = (int)(r / g.nf[1]);
}

__host__ __device__ inline int coarse_class(const Geo& g, int x, int y, int z) {
  if (!g.has_fine) return CC_MIDDLE;
  const int c[3] = {x, y, z};
  bool in_tn = true, on_tn = false, in_tf = true, on_tf = false;
  for (int d = 0; d < g.D; ++d) {
    const int lo = g.a[d], hi = g.a[d] + g.m[d];
    if (c[d] < lo + 1 || c[d] > hi - 1) in_tn = false;
    if (c[d] == lo + 1 || c[d] == hi - 1) on_tn = true;
    if (c[d] < lo || c[d] > hi) in_tf = false;
    if (c[d] == lo || c[d] == hi) on_tf = true;
  }
  if (in_tn) return on_tn ? CC_TN : CC_COVERED;
  return (in_tf && on_tf) ? CC_TF : CC_MIDDLE;
}

__host__ __device__ inline bool fine_is_ring(const Geo& g, int x, int y, int z) {
  return x == 0 || x == g.nf[0] - 1 || y == 0 || y == g.nf[1] - 1 ||
         (g.D == 3 && (z == 0 || z == g.nf[2] - 1));
}

__host__ __device__ inline int fine_class(const Geo& g, int x, int y, int z) {
  const int j[3] = {x, y, z};
  int odd = 0;
  bool even = true, in_tn = true, on_tn = false;
  for (int d = 0; d < g.D; ++d) {
    const int M = g.nf[d] - 1;
    if (j[d] & 1) {
      odd++;
      even = false;
    }
    if (j[d] < 2 || j[d] > M - 2) in_tn = false;
    if (j[d] == 2 || j[d] == M - 2) on_tn = true;
  }
  if (fine_is_ring(g, x, y, z)) return odd == 0 ? FC_TF : (odd == 1 ? FC_IE : FC_IEFACE);
  return (even && in_tn && on_tn) ? FC_TN : FC_MIDDLE;
}

// Compact copy of the fine state in the two x-normal bands of the patch,
// x in [0, 4] (side 0) and [nx - 5, nx - 1] (side 1), five nodes per row:
// [side][population][z][y][x offset].  In the row-major layout every
// population of those nodes fills its own cache line; here consecutive rows
// are 5 values apart.  (The bands overlap when nx < 10: a node may sit on
// both sides.)
__host__ __device__ inline int64_t xband_at(const Geo& g, int Q, int side, int q, int y, int z, int xo) {
  return ((((int64_t)side * Q + q) * g.nf[2] + z) * g.nf[1] + y) * 5 + xo;
}
__host__ __device__ inline int64_t xband_elems(const Geo& g, int Q) { return (int64_t)2 * Q * g.nf[2] * g.nf[1] * 5; }

// Periodic wrap of a coarse coordinate displaced by at most one period.
__host__ __device__ inline int wrap(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Population storage, array of structure-of-arrays: the padded node positions
// p of a level are cut into blocks of PB consecutive positions; block b holds
// Q sub-blocks of 32 KB, one per population, each with the PB values of that
// block.  A pull-stream step then keeps its 2Q concurrent memory streams
// within two windows of Q x 32 KB instead of 2Q planes spread over the whole
// buffer, which HBM serves markedly faster than plain structure-of-arrays.
template <typename S>
struct PopBlock {
  static constexpr int SHIFT = sizeof(S) == 4 ? 13 : 12;  // 8192 floats or 4096 doubles
  static constexpr int64_t B = (int64_t)1 << SHIFT;
};
// Written as base(p) + q B, base(p) = p + (Q - 1) B floor(p / B), which is
// ((p / B) Q + q) B + p mod B: the Q populations of a node share base(p).
template <typename S, int Q>
__host__ __device__ inline int64_t pop_at(int64_t p, int q) {
  constexpr int SH = PopBlock<S>::SHIFT;
  constexpr int64_t B = PopBlock<S>::B;
  return p + (int64_t)(Q - 1) * B * (p >> SH) + (int64_t)q * B;
}
// Elements of a population buffer for NP padded positions: whole blocks up
// to and including position NP (the last x-vector of a fine row reaches one
// position past the end of its row).
template <typename S>
__host__ __device__ inline int64_t pop_elems(int64_t NP, int Q) {
  return ((NP >> PopBlock<S>::SHIFT) + 1) * (int64_t)Q * PopBlock<S>::B;
}

}  // namespace lbm
