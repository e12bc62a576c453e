// batch.hpp -- many independent two-level grids advanced by one set of
// launches per coarse step.
//
// Every grid ("instance") of a batch keeps its own device buffers; a device
// table of InstDev descriptors holds their geometry, buffer pointers and
// time-level state (coarse ping-pong parity, history rotation).  For each
// phase of the coarse step there is one work list of (instance, index)
// items: a bulk chunk of 256 vectors, a fused fine tile (D2Q9 BGK / RR: both
// fine substeps, as k_fine2), a block of 64 interface nodes, or a block of
// TN nodes.  A phase is one launch with one work group per list entry (two
// phases that touch disjoint data may share a launch, each part with its
// own list); the list is split into 8 contiguous parts, one per XCD, so the
// chunks of one instance stay in one L2.  The last launch of a step flips
// each instance's parity and rotates its history on the device, so the
// launch sequence of a step is the same every step and is captured once as a
// hipGraph.  Instances join or leave by rewriting the tables and lists
// between steps; the captured graph reads list lengths from device memory and
// is captured again only when a list outgrows its buffer.
#pragma once
#include "kernels.hpp"

namespace lbm {

struct InstDev {
  Geo g;
  Iface itf;
  Flat fc, ff;  // flat numbering of the coarse / fine bulk vectors
  void* cbuf[2];
  void* fbuf[2];  // fbuf[fpar] holds the fine state at integer times
  void* fh;       // fused: the t+1/2 ring and band (fine-to-coarse source)
  void* xb;       // D3Q19 BGK / RR: compact copy of the fine x-bands at t+1/2 (xband_at)
  void* mac_c;
  void* mac_f;
  double* hist[3];
  double* G;
  double tau_c, tau_f, sig;
  void* ccur;  // coarse buffer holding the current state (cbuf[cpar]) and the
  void* cnext; // other one, kept as pointers so kernels read them directly
  int cpar;    // coarse buffer holding the current state
  int hs[3];  // history buffers holding t-1, t, t+1
  int active;
  int fpar;   // fine buffer holding the state at integer times
  int fused;  // both fine substeps in one phase (D2Q9 BGK / RR): fpar flips every step
  int ntx;    // fused: fine tiles per row of tiles (of the batch's tile shape)
};

// Pointers read from the descriptor table are generic to the compiler, which
// then issues flat memory instructions; every buffer lives in device global
// memory, and saying so gives global loads and stores (vector memory
// counters only, immediate offsets).
template <typename T>
__device__ __forceinline__ T* glob(T* p) {
  using GT = __attribute__((address_space(1))) T;
  return (T*)(GT*)(uintptr_t)p;  // through an integer, so the cast is not folded away
}
__device__ __forceinline__ Iface glob(const Iface& a) {
  Iface b = a;
  b.hnode = glob(a.hnode);
  b.rnode = glob(a.rnode);
  b.rnp = glob(a.rnp);
  b.rpt = glob(a.rpt);
  b.tnf = glob(a.tnf);
  b.tnc = glob(a.tnc);
  return b;
}

struct Work {
  int inst;
  int idx;
};

// Work-list kinds.
enum WorkKind : int {
  W_COARSE = 0,  // coarse bulk chunks
  W_FINE = 1,    // fine bulk chunks
  W_HIST = 2,    // 64 history nodes
  W_HTIME = 3,   // 64 history values (all fields)
  W_RING = 4,    // 64 ring nodes
  W_TN = 5,      // 64 TN nodes
  W_TNB = 6,     // PER TN nodes (one fine-to-coarse work group)
  W_TILE = 7,    // fused fine tile (the batch's tile shape)
  W_KINDS = 8
};

// Fused fine tile shapes of the batch (lanes, vectors x rows), chosen by its
// autotuner: wide tiles suit long fine rows, narrow ones short rows.
constexpr int kNTile = 2;
constexpr int kTileX[kNTile] = {64, 32}, kTileY[kNTile] = {8, 8};

// Item of this work group, or -1.  A phase launches one work group per entry
// of its list's capacity (a multiple of 8); the live count is read from
// device memory, so a captured launch stays valid while grids join and leave.
// Groups are handed to the XCDs round-robin; the item index is remapped so
// each XCD serves one contiguous part of the list, in dispatch order.
// item_in: the same for block b of one part of a launch that serves two
// lists (each part's block count a multiple of 8).
__device__ __forceinline__ int item_in(int b, int n) {
  const int per = (n + kXCD - 1) / kXCD;
  const int w = b / kXCD;
  if (w >= per) return -1;
  const int it = (b % kXCD) * per + w;
  return it < n ? it : -1;
}
__device__ __forceinline__ int item_of(int n) { return item_in(blockIdx.x, n); }

__device__ __forceinline__ Work load_item(const Work* __restrict__ items, int it) {
  Work w = items[it];
  w.inst = __builtin_amdgcn_readfirstlane(w.inst);
  w.idx = __builtin_amdgcn_readfirstlane(w.idx);
  return w;
}

// Bulk stream of one level; SUB selects the fine buffer direction (0: A->B,
// 1: B->A, with A = fbuf[fpar]).
template <int LAT, bool DEV, typename S, int MODEL, int LEVEL, int SUB, bool NT>
__global__ __launch_bounds__(256) void kb_stream(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                                 const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    const InstDev& I = inst[w.inst];
    if (LEVEL == 0) {
      const S* src = glob((const S*)I.ccur);
      S* dst = glob((S*)I.cnext);
      stream_body<LAT, DEV, S, MODEL, 0, NT>(src, dst, glob((S*)I.mac_c), I.g, I.fc, (S)(1.0 - 1.0 / I.tau_c), w.idx);
    } else {
      const S* src = glob((const S*)I.fbuf[I.fpar ^ SUB]);
      S* dst = glob((S*)I.fbuf[I.fpar ^ SUB ^ 1]);
      // the first substep also fills the x-band copy (as the single grid)
      S* xb = (SUB == 0 && I.xb) ? glob((S*)I.xb) : nullptr;
      stream_body<LAT, DEV, S, MODEL, 1, NT>(src, dst, glob((S*)I.mac_f), I.g, I.ff, (S)(1.0 - 1.0 / I.tau_f), w.idx,
                                             xb);
    }
  }
}

// H-RR pull-stream and collision.  LEVEL 0: coarse current -> other buffer;
// LEVEL 1: fine A -> B (SUB 0) or B -> A (SUB 1).
template <int LAT, bool DEV, typename S, int LEVEL, int SUB, bool NT>
__global__ __launch_bounds__(256) void kb_collide(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                                  const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    const InstDev& I = inst[w.inst];
    if (LEVEL == 0) {
      collide_hrr_body<LAT, DEV, S, 0, NT>(glob((const S*)I.ccur), glob((S*)I.cnext), glob((const S*)I.mac_c), I.g,
                                           I.fc, (S)(1.0 - 1.0 / I.tau_c), (S)I.tau_c, (S)I.sig, w.idx);
    } else {
      collide_hrr_body<LAT, DEV, S, 1, NT>(glob((const S*)I.fbuf[I.fpar ^ SUB]), glob((S*)I.fbuf[I.fpar ^ SUB ^ 1]),
                                           glob((const S*)I.mac_f), I.g, I.ff,
                                           (S)(1.0 - 1.0 / I.tau_f), (S)I.tau_f, (S)I.sig, w.idx);
    }
  }
}

template <int LAT, bool DEV, typename S, int MODEL>
__global__ __launch_bounds__(64) void kb_hist_capture(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                                      const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    const InstDev& I = inst[w.inst];
    // BGK / RR: also the t+1/2 interpolation into G (H-RR: kb_hist_time)
    hist_capture_body<LAT, DEV, S, MODEL>(glob((const S*)I.ccur), glob(I.hist[I.hs[2]]), I.g, glob(I.itf),
                                          (int64_t)w.idx * 64 + threadIdx.x, MODEL == M_HRR ? nullptr : glob(I.G),
                                          glob(I.hist[I.hs[0]]), glob(I.hist[I.hs[1]]));
  }
}

template <int LAT, bool DEV, typename S>
__global__ __launch_bounds__(64) void kb_hist_strain(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                                     const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    const InstDev& I = inst[w.inst];
    hist_strain_body<LAT, DEV, S, false>(nullptr, glob((const S*)I.mac_c), glob(I.hist[I.hs[2]]), I.g, glob(I.itf), (int64_t)w.idx * 64 + threadIdx.x);
  }
}

// Temporal interpolation (eq TempInt) of all history values of an instance.
template <int NFIELD>
__global__ __launch_bounds__(64) void kb_hist_time(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                                   const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    const InstDev& I = inst[w.inst];
    const int64_t k = (int64_t)w.idx * 64 + threadIdx.x;
    if (k < I.itf.NH * NFIELD)
      glob(I.G)[k] = time_half(glob(I.hist[I.hs[0]])[k], glob(I.hist[I.hs[1]])[k], glob(I.hist[I.hs[2]])[k]);
  }
}

// Ring reconstruction of one 64-node item: SUB 0 (t+1/2, from G, into the
// half-time buffer: fh when fused, else B), SUB 1 (t+1, from the t+1
// history, into the buffer that holds t+1 after the step: B when fused, else
// A); only the populations the stepping reads (the full ring of A is
// completed before it is observed).
template <int LAT, bool DEV, typename S, int MODEL, int SUB>
__device__ __forceinline__ void kb_ring_item(const InstDev& I, int idx, int lane) {
  const double* G = glob(SUB == 0 ? I.G : I.hist[I.hs[2]]);
  S* dst = glob((S*)(SUB == 0 ? (I.fused ? I.fh : I.fbuf[I.fpar ^ 1]) : I.fbuf[I.fpar ^ I.fused]));
  S* xb = (SUB == 0 && I.xb) ? glob((S*)I.xb) : nullptr;  // the t+1/2 ring fills the x-band copy
  ring_body<LAT, DEV, S, MODEL, true>(G, dst, I.g, glob(I.itf), I.tau_f / (2.0 * I.tau_c), 1.0 - 1.0 / I.tau_f, I.tau_f, I.sig,
                                      (int64_t)idx * 64 + lane, xb);
}
template <int LAT, bool DEV, typename S, int MODEL, int SUB>
__global__ __launch_bounds__(64) void kb_ring(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                              const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    kb_ring_item<LAT, DEV, S, MODEL, SUB>(inst[w.inst], w.idx, threadIdx.x);
  }
}

// Coarse stream (BGK, RR) and the t+1/2 ring in one launch: blocks [0, nrb)
// take ring items (64 lanes each), the rest coarse chunks.
template <int LAT, bool DEV, typename S, int MODEL, bool NT>
__global__ __launch_bounds__(256) void kb_stream_ring(const InstDev* __restrict__ inst, const Work* __restrict__ ritems,
                                                      const int* __restrict__ rcount, const Work* __restrict__ citems,
                                                      const int* __restrict__ ccount, int nrb) {
  const int b = blockIdx.x;
  if (b < nrb) {
    if (threadIdx.x >= 64) return;
    const int it = item_in(b, *rcount);
    if (it < 0) return;
    const Work w = load_item(ritems, it);
    kb_ring_item<LAT, DEV, S, MODEL, 0>(inst[w.inst], w.idx, threadIdx.x);
  } else {
    const int it = item_in(b - nrb, *ccount);
    if (it < 0) return;
    const Work w = load_item(citems, it);
    const InstDev& I = inst[w.inst];
    stream_body<LAT, DEV, S, MODEL, 0, NT>(glob((const S*)I.ccur), glob((S*)I.cnext), nullptr, I.g, I.fc, (S)(1.0 - 1.0 / I.tau_c),
                                           w.idx);
  }
}

// Both fine substeps of one tile (D2Q9 BGK / RR), A -> B with the t+1/2 ring
// and band in fh.
template <int LAT, bool DEV, typename S, int MODEL, bool NT, int HXV, int HYR>
__global__ __launch_bounds__(HXV * HYR) void kb_fine2(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                                      const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  const Work w = load_item(items, it);
  const InstDev& I = inst[w.inst];
  fine2_tile<LAT, DEV, S, MODEL, NT, HXV, HYR>(glob((const S*)I.fbuf[I.fpar]),
                                                             glob((S*)I.fbuf[I.fpar ^ 1]), glob((S*)I.fh), I.g, (S)(1.0 - 1.0 / I.tau_f), I.ntx, w.idx);
}

// H-RR ring rho, u at t+1/2 (SUB 0) or t+1 (SUB 1).
template <int LAT, typename S, int SUB>
__global__ __launch_bounds__(64) void kb_ring_macro(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                                    const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    const InstDev& I = inst[w.inst];
    const double c0 = SUB == 0 ? -0.125 : 0.0, c1 = SUB == 0 ? 0.75 : 0.0, c2 = SUB == 0 ? 0.375 : 1.0;
    ring_macro_body<LAT, S>(glob(I.hist[I.hs[0]]), glob(I.hist[I.hs[1]]), glob(I.hist[I.hs[2]]), c0, c1, c2,
                            glob((S*)I.mac_f), I.g, glob(I.itf),
                            (int64_t)w.idx * 64 + threadIdx.x);
  }
}

template <int LAT, bool DEV, typename S>
__global__ __launch_bounds__(64) void kb_fict(const InstDev* __restrict__ inst, const Work* __restrict__ items,
                                              const int* __restrict__ count) {
  const int it = item_of(*count);
  if (it < 0) return;
  {
    const Work w = load_item(items, it);
    const InstDev& I = inst[w.inst];
    fict_body<LAT, DEV, S, S>(glob((const S*)I.fbuf[I.fpar ^ 1]), glob((S*)I.mac_c), I.g, glob(I.itf), (int64_t)w.idx * 64 + threadIdx.x);
  }
}

// Fine-to-coarse transfer from the t+1/2 state (fh when fused, else B).
template <int LAT, bool DEV, typename S, int MODEL>
__device__ __forceinline__ void kb_coalesce_item(const InstDev& I, int idx) {
  const S* xb = I.xb ? glob((const S*)I.xb) : nullptr;
  coalesce_body<LAT, DEV, S, MODEL>(glob((const S*)(I.fused ? I.fh : I.fbuf[I.fpar ^ 1])), glob((S*)I.cnext), I.g,
                                    glob(I.itf),
                                    2.0 * I.tau_c / I.tau_f, 1.0 - 1.0 / I.tau_c, I.tau_c, I.sig, idx, xb);
}

// The t+1 ring and the fine-to-coarse transfer in one launch: blocks
// [0, nrb) take ring items (64 lanes each), the rest TN blocks.
template <int LAT, bool DEV, typename S, int MODEL>
__global__ __launch_bounds__(256) void kb_ring_coalesce(const InstDev* __restrict__ inst, const Work* __restrict__ ritems,
                                                        const int* __restrict__ rcount, const Work* __restrict__ titems,
                                                        const int* __restrict__ tcount, int nrb) {
  const int b = blockIdx.x;
  if (b < nrb) {
    if (threadIdx.x >= 64) return;
    const int it = item_in(b, *rcount);
    if (it < 0) return;
    const Work w = load_item(ritems, it);
    kb_ring_item<LAT, DEV, S, MODEL, 1>(inst[w.inst], w.idx, threadIdx.x);
  } else {
    const int it = item_in(b - nrb, *tcount);
    if (it < 0) return;  // whole work group: the transfer synchronises its lanes
    const Work w = load_item(titems, it);
    kb_coalesce_item<LAT, DEV, S, MODEL>(inst[w.inst], w.idx);
  }
}

// Uniform (single-level) instances: stream (+ collide) of the coarse level.
// Handled by kb_stream LEVEL 0; nothing else runs for them.

// End of a coarse step: every active instance moves to the next time level.
__global__ void kb_advance(InstDev* __restrict__ inst, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || !inst[k].active) return;
  inst[k].cpar ^= 1;
  inst[k].fpar ^= inst[k].fused;
  void* t = inst[k].ccur;
  inst[k].ccur = inst[k].cnext;
  inst[k].cnext = t;
  const int old = inst[k].hs[0];
  inst[k].hs[0] = inst[k].hs[1];
  inst[k].hs[1] = inst[k].hs[2];
  inst[k].hs[2] = old;
}

}  // namespace lbm
