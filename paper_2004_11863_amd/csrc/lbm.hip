// lbm.hip -- host side of the MI355X two-level LBM library: descriptor
// validation, interface table builder, device state, the per-coarse-step
// launch schedule (Sec. 4.3) and the C ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "batch.hpp"
#include "kernels.hpp"
#include "lbm.h"

namespace lbm {

static thread_local std::string g_create_error;

// A blocking HIP call (synchronous copy or memset, allocation, free, device
// or stream wait) made by one thread while another thread captures a
// hipGraph invalidates that capture.  Every entry point that makes such calls
// holds this lock for its whole call, and a batch holds it while it captures
// its step graph, so calls from several threads never overlap a capture.
// lbm_batch_step (launches only, apart from a capture) and the host-only
// queries do not take it.  Recursive: a call may re-enter it.
static std::recursive_mutex g_api_mu;

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      throw LbmError(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    }                                                                                      \
  } while (0)

struct LbmError {
  int code;
  std::string msg;
  LbmError(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// Device allocation owned by a grid.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool own = true;  // false: a view of another grid's buffer
  void alloc(size_t b) {
    bytes = b;
    own = true;
    if (b == 0) return;
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      throw LbmError(LBM_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
  }
  void view(void* q, size_t b) {
    p = q;
    bytes = b;
    own = false;
  }
  ~DevBuf() {
    if (p && own) (void)hipFree(p);
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// ---------------------------------------------------------------------------
// Interface tables (host).  History nodes: coarse vertices on a face plane of
// the patch box within [a-1, a+m+1]^D (TF plus the nodes one step beyond the
// box that the cubic stencils of ring nodes next to edges and corners reach).
// Ring stencils: 1 point (TF), 4 collinear points (IE, weights of eq
// spaceInt) or 4 x 4 points on a face (IEFACE, first odd axis fastest).
struct HostTables {
  std::vector<uint8_t> cls_c, cls_f;
  std::vector<int64_t> hnode, rnode, tnf, tnc;
  std::vector<int32_t> rnp, rpt;
};

static void build_tables(const Geo& g, HostTables& t) {
  t.cls_c.resize((size_t)g.Nc);
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y)
      for (int x = 0; x < g.n[0]; ++x)
        t.cls_c[(size_t)x + (size_t)g.n[0] * ((size_t)y + (size_t)g.n[1] * z)] = (uint8_t)coarse_class(g, x, y, z);
  if (!g.has_fine) return;
  t.cls_f.resize((size_t)g.Nf);
  for (int z = 0; z < g.nf[2]; ++z)
    for (int y = 0; y < g.nf[1]; ++y)
      for (int x = 0; x < g.nf[0]; ++x)
        t.cls_f[(size_t)x + (size_t)g.nf[0] * ((size_t)y + (size_t)g.nf[1] * z)] = (uint8_t)fine_class(g, x, y, z);
  // history nodes in coarse index order
  std::vector<int64_t> hof((size_t)g.Nc, -1);
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y)
      for (int x = 0; x < g.n[0]; ++x) {
        const int c[3] = {x, y, z};
        bool inb = true, onp = false;
        for (int d = 0; d < g.D; ++d) {
          if (c[d] < g.a[d] - 1 || c[d] > g.a[d] + g.m[d] + 1) inb = false;
          if (c[d] == g.a[d] || c[d] == g.a[d] + g.m[d]) onp = true;
        }
        if (inb && onp) {
          const int64_t ci = (int64_t)x + (int64_t)g.n[0] * ((int64_t)y + (int64_t)g.n[1] * z);
          hof[(size_t)ci] = (int64_t)t.hnode.size();
          t.hnode.push_back(ci);
        }
      }
  auto cidx = [&](int x, int y, int z) -> int64_t {
    return (int64_t)wrap(x, g.n[0]) + (int64_t)g.n[0] * ((int64_t)wrap(y, g.n[1]) + (int64_t)g.n[1] * wrap(z, g.n[2]));
  };
  for (int z = 0; z < g.nf[2]; ++z)
    for (int y = 0; y < g.nf[1]; ++y)
      for (int x = 0; x < g.nf[0]; ++x) {
        const int64_t fi = (int64_t)x + (int64_t)g.nf[0] * ((int64_t)y + (int64_t)g.nf[1] * z);
        const int cl = t.cls_f[(size_t)fi];
        if (cl == FC_TN) {
          t.tnf.push_back(fi);
          t.tnc.push_back(cidx(g.a[0] + x / 2, g.a[1] + y / 2, g.D == 3 ? g.a[2] + z / 2 : 0));
          continue;
        }
        if (cl != FC_TF && cl != FC_IE && cl != FC_IEFACE) continue;
        const int j[3] = {x, y, z};
        int odd[2] = {-1, -1}, no = 0;
        int base[3] = {0, 0, 0};
        for (int d = 0; d < g.D; ++d) {
          if (j[d] & 1) odd[no++] = d;
          else base[d] = g.a[d] + j[d] / 2;
        }
        int32_t pts[16];
        int np = 1;
        if (no == 0) {
          pts[0] = (int32_t)hof[(size_t)cidx(base[0], base[1], base[2])];
        } else if (no == 1) {
          np = 4;
          for (int s = 0; s < 4; ++s) {
            int c[3] = {base[0], base[1], base[2]};
            c[odd[0]] = g.a[odd[0]] + (j[odd[0]] - 3) / 2 + s;
            pts[s] = (int32_t)hof[(size_t)cidx(c[0], c[1], c[2])];
          }
        } else {
          np = 16;
          for (int s1 = 0; s1 < 4; ++s1)
            for (int s0 = 0; s0 < 4; ++s0) {
              int c[3] = {base[0], base[1], base[2]};
              c[odd[0]] = g.a[odd[0]] + (j[odd[0]] - 3) / 2 + s0;
              c[odd[1]] = g.a[odd[1]] + (j[odd[1]] - 3) / 2 + s1;
              pts[4 * s1 + s0] = (int32_t)hof[(size_t)cidx(c[0], c[1], c[2])];
            }
        }
        for (int s = 0; s < np; ++s)
          if (pts[s] < 0) throw LbmError(LBM_EINVAL, "ring stencil leaves the history set");
        t.rnode.push_back(fi);
        t.rnp.push_back(np);
        for (int s = 0; s < 16; ++s) t.rpt.push_back(s < np ? pts[s] : -1);
      }
}

// ---------------------------------------------------------------------------
// Grid implementation (virtual over lattice and storage precision).
struct GridBase {
  lbm_grid_desc desc{};
  Geo g{};
  HostTables tabs;
  std::string err;
  hipStream_t stream = nullptr;
  int device = 0;
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  int64_t prof_launches = 0;
  double prof_ms = 0.0;
  int timed_factor = 1;  // fine substeps one timed launch performs
  // Nested refinement: the fine level carries a patch of its own.  child is
  // the pair (fine level, its patch), a grid whose periodic coarse level is
  // this grid's fine level -- the same buffers and layout; its wrap reaches
  // only the fine ring, which this grid rebuilds -- and whose steps replace
  // this grid's fine substeps.  Levels 1 and 2 of the nested grid are the
  // child's levels 0 and 1.
  std::unique_ptr<GridBase> child;
  // Set on the child of a nested grid.  Its coarse level is the parent's
  // fine level, whose ring the parent rebuilds: with H-RR the parent writes
  // the ring's rho and u at the child's time into the child's coarse
  // velocity planes (coarse_vel_hook, run right after the child's coarse
  // velocity pass), so that the child's centred differences next to the
  // ring take them; the child's coarse level never takes the one-pass form,
  // which computes every velocity itself.
  bool nested_child = false;
  std::function<void(hipStream_t)> coarse_vel_hook;
  virtual ~GridBase() {
    for (auto& e : events) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    if (stream) (void)hipStreamDestroy(stream);
  }
  virtual void init() = 0;
  virtual void step(int n, hipStream_t s) = 0;
  virtual void set_state(int level, const double* rho, const double* u, bool dev) = 0;
  virtual void get_macros(int level, double* rho, double* u, bool dev) = 0;
  virtual void set_pops(int level, const double* f, bool dev) = 0;
  virtual void get_pops(int level, double* f, bool dev) = 0;
  virtual void totals(double* mass, double* mom) = 0;
  // The same reduction with its partial sums in `part` (4 doubles per block
  // of 256 nodes) and its four final sums in `fin`, both device memory.
  virtual void totals_in(double* mass, double* mom, double* part, double* fin) = 0;
  virtual void tune(int reps, int32_t* out) = 0;
  virtual void set_variants(const int32_t* v) = 0;
  virtual void sensors_enable(bool on) = 0;
  virtual void set_dynamic_sigma(bool on, double sigma_dyn, double thr) = 0;
  virtual void sensors(int level, double thr, uint8_t* flags, double* prod, bool dev) = 0;
  virtual void probe_enable(int level, const int32_t* node, int64_t capacity) = 0;
  virtual int64_t probe_read(double* out, int64_t max) = 0;
  virtual void* coarse_buffer(int i) const = 0;
  virtual size_t coarse_bytes() const = 0;
  virtual void* coarse_mac() const = 0;
  virtual size_t coarse_mac_bytes() const = 0;
  int64_t nodes(int level) const {
    if (child && level >= 1) return child->nodes(level - 1);
    return level == 0 ? g.Nc : g.Nf;
  }
  int levels() const { return child ? 3 : (g.has_fine ? 2 : 1); }
  int64_t updates() const {
    if (!g.has_fine) return g.Nc;
    int64_t cov = 1;
    for (int d = 0; d < g.D; ++d) cov *= (g.m[d] - 3);
    // a nested fine level: its own evolving nodes plus twice its patch, twice
    return g.Nc - cov + 2 * (child ? child->updates() : g.Nf);
  }
};

template <int LAT, int PREC>
struct Grid final : GridBase {
  using L = Lattice<LAT>;
  static constexpr bool DEV = PREC == LBM_FP32_DEV;
  using S = typename std::conditional<DEV, float, double>::type;  // stored and bulk compute type
  static constexpr int Q = L::Q, D = L::D;
  // history fields per node: the largest layout over the collision models
  static constexpr int HN = HF<LAT, M_BGK>::N > HF<LAT, M_HRR>::N ? HF<LAT, M_BGK>::N : HF<LAT, M_HRR>::N;
  static constexpr bool NT = true;  // non-temporal stores of the streamed populations
  static constexpr int V = VecOf<S>::V;
  // Bulk-kernel launch variants: residency caps through dynamic LDS
  // (kVarLds); the chosen variant per role: 0 coarse stream, 1 fine stream,
  // 2 coarse H-RR collision, 3 fine H-RR collision.
  static constexpr int NVAR = kNVar;
  static constexpr int kDefaultVar = 2;
  int var[4] = {kDefaultVar, kDefaultVar, kDefaultVar, kDefaultVar};

  DevBuf cbuf[2], fbuf[3], mac_c, mac_f, hist[3], G, tmp_rho, tmp_u, tmp_f, part, tot;
  DevBuf xbuf;  // D3Q19 BGK / RR: compact copy of the fine x-bands at t+1/2 (xband_at)
  DevBuf d_hnode, d_rnode, d_rnp, d_rpt, d_tnf, d_tnc;
  int cpar = 0;  // coarse buffer holding the current state
  // Fine buffers: fbuf[fpar] holds the state at integer times.  A fused step
  // (BGK / RR: always in 2D, k_fine2; in 3D when the fine-role variant picks
  // k_fine3s) runs both fine substeps in one kernel from fbuf[fpar] into the
  // other buffer, which then becomes current; fbuf[2] receives the t+1/2
  // ring and the t+1/2 band the fine-to-coarse transfer pulls from.
  // Otherwise the substeps go fbuf[fpar] -> other -> fbuf[fpar].
  int fpar = 0;
  bool fused = false;
  int n_cu = 0;
  int f3_slots[kNVar] = {0, 0, 0, 0};  // resident k_fine3s work groups per device, per variant
  int h3_slots[kNVar] = {0, 0, 0, 0};  // the same for k_hrr3 / k_hrr3s
  int hs[3] = {0, 1, 2};
  Iface itf{};
  double tau_c = 0, tau_f = 0, sig = 0;
  // The stepping stores only the ring populations it reads again (k_ring
  // PARTIAL); true while fine A holds such a partial ring.
  bool ring_partial = false;
  // NH sensors: while on, the last step of each lbm_step call (rec_fine:
  // the read-out sees no other) records the velocities of the iteration
  // before its last one (coarse t, fine t+1/2) in sUc[sc_cur] / sUf (double
  // planes [1 + D][padded positions]) and keeps the t+1/2 state: D2Q9 BGK /
  // RR in the fused kernel (k_fine2 SENS writes both, the state into
  // fbuf[2]); otherwise a recording pass before the step and the fine
  // substeps as two launches (the t+1/2 state in fine B).  Coarse, BGK / RR
  // two-level: the last two steps' stream and transfer (SENS, rec_coarse)
  // record the state they leave into sUc[sc_cur ^ 1], which the next step
  // takes over instead of a recording pass (sens_coarse_next).  sens_ready:
  // a step has been recorded and nothing has touched the state since.
  bool sensors_on = false, sens_ready = false;
  bool rec_fine = false, rec_coarse = false;
  bool sens_pre_half = false;  // the last step was fused: its t+1/2 state is in fbuf[2]
  bool sens_coarse_next = false;
  int sc_cur = 0;
  DevBuf sUc[2], sUf, sFlags, sProd;
  // Dynamic sigma (H-RR): while on, the bulk H-RR collisions take sig_dyn
  // where the sensors' divergence or curl product falls below -dyn_thr
  // (k_collide_hrr DYN); dynC / dynF hold each node's previous divergence
  // and curl ([4][padded positions] in the storage type).  D2Q9 keeps its
  // one-pass kernels (k_hrr2, k_hrr2c DYN); D3Q19 takes the two-pass H-RR
  // substeps (its one-pass kernels carry no such state).
  bool dyn_on = false;
  double sig_dyn = 0.0, dyn_thr = 0.0;
  DevBuf dynC, dynF;
  // probe: density at one node of a level appended to pSeries each step
  int probe_level = -1;
  int64_t probe_pos = 0, probe_cap = 0;
  DevBuf pSeries, pCount;

  // Velocity planes (H-RR): padded planes plus 64 spare elements.
  static size_t plane_bytes(int64_t NP, int nplanes) { return sizeof(S) * ((size_t)NP * nplanes + 64); }
  // Populations: whole storage blocks up to and including position NP.
  static size_t pop_bytes(int64_t NP) { return sizeof(S) * (size_t)pop_elems<S>(NP, Q); }

  void init() override {
    fused = desc.collision != LBM_HRR && g.has_fine && !child;
    HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
    if (fused) var[1] = 0;
    if (D == 3 && desc.collision == LBM_HRR) var[3] = 0;
    timed_factor = fused_now() ? 2 : 1;
    // every state buffer starts at zero: the state is zero until
    // lbm_set_state, and values no step writes (the populations of covered
    // coarse nodes in the buffer they are not set in) stay the same from
    // run to run
    auto zalloc = [](DevBuf& b, size_t bytes) {
      b.alloc(bytes);
      if (bytes) HIPCHK(hipMemset(b.p, 0, bytes));
    };
    for (int p = 0; p < 2; ++p) zalloc(cbuf[p], pop_bytes(g.Ncp));
    if (child) {
      // the fine level is the child's coarse level: its two state buffers
      for (int p = 0; p < 2; ++p) fbuf[p].view(child->coarse_buffer(p), child->coarse_bytes());
    } else if (g.has_fine) {
      for (int p = 0; p < (fused ? 3 : 2); ++p) zalloc(fbuf[p], pop_bytes(g.Nfp));
    }
    if (g.has_fine && !child && D == 3 && desc.collision != LBM_HRR)
      zalloc(xbuf, sizeof(S) * (size_t)xband_elems(g, Q));
    if (desc.collision == LBM_HRR) {
      zalloc(mac_c, plane_bytes(g.Ncp, 1 + D));
      // a nested grid's fine velocity planes are the child's coarse ones
      if (child) mac_f.view(child->coarse_mac(), child->coarse_mac_bytes());
      else if (g.has_fine) zalloc(mac_f, plane_bytes(g.Nfp, 1 + D));
    }
    tau_c = desc.tau_coarse;
    tau_f = 2.0 * tau_c - 0.5;
    sig = desc.sigma;
    if (g.has_fine) {
      const size_t NH = tabs.hnode.size();
      for (int s = 0; s < 3; ++s) zalloc(hist[s], sizeof(double) * HN * NH);
      zalloc(G, sizeof(double) * HN * NH);
      auto up = [&](DevBuf& b, const void* src, size_t bytes) {
        b.alloc(bytes);
        if (bytes) HIPCHK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
      };
      up(d_hnode, tabs.hnode.data(), sizeof(int64_t) * tabs.hnode.size());
      up(d_rnode, tabs.rnode.data(), sizeof(int64_t) * tabs.rnode.size());
      up(d_rnp, tabs.rnp.data(), sizeof(int32_t) * tabs.rnp.size());
      up(d_rpt, tabs.rpt.data(), sizeof(int32_t) * tabs.rpt.size());
      up(d_tnf, tabs.tnf.data(), sizeof(int64_t) * tabs.tnf.size());
      up(d_tnc, tabs.tnc.data(), sizeof(int64_t) * tabs.tnc.size());
      itf.NH = (int64_t)tabs.hnode.size();
      itf.hnode = d_hnode.as<int64_t>();
      itf.NR = (int64_t)tabs.rnode.size();
      itf.rnode = d_rnode.as<int64_t>();
      itf.rnp = d_rnp.as<int32_t>();
      itf.rpt = d_rpt.as<int32_t>();
      itf.NT = (int64_t)tabs.tnf.size();
      itf.tnf = d_tnf.as<int64_t>();
      itf.tnc = d_tnc.as<int64_t>();
    }
    const size_t Nmax = (size_t)std::max(g.Nc, g.Nf);
    tmp_rho.alloc(sizeof(double) * Nmax);
    tmp_u.alloc(sizeof(double) * D * Nmax);
    part.alloc(sizeof(double) * 4 * ((Nmax + 255) / 256));
    tot.alloc(sizeof(double) * 4);
    for (int p = 0; p < 2; ++p) HIPCHK(hipMemset(cbuf[p].p, 0, cbuf[p].bytes));
    if (g.has_fine && !child)
      for (int p = 0; p < (fused ? 3 : 2); ++p) HIPCHK(hipMemset(fbuf[p].p, 0, fbuf[p].bytes));
    if (mac_c.p) HIPCHK(hipMemset(mac_c.p, 0, mac_c.bytes));
    if (mac_f.p) HIPCHK(hipMemset(mac_f.p, 0, mac_f.bytes));
  }

  static unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
  // Grid of an interface-node kernel (xcd_block): a multiple of the XCD count.
  static unsigned xblocks(int64_t n, int bs) { return (blocks(n, bs) + kXCD - 1) / kXCD * kXCD; }

  Flat flat(int level) const {
    if (level == 0) return make_flat(g.n[0], g.n[1], g.n[2], V, false, D);
    return make_flat(g.nf[0], g.nf[1], g.nf[2], V, true, D);
  }

  void* coarse_buffer(int i) const override { return cbuf[i].p; }
  size_t coarse_bytes() const override { return cbuf[0].bytes; }
  void* coarse_mac() const override { return mac_c.p; }
  size_t coarse_mac_bytes() const override { return mac_c.bytes; }
  void no_nesting(const char* what) const {
    if (child) throw LbmError(LBM_EUNSUPPORTED, std::string(what) + " is not available for a nested grid");
  }
  S* cur_c() { return cbuf[cpar].as<S>(); }
  S* fineA() { return fbuf[fpar].as<S>(); }       // state at integer times
  S* fineB() { return fbuf[fpar ^ 1].as<S>(); }   // the other buffer

  template <int MODEL, int LEVEL>
  void launch_stream(const S* src, S* dst, S* mac, double tau, hipStream_t s, int v = -1, S* xb = nullptr) {
    if (v < 0) v = var[LEVEL];
    const Flat f = flat(LEVEL);
    if (f.nchunks == 0) return;
    hipLaunchKernelGGL((k_stream<LAT, DEV, S, MODEL, LEVEL, NT>), dim3((unsigned)(f.per_xcd * kXCD)), dim3(256),
                       (unsigned)kVarLds[v], s, src, dst, mac, g, f, (S)(1.0 - 1.0 / tau), xb);
  }
  // Coarse stream (BGK, RR) and the t+1/2 ring reconstruction from G into
  // fdst, one launch (k_stream_ring).
  template <int MODEL>
  // su: the NH sensors' record of the coarse state it leaves (SENS), or null
  void launch_stream_ring(const S* src, S* dst, S* fdst, double kf, double omf, hipStream_t s, S* xb = nullptr,
                          double* su = nullptr) {
    const Flat f = flat(0);
    const unsigned nrb = xblocks(itf.NR, 256);
    const dim3 gr(nrb + (unsigned)(f.per_xcd * kXCD)), bl(256);
    const unsigned lds = (unsigned)kVarLds[var[0]];
    const S om = (S)(1.0 - 1.0 / tau_c);
    if (su)
      hipLaunchKernelGGL((k_stream_ring<LAT, DEV, S, MODEL, NT, true>), gr, bl, lds, s, src, dst, g, f, om,
                         G.as<double>(), fdst, itf, kf, omf, tau_f, sig, (int)nrb, xb, su);
    else
      hipLaunchKernelGGL((k_stream_ring<LAT, DEV, S, MODEL, NT, false>), gr, bl, lds, s, src, dst, g, f, om,
                         G.as<double>(), fdst, itf, kf, omf, tau_f, sig, (int)nrb, xb, (double*)nullptr);
  }
  // The t+1 ring (Hp -> fdst) and the fine-to-coarse transfer (src_f ->
  // the TN nodes of cdst), one launch (k_ring_coalesce); su as above.
  template <int MODEL>
  void launch_ring_coalesce(const double* Hp, S* fdst, const S* src_f, S* cdst, const S* xb, double* su,
                            hipStream_t s) {
    constexpr int PER = 256 / (D == 2 ? 9 : 27);
    const unsigned br2 = xblocks(itf.NR, 256), bc = xblocks(itf.NT, PER);
    const double kf = tau_f / (2.0 * tau_c), kc = 2.0 * tau_c / tau_f;
    const double omf = 1.0 - 1.0 / tau_f, omc = 1.0 - 1.0 / tau_c;
    if (su)
      hipLaunchKernelGGL((k_ring_coalesce<LAT, DEV, S, MODEL, true>), dim3(br2 + bc), dim3(256), 0, s, Hp, fdst, src_f,
                         cdst, g, itf, kf, omf, tau_f, kc, omc, tau_c, sig, (int)br2, xb, su);
    else
      hipLaunchKernelGGL((k_ring_coalesce<LAT, DEV, S, MODEL, false>), dim3(br2 + bc), dim3(256), 0, s, Hp, fdst,
                         src_f, cdst, g, itf, kf, omf, tau_f, kc, omc, tau_c, sig, (int)br2, xb, (double*)nullptr);
  }

  // One H-RR fine substep in one pass (D2Q9, k_hrr2): variants of the fine
  // H-RR role are tile shapes (lanes, vectors x rows) 64 x 8, 32 x 8,
  // 32 x 16, 128 x 4.
  // dyn: with dynamic sigma on, the DYN kernels and the fine level's state
  // (stepping only; the tuner's trial launches leave the state alone)
  template <int HXV, int HYR>
  void go_hrr2(const S* src, S* dst, const S* mac, hipStream_t s, bool dyn) {
    if constexpr (D == 2) {
      const int ntx = fine2_ntx<S>(g, HXV), nty = fine2_nty(g, HYR);
      const int per = (ntx * nty + kXCD - 1) / kXCD;
      const dim3 gr((unsigned)(per * kXCD)), bl(HXV * HYR);
      if (dyn && dyn_on)
        hipLaunchKernelGGL((k_hrr2<LAT, DEV, S, NT, HXV, HYR, true>), gr, bl, 0, s, src, dst, mac, g,
                           (S)(1.0 - 1.0 / tau_f), (S)tau_f, (S)sig, ntx, nty, per, dynF.as<S>(), (S)sig_dyn,
                           (S)dyn_thr);
      else
        hipLaunchKernelGGL((k_hrr2<LAT, DEV, S, NT, HXV, HYR, false>), gr, bl, 0, s, src, dst, mac, g,
                           (S)(1.0 - 1.0 / tau_f), (S)tau_f, (S)sig, ntx, nty, per, (S*)nullptr, (S)0, (S)0);
    }
  }
  // The coarse level in one pass (D2Q9 H-RR, rows a whole number of vectors:
  // coarse_one_pass()); same tile variants, role 2.
  bool coarse_one_pass() const {
    return D == 2 && desc.collision == LBM_HRR && g.n[0] % V == 0 && !nested_child;
  }
  // D2Q9 H-RR fine substeps in one pass (k_hrr2)
  bool fine_one_pass2() const { return D == 2; }
  template <int HXV, int HYR>
  void go_hrr2c(const S* src, S* dst, const S* mac, hipStream_t s, bool dyn) {
    if constexpr (D == 2) {
      const int ntx = (g.n[0] / V + HXV - 3) / (HXV - 2), nty = (g.n[1] + HYR - 3) / (HYR - 2);
      const int per = (ntx * nty + kXCD - 1) / kXCD;
      const dim3 gr((unsigned)(per * kXCD)), bl(HXV * HYR);
      if (dyn && dyn_on)
        hipLaunchKernelGGL((k_hrr2c<LAT, DEV, S, NT, HXV, HYR, true>), gr, bl, 0, s, src, dst, mac, g,
                           (S)(1.0 - 1.0 / tau_c), (S)tau_c, (S)sig, ntx, nty, per, dynC.as<S>(), (S)sig_dyn,
                           (S)dyn_thr);
      else
        hipLaunchKernelGGL((k_hrr2c<LAT, DEV, S, NT, HXV, HYR, false>), gr, bl, 0, s, src, dst, mac, g,
                           (S)(1.0 - 1.0 / tau_c), (S)tau_c, (S)sig, ntx, nty, per, (S*)nullptr, (S)0, (S)0);
    }
  }
  void launch_hrr2c(const S* src, S* dst, const S* mac, hipStream_t s, int v = -1, bool dyn = false) {
    if (v < 0) v = var[2];
    switch (v) {
      case 0: go_hrr2c<64, 8>(src, dst, mac, s, dyn); break;
      case 1: go_hrr2c<32, 8>(src, dst, mac, s, dyn); break;
      case 2: go_hrr2c<32, 16>(src, dst, mac, s, dyn); break;
      default: go_hrr2c<128, 4>(src, dst, mac, s, dyn); break;
    }
  }
  void launch_hrr2(const S* src, S* dst, const S* mac, hipStream_t s, int v = -1, bool dyn = false) {
    if (v < 0) v = var[3];
    switch (v) {
      case 0: go_hrr2<64, 8>(src, dst, mac, s, dyn); break;
      case 1: go_hrr2<32, 8>(src, dst, mac, s, dyn); break;
      case 2: go_hrr2<32, 16>(src, dst, mac, s, dyn); break;
      default: go_hrr2<128, 4>(src, dst, mac, s, dyn); break;
    }
  }

  // dyn: use the dynamic-sigma state (stepping only; the tuner's trial
  // launches leave it alone)
  template <int LEVEL>
  void launch_collide_hrr(const S* src, S* dst, const S* mac, double tau, hipStream_t s, int v = -1,
                          bool dyn = false) {
    if (v < 0) v = var[2 + LEVEL];
    const Flat f = flat(LEVEL);
    if (f.nchunks == 0) return;
    const dim3 gr((unsigned)(f.per_xcd * kXCD)), bl(256);
    if (dyn && dyn_on)
      hipLaunchKernelGGL((k_collide_hrr<LAT, DEV, S, LEVEL, NT, true>), gr, bl, (unsigned)kVarLds[v], s, src, dst, mac,
                         g, f, (S)(1.0 - 1.0 / tau), (S)tau, (S)sig, (LEVEL == 0 ? dynC : dynF).as<S>(), (S)sig_dyn,
                         (S)dyn_thr);
    else
      hipLaunchKernelGGL((k_collide_hrr<LAT, DEV, S, LEVEL, NT, false>), gr, bl, (unsigned)kVarLds[v], s, src, dst,
                         mac, g, f, (S)(1.0 - 1.0 / tau), (S)tau, (S)sig, (S*)nullptr, (S)0, (S)0);
  }

  // Both fine substeps (BGK / RR), src -> dst, t+1/2 ring and band in half.
  // D2Q9 variants of the fine role (halo-tile lanes, vectors x rows): 64 x 8,
  // 64 x 16, 32 x 16 and 32 x 8 (measured on the 4097 x 2049 patch, FP32:
  // 119, 134-147, 135 and 135 us; narrower or non-power-of-two widths and
  // 1024-lane tiles were slower still).
  // su: the NH sensors' velocity planes of the t+1/2 iteration (k_fine2
  // SENS records them, and the whole t+1/2 state into half), or null.
  template <int MODEL, int HXV, int HYR>
  void go_fine2(const S* src, S* dst, S* half, hipStream_t s, double* su = nullptr) {
    if constexpr (D == 2 && MODEL != M_HRR) {
      const int ntx = fine2_ntx<S>(g, HXV), nty = fine2_nty(g, HYR);
      const int per = (ntx * nty + kXCD - 1) / kXCD;
      const dim3 gr((unsigned)(per * kXCD)), bl(HXV * HYR);
      if (su)
        hipLaunchKernelGGL((k_fine2<LAT, DEV, S, MODEL, NT, HXV, HYR, 4, true>), gr, bl, 0, s, src, dst, half, g,
                           (S)(1.0 - 1.0 / tau_f), ntx, nty, per, su);
      else
        hipLaunchKernelGGL((k_fine2<LAT, DEV, S, MODEL, NT, HXV, HYR, 4, false>), gr, bl, 0, s, src, dst, half, g,
                           (S)(1.0 - 1.0 / tau_f), ntx, nty, per, (double*)nullptr);
    }
  }
  // Work decomposition of a marching fine kernel (k_hrr3) with TXV x TY
  // tiles of vectors, for `slots` resident work groups on the device: a run
  // of zlen planes costs zlen + 2 planes of work (its first step needs two
  // more), and runs are at least kMinZRun planes long so that this overhead
  // stays small, while the work groups fill the device in few rounds.
  struct ZRuns {
    int ntx, nty, nzc, zlen, per;
  };
  ZRuns zruns(int TXV, int TY, int slots) const {
    const int nv = (g.nf[0] - 1 + V - 1) / V;
    return zruns_tiles((nv + TXV - 1) / TXV, (g.nf[1] - 2 + TY - 1) / TY, slots);
  }
  // zcap: longest run allowed (runs of the one-node-per-lane kernels address
  // their storage window with 32-bit byte offsets).
  ZRuns zruns_tiles(int ntx, int nty, int slots, int zcap = 1 << 30) const {
    ZRuns r;
    r.ntx = ntx;
    r.nty = nty;
    const int nzm = g.nf[2] - 2;
    const int64_t ntile = (int64_t)r.ntx * r.nty;
    r.zlen = std::min(nzm, zcap);
    double best = -1.0;
    constexpr int kMinZRun = 8;
    for (int nzc = 1; nzc <= nzm; ++nzc) {
      const int zl = (nzm + nzc - 1) / nzc;
      if (zl > zcap) continue;
      if (zl < kMinZRun && nzc > 1 && zl < zcap) break;
      if ((nzm + zl - 1) / zl != nzc) continue;
      const int64_t rounds = (ntile * nzc + slots - 1) / slots;
      const double cost = (double)rounds * (zl + 2);
      if (best < 0.0 || cost < best) {
        best = cost;
        r.zlen = zl;
      }
    }
    r.nzc = (nzm + r.zlen - 1) / r.zlen;
    r.per = (int)((ntile * r.nzc + kXCD - 1) / kXCD);
    return r;
  }
  template <typename K>
  int occupancy_slots(K kern, int& cache, int lanes = 256) {
    if (cache == 0) {
      int nb = 0;
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, lanes, 0));
      cache = std::max(1, nb) * std::max(1, n_cu);
    }
    return cache;
  }
  // Both fine substeps in one marching kernel with one node per lane
  // (k_fine3s): tiles of (TXH - 2) x (TYH - 2) middle nodes.  The tile
  // counts come from nodes, not vectors; the runs are cut as for k_hrr3.
  // Longest run of a one-node-per-lane marching kernel: its storage window
  // (zlen + 4 planes and one storage block) stays below 2^32 bytes.
  int window_zcap() const {
    const double plane = (double)g.pf * g.nf[1] * Q * sizeof(S);
    const double room = 2147483648.0 - 2.0 * (double)PopBlock<S>::B * Q * sizeof(S);
    return std::max(0, (int)std::floor(room / plane) - 4);
  }
  template <int MODEL, int TXH, int TYH, int MINW>
  void go_fine3s(const S* src, S* dst, S* half, hipStream_t s, int v) {
    if constexpr (D == 3 && MODEL != M_HRR) {
      auto kern = k_fine3s<LAT, DEV, S, MODEL, NT, TXH, TYH, MINW>;
      const int ntx = (g.nf[0] - 2 + TXH - 3) / (TXH - 2), nty = (g.nf[1] - 2 + TYH - 3) / (TYH - 2);
      const int zcap = window_zcap();
      if (zcap < 1) throw LbmError(LBM_EUNSUPPORTED, "fine planes too large for the one-pass fused kernel");
      // the compact x-band copy is addressed with 32-bit byte offsets too
      if ((double)xband_elems(g, Q) * sizeof(S) >= 2147483648.0)
        throw LbmError(LBM_EUNSUPPORTED, "fine x-bands too large for the one-pass fused kernel");
      const ZRuns r = zruns_tiles(ntx, nty, occupancy_slots(kern, f3_slots[v], TXH * TYH), zcap);
      hipLaunchKernelGGL(kern, dim3((unsigned)(r.per * kXCD)), dim3(TXH * TYH), 0, s, src, dst, half, xbuf.as<S>(),
                         g, (S)(1.0 - 1.0 / tau_f), r.ntx, r.nty, r.nzc, r.zlen, r.per);
    }
  }
  // One H-RR fine substep in one pass (D3Q19): fine H-RR role variant 2 is
  // k_hrr3 (30 x 6 tiles of vectors), variant 3 k_hrr3s (one node per lane,
  // 64 x 8 lanes in FP32, 34 x 8 in FP64); variants 0 and 1 run the velocity
  // pass and k_collide_hrr (capped at 2 / 3 resident work groups).  On the
  // 385^3 patch in FP32, per substep: k_hrr3 2.78 ms, k_hrr3s 2.91 ms, the
  // two-pass form 1.0 + 1.78 ms; the one-pass kernels save the velocity
  // pass's traffic but re-read their tile halos from HBM.
  bool hrr_one_pass3() const { return D == 3 && desc.collision == LBM_HRR && var[3] >= 2 && !dyn_on; }
  int hrr_lds_var(int v) const { return (D == 3 && desc.collision == LBM_HRR) ? (v == 0 ? 2 : 1) : v; }
  template <int TXV, int TY>
  void go_hrr3(const S* src, S* dst, const S* mac, hipStream_t s, int v) {
    if constexpr (D == 3) {
      auto kern = k_hrr3<LAT, DEV, S, NT, TXV, TY, 2>;
      const ZRuns r = zruns(TXV, TY, occupancy_slots(kern, h3_slots[v]));
      hipLaunchKernelGGL(kern, dim3((unsigned)(r.per * kXCD)), dim3(256), 0, s, src, dst, mac, g,
                         (S)(1.0 - 1.0 / tau_f), (S)tau_f, (S)sig, r.ntx, r.nty, r.nzc, r.zlen, r.per);
    }
  }
  template <int TXH, int TYH>
  void go_hrr3s(const S* src, S* dst, const S* mac, hipStream_t s, int v) {
    if constexpr (D == 3) {
      auto kern = k_hrr3s<LAT, DEV, S, NT, TXH, TYH, 1>;
      const int ntx = (g.nf[0] - 2 + TXH - 3) / (TXH - 2), nty = (g.nf[1] - 2 + TYH - 3) / (TYH - 2);
      const int zcap = window_zcap();
      // the velocity planes are read through a window of 2^31 bytes as well
      if (zcap < 1 || (double)(1 + D) * g.Nfp * sizeof(S) >= 2147483648.0)
        throw LbmError(LBM_EUNSUPPORTED, "fine level too large for the one-pass H-RR kernel");
      const ZRuns r = zruns_tiles(ntx, nty, occupancy_slots(kern, h3_slots[v], TXH * TYH), zcap);
      hipLaunchKernelGGL(kern, dim3((unsigned)(r.per * kXCD)), dim3(TXH * TYH), 0, s, src, dst, mac, g,
                         (S)(1.0 - 1.0 / tau_f), (S)tau_f, (S)sig, r.ntx, r.nty, r.nzc, r.zlen, r.per);
    }
  }
  void launch_hrr3(const S* src, S* dst, const S* mac, hipStream_t s, int v = -1) {
    if (v < 0) v = var[3];
    if constexpr (sizeof(S) == 4) {
      if (v == 2) go_hrr3<30, 6>(src, dst, mac, s, 2);
      else go_hrr3s<64, 8>(src, dst, mac, s, 3);
    } else {
      if (v == 2) go_hrr3<30, 6>(src, dst, mac, s, 2);
      else go_hrr3s<34, 8>(src, dst, mac, s, 3);
    }
  }
  template <int MODEL>
  void launch_fused(const S* src, S* dst, S* half, hipStream_t s, int v = -1, double* su = nullptr) {
    if (v < 0) v = var[1];
    if constexpr (D == 2) {
      switch (v) {
        case 0: go_fine2<MODEL, 64, 8>(src, dst, half, s, su); break;
        case 1: go_fine2<MODEL, 64, 16>(src, dst, half, s, su); break;
        case 2: go_fine2<MODEL, 32, 16>(src, dst, half, s, su); break;
        default: go_fine2<MODEL, 32, 8>(src, dst, half, s, su); break;
      }
    } else if constexpr (sizeof(S) == 4) {
      if (v == 2) go_fine3s<MODEL, 64, 16, 1>(src, dst, half, s, 2);
      else go_fine3s<MODEL, 64, 8, 1>(src, dst, half, s, 3);
    } else {
      if (v == 2) go_fine3s<MODEL, 34, 14, 1>(src, dst, half, s, 2);
      else go_fine3s<MODEL, 34, 8, 1>(src, dst, half, s, 3);
    }
  }

  // Runs fn (one launch) between HIP events on s when profiling is on.
  template <typename Fn>
  void timed(hipStream_t s, Fn&& fn) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, s));
    }
    fn();
    if (profile) {
      HIPCHK(hipEventRecord(e1, s));
      events.emplace_back(e0, e1);
    }
  }
  // True when this step runs both fine substeps in one kernel.
  // (D2Q9 stays fused when it records the NH sensors: k_fine2 SENS does)
  bool fused_now() const { return fused && (D == 2 || (!rec_fine && var[1] >= 2)); }
  // LDS variant of the fine k_stream launches for fine-role variant v.
  int fine_lds_var(int v) const { return (fused && D == 3) ? (v == 0 ? 2 : 1) : v; }
  // Fine-level pull-stream + collide (BGK, RR): the timed kernel.
  void fine_stream_timed(int model, const S* src, S* dst, hipStream_t s, S* xb = nullptr) {
    const int lv = fine_lds_var(var[1]);
    timed(s, [&] {
      if (model == M_BGK) launch_stream<M_BGK, 1>(src, dst, nullptr, tau_f, s, lv, xb);
      else launch_stream<M_RR, 1>(src, dst, nullptr, tau_f, s, lv, xb);
    });
  }

  // Autotuner: times every bulk-kernel variant of each role on this grid
  // (reps launches each, after one warm-up) and keeps the fastest.  Only
  // buffers that the next step rewrites are touched (the coarse and fine
  // buffers not holding the current state, and the macro planes).
  void role_launch(int role, int v, hipStream_t s) {
    const int model = desc.collision;
    S* c_cur = cur_c();
    S* c_oth = cbuf[cpar ^ 1].as<S>();
    if (role == 0) {
      if (model == M_BGK) launch_stream<M_BGK, 0>(c_cur, c_oth, nullptr, tau_c, s, v);
      else if (model == M_RR) launch_stream<M_RR, 0>(c_cur, c_oth, nullptr, tau_c, s, v);
      else launch_stream<M_HRR, 0>(c_cur, c_oth, mac_c.as<S>(), tau_c, s, v);
    } else if (role == 1 && fused && D == 3 && v < 2) {
      // both substeps as two launches (timed on the same buffers)
      for (int k = 0; k < 2; ++k) {
        if (model == M_BGK) launch_stream<M_BGK, 1>(fineA(), fineB(), nullptr, tau_f, s, fine_lds_var(v));
        else launch_stream<M_RR, 1>(fineA(), fineB(), nullptr, tau_f, s, fine_lds_var(v));
      }
    } else if (role == 1 && fused) {
      // both substeps: writes the other buffer and the t+1/2 band, which the
      // next step rewrites
      if (model == M_BGK) launch_fused<M_BGK>(fineA(), fineB(), fbuf[2].as<S>(), s, v);
      else launch_fused<M_RR>(fineA(), fineB(), fbuf[2].as<S>(), s, v);
    } else if (role == 1) {
      if (model == M_BGK) launch_stream<M_BGK, 1>(fineA(), fineB(), nullptr, tau_f, s, v);
      else if (model == M_RR) launch_stream<M_RR, 1>(fineA(), fineB(), nullptr, tau_f, s, v);
      else launch_stream<M_HRR, 1>(fineA(), fineB(), mac_f.as<S>(), tau_f, s, v);
    } else if (role == 2 && coarse_one_pass()) {
      launch_hrr2c(c_cur, c_oth, mac_c.as<S>(), s, v);
    } else if (role == 2) {
      launch_collide_hrr<0>(c_cur, c_oth, mac_c.as<S>(), tau_c, s, v);
    } else if (D == 2) {
      launch_hrr2(fineA(), fineB(), mac_f.as<S>(), s, v);
    } else if (v >= 2) {
      launch_hrr3(fineA(), fineB(), mac_f.as<S>(), s, v);
    } else {
      // the two passes the one-pass variants replace
      launch_stream<M_HRR, 1>(fineA(), fineB(), mac_f.as<S>(), tau_f, s);
      launch_collide_hrr<1>(fineA(), fineB(), mac_f.as<S>(), tau_f, s, hrr_lds_var(v));
    }
  }

  void set_variants(const int32_t* v) override {
    no_nesting("launch variants");
    for (int r = 0; r < 4; ++r)
      if (v[r] < 0 || v[r] >= NVAR) throw LbmError(LBM_EINVAL, "variant index out of range");
    for (int r = 0; r < 4; ++r) var[r] = v[r];
  }

  void tune(int reps, int32_t* out) override {
    HIPCHK(hipSetDevice(device));
    no_nesting("tuning");
    HIPCHK(hipStreamSynchronize(stream));
    sens_ready = sens_coarse_next = false;  // the trial launches overwrite the previous states
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int role = 0; role < 4; ++role) {
      const bool used = (role & 1) ? g.has_fine : true;
      const bool hrr_role = role >= 2;
      if (!used || (hrr_role && desc.collision != LBM_HRR)) continue;
      if (role == 1 && D == 2 && desc.collision == LBM_HRR) continue;  // no fine velocity pass (k_hrr2)
      if (role == 0 && coarse_one_pass()) continue;                    // no coarse velocity pass (k_hrr2c)

      float best = -1.f;
      for (int v = 0; v < NVAR; ++v) {
        try {
          role_launch(role, v, stream);
        } catch (const LbmError& e) {
          if (e.code != LBM_EUNSUPPORTED) throw;
          continue;  // this variant does not apply to the grid
        }
        HIPCHK(hipEventRecord(e0, stream));
        for (int k = 0; k < reps; ++k) role_launch(role, v, stream);
        HIPCHK(hipEventRecord(e1, stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (best < 0.f || ms < best) {
          best = ms;
          var[role] = v;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    for (int r = 0; r < 4; ++r) out[r] = var[r];
  }

  void step_uniform(hipStream_t s) {
    const int model = desc.collision;
    S* src = cbuf[cpar].as<S>();
    S* dst = cbuf[cpar ^ 1].as<S>();
    if (model == M_BGK) launch_stream<M_BGK, 0>(src, dst, nullptr, tau_c, s);
    else if (model == M_RR) launch_stream<M_RR, 0>(src, dst, nullptr, tau_c, s);
    else {
      launch_stream<M_HRR, 0>(src, dst, mac_c.as<S>(), tau_c, s);
      launch_collide_hrr<0>(src, dst, mac_c.as<S>(), tau_c, s, -1, true);
    }
    cpar ^= 1;
  }

  // One coarse step, Sec. 4.3: asynchronous iteration (coarse t -> t+1, fine
  // t -> t+1/2) then synchronous iteration (fine t+1/2 -> t+1).  Fine buffer
  // A holds the state at integer times, B at half times.
  template <int MODEL>
  void step_two_level(hipStream_t s) {
    S* csrc = cbuf[cpar].as<S>();
    S* cdst = cbuf[cpar ^ 1].as<S>();
    S* fA = fineA();
    S* fB = fineB();
    double* Hm = hist[hs[0]].as<double>();
    double* H0 = hist[hs[1]].as<double>();
    double* Hp = hist[hs[2]].as<double>();
    const int64_t NH = itf.NH;
    const double kf = tau_f / (2.0 * tau_c), kc = 2.0 * tau_c / tau_f;
    const double omf = 1.0 - 1.0 / tau_f, omc = 1.0 - 1.0 / tau_c;
    const double c0 = -1.0 / 8.0, c1 = 3.0 / 4.0, c2 = 3.0 / 8.0;  // eq TempInt at t+1/2
    constexpr int IB = kIfaceBlock;
    constexpr int PER = 256 / (D == 2 ? 9 : 27);
    const unsigned bh = xblocks(NH, IB), br = xblocks(itf.NR, IB), bt = xblocks(itf.NT, IB);
    const unsigned bc = xblocks(itf.NT, PER), br2 = xblocks(itf.NR, 256);
    // BGK / RR: the capture also interpolates every history value to t+1/2
    // (G); H-RR fills its strain-rate fields later and interpolates then
    hipLaunchKernelGGL((k_hist_capture<LAT, DEV, S, MODEL>), dim3(bh), dim3(IB), 0, s, csrc, Hp, g, itf,
                       MODEL == M_HRR ? nullptr : G.as<double>(), Hm, H0);
    timed_factor = fused_now() ? 2 : 1;
    sens_pre_half = MODEL != M_HRR && fused_now();
    // BGK / RR: the coarse record of the state this step leaves
    double* scn = MODEL != M_HRR && rec_coarse ? sUc[sc_cur ^ 1].as<double>() : nullptr;
    sens_coarse_next = scn != nullptr;
    if (MODEL != M_HRR && fused_now()) {
      S* fH = fbuf[2].as<S>();
      // D3Q19: the t+1/2 ring and the fused kernel also fill the compact
      // x-band copy, from which the transfer reads the x-bands
      S* xb = D == 3 ? xbuf.as<S>() : nullptr;
      launch_stream_ring<MODEL>(csrc, cdst, fH, kf, omf, s, xb, scn);
      timed(s, [&] { launch_fused<MODEL>(fA, fB, fH, s, -1, rec_fine ? sUf.as<double>() : nullptr); });
      launch_ring_coalesce<MODEL>(Hp, fB, fH, cdst, xb, scn, s);
      fpar ^= 1;
    } else if (MODEL != M_HRR) {
      // substep 1 writes the ring column x = nx - 1 of B, so the t+1/2 ring
      // (sharing a launch with the coarse stream) follows it; both also fill
      // the compact copy of the x-bands, from which the transfer reads
      S* xb = xbuf.as<S>();
      fine_stream_timed(MODEL, fA, fB, s, xb);
      launch_stream_ring<MODEL>(csrc, cdst, fB, kf, omf, s, xb, scn);
      fine_stream_timed(MODEL, fB, fA, s);
      launch_ring_coalesce<MODEL>(Hp, fA, fB, cdst, xb, scn, s);
    } else {
      S* mc = mac_c.as<S>();
      S* mf = mac_f.as<S>();
      // velocity passes (rho, u of the pulled states), ring rho, u, then
      // pull-stream + collide with the strain rate of those velocities
      const bool one_c = coarse_one_pass();
      if (!one_c) launch_stream<M_HRR, 0>(csrc, cdst, mc, tau_c, s);
      if (coarse_vel_hook) coarse_vel_hook(s);  // nested child: the parent's ring rho, u
      if (fine_one_pass2()) {
        // one pass per fine substep (k_hrr2): ring rho, u first
        hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, s, Hm, H0, Hp, c0, c1, c2, mf, g, itf);
        timed(s, [&] { launch_hrr2(fA, fB, mf, s, -1, true); });
      } else if (hrr_one_pass3()) {
        hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, s, Hm, H0, Hp, c0, c1, c2, mf, g, itf);
        timed(s, [&] { launch_hrr3(fA, fB, mf, s); });
      } else {
        launch_stream<M_HRR, 1>(fA, fB, mf, tau_f, s);
        hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, s, Hm, H0, Hp, c0, c1, c2, mf, g, itf);
        timed(s, [&] { launch_collide_hrr<1>(fA, fB, mf, tau_f, s, hrr_lds_var(var[3]), true); });
      }
      hipLaunchKernelGGL((k_fict<LAT, DEV, S, S>), dim3(bt), dim3(IB), 0, s, fB, mc, g, itf);
      // the coarse velocities at the history nodes' neighbours: from the
      // velocity pass, or (one-pass coarse level) pulled here
      // strain rate at the history nodes, then the temporal interpolation
      // of their fields (one thread per history node, one launch)
      if (one_c)
        hipLaunchKernelGGL((k_hist_strain_time<LAT, DEV, S, true>), dim3(bh), dim3(IB), 0, s, csrc, mc, Hm, H0, Hp,
                           G.as<double>(), g, itf);
      else
        hipLaunchKernelGGL((k_hist_strain_time<LAT, DEV, S, false>), dim3(bh), dim3(IB), 0, s, csrc, mc, Hm, H0, Hp,
                           G.as<double>(), g, itf);
      if (fine_one_pass2() || hrr_one_pass3()) {
        // the t+1/2 ring and the t+1 ring velocities in one launch
        hipLaunchKernelGGL((k_ring_half_macro<LAT, DEV, S, M_HRR>), dim3(2 * br), dim3(IB), 0, s, G.as<double>(), fB, Hm,
                           H0, Hp, mf, g, itf, kf, omf, tau_f, sig, (int)br);
      } else {
        hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_HRR, true>), dim3(br), dim3(IB), 0, s, G.as<double>(), fB, g, itf, kf,
                           omf, tau_f, sig);
      }
      if (fine_one_pass2()) {
        timed(s, [&] { launch_hrr2(fB, fA, mf, s, -1, true); });
      } else if (hrr_one_pass3()) {
        timed(s, [&] { launch_hrr3(fB, fA, mf, s); });
      } else {
        launch_stream<M_HRR, 1>(fB, fA, mf, tau_f, s);
        hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, s, Hm, H0, Hp, 0.0, 0.0, 1.0, mf, g, itf);
        timed(s, [&] { launch_collide_hrr<1>(fB, fA, mf, tau_f, s, hrr_lds_var(var[3]), true); });
      }
      // coarse collision before the TN transfer: the vector kernel also
      // passes over TN nodes, which the transfer then overwrites; the t+1
      // ring (into fine A, independent of both) shares the transfer's launch
      if (one_c) launch_hrr2c(csrc, cdst, mc, s, -1, true);
      else launch_collide_hrr<0>(csrc, cdst, mc, tau_c, s, -1, true);
      hipLaunchKernelGGL((k_ring_coalesce<LAT, DEV, S, M_HRR>), dim3(br2 + bc), dim3(256), 0, s, Hp, fA, fB, cdst, g,
                         itf, kf, omf, tau_f, kc, omc, tau_c, sig, (int)br2, (const S*)nullptr, (double*)nullptr);
    }
    HIPCHK(hipGetLastError());
    cpar ^= 1;
    const int old = hs[0];
    hs[0] = hs[1];
    hs[1] = hs[2];
    hs[2] = old;
    ring_partial = true;
  }

  // One coarse step of a nested grid (BGK / RR): the two-level step of Sec.
  // 4.3 with each fine substep replaced by one step of the child pair (the
  // fine level and its patch), applied recursively.  Fine A / B are the
  // child's coarse buffers: the child steps A -> B (t -> t+1/2), the t+1/2
  // ring (with the coarse stream) goes into B, the child steps B -> A
  // (t+1/2 -> t+1), then the t+1 ring into A and the transfer to TN^c.
  template <int MODEL>
  void step_nested(hipStream_t s) {
    S* csrc = cbuf[cpar].as<S>();
    S* cdst = cbuf[cpar ^ 1].as<S>();
    S* fA = fineA();
    S* fB = fineB();
    double* Hm = hist[hs[0]].as<double>();
    double* H0 = hist[hs[1]].as<double>();
    double* Hp = hist[hs[2]].as<double>();
    const int64_t NH = itf.NH;
    const double kf = tau_f / (2.0 * tau_c), kc = 2.0 * tau_c / tau_f;
    const double omf = 1.0 - 1.0 / tau_f, omc = 1.0 - 1.0 / tau_c;
    constexpr int IB = kIfaceBlock;
    constexpr int PER = 256 / (D == 2 ? 9 : 27);
    const unsigned bh = xblocks(NH, IB), bc = xblocks(itf.NT, PER), br2 = xblocks(itf.NR, 256);
    hipLaunchKernelGGL((k_hist_capture<LAT, DEV, S, MODEL>), dim3(bh), dim3(IB), 0, s, csrc, Hp, g, itf,
                       G.as<double>(), Hm, H0);
    child->step(1, s);
    launch_stream_ring<MODEL>(csrc, cdst, fB, kf, omf, s, nullptr);
    child->step(1, s);
    hipLaunchKernelGGL((k_ring_coalesce<LAT, DEV, S, MODEL>), dim3(br2 + bc), dim3(256), 0, s, Hp, fA, fB, cdst, g, itf,
                       kf, omf, tau_f, kc, omc, tau_c, sig, (int)br2, (const S*)nullptr, (double*)nullptr);
    HIPCHK(hipGetLastError());
    cpar ^= 1;
    const int old = hs[0];
    hs[0] = hs[1];
    hs[1] = hs[2];
    hs[2] = old;
    ring_partial = true;
  }

  // One coarse step of a nested grid with H-RR: as step_nested, with the
  // H-RR phases of the two-level step around the child's steps -- the
  // coarse velocity pass first; before each child step the ring's rho, u at
  // the child's time (t+1/2, then t+1) for the child's coarse collision
  // (coarse_vel_hook); after the first, the fictitious propagation onto
  // TN^f (u(TN^c, t+1)), the strain rate at the history nodes and the t+1/2
  // ring; at the end the coarse collision, the t+1 ring and the transfer.
  void step_nested_hrr(hipStream_t s) {
    S* csrc = cbuf[cpar].as<S>();
    S* cdst = cbuf[cpar ^ 1].as<S>();
    S* fA = fineA();
    S* fB = fineB();
    S* mc = mac_c.as<S>();
    S* mf = mac_f.as<S>();  // the child's coarse velocity planes
    double* Hm = hist[hs[0]].as<double>();
    double* H0 = hist[hs[1]].as<double>();
    double* Hp = hist[hs[2]].as<double>();
    const int64_t NH = itf.NH;
    const double kf = tau_f / (2.0 * tau_c), kc = 2.0 * tau_c / tau_f;
    const double omf = 1.0 - 1.0 / tau_f, omc = 1.0 - 1.0 / tau_c;
    const double c0 = -1.0 / 8.0, c1 = 3.0 / 4.0, c2 = 3.0 / 8.0;  // eq TempInt at t+1/2
    constexpr int IB = kIfaceBlock;
    constexpr int PER = 256 / (D == 2 ? 9 : 27);
    const unsigned bh = xblocks(NH, IB), br = xblocks(itf.NR, IB), bt = xblocks(itf.NT, IB);
    const unsigned bc = xblocks(itf.NT, PER), br2 = xblocks(itf.NR, 256);
    const Geo gg = g;
    const Iface it = itf;
    hipLaunchKernelGGL((k_hist_capture<LAT, DEV, S, M_HRR>), dim3(bh), dim3(IB), 0, s, csrc, Hp, g, itf, nullptr, Hm,
                       H0);
    const bool one_c = coarse_one_pass();
    if (!one_c) launch_stream<M_HRR, 0>(csrc, cdst, mc, tau_c, s);
    child->coarse_vel_hook = [=](hipStream_t st) {
      hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, st, Hm, H0, Hp, c0, c1, c2, mf, gg, it);
    };
    child->step(1, s);
    hipLaunchKernelGGL((k_fict<LAT, DEV, S, S>), dim3(bt), dim3(IB), 0, s, fB, mc, g, itf);
    if (one_c)
      hipLaunchKernelGGL((k_hist_strain_time<LAT, DEV, S, true>), dim3(bh), dim3(IB), 0, s, csrc, mc, Hm, H0, Hp,
                         G.as<double>(), g, itf);
    else
      hipLaunchKernelGGL((k_hist_strain_time<LAT, DEV, S, false>), dim3(bh), dim3(IB), 0, s, csrc, mc, Hm, H0, Hp,
                         G.as<double>(), g, itf);
    hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_HRR, true>), dim3(br), dim3(IB), 0, s, G.as<double>(), fB, g, itf, kf,
                       omf, tau_f, sig);
    child->coarse_vel_hook = [=](hipStream_t st) {
      hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, st, Hm, H0, Hp, 0.0, 0.0, 1.0, mf, gg, it);
    };
    child->step(1, s);
    child->coarse_vel_hook = nullptr;
    if (one_c) launch_hrr2c(csrc, cdst, mc, s);
    else launch_collide_hrr<0>(csrc, cdst, mc, tau_c, s, -1, true);
    hipLaunchKernelGGL((k_ring_coalesce<LAT, DEV, S, M_HRR>), dim3(br2 + bc), dim3(256), 0, s, Hp, fA, fB, cdst, g,
                       itf, kf, omf, tau_f, kc, omc, tau_c, sig, (int)br2, (const S*)nullptr, (double*)nullptr);
    HIPCHK(hipGetLastError());
    cpar ^= 1;
    const int old = hs[0];
    hs[0] = hs[1];
    hs[1] = hs[2];
    hs[2] = old;
    ring_partial = true;
  }

  // Completes the ring of fine A: rebuilds every population of the ring
  // nodes from the history level the last step's synchronous ring used (now
  // the middle level), which reproduces bitwise the populations stored then.
  void complete_ring() {
    if (!ring_partial || !g.has_fine) return;
    const double kf = tau_f / (2.0 * tau_c), omf = 1.0 - 1.0 / tau_f;
    const dim3 gr(xblocks(itf.NR, kIfaceBlock)), bl(kIfaceBlock);
    const double* H = hist[hs[1]].as<double>();
    if (desc.collision == LBM_BGK)
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_BGK, false>), gr, bl, 0, stream, H, fineA(), g, itf, kf, omf, tau_f, sig);
    else if (desc.collision == LBM_RR)
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_RR, false>), gr, bl, 0, stream, H, fineA(), g, itf, kf, omf, tau_f, sig);
    else
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_HRR, false>), gr, bl, 0, stream, H, fineA(), g, itf, kf, omf, tau_f, sig);
    HIPCHK(hipGetLastError());
    ring_partial = false;
  }

  void step(int n, hipStream_t s) override {
    HIPCHK(hipSetDevice(device));
    if (child) {
      for (int k = 0; k < n; ++k) {
        if (desc.collision == LBM_BGK) step_nested<M_BGK>(s);
        else if (desc.collision == LBM_RR) step_nested<M_RR>(s);
        else step_nested_hrr(s);
      }
      HIPCHK(hipGetLastError());
      return;
    }
    for (int k = 0; k < n; ++k) {
      rec_fine = sensors_on && k == n - 1;
      rec_coarse = sensors_on && k >= n - 2;
      if (rec_fine) sensors_before(s);
      sens_coarse_next = false;  // set again by a step that records
      if (!g.has_fine) step_uniform(s);
      else if (desc.collision == LBM_BGK) step_two_level<M_BGK>(s);
      else if (desc.collision == LBM_RR) step_two_level<M_RR>(s);
      else step_two_level<M_HRR>(s);
      if (rec_fine) sensors_after(s);
      if (probe_level >= 0) {
        // the level's post-collision state at the probe (its density is
        // the pre-collision one); the ring is complete at interior nodes
        const S* src = probe_level == 0 ? cur_c() : fineA();
        hipLaunchKernelGGL((k_probe<LAT, DEV, S>), dim3(1), dim3(64), 0, s, src, probe_pos, pSeries.as<double>(),
                           pCount.as<int64_t>(), probe_cap);
      }
    }
    rec_fine = rec_coarse = false;
    if (n > 0) sens_ready = sensors_on;
    HIPCHK(hipGetLastError());
  }

  // NH sensors (Sec. 7): velocities of the iteration before the step's last
  // one.  Coarse: the state at t.  Fine: the moments of what the non-ring
  // nodes pull from the state at t (the pre-collision state at t+1/2); the
  // ring's t+1/2 velocities are interpolated from the history after the
  // step, when its t+1 level exists.
  // (a fused D2Q9 step records the fine level's in k_fine2; a BGK / RR
  // two-level step the coarse level's of the next step)
  void sensors_before(hipStream_t s) {
    if (sens_coarse_next) sc_cur ^= 1;
    else
      hipLaunchKernelGGL((k_sens_vel<LAT, DEV, S, 0, false>), dim3(blocks(g.Nc, 256)), dim3(256), 0, s, cur_c(),
                         sUc[sc_cur].as<double>(), g);
    if (g.has_fine && !(desc.collision != LBM_HRR && fused_now()))
      hipLaunchKernelGGL((k_sens_vel<LAT, DEV, S, 1, true>), dim3(blocks(g.Nf, 256)), dim3(256), 0, s, fineA(),
                         sUf.as<double>(), g);
  }
  void sensors_after(hipStream_t s) {
    if (!g.has_fine) return;
    // after the step the history levels t-1, t, t+1 are hs[2], hs[0], hs[1]
    hipLaunchKernelGGL((k_ring_macro<LAT, double>), dim3(xblocks(itf.NR, kIfaceBlock)), dim3(kIfaceBlock), 0, s,
                       hist[hs[2]].as<double>(), hist[hs[0]].as<double>(), hist[hs[1]].as<double>(), -1.0 / 8.0,
                       3.0 / 4.0, 3.0 / 8.0, sUf.as<double>(), g, itf);
  }
  void set_dynamic_sigma(bool on, double sigma_dyn, double thr) override {
    HIPCHK(hipSetDevice(device));
    no_nesting("dynamic sigma");
    HIPCHK(hipStreamSynchronize(stream));
    if (on) {
      // a fresh start: no previous divergences and curls
      auto zalloc = [](DevBuf& b, size_t bytes) {
        if (!b.p) b.alloc(bytes);
        HIPCHK(hipMemset(b.p, 0, bytes));
      };
      zalloc(dynC, sizeof(S) * 4 * (size_t)g.Ncp);
      if (g.has_fine) zalloc(dynF, sizeof(S) * 4 * (size_t)g.Nfp);
    }
    dyn_on = on;
    sig_dyn = sigma_dyn;
    dyn_thr = thr;
  }
  void sensors_enable(bool on) override {
    HIPCHK(hipSetDevice(device));
    no_nesting("the NH sensors");
    HIPCHK(hipStreamSynchronize(stream));
    if (on && !sUc[0].p) {
      auto zalloc = [](DevBuf& b, size_t bytes) {
        b.alloc(bytes);
        HIPCHK(hipMemset(b.p, 0, bytes));
      };
      zalloc(sUc[0], sizeof(double) * (1 + D) * (size_t)g.Ncp);
      zalloc(sUc[1], sizeof(double) * (1 + D) * (size_t)g.Ncp);
      if (g.has_fine) zalloc(sUf, sizeof(double) * (1 + D) * (size_t)g.Nfp);
      const size_t Nmax = (size_t)std::max(g.Nc, g.Nf);
      sFlags.alloc(Nmax);
      sProd.alloc(sizeof(double) * 3 * Nmax);
    }
    sensors_on = on;
    sens_ready = sens_coarse_next = false;
  }
  void sensors(int level, double thr, uint8_t* flags, double* prod, bool dev) override {
    HIPCHK(hipSetDevice(device));
    if (!sensors_on || !sens_ready)
      throw LbmError(LBM_EINVAL, "NH sensors: enable them, then step at least once before reading them");
    complete_ring();
    const int64_t N = nodes(level);
    double* pr = prod ? sProd.as<double>() : nullptr;
    uint8_t* fl = sFlags.as<uint8_t>();
    if (level == 0)
      hipLaunchKernelGGL((k_sensors<LAT, DEV, S, 0>), dim3(blocks(N, 256)), dim3(256), 0, stream, sUc[sc_cur].as<double>(),
                         cur_c(), cbuf[cpar ^ 1].as<S>(), fl, pr, g, thr);
    else
      hipLaunchKernelGGL((k_sensors<LAT, DEV, S, 1>), dim3(blocks(N, 256)), dim3(256), 0, stream, sUf.as<double>(),
                         fineA(), sens_pre_half ? fbuf[2].as<S>() : fineB(), fl, pr, g, thr);
    HIPCHK(hipGetLastError());
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(flags, fl, (size_t)N, k, stream));
    if (prod) HIPCHK(hipMemcpyAsync(prod, pr, sizeof(double) * 3 * (size_t)N, k, stream));
    HIPCHK(hipStreamSynchronize(stream));
  }
  void probe_enable(int level, const int32_t* node, int64_t capacity) override {
    HIPCHK(hipSetDevice(device));
    no_nesting("probe recording");
    HIPCHK(hipStreamSynchronize(stream));
    if (level < 0) {
      probe_level = -1;
      return;
    }
    const int nx = level == 0 ? g.n[0] : g.nf[0], ny = level == 0 ? g.n[1] : g.nf[1],
              nz = level == 0 ? g.n[2] : g.nf[2];
    for (int d = 0; d < 3; ++d)
      if (node[d] < 0 || node[d] >= (d == 0 ? nx : d == 1 ? ny : nz))
        throw LbmError(LBM_EINVAL, "probe node outside the level");
    if (level == 0 && g.has_fine && coarse_class(g, node[0], node[1], node[2]) == CC_COVERED)
      throw LbmError(LBM_EINVAL, "probe on a covered coarse node (not evolved): probe the fine level there");
    if (level == 1 && fine_is_ring(g, node[0], node[1], node[2]))
      throw LbmError(LBM_EINVAL, "probe on a fine ring node (rebuilt, not evolved)");
    if (capacity < 1) throw LbmError(LBM_EINVAL, "probe capacity must be positive");
    if (pSeries.p) HIPCHK(hipFree(pSeries.p));
    pSeries.p = nullptr;
    pSeries.alloc(sizeof(double) * (size_t)capacity);
    if (!pCount.p) pCount.alloc(sizeof(int64_t));
    HIPCHK(hipMemset(pCount.p, 0, sizeof(int64_t)));
    probe_level = level;
    probe_pos = level == 0 ? cpos(g, node[0], node[1], node[2]) : fpos(g, node[0], node[1], node[2]);
    probe_cap = capacity;
  }
  int64_t probe_read(double* out, int64_t max) override {
    HIPCHK(hipSetDevice(device));
    if (probe_level < 0) throw LbmError(LBM_EINVAL, "no probe enabled");
    HIPCHK(hipStreamSynchronize(stream));
    int64_t c = 0;
    HIPCHK(hipMemcpy(&c, pCount.p, sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t n = std::min(c, max);
    if (n > 0) HIPCHK(hipMemcpy(out, pSeries.p, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
    return c;
  }

  void upload(DevBuf& dst, const double* src, size_t n, bool dev) {
    HIPCHK(hipMemcpyAsync(dst.p, src, sizeof(double) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          stream));
  }

  void reset_history_from_tmp() {
    hs[0] = 0;
    hs[1] = 1;
    hs[2] = 2;
    const dim3 gb(blocks(itf.NH, kIfaceBlock)), bb(kIfaceBlock);
    double *h0 = hist[0].as<double>(), *h1 = hist[1].as<double>(), *h2 = hist[2].as<double>();
    if (desc.collision == LBM_BGK)
      hipLaunchKernelGGL((k_hist_init<LAT, M_BGK>), gb, bb, 0, stream, tmp_rho.as<double>(), tmp_u.as<double>(), h0,
                         h1, h2, g, itf);
    else if (desc.collision == LBM_RR)
      hipLaunchKernelGGL((k_hist_init<LAT, M_RR>), gb, bb, 0, stream, tmp_rho.as<double>(), tmp_u.as<double>(), h0,
                         h1, h2, g, itf);
    else
      hipLaunchKernelGGL((k_hist_init<LAT, M_HRR>), gb, bb, 0, stream, tmp_rho.as<double>(), tmp_u.as<double>(), h0,
                         h1, h2, g, itf);
  }

  void set_state(int level, const double* rho, const double* u, bool dev) override {
    HIPCHK(hipSetDevice(device));
    if (child && level >= 1) {
      HIPCHK(hipDeviceSynchronize());
      ring_partial = false;
      child->set_state(level - 1, rho, u, dev);
      return;
    }
    sens_ready = sens_coarse_next = false;
    HIPCHK(hipDeviceSynchronize());
    // a coarse reset replaces the history the ring completion reads
    if (level == 0) complete_ring();
    else ring_partial = false;
    const int64_t N = nodes(level);
    upload(tmp_rho, rho, (size_t)N, dev);
    upload(tmp_u, u, (size_t)N * D, dev);
    S* dst = level == 0 ? cur_c() : fineA();
    hipLaunchKernelGGL((k_set_state<LAT, DEV, S>), dim3(blocks(N, 256)), dim3(256), 0, stream, tmp_rho.as<double>(),
                       tmp_u.as<double>(), dst, g, level);
    if (level == 0 && g.has_fine) reset_history_from_tmp();
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
  }

  void compute_macros(int level) {
    const int64_t N = nodes(level);
    const S* src = level == 0 ? cur_c() : fineA();
    hipLaunchKernelGGL((k_macros<LAT, DEV, S>), dim3(blocks(N, 256)), dim3(256), 0, stream, src,
                       g.has_fine ? fineA() : nullptr, tmp_rho.as<double>(), tmp_u.as<double>(), g, level);
    HIPCHK(hipGetLastError());
  }

  void get_macros(int level, double* rho, double* u, bool dev) override {
    HIPCHK(hipSetDevice(device));
    const int64_t N = nodes(level);
    complete_ring();
    if (child && level >= 1) {
      HIPCHK(hipStreamSynchronize(stream));
      child->get_macros(level - 1, rho, u, dev);
      return;
    }
    compute_macros(level);
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(rho, tmp_rho.p, sizeof(double) * N, k, stream));
    HIPCHK(hipMemcpyAsync(u, tmp_u.p, sizeof(double) * N * D, k, stream));
    HIPCHK(hipStreamSynchronize(stream));
  }

  void ensure_tmp_f(int64_t N) {
    if (tmp_f.bytes < sizeof(double) * Q * N) {
      if (tmp_f.p) HIPCHK(hipFree(tmp_f.p));
      tmp_f.p = nullptr;
      tmp_f.bytes = 0;
      tmp_f.alloc(sizeof(double) * Q * N);
    }
  }

  void set_pops(int level, const double* f, bool dev) override {
    HIPCHK(hipSetDevice(device));
    if (child && level >= 1) {
      HIPCHK(hipDeviceSynchronize());
      ring_partial = false;
      child->set_pops(level - 1, f, dev);
      return;
    }
    sens_ready = sens_coarse_next = false;
    HIPCHK(hipDeviceSynchronize());
    if (level == 0) complete_ring();
    else ring_partial = false;
    const int64_t N = nodes(level);
    ensure_tmp_f(N);
    HIPCHK(hipMemcpyAsync(tmp_f.p, f, sizeof(double) * Q * N, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          stream));
    S* dst = level == 0 ? cur_c() : fineA();
    hipLaunchKernelGGL((k_pops_in<LAT, DEV, S>), dim3(blocks(Q * N, 256)), dim3(256), 0, stream, tmp_f.as<double>(),
                       dst, g, level);
    if (level == 0 && g.has_fine) {
      compute_macros(0);
      reset_history_from_tmp();
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
  }

  void get_pops(int level, double* f, bool dev) override {
    HIPCHK(hipSetDevice(device));
    const int64_t N = nodes(level);
    complete_ring();
    if (child && level >= 1) {
      HIPCHK(hipStreamSynchronize(stream));
      child->get_pops(level - 1, f, dev);
      return;
    }
    ensure_tmp_f(N);
    const S* src = level == 0 ? cur_c() : fineA();
    hipLaunchKernelGGL((k_pops_out<LAT, DEV, S>), dim3(blocks(Q * N, 256)), dim3(256), 0, stream, src,
                       tmp_f.as<double>(), g, level);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(f, tmp_f.p, sizeof(double) * Q * N, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          stream));
    HIPCHK(hipStreamSynchronize(stream));
  }

  void totals(double* mass, double* mom) override { totals_in(mass, mom, part.as<double>(), tot.as<double>()); }

  void totals_in(double* mass, double* mom, double* pbuf, double* fin) override {
    HIPCHK(hipSetDevice(device));
    no_nesting("totals");
    complete_ring();
    for (int lv = 0; lv < 2; ++lv) {
      mass[lv] = 0.0;
      for (int d = 0; d < 3; ++d) mom[3 * lv + d] = 0.0;
      if (lv == 1 && !g.has_fine) continue;
      const int64_t N = nodes(lv);
      const unsigned nb = blocks(N, 256);
      const S* src = lv == 0 ? cur_c() : fineA();
      hipLaunchKernelGGL((k_totals<LAT, DEV, S>), dim3(nb), dim3(256), 0, stream, src, pbuf, g, lv);
      hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(256), 0, stream, pbuf, (int64_t)nb, fin);
      HIPCHK(hipGetLastError());
      double h[4];
      HIPCHK(hipMemcpyAsync(h, fin, sizeof(h), hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));
      mass[lv] = h[0];
      for (int d = 0; d < 3; ++d) mom[3 * lv + d] = h[1 + d];
    }
  }
};

static GridBase* make_grid(const lbm_grid_desc& d) {
  if (d.lattice == LBM_D2Q9 && d.precision == LBM_FP64) return new Grid<0, LBM_FP64>();
  if (d.lattice == LBM_D2Q9 && d.precision == LBM_FP32_DEV) return new Grid<0, LBM_FP32_DEV>();
  if (d.lattice == LBM_D3Q19 && d.precision == LBM_FP64) return new Grid<1, LBM_FP64>();
  if (d.lattice == LBM_D3Q19 && d.precision == LBM_FP32_DEV) return new Grid<1, LBM_FP32_DEV>();
  return nullptr;
}

static Geo validate(const lbm_grid_desc& d) {
  if (d.lattice != LBM_D2Q9 && d.lattice != LBM_D3Q19) throw LbmError(LBM_EINVAL, "unknown lattice");
  if (d.collision < LBM_BGK || d.collision > LBM_HRR) throw LbmError(LBM_EINVAL, "unknown collision model");
  if (d.precision != LBM_FP64 && d.precision != LBM_FP32_DEV) throw LbmError(LBM_EINVAL, "unknown precision");
  if (!(d.tau_coarse > 0.5) || !std::isfinite(d.tau_coarse)) throw LbmError(LBM_EINVAL, "tau_coarse must be > 1/2");
  if (d.collision == LBM_HRR && !(d.sigma >= 0.0 && d.sigma <= 1.0)) throw LbmError(LBM_EINVAL, "sigma outside [0, 1]");
  if (d.reserved != 0) throw LbmError(LBM_EINVAL, "reserved field must be 0");
  Geo g{};
  g.D = d.lattice == LBM_D2Q9 ? 2 : 3;
  bool any = false;
  for (int k = 0; k < 3; ++k) {
    g.n[k] = k < g.D ? d.n[k] : 1;
    if (k >= g.D && d.n[k] != 1 && d.n[k] != 0) throw LbmError(LBM_EINVAL, "n[2] must be 1 for D2Q9");
    if (k < g.D && g.n[k] < 3) throw LbmError(LBM_EINVAL, "coarse grid needs at least 3 nodes per used axis");
    if (k < g.D && d.hi[k] != d.lo[k]) any = true;
    g.nf[k] = 1;
  }
  const int64_t Nc = (int64_t)g.n[0] * g.n[1] * g.n[2];
  if (Nc * 19 > ((int64_t)1 << 40)) throw LbmError(LBM_EINVAL, "grid too large");
  g.Nc = Nc;
  g.has_fine = any ? 1 : 0;
  if (any) {
    for (int k = 0; k < g.D; ++k) {
      g.a[k] = d.lo[k];
      g.m[k] = d.hi[k] - d.lo[k];
      if (g.m[k] < 4) throw LbmError(LBM_EINVAL, "patch must span at least 4 coarse cells per axis");
      if (d.lo[k] < 2 || d.hi[k] > g.n[k] - 3) throw LbmError(LBM_EINVAL, "patch must satisfy lo >= 2, hi <= n - 3");
      g.nf[k] = 2 * g.m[k] + 1;
    }
    g.Nf = (int64_t)g.nf[0] * g.nf[1] * g.nf[2];
  }
  g.pc = pitch_of(g.n[0]);
  g.Ncp = (int64_t)g.pc * g.n[1] * g.n[2];
  g.fxo = d.precision == LBM_FP32_DEV ? 3 : 1;
  g.pf = g.has_fine ? pitch_of(g.nf[0] + g.fxo) : 0;
  g.Nfp = g.has_fine ? (int64_t)g.pf * g.nf[1] * g.nf[2] : 0;
  // the bulk kernels number node positions and vectors in 32 bits
  if (g.Ncp >= ((int64_t)1 << 31) || g.Nfp >= ((int64_t)1 << 31)) throw LbmError(LBM_EINVAL, "grid too large");
  return g;
}


// ---------------------------------------------------------------------------
// Batch of independent grids (same lattice, collision model and precision),
// advanced together by one launch per phase; one coarse step is captured as a
// hipGraph and replayed.
struct BatchBase {
  int lattice = 0, collision = 0, precision = 0, device = 0, capacity = 0;
  hipStream_t stream = nullptr;
  // Recorded on the caller's stream after each step: the batch's own host
  // calls wait for it and for `stream`, never for the whole device, so work
  // of other batches (other streams) keeps running meanwhile.
  hipEvent_t stepped = nullptr;
  bool stepped_rec = false;
  std::string err;
  virtual ~BatchBase() {
    if (stepped) (void)hipEventDestroy(stepped);
    if (stream) (void)hipStreamDestroy(stream);
  }
  void quiesce() {
    if (stepped_rec) HIPCHK(hipEventSynchronize(stepped));
    HIPCHK(hipStreamSynchronize(stream));
  }
  virtual int add(const lbm_grid_desc& d) = 0;
  virtual void remove(int slot) = 0;
  virtual void set_state(int slot, int level, const double* rho, const double* u, bool dev) = 0;
  virtual void get_macros(int slot, int level, double* rho, double* u, bool dev) = 0;
  virtual void get_pops(int slot, int level, double* f, bool dev) = 0;
  virtual void step(int n, hipStream_t s) = 0;
  virtual void tune(int reps, int32_t* out) = 0;
  virtual void set_variants(const int32_t* v) = 0;
  virtual void set_graph(bool on) = 0;
  virtual void info(int64_t* out) = 0;
  virtual int64_t slot_steps(int slot) = 0;
};

// Device bytes one grid of this descriptor needs in a batch slot
// (populations, macro planes, history, interface tables), without any
// scratch.  D2Q9 BGK / RR keep a third fine population buffer (the fused
// fine phase's t+1/2 ring and band), D3Q19 BGK / RR the compact copy of the
// fine x-bands.
static int64_t grid_footprint(const lbm_grid_desc& d, const Geo& g) {
  const int Q = d.lattice == LBM_D2Q9 ? 9 : 19;
  const int D = g.D;
  const bool f32 = d.precision == LBM_FP32_DEV;
  const int64_t sb = f32 ? 4 : 8;
  auto pops = [&](int64_t NP) { return sb * (f32 ? pop_elems<float>(NP, Q) : pop_elems<double>(NP, Q)); };
  const int nfine = (g.D == 2 && d.collision != LBM_HRR) ? 3 : 2;
  int64_t bytes = 2 * pops(g.Ncp) + (g.has_fine ? nfine * pops(g.Nfp) : 0);
  if (g.has_fine && g.D == 3 && d.collision != LBM_HRR) bytes += sb * xband_elems(g, Q);
  if (d.collision == LBM_HRR) bytes += sb * (1 + D) * (g.Ncp + g.Nfp + 128);
  if (g.has_fine) {
    int64_t nh = 0, ring_out = 1, ring_in = 1, tn_out = 1, tn_in = 1;
    for (int a = 0; a < D; ++a) {
      int64_t face = 2;
      for (int b = 0; b < D; ++b)
        if (b != a) face *= (g.m[b] + 3);
      nh += face;
      ring_out *= 2 * g.m[a] + 1;
      ring_in *= 2 * g.m[a] - 1;
      tn_out *= g.m[a] - 1;
      tn_in *= g.m[a] - 3;
    }
    const int64_t nr = ring_out - ring_in, nt = tn_out - tn_in;
    const int64_t hn = 1 + D + Q + (D == 2 ? 3 : 6);
    bytes += 4 * 8 * hn * nh + nh * 8 + nr * (8 + 4 + 64) + nt * 16;
  }
  return bytes;
}

template <int LAT, int PREC>
struct Batch final : BatchBase {
  using L = Lattice<LAT>;
  static constexpr bool DEV = PREC == LBM_FP32_DEV;
  using S = typename std::conditional<DEV, float, double>::type;
  static constexpr int Q = L::Q, D = L::D;
  static constexpr bool NT = true;
  static constexpr int NVAR = kNVar;
  static constexpr int V = VecOf<S>::V;
  static constexpr int HN = Grid<LAT, PREC>::HN;

  struct Inst {
    lbm_grid_desc desc{};
    Geo g{};
    HostTables tabs;
    DevBuf cbuf[2], fbuf[3], xb, mac_c, mac_f, hist[3], G, d_hnode, d_rnode, d_rnp, d_rpt, d_tnf, d_tnc;
    Iface itf{};
  };
  // D2Q9 BGK / RR instances run both fine substeps in one phase (kb_fine2),
  // in tiles of shape tile_var (kTileX, kTileY).
  bool fused() const { return D == 2 && collision != LBM_HRR; }
  int tile_var = 0;
  std::vector<std::unique_ptr<Inst>> slots;
  std::vector<InstDev> hinst;
  std::vector<int64_t> steps_done;
  std::vector<char> ring_partial;  // per slot: fine A holds a partial ring (see Grid)
  DevBuf d_inst, d_counts, d_items[W_KINDS];
  size_t item_cap[W_KINDS] = {};
  int counts[W_KINDS] = {};
  DevBuf tmp_rho, tmp_u, tmp_f;
  int var_c = Grid<LAT, PREC>::kDefaultVar, var_f = Grid<LAT, PREC>::kDefaultVar;
  bool use_graph = true, graph_ok = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~Batch() override { drop_graph(); }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    graph_ok = false;
  }

  void init(int cap) {
    capacity = cap;
    slots.resize((size_t)cap);
    hinst.assign((size_t)cap, InstDev{});
    steps_done.assign((size_t)cap, 0);
    ring_partial.assign((size_t)cap, 0);
    d_inst.alloc(sizeof(InstDev) * (size_t)cap);
    HIPCHK(hipMemset(d_inst.p, 0, d_inst.bytes));
    d_counts.alloc(sizeof(int) * W_KINDS);
    HIPCHK(hipMemset(d_counts.p, 0, d_counts.bytes));
    for (int k = 0; k < W_KINDS; ++k) grow_items(k, 64);
  }

  void grow_items(int k, size_t n) {
    if (n <= item_cap[k]) return;
    size_t cap = std::max(n, 2 * item_cap[k]);
    if (d_items[k].p) HIPCHK(hipFree(d_items[k].p));
    d_items[k].p = nullptr;
    d_items[k].alloc(sizeof(Work) * cap);
    item_cap[k] = cap;
    drop_graph();  // the graph holds the old list addresses
  }

  static Flat flat(const Geo& g, int level) {
    if (level == 0) return make_flat(g.n[0], g.n[1], g.n[2], V, false, D);
    return make_flat(g.nf[0], g.nf[1], g.nf[2], V, true, D);
  }

  void upload_inst(int slot) {
    HIPCHK(hipMemcpy(d_inst.template as<InstDev>() + slot, &hinst[(size_t)slot], sizeof(InstDev), hipMemcpyHostToDevice));
  }
  void fetch_inst(int slot) {
    HIPCHK(hipMemcpy(&hinst[(size_t)slot], d_inst.template as<InstDev>() + slot, sizeof(InstDev), hipMemcpyDeviceToHost));
  }

  // Work lists of every phase from the active instances.
  void rebuild_lists() {
    std::vector<Work> lists[W_KINDS];
    constexpr int PER = 256 / (D == 2 ? 9 : 27);
    const int hfields = collision == LBM_BGK ? HF<LAT, M_BGK>::N : (collision == LBM_RR ? HF<LAT, M_RR>::N
                                                                                         : HF<LAT, M_HRR>::N);
    for (int sl = 0; sl < capacity; ++sl) {
      if (!slots[(size_t)sl]) continue;
      const InstDev& I = hinst[(size_t)sl];
      for (int t = 0; t < I.fc.nchunks; ++t) lists[W_COARSE].push_back({sl, t});
      if (!I.g.has_fine) continue;
      for (int t = 0; t < I.ff.nchunks; ++t) lists[W_FINE].push_back({sl, t});
      const int64_t nh = I.itf.NH, nr = I.itf.NR, nt = I.itf.NT;
      for (int64_t c = 0; c < (nh + 63) / 64; ++c) lists[W_HIST].push_back({sl, (int)c});
      for (int64_t c = 0; c < (nh * hfields + 63) / 64; ++c) lists[W_HTIME].push_back({sl, (int)c});
      for (int64_t c = 0; c < (nr + 63) / 64; ++c) lists[W_RING].push_back({sl, (int)c});
      for (int64_t c = 0; c < (nt + 63) / 64; ++c) lists[W_TN].push_back({sl, (int)c});
      for (int64_t c = 0; c < (nt + PER - 1) / PER; ++c) lists[W_TNB].push_back({sl, (int)c});
      if (I.fused) {
        const int ntile = fine2_ntx<S>(I.g, kTileX[tile_var]) * fine2_nty(I.g, kTileY[tile_var]);
        for (int c = 0; c < ntile; ++c) lists[W_TILE].push_back({sl, c});
      }
    }
    for (int k = 0; k < W_KINDS; ++k) {
      grow_items(k, lists[k].size());
      counts[k] = (int)lists[k].size();
      if (!lists[k].empty())
        HIPCHK(hipMemcpy(d_items[k].p, lists[k].data(), sizeof(Work) * lists[k].size(), hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(d_counts.p, counts, sizeof(counts), hipMemcpyHostToDevice));
  }

  int add(const lbm_grid_desc& d) override {
    if (d.lattice != lattice || d.collision != collision || d.precision != precision)
      throw LbmError(LBM_EINVAL, "descriptor does not match the batch's lattice, collision and precision");
    int sl = -1;
    for (int k = 0; k < capacity; ++k)
      if (!slots[(size_t)k]) {
        sl = k;
        break;
      }
    if (sl < 0) throw LbmError(LBM_ENOMEM, "batch is full");
    Geo g = validate(d);
    auto in = std::make_unique<Inst>();
    in->desc = d;
    in->g = g;
    HIPCHK(hipSetDevice(device));
    quiesce();
    build_tables(g, in->tabs);
    const size_t sb = sizeof(S);
    for (int p = 0; p < 2; ++p) {
      in->cbuf[p].alloc(sb * (size_t)pop_elems<S>(g.Ncp, Q));
      HIPCHK(hipMemset(in->cbuf[p].p, 0, in->cbuf[p].bytes));
    }
    if (collision == LBM_HRR) {
      in->mac_c.alloc(sb * ((size_t)g.Ncp * (1 + D) + 64));
      HIPCHK(hipMemset(in->mac_c.p, 0, in->mac_c.bytes));
    }
    if (g.has_fine) {
      for (int p = 0; p < (fused() ? 3 : 2); ++p) {
        in->fbuf[p].alloc(sb * (size_t)pop_elems<S>(g.Nfp, Q));
        HIPCHK(hipMemset(in->fbuf[p].p, 0, in->fbuf[p].bytes));
      }
      if (collision == LBM_HRR) {
        in->mac_f.alloc(sb * ((size_t)g.Nfp * (1 + D) + 64));
        HIPCHK(hipMemset(in->mac_f.p, 0, in->mac_f.bytes));
      }
      if (D == 3 && collision != LBM_HRR) {
        in->xb.alloc(sb * (size_t)xband_elems(g, Q));
        HIPCHK(hipMemset(in->xb.p, 0, in->xb.bytes));
      }
      const size_t NH = in->tabs.hnode.size();
      for (int k = 0; k < 3; ++k) in->hist[k].alloc(sizeof(double) * HN * NH);
      in->G.alloc(sizeof(double) * HN * NH);
      auto up = [&](DevBuf& b, const void* src, size_t bytes) {
        b.alloc(bytes);
        if (bytes) HIPCHK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
      };
      const HostTables& t = in->tabs;
      up(in->d_hnode, t.hnode.data(), sizeof(int64_t) * t.hnode.size());
      up(in->d_rnode, t.rnode.data(), sizeof(int64_t) * t.rnode.size());
      up(in->d_rnp, t.rnp.data(), sizeof(int32_t) * t.rnp.size());
      up(in->d_rpt, t.rpt.data(), sizeof(int32_t) * t.rpt.size());
      up(in->d_tnf, t.tnf.data(), sizeof(int64_t) * t.tnf.size());
      up(in->d_tnc, t.tnc.data(), sizeof(int64_t) * t.tnc.size());
      in->itf = Iface{(int64_t)t.hnode.size(), in->d_hnode.template as<int64_t>(), (int64_t)t.rnode.size(),
                      in->d_rnode.template as<int64_t>(), in->d_rnp.template as<int32_t>(), in->d_rpt.template as<int32_t>(),
                      (int64_t)t.tnf.size(), in->d_tnf.template as<int64_t>(), in->d_tnc.template as<int64_t>()};
    }
    const int64_t Nmax = std::max(g.Nc, g.Nf);
    if (tmp_rho.bytes < sizeof(double) * (size_t)Nmax) {
      if (tmp_rho.p) HIPCHK(hipFree(tmp_rho.p));
      if (tmp_u.p) HIPCHK(hipFree(tmp_u.p));
      tmp_rho.p = tmp_u.p = nullptr;
      tmp_rho.alloc(sizeof(double) * (size_t)Nmax);
      tmp_u.alloc(sizeof(double) * D * (size_t)Nmax);
    }
    InstDev I{};
    I.g = g;
    I.itf = in->itf;
    I.fc = flat(g, 0);
    if (g.has_fine) I.ff = flat(g, 1);
    I.cbuf[0] = in->cbuf[0].p;
    I.cbuf[1] = in->cbuf[1].p;
    I.fbuf[0] = in->fbuf[0].p;
    I.fbuf[1] = in->fbuf[1].p;
    I.fh = in->fbuf[2].p;
    I.xb = in->xb.p;
    I.fpar = 0;
    I.fused = (g.has_fine && fused()) ? 1 : 0;
    I.ntx = g.has_fine ? fine2_ntx<S>(g, kTileX[tile_var]) : 0;
    I.mac_c = in->mac_c.p;
    I.mac_f = in->mac_f.p;
    for (int k = 0; k < 3; ++k) I.hist[k] = in->hist[k].template as<double>();
    I.G = in->G.template as<double>();
    I.tau_c = d.tau_coarse;
    I.tau_f = 2.0 * d.tau_coarse - 0.5;
    I.sig = d.sigma;
    I.cpar = 0;
    I.ccur = I.cbuf[0];
    I.cnext = I.cbuf[1];
    I.hs[0] = 0;
    I.hs[1] = 1;
    I.hs[2] = 2;
    I.active = 1;
    slots[(size_t)sl] = std::move(in);
    hinst[(size_t)sl] = I;
    steps_done[(size_t)sl] = 0;
    ring_partial[(size_t)sl] = 0;
    upload_inst(sl);
    rebuild_lists();
    return sl;
  }

  Inst& slot_ref(int sl) {
    if (sl < 0 || sl >= capacity || !slots[(size_t)sl]) throw LbmError(LBM_EINVAL, "no grid in this slot");
    return *slots[(size_t)sl];
  }

  void remove(int sl) override {
    slot_ref(sl);
    HIPCHK(hipSetDevice(device));
    quiesce();
    hinst[(size_t)sl] = InstDev{};
    upload_inst(sl);
    slots[(size_t)sl].reset();
    rebuild_lists();
  }

  // Completes the ring of a slot's fine A (as Grid::complete_ring) from its
  // middle history level.  Expects hinst[sl] fetched.
  void complete_ring(int sl) {
    if (!ring_partial[(size_t)sl]) return;
    const Inst& in = *slots[(size_t)sl];
    const InstDev& I = hinst[(size_t)sl];
    const double kf = I.tau_f / (2.0 * I.tau_c), omf = 1.0 - 1.0 / I.tau_f;
    const dim3 gr((unsigned)((in.itf.NR + 8 * kIfaceBlock - 1) / (8 * kIfaceBlock) * 8)), bl(kIfaceBlock);
    const double* H = I.hist[I.hs[1]];
    S* A = (S*)I.fbuf[I.fpar];
    if (collision == LBM_BGK)
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_BGK, false>), gr, bl, 0, stream, H, A, in.g, in.itf, kf, omf, I.tau_f, I.sig);
    else if (collision == LBM_RR)
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_RR, false>), gr, bl, 0, stream, H, A, in.g, in.itf, kf, omf, I.tau_f, I.sig);
    else
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_HRR, false>), gr, bl, 0, stream, H, A, in.g, in.itf, kf, omf, I.tau_f,
                         I.sig);
    HIPCHK(hipGetLastError());
    ring_partial[(size_t)sl] = 0;
  }

  void set_state(int sl, int level, const double* rho, const double* u, bool dev) override {
    Inst& in = slot_ref(sl);
    if (level == 1 && !in.g.has_fine) throw LbmError(LBM_EINVAL, "no fine level");
    HIPCHK(hipSetDevice(device));
    quiesce();
    fetch_inst(sl);
    InstDev& I = hinst[(size_t)sl];
    // a coarse reset replaces the history the ring completion reads
    if (level == 0) complete_ring(sl);
    else ring_partial[(size_t)sl] = 0;
    const int64_t N = level == 0 ? in.g.Nc : in.g.Nf;
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpy(tmp_rho.p, rho, sizeof(double) * N, k));
    HIPCHK(hipMemcpy(tmp_u.p, u, sizeof(double) * N * D, k));
    S* dst = (S*)(level == 0 ? I.cbuf[I.cpar] : I.fbuf[I.fpar]);
    hipLaunchKernelGGL((k_set_state<LAT, DEV, S>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream,
                       tmp_rho.template as<double>(), tmp_u.template as<double>(), dst, in.g, level);
    if (level == 0 && in.g.has_fine) {
      I.hs[0] = 0;
      I.hs[1] = 1;
      I.hs[2] = 2;
      const dim3 gb((unsigned)((in.itf.NH + 63) / 64)), bb(64);
      if (collision == LBM_BGK)
        hipLaunchKernelGGL((k_hist_init<LAT, M_BGK>), gb, bb, 0, stream, tmp_rho.template as<double>(), tmp_u.template as<double>(),
                           I.hist[0], I.hist[1], I.hist[2], in.g, in.itf);
      else if (collision == LBM_RR)
        hipLaunchKernelGGL((k_hist_init<LAT, M_RR>), gb, bb, 0, stream, tmp_rho.template as<double>(), tmp_u.template as<double>(),
                           I.hist[0], I.hist[1], I.hist[2], in.g, in.itf);
      else
        hipLaunchKernelGGL((k_hist_init<LAT, M_HRR>), gb, bb, 0, stream, tmp_rho.template as<double>(), tmp_u.template as<double>(),
                           I.hist[0], I.hist[1], I.hist[2], in.g, in.itf);
      upload_inst(sl);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    if (level == 0) steps_done[(size_t)sl] = 0;
  }

  void get_macros(int sl, int level, double* rho, double* u, bool dev) override {
    Inst& in = slot_ref(sl);
    if (level == 1 && !in.g.has_fine) throw LbmError(LBM_EINVAL, "no fine level");
    HIPCHK(hipSetDevice(device));
    quiesce();
    fetch_inst(sl);
    complete_ring(sl);
    const InstDev& I = hinst[(size_t)sl];
    const int64_t N = level == 0 ? in.g.Nc : in.g.Nf;
    const S* src = (const S*)(level == 0 ? I.cbuf[I.cpar] : I.fbuf[I.fpar]);
    hipLaunchKernelGGL((k_macros<LAT, DEV, S>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream, src,
                       (const S*)I.fbuf[I.fpar], tmp_rho.template as<double>(), tmp_u.template as<double>(), in.g, level);
    HIPCHK(hipGetLastError());
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(rho, tmp_rho.p, sizeof(double) * N, k, stream));
    HIPCHK(hipMemcpyAsync(u, tmp_u.p, sizeof(double) * N * D, k, stream));
    HIPCHK(hipStreamSynchronize(stream));
  }

  void get_pops(int sl, int level, double* f, bool dev) override {
    Inst& in = slot_ref(sl);
    if (level == 1 && !in.g.has_fine) throw LbmError(LBM_EINVAL, "no fine level");
    HIPCHK(hipSetDevice(device));
    quiesce();
    fetch_inst(sl);
    complete_ring(sl);
    const InstDev& I = hinst[(size_t)sl];
    const int64_t N = level == 0 ? in.g.Nc : in.g.Nf;
    if (tmp_f.bytes < sizeof(double) * Q * (size_t)N) {
      if (tmp_f.p) HIPCHK(hipFree(tmp_f.p));
      tmp_f.p = nullptr;
      tmp_f.alloc(sizeof(double) * Q * (size_t)N);
    }
    const S* src = (const S*)(level == 0 ? I.cbuf[I.cpar] : I.fbuf[I.fpar]);
    hipLaunchKernelGGL((k_pops_out<LAT, DEV, S>), dim3((unsigned)((Q * N + 255) / 256)), dim3(256), 0, stream, src,
                       tmp_f.template as<double>(), in.g, level);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(f, tmp_f.p, sizeof(double) * Q * N, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          stream));
    HIPCHK(hipStreamSynchronize(stream));
  }

  // ---- phase launches ----
  const InstDev* di() const { return d_inst.template as<InstDev>(); }
  // One work group per entry of list k's capacity (a multiple of 8).
  dim3 grid_of(int k) const { return dim3((unsigned)((item_cap[k] + kXCD - 1) / kXCD * kXCD)); }
  const Work* items(int k) const { return d_items[k].template as<Work>(); }
  const int* cnt(int k) const { return d_counts.template as<int>() + k; }

  template <int MODEL, int LEVEL, int SUB>
  void phase_stream(hipStream_t s, int v) {
    hipLaunchKernelGGL((kb_stream<LAT, DEV, S, MODEL, LEVEL, SUB, NT>), grid_of(LEVEL == 0 ? W_COARSE : W_FINE), dim3(256),
                       (unsigned)kVarLds[v], s, di(), items(LEVEL == 0 ? W_COARSE : W_FINE),
                       cnt(LEVEL == 0 ? W_COARSE : W_FINE));
  }
  template <int LEVEL, int SUB>
  void phase_collide(hipStream_t s, int v) {
    hipLaunchKernelGGL((kb_collide<LAT, DEV, S, LEVEL, SUB, NT>), grid_of(LEVEL == 0 ? W_COARSE : W_FINE), dim3(256),
                       (unsigned)kVarLds[v], s,
                       di(), items(LEVEL == 0 ? W_COARSE : W_FINE), cnt(LEVEL == 0 ? W_COARSE : W_FINE));
  }

  // Fused fine phase (D2Q9 BGK / RR) in the current tile shape.
  template <int MODEL>
  void phase_fine2(hipStream_t s) {
    if constexpr (D == 2 && MODEL != M_HRR) {
      if (tile_var == 0)
        hipLaunchKernelGGL((kb_fine2<LAT, DEV, S, MODEL, NT, kTileX[0], kTileY[0]>), grid_of(W_TILE),
                           dim3(kTileX[0] * kTileY[0]), 0, s, di(), items(W_TILE), cnt(W_TILE));
      else
        hipLaunchKernelGGL((kb_fine2<LAT, DEV, S, MODEL, NT, kTileX[1], kTileY[1]>), grid_of(W_TILE),
                           dim3(kTileX[1] * kTileY[1]), 0, s, di(), items(W_TILE), cnt(W_TILE));
    }
  }
  // Sets the fused tile shape: every instance's tile count per row on the
  // device (that field only: the rest of a descriptor advances on the device)
  // and the tile list.
  void set_tile_var(int tv) {
    tile_var = tv;
    for (int sl = 0; sl < capacity; ++sl) {
      if (!slots[(size_t)sl] || !hinst[(size_t)sl].fused) continue;
      const int ntx = fine2_ntx<S>(hinst[(size_t)sl].g, kTileX[tv]);
      hinst[(size_t)sl].ntx = ntx;
      HIPCHK(hipMemcpy(&(d_inst.template as<InstDev>() + sl)->ntx, &ntx, sizeof(int), hipMemcpyHostToDevice));
    }
    rebuild_lists();
    drop_graph();
  }

  template <int MODEL>
  void launch_step_model(hipStream_t s) {
    using F = HF<LAT, MODEL>;
    const dim3 ib(64);
    hipLaunchKernelGGL((kb_hist_capture<LAT, DEV, S, MODEL>), grid_of(W_HIST), ib, 0, s, di(), items(W_HIST),
                       cnt(W_HIST));
    if (MODEL != M_HRR) {
      // as Grid::step_two_level: the capture interpolated G; the t+1/2 ring
      // shares the coarse launch; the t+1 ring shares the transfer's launch
      const unsigned nrb = grid_of(W_RING).x;
      auto stream_ring = [&] {
        hipLaunchKernelGGL((kb_stream_ring<LAT, DEV, S, MODEL, NT>), dim3(nrb + grid_of(W_COARSE).x), dim3(256),
                           (unsigned)kVarLds[var_c], s, di(), items(W_RING), cnt(W_RING), items(W_COARSE),
                           cnt(W_COARSE), (int)nrb);
      };
      if constexpr (D == 2) {  // fused() for BGK / RR
        stream_ring();
        phase_fine2<MODEL>(s);
      } else {
        phase_stream<MODEL, 1, 0>(s, var_f);  // writes B's ring column: the t+1/2 ring follows
        stream_ring();
        phase_stream<MODEL, 1, 1>(s, var_f);
      }
      hipLaunchKernelGGL((kb_ring_coalesce<LAT, DEV, S, MODEL>), dim3(nrb + grid_of(W_TNB).x), dim3(256), 0, s, di(),
                         items(W_RING), cnt(W_RING), items(W_TNB), cnt(W_TNB), (int)nrb);
    } else {
      phase_stream<M_HRR, 0, 0>(s, var_c);
      phase_stream<M_HRR, 1, 0>(s, var_f);
      hipLaunchKernelGGL((kb_ring_macro<LAT, S, 0>), grid_of(W_RING), ib, 0, s, di(), items(W_RING), cnt(W_RING));
      phase_collide<1, 0>(s, var_f);
      hipLaunchKernelGGL((kb_fict<LAT, DEV, S>), grid_of(W_TN), ib, 0, s, di(), items(W_TN), cnt(W_TN));
      hipLaunchKernelGGL((kb_hist_strain<LAT, DEV, S>), grid_of(W_HIST), ib, 0, s, di(), items(W_HIST), cnt(W_HIST));
      hipLaunchKernelGGL((kb_hist_time<F::N>), grid_of(W_HTIME), ib, 0, s, di(), items(W_HTIME), cnt(W_HTIME));
      hipLaunchKernelGGL((kb_ring<LAT, DEV, S, M_HRR, 0>), grid_of(W_RING), ib, 0, s, di(), items(W_RING), cnt(W_RING));
      phase_stream<M_HRR, 1, 1>(s, var_f);
      hipLaunchKernelGGL((kb_ring_macro<LAT, S, 1>), grid_of(W_RING), ib, 0, s, di(), items(W_RING), cnt(W_RING));
      phase_collide<1, 1>(s, var_f);
      phase_collide<0, 0>(s, var_c);
      // the t+1 ring shares the transfer's launch (as for BGK / RR)
      const unsigned nrb = grid_of(W_RING).x;
      hipLaunchKernelGGL((kb_ring_coalesce<LAT, DEV, S, M_HRR>), dim3(nrb + grid_of(W_TNB).x), dim3(256), 0, s, di(),
                         items(W_RING), cnt(W_RING), items(W_TNB), cnt(W_TNB), (int)nrb);
    }
    hipLaunchKernelGGL(kb_advance, dim3((unsigned)((capacity + 255) / 256)), dim3(256), 0, s, d_inst.template as<InstDev>(),
                       capacity);
  }
  void launch_step(hipStream_t s) {
    if (collision == LBM_BGK) launch_step_model<M_BGK>(s);
    else if (collision == LBM_RR) launch_step_model<M_RR>(s);
    else launch_step_model<M_HRR>(s);
  }

  void capture() {
    std::lock_guard<std::recursive_mutex> lk(g_api_mu);
    drop_graph();
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    launch_step(stream);
    hipGraph_t gr = nullptr;
    HIPCHK(hipStreamEndCapture(stream, &gr));
    graph = gr;
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    graph_ok = true;
  }

  void step(int n, hipStream_t s) override {
    HIPCHK(hipSetDevice(device));
    int64_t active = 0;
    for (int k = 0; k < capacity; ++k) active += slots[(size_t)k] ? 1 : 0;
    if (active == 0 || n <= 0) return;
    if (use_graph && !graph_ok) capture();
    for (int k = 0; k < n; ++k) {
      if (use_graph) HIPCHK(hipGraphLaunch(exec, s));
      else launch_step(s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(stepped, s));
    stepped_rec = true;
    for (int k = 0; k < capacity; ++k)
      if (slots[(size_t)k]) {
        steps_done[(size_t)k] += n;
        if (slots[(size_t)k]->g.has_fine) ring_partial[(size_t)k] = 1;
      }
  }

  void set_graph(bool on) override {
    use_graph = on;
    if (!on) drop_graph();
  }

  // Autotuner over the bulk variants of the whole batch.  Times the coarse and
  // fine stream phases (writing only buffers the next step rewrites).
  void tune(int reps, int32_t* out) override {
    HIPCHK(hipSetDevice(device));
    quiesce();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    if (fused() && counts[W_FINE] > 0) {
      // fused fine phase: one variant per tile shape (it rewrites B and the
      // half-step buffer, which the next step rewrites)
      float best = -1.f;
      int bt = 0;
      for (int tv = 0; tv < kNTile; ++tv) {
        set_tile_var(tv);
        auto run = [&] {
          if (collision == LBM_BGK) phase_fine2<M_BGK>(stream);
          else phase_fine2<M_RR>(stream);
        };
        run();
        HIPCHK(hipEventRecord(e0, stream));
        for (int k = 0; k < reps; ++k) run();
        HIPCHK(hipEventRecord(e1, stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (best < 0.f || ms < best) {
          best = ms;
          bt = tv;
        }
      }
      set_tile_var(bt);
      var_f = bt;
    }
    for (int level = 0; level < 2; ++level) {
      if (counts[level == 0 ? W_COARSE : W_FINE] == 0) continue;
      if (level == 1 && fused()) continue;  // tuned above
      float best = -1.f;
      int bv = 0;
      for (int v = 0; v < NVAR; ++v) {
        auto run = [&] {
          if (collision == LBM_BGK) {
            if (level == 0) phase_stream<M_BGK, 0, 0>(stream, v);
            else phase_stream<M_BGK, 1, 0>(stream, v);
          } else if (collision == LBM_RR) {
            if (level == 0) phase_stream<M_RR, 0, 0>(stream, v);
            else phase_stream<M_RR, 1, 0>(stream, v);
          } else {
            if (level == 0) phase_stream<M_HRR, 0, 0>(stream, v);
            else phase_stream<M_HRR, 1, 0>(stream, v);
          }
        };
        run();
        HIPCHK(hipEventRecord(e0, stream));
        for (int k = 0; k < reps; ++k) run();
        HIPCHK(hipEventRecord(e1, stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (best < 0.f || ms < best) {
          best = ms;
          bv = v;
        }
      }
      if (level == 0) var_c = bv;
      else var_f = bv;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graph();
    out[0] = var_c;
    out[1] = var_f;
  }

  // Applies variants a previous tune returned (same meaning as its output).
  void set_variants(const int32_t* v) override {
    const int nf = fused() ? kNTile : NVAR;
    if (v[0] < 0 || v[0] >= NVAR || v[1] < 0 || v[1] >= nf)
      throw LbmError(LBM_EINVAL, "variant index out of range");
    HIPCHK(hipSetDevice(device));
    quiesce();
    var_c = v[0];
    var_f = v[1];
    if (fused()) set_tile_var(v[1]);
    drop_graph();
  }

  void info(int64_t* out) override {
    int64_t active = 0, ups = 0, bytes = 0;
    for (int k = 0; k < capacity; ++k) {
      if (!slots[(size_t)k]) continue;
      const Inst& in = *slots[(size_t)k];
      active++;
      int64_t u = in.g.Nc;
      if (in.g.has_fine) {
        int64_t cov = 1;
        for (int d = 0; d < D; ++d) cov *= (in.g.m[d] - 3);
        u = in.g.Nc - cov + 2 * in.g.Nf;
      }
      ups += u;
      bytes += grid_footprint(in.desc, in.g);
    }
    out[0] = active;
    out[1] = ups;
    out[2] = bytes;
  }

  int64_t slot_steps(int sl) override {
    slot_ref(sl);
    return steps_done[(size_t)sl];
  }
};

static BatchBase* make_batch(int lattice, int precision) {
  if (lattice == LBM_D2Q9 && precision == LBM_FP64) return new Batch<0, LBM_FP64>();
  if (lattice == LBM_D2Q9 && precision == LBM_FP32_DEV) return new Batch<0, LBM_FP32_DEV>();
  if (lattice == LBM_D3Q19 && precision == LBM_FP64) return new Batch<1, LBM_FP64>();
  if (lattice == LBM_D3Q19 && precision == LBM_FP32_DEV) return new Batch<1, LBM_FP32_DEV>();
  return nullptr;
}

}  // namespace lbm

using namespace lbm;

struct lbm_grid {
  std::unique_ptr<GridBase> impl;
};


// Streaming copy for the bandwidth reference: 16-byte non-temporal loads
// and stores, four per lane in flight; work group b copies vectors
// [1024 b, 1024 b + 1024) of n (a fixed grid walking the buffer with a
// stride measured 15 % slower on gfx950).
using F4 = VT<float, 4>::a;
__global__ __launch_bounds__(256) void k_copy16(const F4* __restrict__ a, F4* __restrict__ b, int64_t n) {
  const int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  F4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = i0 + (int64_t)k * 256;
    if (i < n) v[k] = __builtin_nontemporal_load(a + i);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = i0 + (int64_t)k * 256;
    if (i < n) __builtin_nontemporal_store(v[k], b + i);
  }
}

template <typename F>
static int guard(lbm_handle h, F&& fn) {
  std::lock_guard<std::recursive_mutex> lk(g_api_mu);
  try {
    fn();
    return LBM_OK;
  } catch (const LbmError& e) {
    if (h && h->impl) h->impl->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (h && h->impl) h->impl->err = "host allocation failed";
    return LBM_ENOMEM;
  } catch (...) {
    if (h && h->impl) h->impl->err = "unexpected exception";
    return LBM_EDEVICE;
  }
}

extern "C" {

int lbm_create_grid(const lbm_grid_desc* d, lbm_handle* out) {
  std::lock_guard<std::recursive_mutex> lk(g_api_mu);
  if (!d || !out) {
    g_create_error = "null argument";
    return LBM_EINVAL;
  }
  *out = nullptr;
  std::unique_ptr<GridBase> gb;
  try {
    Geo geo = validate(*d);
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (d->device < 0 || d->device >= ndev) throw LbmError(LBM_EINVAL, "no such HIP device");
    gb.reset(make_grid(*d));
    gb->desc = *d;
    gb->g = geo;
    gb->device = d->device;
    HIPCHK(hipSetDevice(d->device));
    HIPCHK(hipStreamCreateWithFlags(&gb->stream, hipStreamNonBlocking));
    build_tables(geo, gb->tabs);
    gb->init();
    HIPCHK(hipDeviceSynchronize());
  } catch (const LbmError& e) {
    g_create_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    return LBM_ENOMEM;
  }
  auto* h = new lbm_grid;
  h->impl = std::move(gb);
  *out = h;
  return LBM_OK;
}

int lbm_create_nested(const lbm_grid_desc* d, const int32_t lo2[3], const int32_t hi2[3], lbm_handle* out) {
  std::lock_guard<std::recursive_mutex> lk(g_api_mu);
  if (!d || !lo2 || !hi2 || !out) {
    g_create_error = "null argument";
    return LBM_EINVAL;
  }
  *out = nullptr;
  std::unique_ptr<GridBase> gb;
  try {
    Geo geo = validate(*d);
    if (!geo.has_fine) throw LbmError(LBM_EINVAL, "a nested grid needs the level-1 patch");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (d->device < 0 || d->device >= ndev) throw LbmError(LBM_EINVAL, "no such HIP device");
    // the pair (level 1, level 2): level 1 as a periodic coarse grid
    lbm_grid_desc dc = *d;
    for (int k = 0; k < 3; ++k) {
      dc.n[k] = geo.nf[k];
      dc.lo[k] = lo2[k];
      dc.hi[k] = hi2[k];
    }
    dc.tau_coarse = 2.0 * d->tau_coarse - 0.5;
    Geo gc = validate(dc);
    if (!gc.has_fine) throw LbmError(LBM_EINVAL, "a nested grid needs the level-2 patch");
    std::unique_ptr<GridBase> child(make_grid(dc));
    child->desc = dc;
    child->g = gc;
    child->device = d->device;
    HIPCHK(hipSetDevice(d->device));
    HIPCHK(hipStreamCreateWithFlags(&child->stream, hipStreamNonBlocking));
    child->nested_child = true;
    build_tables(gc, child->tabs);
    child->init();
    // level 1 is stored in the child's coarse layout
    geo.pf = gc.pc;
    geo.fxo = 0;
    geo.Nfp = gc.Ncp;
    gb.reset(make_grid(*d));
    gb->desc = *d;
    gb->g = geo;
    gb->device = d->device;
    gb->child = std::move(child);
    HIPCHK(hipStreamCreateWithFlags(&gb->stream, hipStreamNonBlocking));
    build_tables(geo, gb->tabs);
    gb->init();
    HIPCHK(hipDeviceSynchronize());
  } catch (const LbmError& e) {
    g_create_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    return LBM_ENOMEM;
  }
  auto* h = new lbm_grid;
  h->impl = std::move(gb);
  *out = h;
  return LBM_OK;
}

int lbm_destroy(lbm_handle h) {
  if (!h) return LBM_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g_api_mu);
  (void)hipSetDevice(h->impl->device);
  (void)hipStreamSynchronize(h->impl->stream);
  delete h;
  return LBM_OK;
}

static bool bad_level(lbm_handle h, int level) {
  return !h || level < 0 || level >= h->impl->levels();
}

int lbm_set_state(lbm_handle h, int level, const double* rho, const double* u, int mem) {
  if (bad_level(h, level) || !rho || !u || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return guard(h, [&] { h->impl->set_state(level, rho, u, mem == LBM_DEVICE); });
}

int lbm_step(lbm_handle h, int n, void* stream) {
  if (!h || n < 0) return LBM_EINVAL;
  return guard(h, [&] { h->impl->step(n, stream ? (hipStream_t)stream : h->impl->stream); });
}

int lbm_get_macros(lbm_handle h, int level, double* rho, double* u, int mem) {
  if (bad_level(h, level) || !rho || !u || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return guard(h, [&] {
    HIPCHK(hipDeviceSynchronize());
    h->impl->get_macros(level, rho, u, mem == LBM_DEVICE);
  });
}

int lbm_set_populations(lbm_handle h, int level, const double* f, int mem) {
  if (bad_level(h, level) || !f || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return guard(h, [&] { h->impl->set_pops(level, f, mem == LBM_DEVICE); });
}

int lbm_get_populations(lbm_handle h, int level, double* f, int mem) {
  if (bad_level(h, level) || !f || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return guard(h, [&] {
    HIPCHK(hipDeviceSynchronize());
    h->impl->get_pops(level, f, mem == LBM_DEVICE);
  });
}

int lbm_get_totals(lbm_handle h, double mass[2], double momentum[6]) {
  if (!h || !mass || !momentum) return LBM_EINVAL;
  int rc = guard(h, [&] {
    HIPCHK(hipDeviceSynchronize());
    h->impl->totals(mass, momentum);
  });
  if (rc != LBM_OK) return rc;
  for (int k = 0; k < 2; ++k)
    if (!std::isfinite(mass[k])) {
      h->impl->err = "non-finite mass";
      return LBM_EUNSTABLE;
    }
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(momentum[k])) {
      h->impl->err = "non-finite momentum";
      return LBM_EUNSTABLE;
    }
  return LBM_OK;
}

// Allocation-free totals.  The partial sums and the final sums live in a
// file-scope device array instead of buffers of the grid: 4 doubles per block
// of 256 nodes for up to kNoAllocBlocks blocks (levels of at most 2^26 nodes),
// then the 4 final sums; 8 MiB + 32 B per GPU, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): its device address is looked up once per
// device, with that device current, and kept in g_scratch_ptr.
static constexpr int64_t kNoAllocBlocks = (int64_t)1 << 18;
static constexpr int64_t kNoAllocMaxNodes = kNoAllocBlocks * 256;
static __device__ __align__(256) double scratch[4 * kNoAllocBlocks + 4];
static constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (caller holds g_api_mu).
static double* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) throw LbmError(LBM_EINVAL, "device ordinal beyond the scratch table");
  if (!g_scratch_ptr[device]) {
    HIPCHK(hipSetDevice(device));
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw LbmError(LBM_EDEVICE, "hipGetSymbolAddress returned no address for the totals scratch");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  return g_scratch_ptr[device];
}

int lbm_get_totals_noalloc(lbm_handle h, double mass[2], double momentum[6]) {
  if (!h || !mass || !momentum) return LBM_EINVAL;
  int rc = guard(h, [&] {
    const GridBase& gb = *h->impl;
    const int64_t nmax = std::max(gb.g.Nc, gb.g.has_fine ? gb.g.Nf : (int64_t)0);
    if (nmax > kNoAllocMaxNodes)
      throw LbmError(LBM_EINVAL, "lbm_get_totals_noalloc: a level has " + std::to_string(nmax) +
                                     " nodes; its scratch holds the partial sums of at most " +
                                     std::to_string(kNoAllocMaxNodes) + " nodes per level");
    double* p = scratch_on(gb.device);
    HIPCHK(hipSetDevice(gb.device));
    HIPCHK(hipDeviceSynchronize());
    h->impl->totals_in(mass, momentum, p, p + 4 * kNoAllocBlocks);
  });
  if (rc != LBM_OK) return rc;
  for (int k = 0; k < 2; ++k)
    if (!std::isfinite(mass[k])) {
      h->impl->err = "non-finite mass";
      return LBM_EUNSTABLE;
    }
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(momentum[k])) {
      h->impl->err = "non-finite momentum";
      return LBM_EUNSTABLE;
    }
  return LBM_OK;
}

int lbm_sensors_enable(lbm_handle h, int on) {
  if (!h) return LBM_EINVAL;
  return guard(h, [&] { h->impl->sensors_enable(on != 0); });
}

int lbm_set_dynamic_sigma(lbm_handle h, int on, double sigma_dyn, double threshold) {
  if (!h) return LBM_EINVAL;
  if (on && (h->impl->desc.collision != LBM_HRR || !(sigma_dyn >= 0.0 && sigma_dyn <= 1.0) ||
             !(threshold >= 0.0) || !std::isfinite(threshold)))
    return LBM_EINVAL;
  return guard(h, [&] { h->impl->set_dynamic_sigma(on != 0, sigma_dyn, threshold); });
}

int lbm_sensors(lbm_handle h, int level, double threshold, uint8_t* flags, double* diag, int mem) {
  if (bad_level(h, level) || !flags || (mem != LBM_HOST && mem != LBM_DEVICE) || !(threshold >= 0.0))
    return LBM_EINVAL;
  return guard(h, [&] {
    HIPCHK(hipDeviceSynchronize());
    h->impl->sensors(level, threshold, flags, diag, mem == LBM_DEVICE);
  });
}

int lbm_probe_enable(lbm_handle h, int level, const int32_t node[3], int64_t capacity) {
  if (!h || level < -1 || level > 1 || (level == 1 && !h->impl->g.has_fine) || (level >= 0 && !node))
    return LBM_EINVAL;
  return guard(h, [&] { h->impl->probe_enable(level, node, capacity); });
}

int lbm_probe_read(lbm_handle h, double* out, int64_t max, int64_t* count) {
  if (!h || !count || max < 0 || (max > 0 && !out)) return LBM_EINVAL;
  return guard(h, [&] { *count = h->impl->probe_read(out, max); });
}

int lbm_get_index_maps(lbm_handle h, int level, uint8_t* cls, int mem) {
  if (bad_level(h, level) || !cls || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return guard(h, [&] {
    // nested: level 1 has the classes of the parent pair (its ring, TN^f),
    // level 2 those of the child pair
    const GridBase& G = level == 2 ? *h->impl->child : *h->impl;
    const auto& v = level == 0 ? G.tabs.cls_c : G.tabs.cls_f;
    if (mem == LBM_HOST) std::memcpy(cls, v.data(), v.size());
    else HIPCHK(hipMemcpy(cls, v.data(), v.size(), hipMemcpyHostToDevice));
  });
}

int lbm_level_dims(lbm_handle h, int level, int32_t dims[3]) {
  if (bad_level(h, level) || !dims) return LBM_EINVAL;
  const Geo& G = level == 2 ? h->impl->child->g : h->impl->g;
  for (int k = 0; k < 3; ++k) dims[k] = level == 0 ? G.n[k] : G.nf[k];
  return LBM_OK;
}

int lbm_lattice_info(int lattice, int32_t* D, int32_t* Q, int32_t* xi, double* w) {
  if (!D || !Q || !xi || !w) return LBM_EINVAL;
  if (lattice == LBM_D2Q9) {
    *D = 2;
    *Q = 9;
    for (int i = 0; i < 9; ++i) {
      xi[3 * i] = Lattice<0>::cx(i);
      xi[3 * i + 1] = Lattice<0>::cy(i);
      xi[3 * i + 2] = 0;
      w[i] = Lattice<0>::w(i);
    }
    return LBM_OK;
  }
  if (lattice == LBM_D3Q19) {
    *D = 3;
    *Q = 19;
    for (int i = 0; i < 19; ++i) {
      xi[3 * i] = Lattice<1>::cx(i);
      xi[3 * i + 1] = Lattice<1>::cy(i);
      xi[3 * i + 2] = Lattice<1>::cz(i);
      w[i] = Lattice<1>::w(i);
    }
    return LBM_OK;
  }
  return LBM_EINVAL;
}

int lbm_interface_counts(lbm_handle h, int64_t counts[3]) {
  if (!h || !counts) return LBM_EINVAL;
  counts[0] = (int64_t)h->impl->tabs.hnode.size();
  counts[1] = (int64_t)h->impl->tabs.rnode.size();
  counts[2] = (int64_t)h->impl->tabs.tnf.size();
  return LBM_OK;
}

int lbm_interface_tables(lbm_handle h, int64_t* hist_nodes, int64_t* ring_nodes, int32_t* ring_npts,
                         int64_t* ring_pts) {
  if (!h) return LBM_EINVAL;
  const auto& t = h->impl->tabs;
  if (hist_nodes) std::memcpy(hist_nodes, t.hnode.data(), sizeof(int64_t) * t.hnode.size());
  if (ring_nodes) std::memcpy(ring_nodes, t.rnode.data(), sizeof(int64_t) * t.rnode.size());
  if (ring_npts) std::memcpy(ring_npts, t.rnp.data(), sizeof(int32_t) * t.rnp.size());
  if (ring_pts)
    for (size_t k = 0; k < t.rpt.size(); ++k) ring_pts[k] = t.rpt[k];
  return LBM_OK;
}

int lbm_updates_per_step(lbm_handle h, int64_t* updates) {
  if (!h || !updates) return LBM_EINVAL;
  *updates = h->impl->updates();
  return LBM_OK;
}

int lbm_profile_enable(lbm_handle h, int on) {
  if (!h) return LBM_EINVAL;
  return guard(h, [&] {
    auto& G = *h->impl;
    HIPCHK(hipSetDevice(G.device));
    HIPCHK(hipDeviceSynchronize());
    for (auto& e : G.events) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    G.events.clear();
    G.prof_launches = 0;
    G.prof_ms = 0.0;
    G.profile = on != 0;
  });
}

int lbm_kernel_time(lbm_handle h, int64_t* launches, double* mean_ms, int64_t* nodes_per_launch) {
  if (!h || !launches || !mean_ms || !nodes_per_launch) return LBM_EINVAL;
  return guard(h, [&] {
    auto& G = *h->impl;
    HIPCHK(hipSetDevice(G.device));
    HIPCHK(hipDeviceSynchronize());
    for (auto& e : G.events) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
      G.prof_ms += ms;
      G.prof_launches++;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    G.events.clear();
    *launches = G.prof_launches;
    *mean_ms = G.prof_launches ? G.prof_ms / (double)G.prof_launches : 0.0;
    int64_t mid = 1;
    for (int d = 0; d < G.g.D; ++d) mid *= (G.g.has_fine ? G.g.nf[d] - 2 : 0);
    *nodes_per_launch = mid * G.timed_factor;
  });
}

int lbm_tune(lbm_handle h, int reps, int32_t variants[4]) {
  if (!h || reps < 1 || !variants) return LBM_EINVAL;
  return guard(h, [&] {
    HIPCHK(hipDeviceSynchronize());
    h->impl->tune(reps, variants);
  });
}

int lbm_set_variants(lbm_handle h, const int32_t variants[4]) {
  if (!h || !variants) return LBM_EINVAL;
  return guard(h, [&] { h->impl->set_variants(variants); });
}

const char* lbm_last_error(lbm_handle h) {
  if (!h) return g_create_error.c_str();
  return h->impl->err.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batch ABI.
struct lbm_batch {
  std::unique_ptr<BatchBase> impl;
};

template <bool LOCK = true, typename F>
static int bguard(lbm_batch_handle b, F&& fn) {
  std::unique_lock<std::recursive_mutex> lk(g_api_mu, std::defer_lock);
  if (LOCK) lk.lock();
  try {
    fn();
    return LBM_OK;
  } catch (const LbmError& e) {
    if (b && b->impl) b->impl->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (b && b->impl) b->impl->err = "host allocation failed";
    return LBM_ENOMEM;
  } catch (...) {
    if (b && b->impl) b->impl->err = "unexpected exception";
    return LBM_EDEVICE;
  }
}

extern "C" {

int lbm_batch_create(int lattice, int collision, int precision, int device, int capacity, lbm_batch_handle* out) {
  if (!out) return LBM_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g_api_mu);
  *out = nullptr;
  if ((lattice != LBM_D2Q9 && lattice != LBM_D3Q19) || collision < LBM_BGK || collision > LBM_HRR ||
      (precision != LBM_FP64 && precision != LBM_FP32_DEV) || capacity < 1 || capacity > (1 << 20)) {
    g_create_error = "invalid batch parameters";
    return LBM_EINVAL;
  }
  try {
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw LbmError(LBM_EINVAL, "no such HIP device");
    std::unique_ptr<BatchBase> b(make_batch(lattice, precision));
    b->lattice = lattice;
    b->collision = collision;
    b->precision = precision;
    b->device = device;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->stepped, hipEventDisableTiming));
    if (lattice == LBM_D2Q9 && precision == LBM_FP64) static_cast<Batch<0, LBM_FP64>*>(b.get())->init(capacity);
    if (lattice == LBM_D2Q9 && precision == LBM_FP32_DEV) static_cast<Batch<0, LBM_FP32_DEV>*>(b.get())->init(capacity);
    if (lattice == LBM_D3Q19 && precision == LBM_FP64) static_cast<Batch<1, LBM_FP64>*>(b.get())->init(capacity);
    if (lattice == LBM_D3Q19 && precision == LBM_FP32_DEV)
      static_cast<Batch<1, LBM_FP32_DEV>*>(b.get())->init(capacity);
    auto* h = new lbm_batch;
    h->impl = std::move(b);
    *out = h;
    return LBM_OK;
  } catch (const LbmError& e) {
    g_create_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    return LBM_ENOMEM;
  }
}

int lbm_batch_destroy(lbm_batch_handle b) {
  if (!b) return LBM_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g_api_mu);
  (void)hipSetDevice(b->impl->device);
  (void)hipDeviceSynchronize();
  delete b;
  return LBM_OK;
}

int lbm_batch_add(lbm_batch_handle b, const lbm_grid_desc* d, int32_t* slot) {
  if (!b || !d || !slot) return LBM_EINVAL;
  return bguard(b, [&] { *slot = b->impl->add(*d); });
}

int lbm_batch_remove(lbm_batch_handle b, int slot) {
  if (!b) return LBM_EINVAL;
  return bguard(b, [&] { b->impl->remove(slot); });
}

int lbm_batch_set_state(lbm_batch_handle b, int slot, int level, const double* rho, const double* u, int mem) {
  if (!b || !rho || !u || level < 0 || level > 1 || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return bguard(b, [&] { b->impl->set_state(slot, level, rho, u, mem == LBM_DEVICE); });
}

int lbm_batch_get_macros(lbm_batch_handle b, int slot, int level, double* rho, double* u, int mem) {
  if (!b || !rho || !u || level < 0 || level > 1 || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return bguard(b, [&] { b->impl->get_macros(slot, level, rho, u, mem == LBM_DEVICE); });
}

int lbm_batch_get_populations(lbm_batch_handle b, int slot, int level, double* f, int mem) {
  if (!b || !f || level < 0 || level > 1 || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return bguard(b, [&] { b->impl->get_pops(slot, level, f, mem == LBM_DEVICE); });
}

int lbm_batch_step(lbm_batch_handle b, int n, void* stream) {
  if (!b || n < 0) return LBM_EINVAL;
  return bguard<false>(b, [&] { b->impl->step(n, stream ? (hipStream_t)stream : b->impl->stream); });
}

int lbm_batch_use_graph(lbm_batch_handle b, int on) {
  if (!b) return LBM_EINVAL;
  return bguard(b, [&] { b->impl->set_graph(on != 0); });
}

int lbm_batch_tune(lbm_batch_handle b, int reps, int32_t variants[2]) {
  if (!b || reps < 1 || !variants) return LBM_EINVAL;
  return bguard(b, [&] { b->impl->tune(reps, variants); });
}

int lbm_batch_set_variants(lbm_batch_handle b, const int32_t variants[2]) {
  if (!b || !variants) return LBM_EINVAL;
  return bguard(b, [&] { b->impl->set_variants(variants); });
}

int lbm_batch_info(lbm_batch_handle b, int64_t info[3]) {
  if (!b || !info) return LBM_EINVAL;
  return bguard<false>(b, [&] { b->impl->info(info); });
}

int lbm_batch_slot_steps(lbm_batch_handle b, int slot, int64_t* steps) {
  if (!b || !steps) return LBM_EINVAL;
  return bguard<false>(b, [&] { *steps = b->impl->slot_steps(slot); });
}

int lbm_footprint(const lbm_grid_desc* d, int64_t* bytes) {
  if (!d || !bytes) return LBM_EINVAL;
  try {
    const Geo g = validate(*d);
    *bytes = grid_footprint(*d, g);
    return LBM_OK;
  } catch (const LbmError& e) {
    g_create_error = e.msg;
    return e.code;
  }
}

int lbm_copy_probe(int device, int64_t bytes, int reps, double* gbs) {
  if (!gbs || bytes < 16 || reps < 1) return LBM_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g_api_mu);
  try {
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw LbmError(LBM_EINVAL, "no such HIP device");
    HIPCHK(hipSetDevice(device));
    const int64_t n = bytes / 16;
    DevBuf a, b;
    a.alloc((size_t)n * 16);
    b.alloc((size_t)n * 16);
    HIPCHK(hipMemset(a.p, 0, a.bytes));
    if ((n + 1023) / 1024 > (int64_t)INT32_MAX) throw LbmError(LBM_EINVAL, "copy too large");
    const unsigned grid = (unsigned)((n + 1023) / 1024);
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, st, a.as<const F4>(), b.as<F4>(), n);
    HIPCHK(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r)
      hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, st, a.as<const F4>(), b.as<F4>(), n);
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    *gbs = 2.0 * (double)n * 16.0 * reps / ((double)ms * 1e-3) / 1e9;
    return LBM_OK;
  } catch (const LbmError& e) {
    g_create_error = e.msg;
    return e.code;
  }
}

const char* lbm_batch_last_error(lbm_batch_handle b) {
  if (!b) return g_create_error.c_str();
  return b->impl->err.c_str();
}

}  // extern "C"
