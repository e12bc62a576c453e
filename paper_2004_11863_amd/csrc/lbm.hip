// lbm.hip -- host side of the MI355X two-level LBM library: descriptor
// validation, interface table builder, device state, the per-coarse-step
// launch schedule (Sec. 4.3) and the C ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lbm.h"

namespace lbm {

static thread_local std::string g_create_error;

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
  void alloc(size_t b) {
    bytes = b;
    if (b == 0) return;
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      throw LbmError(LBM_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
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
  virtual void tune(int reps, int32_t* out) = 0;
  virtual void set_variants(const int32_t* v) = 0;
  int64_t nodes(int level) const { return level == 0 ? g.Nc : g.Nf; }
  int64_t updates() const {
    if (!g.has_fine) return g.Nc;
    int64_t cov = 1;
    for (int d = 0; d < g.D; ++d) cov *= (g.m[d] - 3);
    return g.Nc - cov + 2 * g.Nf;
  }
};

template <int LAT, int PREC>
struct Grid final : GridBase {
  using L = Lattice<LAT>;
  static constexpr bool DEV = PREC == LBM_FP32_DEV;
  using S = typename std::conditional<DEV, float, double>::type;  // stored and bulk compute type
  using F = HF<LAT>;
  static constexpr int Q = L::Q, D = L::D;
  static constexpr bool NT = true;  // non-temporal stores of the streamed planes
  // Bulk-kernel variants (nodes per lane V, lanes along x LX; work groups are
  // LX x 256/LX).  FP32: 16-byte (V = 4) or 8-byte (V = 2) accesses; FP64:
  // 16-byte (V = 2).
  static constexpr int NVAR = DEV ? 5 : 3;
  static constexpr int kV[5] = {DEV ? 4 : 2, DEV ? 4 : 2, DEV ? 4 : 2, 2, 2};
  static constexpr int kLX[5] = {64, 32, 16, 64, 32};
  // chosen variant per role: 0 coarse stream, 1 fine stream, 2 coarse H-RR
  // collision, 3 fine H-RR collision
  int var[4] = {0, 0, 0, 0};

  DevBuf cbuf[2], fbuf[2], mac_c, mac_f, hist[3], G, tmp_rho, tmp_u, tmp_f, part, tot;
  DevBuf d_hnode, d_rnode, d_rnp, d_rpt, d_tnf, d_tnc;
  int cpar = 0;  // coarse buffer holding the current state
  int hs[3] = {0, 1, 2};
  Iface itf{};
  double tau_c = 0, tau_f = 0, sig = 0;

  // padded plane storage plus slack for the one-element overreach of the
  // x-shifted vector loads at the very end of a buffer
  static size_t plane_bytes(int64_t NP, int nplanes) { return sizeof(S) * ((size_t)NP * nplanes + 64); }

  void init() override {
    for (int p = 0; p < 2; ++p) cbuf[p].alloc(plane_bytes(g.Ncp, Q));
    if (g.has_fine)
      for (int p = 0; p < 2; ++p) fbuf[p].alloc(plane_bytes(g.Nfp, Q));
    if (desc.collision == LBM_HRR) {
      mac_c.alloc(plane_bytes(g.Ncp, 1 + D));
      if (g.has_fine) mac_f.alloc(plane_bytes(g.Nfp, 1 + D));
    }
    tau_c = desc.tau_coarse;
    tau_f = 2.0 * tau_c - 0.5;
    sig = desc.sigma;
    for (int r = 0; r < 4; ++r) var[r] = default_variant(r & 1);
    if (g.has_fine) {
      const size_t NH = tabs.hnode.size();
      for (int s = 0; s < 3; ++s) hist[s].alloc(sizeof(double) * F::N * NH);
      G.alloc(sizeof(double) * F::N * NH);
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
    if (g.has_fine)
      for (int p = 0; p < 2; ++p) HIPCHK(hipMemset(fbuf[p].p, 0, fbuf[p].bytes));
    if (mac_c.p) HIPCHK(hipMemset(mac_c.p, 0, mac_c.bytes));
    if (mac_f.p) HIPCHK(hipMemset(mac_f.p, 0, mac_f.bytes));
  }

  static unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

  Tiling tiling(int level, int v) const {
    const int V = kV[v], LX = kLX[v];
    if (level == 0) return make_tiling(g.n[0], g.n[1], g.n[2], 0, V, LX, 256 / LX);
    return make_tiling(g.nf[0], g.nf[1], g.nf[2], 1, V, LX, 256 / LX);
  }
  // Variant with the fewest idle lanes along x (ties: the earlier one).
  int default_variant(int level) const {
    if (level == 1 && !g.has_fine) return 0;
    int best = 0;
    int64_t bw = -1;
    for (int v = 0; v < NVAR; ++v) {
      if (kV[v] != kV[0]) continue;
      const Tiling t = tiling(level, v);
      const int64_t waste = (int64_t)t.ntx * kLX[v] - t.nv;
      if (bw < 0 || waste < bw) {
        bw = waste;
        best = v;
      }
    }
    return best;
  }

  S* cur_c() { return cbuf[cpar].as<S>(); }
  S* fineA() { return fbuf[0].as<S>(); }
  S* fineB() { return fbuf[1].as<S>(); }

  template <int MODEL, int LEVEL, int V, int LX>
  void go_stream(const S* src, S* dst, S* mac, double tau, hipStream_t s, int v) {
    const Tiling t = tiling(LEVEL, v);
    const S om = (S)(1.0 - 1.0 / tau);
    hipLaunchKernelGGL((k_stream<LAT, DEV, S, MODEL, LEVEL, V, LX, NT>), dim3((unsigned)(t.per_xcd * kXCD)),
                       dim3(256), 0, s, src, dst, mac, g, t, om);
  }
  template <int MODEL, int LEVEL>
  void launch_stream(const S* src, S* dst, S* mac, double tau, hipStream_t s, int v = -1) {
    if (v < 0) v = var[LEVEL];
    if constexpr (DEV) {
      switch (v) {
        case 0: go_stream<MODEL, LEVEL, 4, 64>(src, dst, mac, tau, s, v); break;
        case 1: go_stream<MODEL, LEVEL, 4, 32>(src, dst, mac, tau, s, v); break;
        case 2: go_stream<MODEL, LEVEL, 4, 16>(src, dst, mac, tau, s, v); break;
        case 3: go_stream<MODEL, LEVEL, 2, 64>(src, dst, mac, tau, s, v); break;
        default: go_stream<MODEL, LEVEL, 2, 32>(src, dst, mac, tau, s, 4); break;
      }
    } else {
      switch (v) {
        case 0: go_stream<MODEL, LEVEL, 2, 64>(src, dst, mac, tau, s, v); break;
        case 1: go_stream<MODEL, LEVEL, 2, 32>(src, dst, mac, tau, s, v); break;
        default: go_stream<MODEL, LEVEL, 2, 16>(src, dst, mac, tau, s, 2); break;
      }
    }
  }

  template <int LEVEL, int V, int LX>
  void go_collide(S* buf, const S* mac, double tau, hipStream_t s, int v) {
    const Tiling t = tiling(LEVEL, v);
    hipLaunchKernelGGL((k_collide_hrr<LAT, DEV, S, LEVEL, V, LX, NT>), dim3((unsigned)(t.per_xcd * kXCD)), dim3(256),
                       0, s, buf, mac, g, t, (S)(1.0 - 1.0 / tau), (S)tau, (S)sig);
  }
  template <int LEVEL>
  void launch_collide_hrr(S* buf, const S* mac, double tau, hipStream_t s, int v = -1) {
    if (v < 0) v = var[2 + LEVEL];
    if constexpr (DEV) {
      switch (v) {
        case 0: go_collide<LEVEL, 4, 64>(buf, mac, tau, s, v); break;
        case 1: go_collide<LEVEL, 4, 32>(buf, mac, tau, s, v); break;
        case 2: go_collide<LEVEL, 4, 16>(buf, mac, tau, s, v); break;
        case 3: go_collide<LEVEL, 2, 64>(buf, mac, tau, s, v); break;
        default: go_collide<LEVEL, 2, 32>(buf, mac, tau, s, 4); break;
      }
    } else {
      switch (v) {
        case 0: go_collide<LEVEL, 2, 64>(buf, mac, tau, s, v); break;
        case 1: go_collide<LEVEL, 2, 32>(buf, mac, tau, s, v); break;
        default: go_collide<LEVEL, 2, 16>(buf, mac, tau, s, 2); break;
      }
    }
  }

  void fine_stream_timed(int model, const S* src, S* dst, hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, s));
    }
    if (model == M_BGK) launch_stream<M_BGK, 1>(src, dst, nullptr, tau_f, s);
    else if (model == M_RR) launch_stream<M_RR, 1>(src, dst, nullptr, tau_f, s);
    else launch_stream<M_HRR, 1>(src, dst, mac_f.as<S>(), tau_f, s);
    if (profile) {
      HIPCHK(hipEventRecord(e1, s));
      events.emplace_back(e0, e1);
    }
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
    } else if (role == 1) {
      if (model == M_BGK) launch_stream<M_BGK, 1>(fineA(), fineB(), nullptr, tau_f, s, v);
      else if (model == M_RR) launch_stream<M_RR, 1>(fineA(), fineB(), nullptr, tau_f, s, v);
      else launch_stream<M_HRR, 1>(fineA(), fineB(), mac_f.as<S>(), tau_f, s, v);
    } else if (role == 2) {
      launch_collide_hrr<0>(c_oth, mac_c.as<S>(), tau_c, s, v);
    } else {
      launch_collide_hrr<1>(fineB(), mac_f.as<S>(), tau_f, s, v);
    }
  }

  void set_variants(const int32_t* v) override {
    for (int r = 0; r < 4; ++r)
      if (v[r] < 0 || v[r] >= NVAR) throw LbmError(LBM_EINVAL, "variant index out of range");
    for (int r = 0; r < 4; ++r) var[r] = v[r];
  }

  void tune(int reps, int32_t* out) override {
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamSynchronize(stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int role = 0; role < 4; ++role) {
      const bool used = (role & 1) ? g.has_fine : true;
      const bool hrr_role = role >= 2;
      if (!used || (hrr_role && desc.collision != LBM_HRR)) continue;
      float best = -1.f;
      for (int v = 0; v < NVAR; ++v) {
        role_launch(role, v, stream);
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
      launch_collide_hrr<0>(dst, mac_c.as<S>(), tau_c, s);
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
    const double c0 = -1.0 / 8.0, c1 = 3.0 / 4.0, c2 = 3.0 / 8.0;
    constexpr int IB = kIfaceBlock;
    constexpr int PER = 256 / (D == 2 ? 9 : 27);
    const unsigned bh = blocks(NH, IB), br = blocks(itf.NR, IB), bt = blocks(itf.NT, IB), bg = blocks(NH * F::N, 256);
    const unsigned bc = blocks(itf.NT, PER);
    hipLaunchKernelGGL((k_hist_capture<LAT, DEV, S>), dim3(bh), dim3(IB), 0, s, csrc, Hp, g, itf);
    if (MODEL != M_HRR) {
      launch_stream<MODEL, 0>(csrc, cdst, nullptr, tau_c, s);
      fine_stream_timed(MODEL, fA, fB, s);
      hipLaunchKernelGGL(k_hist_time, dim3(bg), dim3(256), 0, s, Hm, H0, Hp, G.as<double>(), NH * F::N, c0, c1, c2);
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, MODEL>), dim3(br), dim3(IB), 0, s, G.as<double>(), fB, g, itf, kf, omf,
                         tau_f, sig);
      fine_stream_timed(MODEL, fB, fA, s);
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, MODEL>), dim3(br), dim3(IB), 0, s, Hp, fA, g, itf, kf, omf, tau_f, sig);
      hipLaunchKernelGGL((k_coalesce<LAT, DEV, S, MODEL>), dim3(bc), dim3(256), 0, s, fB, cdst, g, itf, kc, omc,
                         tau_c, sig);
    } else {
      S* mc = mac_c.as<S>();
      S* mf = mac_f.as<S>();
      launch_stream<M_HRR, 0>(csrc, cdst, mc, tau_c, s);
      fine_stream_timed(M_HRR, fA, fB, s);
      hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, s, Hm, H0, Hp, c0, c1, c2, mf, g, itf);
      launch_collide_hrr<1>(fB, mf, tau_f, s);
      hipLaunchKernelGGL((k_fict<LAT, DEV, S, S>), dim3(bt), dim3(IB), 0, s, fB, mc, g, itf);
      hipLaunchKernelGGL((k_hist_strain<LAT, S>), dim3(bh), dim3(IB), 0, s, mc, Hp, g, itf);
      hipLaunchKernelGGL(k_hist_time, dim3(bg), dim3(256), 0, s, Hm, H0, Hp, G.as<double>(), NH * F::N, c0, c1, c2);
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_HRR>), dim3(br), dim3(IB), 0, s, G.as<double>(), fB, g, itf, kf, omf,
                         tau_f, sig);
      fine_stream_timed(M_HRR, fB, fA, s);
      hipLaunchKernelGGL((k_ring_macro<LAT, S>), dim3(br), dim3(IB), 0, s, Hm, H0, Hp, 0.0, 0.0, 1.0, mf, g, itf);
      launch_collide_hrr<1>(fA, mf, tau_f, s);
      hipLaunchKernelGGL((k_ring<LAT, DEV, S, M_HRR>), dim3(br), dim3(IB), 0, s, Hp, fA, g, itf, kf, omf, tau_f, sig);
      // coarse collision before the TN transfer: the vector kernel also
      // passes over TN nodes, which the transfer then overwrites
      launch_collide_hrr<0>(cdst, mc, tau_c, s);
      hipLaunchKernelGGL((k_coalesce<LAT, DEV, S, M_HRR>), dim3(bc), dim3(256), 0, s, fB, cdst, g, itf, kc, omc,
                         tau_c, sig);
    }
    HIPCHK(hipGetLastError());
    cpar ^= 1;
    const int old = hs[0];
    hs[0] = hs[1];
    hs[1] = hs[2];
    hs[2] = old;
  }

  void step(int n, hipStream_t s) override {
    HIPCHK(hipSetDevice(device));
    for (int k = 0; k < n; ++k) {
      if (!g.has_fine) step_uniform(s);
      else if (desc.collision == LBM_BGK) step_two_level<M_BGK>(s);
      else if (desc.collision == LBM_RR) step_two_level<M_RR>(s);
      else step_two_level<M_HRR>(s);
    }
    HIPCHK(hipGetLastError());
  }

  void upload(DevBuf& dst, const double* src, size_t n, bool dev) {
    HIPCHK(hipMemcpyAsync(dst.p, src, sizeof(double) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          stream));
  }

  void reset_history_from_tmp() {
    hs[0] = 0;
    hs[1] = 1;
    hs[2] = 2;
    hipLaunchKernelGGL((k_hist_init<LAT>), dim3(blocks(itf.NH, kIfaceBlock)), dim3(kIfaceBlock), 0, stream,
                       tmp_rho.as<double>(), tmp_u.as<double>(), hist[0].as<double>(), hist[1].as<double>(),
                       hist[2].as<double>(), g, itf);
  }

  void set_state(int level, const double* rho, const double* u, bool dev) override {
    HIPCHK(hipSetDevice(device));
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
    ensure_tmp_f(N);
    const S* src = level == 0 ? cur_c() : fineA();
    hipLaunchKernelGGL((k_pops_out<LAT, DEV, S>), dim3(blocks(Q * N, 256)), dim3(256), 0, stream, src,
                       tmp_f.as<double>(), g, level);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(f, tmp_f.p, sizeof(double) * Q * N, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          stream));
    HIPCHK(hipStreamSynchronize(stream));
  }

  void totals(double* mass, double* mom) override {
    HIPCHK(hipSetDevice(device));
    for (int lv = 0; lv < 2; ++lv) {
      mass[lv] = 0.0;
      for (int d = 0; d < 3; ++d) mom[3 * lv + d] = 0.0;
      if (lv == 1 && !g.has_fine) continue;
      const int64_t N = nodes(lv);
      const unsigned nb = blocks(N, 256);
      const S* src = lv == 0 ? cur_c() : fineA();
      hipLaunchKernelGGL((k_totals<LAT, DEV, S>), dim3(nb), dim3(256), 0, stream, src, part.as<double>(), g, lv);
      hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(256), 0, stream, part.as<double>(), (int64_t)nb,
                         tot.as<double>());
      HIPCHK(hipGetLastError());
      double h[4];
      HIPCHK(hipMemcpyAsync(h, tot.p, sizeof(h), hipMemcpyDeviceToHost, stream));
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
  return g;
}

}  // namespace lbm

using namespace lbm;

struct lbm_grid {
  std::unique_ptr<GridBase> impl;
};

template <typename F>
static int guard(lbm_handle h, F&& fn) {
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

int lbm_destroy(lbm_handle h) {
  if (!h) return LBM_EINVAL;
  (void)hipSetDevice(h->impl->device);
  (void)hipStreamSynchronize(h->impl->stream);
  delete h;
  return LBM_OK;
}

static bool bad_level(lbm_handle h, int level) {
  return !h || level < 0 || level > 1 || (level == 1 && !h->impl->g.has_fine);
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

int lbm_get_index_maps(lbm_handle h, int level, uint8_t* cls, int mem) {
  if (bad_level(h, level) || !cls || (mem != LBM_HOST && mem != LBM_DEVICE)) return LBM_EINVAL;
  return guard(h, [&] {
    const auto& v = level == 0 ? h->impl->tabs.cls_c : h->impl->tabs.cls_f;
    if (mem == LBM_HOST) std::memcpy(cls, v.data(), v.size());
    else HIPCHK(hipMemcpy(cls, v.data(), v.size(), hipMemcpyHostToDevice));
  });
}

int lbm_level_dims(lbm_handle h, int level, int32_t dims[3]) {
  if (bad_level(h, level) || !dims) return LBM_EINVAL;
  for (int k = 0; k < 3; ++k) dims[k] = level == 0 ? h->impl->g.n[k] : h->impl->g.nf[k];
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
    *nodes_per_launch = mid;
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
