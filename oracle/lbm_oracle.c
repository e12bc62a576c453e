/*
 * lbm_oracle.c -- plain, slow, FP64 CPU reference of the two-level lattice
 * Boltzmann scheme analysed by Astoul, Wissocq, Boussuge, Sengissen and
 * Sagaut, "Analysis and reduction of spurious noise generated at grid
 * refinement interfaces with the lattice Boltzmann method" (arXiv:2004.11863).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path: lattice tables, Hermite algebra, node classification, stencils
 * and the time schedule are all written out here independently.
 *
 * Everything is double precision, IEEE round-to-nearest, built without
 * fast-math and with floating-point contraction disabled.  Every loop is a
 * plain loop over nodes; nothing is fused or reordered beyond what the paper
 * states.  OpenMP only splits independent per-node loops across threads and
 * never changes a result (reductions stay sequential).
 *
 * Where the paper is silent or ambiguous the readings below are taken; each
 * one is marked "Reading:" at the place it applies.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXQ 19
#define NFIELD (1 + 3 + MAXQ + 9) /* rho, u[3], f1[Q], S[3][3]            */
#define F_RHO 0
#define F_U 1
#define F_F1 4
#define F_S (4 + MAXQ)

enum { LAT_D2Q9 = 0, LAT_D3Q19 = 1 };
enum { MOD_BGK = 0, MOD_RR = 1, MOD_HRR = 2 };
/* node classes (values are part of the exported interface) */
enum { C_MIDDLE = 0, C_TFC = 1, C_TNC = 2, C_COVERED = 3 };
enum { F_MIDDLE = 0, F_TFF = 1, F_IE = 2, F_IEFACE = 3, F_TNF = 4 };

static const double CS2 = 1.0 / 3.0; /* c_s^2 of both lattices (Sec. 3.1) */

/* Deliberate-mistake switch used ONLY by the test suite to show that the
 * pins detect plausible errors.  0 = the scheme as written. */
static int g_mut = 0;
void orc_set_mutation(int code) { g_mut = code; }
enum {
  MUT_NONE = 0,
  MUT_RESCALE_SWAP = 1,   /* c->f and f->c rescaling factors exchanged        */
  MUT_TEMPORAL_REV = 2,   /* temporal weights applied to reversed time levels */
  MUT_SPATIAL_LIN = 3,    /* linear instead of cubic midpoint interpolation   */
  MUT_FILTER_SWAP = 4,    /* normal and diagonal filter weights exchanged     */
  MUT_FD_SIGN = 5,        /* centred difference with the wrong sign           */
  MUT_NO_THIRD = 6,       /* third-order regularised terms dropped            */
  MUT_SIGMA_SWAP = 7,     /* sigma and 1-sigma exchanged in the hybrid stress */
  MUT_STREAM_PUSH = 8,    /* populations pulled from x+xi instead of x-xi     */
  MUT_SC_HALF = 9,        /* fine strain rate halved instead of doubled       */
  MUT_TAUF = 10,          /* tau_f = 2 tau_c (missing -1/2)                   */
  MUT_FEQ2 = 11,          /* second-order equilibrium (third order dropped)   */
  MUT_NOFILTER = 12,      /* fine->coarse transfer without the filter         */
  MUT_FILTER_ZOFF = 13,   /* 3D filter sampling shifted by one node along z   */
  MUT_FACE_AXES = 14,     /* face-centre stencil built with its axes swapped  */
  MUT_NEST_SYNC = 15,     /* nested: second child step from the state at t    */
  MUT_NEST_RING = 16,     /* nested: no ring rebuilt at t+1/2 for the child   */
  MUT_NEST_INJ = 17       /* nested H-RR: child without the ring's rho, u     */
};

/* ------------------------------------------------------------------------ */
/* Lattices: D2Q9 velocities and weights as printed in Sec. 3.1 (eqs xi_i,
 * w_i); D3Q19 is the standard 19-velocity lattice (the paper only names it,
 * Sec. 10), in the order fixed below.                                      */
typedef struct {
  int D, Q;
  int xi[MAXQ][3];
  double w[MAXQ];
  int nP;            /* number of third-order basis polynomials            */
  int Pn[6];         /* number of canonical components in basis P          */
  int Pc[6][2][3];   /* canonical component index triples                  */
  double Ps[6][2];   /* their signs                                        */
  double PN[6];      /* lattice norm sum_i w_i P_i^2                       */
  double H2[MAXQ][3][3]; /* H^(2) evaluated at each velocity (tabulated once) */
  double PV[MAXQ][6];    /* basis polynomials evaluated at each velocity     */
} lattice_t;

static double herm2(const int* xi, int a, int b) {
  return (double)(xi[a] * xi[b]) - (a == b ? CS2 : 0.0);
}
static double herm3(const int* xi, int a, int b, int c) {
  double v = (double)(xi[a] * xi[b] * xi[c]);
  if (b == c) v -= CS2 * xi[a];
  if (a == c) v -= CS2 * xi[b];
  if (a == b) v -= CS2 * xi[c];
  return v;
}
static double basisP(const lattice_t* L, int p, const int* xi) {
  double v = 0.0;
  for (int k = 0; k < L->Pn[p]; ++k)
    v += L->Ps[p][k] * herm3(xi, L->Pc[p][k][0], L->Pc[p][k][1], L->Pc[p][k][2]);
  return v;
}

static void lattice_init(int lat, lattice_t* L) {
  memset(L, 0, sizeof(*L));
  if (lat == LAT_D2Q9) {
    static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    L->D = 2;
    L->Q = 9;
    for (int i = 0; i < 9; ++i) {
      L->xi[i][0] = ex[i];
      L->xi[i][1] = ey[i];
      L->xi[i][2] = 0;
      L->w[i] = (i == 0) ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    /* third-order Hermite terms present in eq f1RR: H_xxy and H_xyy */
    L->nP = 2;
    L->Pn[0] = 1; L->Pc[0][0][0] = 0; L->Pc[0][0][1] = 0; L->Pc[0][0][2] = 1; L->Ps[0][0] = 1;
    L->Pn[1] = 1; L->Pc[1][0][0] = 0; L->Pc[1][0][1] = 1; L->Pc[1][0][2] = 1; L->Ps[1][0] = 1;
  } else {
    static const int v[19][3] = {
        {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
        {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
        {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    L->D = 3;
    L->Q = 19;
    for (int i = 0; i < 19; ++i) {
      for (int d = 0; d < 3; ++d) L->xi[i][d] = v[i][d];
      L->w[i] = (i == 0) ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    /* Reading: D3Q19 cannot separate H_xxy from H_yzz (and the two other
     * pairs); the third order is carried by their sums and differences,
     * which are orthogonal in the lattice inner product. */
    static const int pairs[3][2][3] = {{{0, 0, 1}, {1, 2, 2}},  /* xxy, yzz */
                                       {{0, 2, 2}, {0, 1, 1}},  /* xzz, xyy */
                                       {{1, 1, 2}, {0, 0, 2}}}; /* yyz, xxz */
    L->nP = 6;
    for (int p = 0; p < 6; ++p) {
      int pr = p % 3;
      L->Pn[p] = 2;
      for (int k = 0; k < 2; ++k)
        for (int d = 0; d < 3; ++d) L->Pc[p][k][d] = pairs[pr][k][d];
      L->Ps[p][0] = 1.0;
      L->Ps[p][1] = (p < 3) ? 1.0 : -1.0;
    }
  }
  for (int p = 0; p < L->nP; ++p) {
    double s = 0.0;
    for (int i = 0; i < L->Q; ++i) {
      double P = basisP(L, p, L->xi[i]);
      s += L->w[i] * P * P;
    }
    L->PN[p] = s;
  }
  for (int i = 0; i < L->Q; ++i) {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) L->H2[i][a][b] = herm2(L->xi[i], a, b);
    for (int p = 0; p < L->nP; ++p) L->PV[i][p] = basisP(L, p, L->xi[i]);
  }
}

int orc_lattice_info(int lat, int* D, int* Q, int* xi, double* w) {
  lattice_t L;
  if (lat != LAT_D2Q9 && lat != LAT_D3Q19) return -1;
  lattice_init(lat, &L);
  *D = L.D;
  *Q = L.Q;
  for (int i = 0; i < L.Q; ++i) {
    for (int d = 0; d < 3; ++d) xi[3 * i + d] = L.xi[i][d];
    w[i] = L.w[i];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Hermite equilibrium truncated at third order, eq fEqH with the moments
 * a0^(n) = rho u^n.  The second order is contracted over the full tensor
 * (xy counted twice), the third order over the basis polynomials P with the
 * lattice norm, which reproduces eq fEqO3 on D2Q9.                         */
static void feq_L(const lattice_t* L, double rho, const double* u, double* out) {
  const int D = L->D;
  double a2[3][3], a3[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      a2[a][b] = rho * u[a] * u[b];
      for (int c = 0; c < 3; ++c) a3[a][b][c] = rho * u[a] * u[b] * u[c];
    }
  for (int i = 0; i < L->Q; ++i) {
    const int* xi = L->xi[i];
    double t1 = 0.0, t2 = 0.0, t3 = 0.0;
    for (int a = 0; a < D; ++a) t1 += xi[a] * rho * u[a];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) t2 += L->H2[i][a][b] * a2[a][b];
    if (g_mut != MUT_FEQ2) {
      for (int p = 0; p < L->nP; ++p) {
        double aP = 0.0;
        for (int k = 0; k < L->Pn[p]; ++k)
          aP += L->Ps[p][k] * a3[L->Pc[p][k][0]][L->Pc[p][k][1]][L->Pc[p][k][2]];
        t3 += L->PV[i][p] * aP / L->PN[p];
      }
    }
    out[i] = L->w[i] * (rho + t1 / CS2 + t2 / (2.0 * CS2 * CS2) + t3);
  }
}

int orc_feq(int lat, double rho, const double* u, double* out) {
  lattice_t L;
  lattice_init(lat, &L);
  feq_L(&L, rho, u, out);
  return 0;
}

/* eqs moment_rho and moment_rhoU, summed in ascending population order */
static void moments_L(const lattice_t* L, const double* f, long stride, double* rho, double* u) {
  double r = 0.0, m[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < L->Q; ++i) {
    double fi = f[i * stride];
    r += fi;
    for (int d = 0; d < 3; ++d) m[d] += L->xi[i][d] * fi;
  }
  *rho = r;
  for (int d = 0; d < 3; ++d) u[d] = m[d] / r;
}

/* ------------------------------------------------------------------------ */
/* Collision, one node.  f: pre-collision populations (contiguous), S: the
 * strain rate used by H-RR (3x3, row-major), tau: the level's relaxation
 * time.  BGK: eq BGKmodel written as f0 + (1-1/tau)(f-f0).  RR: eqs a1Proj,
 * f1RR, a13RR and LBMscheme_reg.  H-RR: eq a1ij_HRR, then the RR recursion.
 * Reading: the third-order coefficients for D3Q19 follow the same recursion
 * a1_abg = u_a a1_bg + u_b a1_ag + u_g a1_ab, which is eq a13RR in 2D.     */
static void collide_L(const lattice_t* L, int model, double tau, double sigma, const double* f,
                      long stride, const double* S, double* out, long ostride) {
  const int D = L->D, Q = L->Q;
  double rho, u[3], f0[MAXQ], f1[MAXQ];
  double fl[MAXQ];
  for (int i = 0; i < Q; ++i) fl[i] = f[i * stride];
  moments_L(L, fl, 1, &rho, u);
  feq_L(L, rho, u, f0);
  for (int i = 0; i < Q; ++i) f1[i] = fl[i] - f0[i];
  const double om = 1.0 - 1.0 / tau;
  if (model == MOD_BGK) {
    for (int i = 0; i < Q; ++i) out[i * ostride] = f0[i] + om * f1[i];
    return;
  }
  double a2[3][3] = {{0}};
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      double s = 0.0;
      for (int i = 0; i < Q; ++i) s += L->H2[i][a][b] * f1[i];
      a2[a][b] = s;
    }
  if (model == MOD_HRR) {
    double sg = sigma, osg = 1.0 - sigma;
    if (g_mut == MUT_SIGMA_SWAP) { sg = 1.0 - sigma; osg = sigma; }
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        a2[a][b] = sg * a2[a][b] + osg * (-2.0 * tau * rho * CS2 * S[3 * a + b]);
  }
  double a3[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) a3[a][b][c] = u[a] * a2[b][c] + u[b] * a2[a][c] + u[c] * a2[a][b];
  for (int i = 0; i < Q; ++i) {
    double t2 = 0.0, t3 = 0.0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) t2 += L->H2[i][a][b] * a2[a][b];
    if (g_mut != MUT_NO_THIRD) {
      for (int p = 0; p < L->nP; ++p) {
        double aP = 0.0;
        for (int k = 0; k < L->Pn[p]; ++k)
          aP += L->Ps[p][k] * a3[L->Pc[p][k][0]][L->Pc[p][k][1]][L->Pc[p][k][2]];
        t3 += L->PV[i][p] * aP / L->PN[p];
      }
    }
    double f1rr = L->w[i] * (t2 / (2.0 * CS2 * CS2) + t3);
    out[i * ostride] = f0[i] + om * f1rr;
  }
}

int orc_collide(int lat, int model, double tau, double sigma, const double* f, const double* S,
                double* out) {
  lattice_t L;
  double Sz[9] = {0};
  lattice_init(lat, &L);
  collide_L(&L, model, tau, sigma, f, 1, S ? S : Sz, out, 1);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Interface primitives.                                                    */

/* eq rescTau */
double orc_tau_fine(double tau_c) {
  if (g_mut == MUT_TAUF) return 2.0 * tau_c;
  return 2.0 * tau_c - 0.5;
}
/* eq rescff: factor applied to a coarse non-equilibrium part on the fine grid */
double orc_rescale_c2f(double tau_c, double tau_f) {
  if (g_mut == MUT_RESCALE_SWAP) return 2.0 * tau_c / tau_f;
  return tau_f / (2.0 * tau_c);
}
/* eq rescfc: factor applied to a filtered fine non-equilibrium part */
double orc_rescale_f2c(double tau_c, double tau_f) {
  if (g_mut == MUT_RESCALE_SWAP) return tau_f / (2.0 * tau_c);
  return 2.0 * tau_c / tau_f;
}
/* eq PijResc: S^c = 2 S^f */
double orc_strain_f2c(void) { return g_mut == MUT_SC_HALF ? 0.5 : 2.0; }

/* eq TempInt.  Reading: the printed time levels (t-1/2, t, t+1) cannot go
 * with the printed weights; the weights are those of the quadratic through
 * t-1, t and t+1 evaluated at t+1/2, so the first level is read as t-1.
 * c[0], c[1], c[2] weight the values at t-1, t, t+1. */
void orc_temporal_weights(int half, double* c) {
  if (half) {
    c[0] = -1.0 / 8.0;
    c[1] = 3.0 / 4.0;
    c[2] = 3.0 / 8.0;
    if (g_mut == MUT_TEMPORAL_REV) { c[0] = 3.0 / 8.0; c[2] = -1.0 / 8.0; }
  } else {
    c[0] = 0.0;
    c[1] = 0.0;
    c[2] = 1.0;
  }
}
double orc_temporal_interp(double gm1, double g0, double gp1) {
  double c[3];
  orc_temporal_weights(1, c);
  return c[0] * gm1 + c[1] * g0 + c[2] * gp1;
}
/* eq spaceInt: weights of the values at -3/2, -1/2, +1/2, +3/2 */
void orc_cubic_weights(double* w) {
  if (g_mut == MUT_SPATIAL_LIN) {
    w[0] = 0.0; w[1] = 0.5; w[2] = 0.5; w[3] = 0.0;
    return;
  }
  w[0] = -1.0 / 16.0;
  w[1] = 9.0 / 16.0;
  w[2] = 9.0 / 16.0;
  w[3] = -1.0 / 16.0;
}
double orc_cubic_mid(const double* g) {
  double w[4];
  orc_cubic_weights(w);
  return w[0] * g[0] + w[1] * g[1] + w[2] * g[2] + w[3] * g[3];
}
/* eq filterFneq: 1/4 centre, 1/8 for the four normal neighbours, 1/16 for
 * the four diagonal ones.  Reading: in 3D the same filter is the product
 * of the 1D weights (1/4, 1/2, 1/4) along each axis, as eq filterFneq is in
 * 2D.  Offsets o in {-1,0,1}^D, listed with o[0] fastest. */
double orc_filter_weight(int D, const int* o) {
  int nz = 0;
  for (int d = 0; d < D; ++d) nz += (o[d] != 0);
  if (g_mut == MUT_NOFILTER) return nz == 0 ? 1.0 : 0.0;
  if (D == 2) {
    if (nz == 0) return 1.0 / 4.0;
    if (nz == 1) return g_mut == MUT_FILTER_SWAP ? 1.0 / 16.0 : 1.0 / 8.0;
    return g_mut == MUT_FILTER_SWAP ? 1.0 / 8.0 : 1.0 / 16.0;
  }
  double w = 1.0;
  for (int d = 0; d < D; ++d) w *= (o[d] == 0) ? 0.5 : 0.25;
  if (g_mut == MUT_FILTER_SWAP && nz == 1) w = 1.0 / 64.0;
  if (g_mut == MUT_FILTER_SWAP && nz == 3) w = 1.0 / 16.0;
  return w;
}

/* ------------------------------------------------------------------------ */
/* Grid state.                                                              */
typedef struct ogrid_s {
  lattice_t L;
  int lat, model, D, Q;
  int n[3], a[3], m[3], nf[3];
  int has_fine;
  long Nc, Nf;
  double tau_c, tau_f, sigma;
  double *fc, *ff;          /* post-collision populations [Q][N]            */
  double *fc_pre, *ff_pre;  /* pre-collision (post-stream) populations      */
  double *ff_half;          /* fine post-collision populations at t+1/2     */
  double *rho_c, *u_c, *rho_f, *u_f; /* u: [3][N]                          */
  double *S_tn;             /* strain rate handed to TN^c nodes [NT][9]     */
  uint8_t *cls_c, *cls_f;
  long NH;
  long* hnode;              /* coarse node of each history entry            */
  double* hist[3];          /* [NFIELD][NH] per time level                  */
  int hs[3];                /* hist buffers holding t-1, t, t+1             */
  long NR;
  long* rnode;              /* fine ring nodes                              */
  int* rnp;                 /* stencil size (1, 4 or 16)                    */
  long* rpt;                /* [NR][16] history entries                     */
  double* rw;               /* [NR][16] spatial weights                     */
  double *r_rho, *r_u, *r_f, *r_S; /* ring scratch                         */
  long NT;
  long *tn_f, *tn_c;
  long steps;
  /* NH sensors (Sec. 7): velocities of the iteration before the last one
   * of each level (coarse: t, fine: t+1/2, for a step t -> t+1) */
  double *u_c_prev, *u_f_prev;
  /* Dynamic sigma (H-RR, suggested in Sec. 9.3 and Sec. 11): on/off, the
   * sigma taken where a node's sensors fire, and per node the divergence and
   * curl of the velocity gradient of its previous bulk collision [4][N]. */
  int dyn;
  double sigma_dyn, dyn_thr;
  double *dyn_c, *dyn_f;
  uint8_t *dyn_mask_c, *dyn_mask_f; /* 1 where the last collision took sigma_dyn */
  /* Nested refinement: the fine level carries a patch of its own.  child is
   * a two-level grid whose coarse level is this grid's fine level (same
   * nodes, same order; its periodic wrap only reaches the fine ring, which
   * this grid rebuilds), evolved by child steps in place of the fine
   * substeps. */
  struct ogrid_s* child;
  /* Set on a child: rho and u of the parent's fine ring at the time of the
   * child's step (n_inj nodes of this grid's coarse level), written over the
   * values its periodic propagation leaves there. */
  const long* inj_node;
  const double *inj_rho, *inj_u;
  long n_inj;
} ogrid;

static long cidx(const ogrid* g, int x, int y, int z) {
  x = ((x % g->n[0]) + g->n[0]) % g->n[0];
  y = ((y % g->n[1]) + g->n[1]) % g->n[1];
  z = ((z % g->n[2]) + g->n[2]) % g->n[2];
  return (long)x + (long)g->n[0] * ((long)y + (long)g->n[1] * z);
}
static long fidx(const ogrid* g, int x, int y, int z) {
  return (long)x + (long)g->nf[0] * ((long)y + (long)g->nf[1] * z);
}
static void cco(const ogrid* g, long i, int* c) {
  c[0] = (int)(i % g->n[0]);
  c[1] = (int)((i / g->n[0]) % g->n[1]);
  c[2] = (int)(i / ((long)g->n[0] * g->n[1]));
}
static void fco(const ogrid* g, long i, int* c) {
  c[0] = (int)(i % g->nf[0]);
  c[1] = (int)((i / g->nf[0]) % g->nf[1]);
  c[2] = (int)(i / ((long)g->nf[0] * g->nf[1]));
}

/* Node classes of the one-coarse-cell overlap of Fig. Overlap.  Reading: the
 * fine patch is the coarse vertex box [a, a+m]^D; fine node j sits at coarse
 * coordinate a + j/2.  Fine ring (j = 0 or 2m on some axis): TF^f where all
 * coordinates are coarse vertices, IE elsewhere (IEFACE when two coordinates
 * are half-integers, i.e. a 3D face centre).  TN^c / TN^f: vertices on the
 * boundary of [a+1, a+m-1]^D.  Covered coarse nodes: the interior of that
 * box.  TF^c: coarse vertices on the boundary of [a, a+m]^D.  */
static int coarse_class(const ogrid* g, const int* x) {
  if (!g->has_fine) return C_MIDDLE;
  int inTN = 1, onTN = 0, inTF = 1, onTF = 0;
  for (int d = 0; d < g->D; ++d) {
    int lo = g->a[d], hi = g->a[d] + g->m[d];
    if (x[d] < lo + 1 || x[d] > hi - 1) inTN = 0;
    if (x[d] == lo + 1 || x[d] == hi - 1) onTN = 1;
    if (x[d] < lo || x[d] > hi) inTF = 0;
    if (x[d] == lo || x[d] == hi) onTF = 1;
  }
  if (inTN) return onTN ? C_TNC : C_COVERED;
  if (inTF && onTF) return C_TFC;
  return C_MIDDLE;
}
static int fine_class(const ogrid* g, const int* j) {
  int ring = 0, nodd = 0, even = 1, inTN = 1, onTN = 0;
  for (int d = 0; d < g->D; ++d) {
    int M = 2 * g->m[d];
    if (j[d] == 0 || j[d] == M) ring = 1;
    if (j[d] & 1) { nodd++; even = 0; }
    if (j[d] < 2 || j[d] > M - 2) inTN = 0;
    if (j[d] == 2 || j[d] == M - 2) onTN = 1;
  }
  if (ring) return nodd == 0 ? F_TFF : (nodd == 1 ? F_IE : F_IEFACE);
  if (even && inTN && onTN) return F_TNF;
  return F_MIDDLE;
}

void orc_destroy(void* hp) {
  ogrid* g = (ogrid*)hp;
  if (!g) return;
  free(g->fc); free(g->ff); free(g->fc_pre); free(g->ff_pre); free(g->ff_half);
  free(g->rho_c); free(g->u_c); free(g->rho_f); free(g->u_f); free(g->S_tn);
  free(g->cls_c); free(g->cls_f); free(g->hnode);
  for (int s = 0; s < 3; ++s) free(g->hist[s]);
  free(g->rnode); free(g->rnp); free(g->rpt); free(g->rw);
  free(g->r_rho); free(g->r_u); free(g->r_f); free(g->r_S);
  free(g->tn_f); free(g->tn_c);
  free(g->u_c_prev); free(g->u_f_prev);
  free(g->dyn_c); free(g->dyn_f); free(g->dyn_mask_c); free(g->dyn_mask_f);
  if (g->child) orc_destroy(g->child);
  free(g);
}

/* lattice: 0 D2Q9, 1 D3Q19; model: 0 BGK, 1 RR, 2 H-RR; n: coarse nodes per
 * axis; lo/hi: patch box in coarse vertices (hi == lo on every axis: single
 * uniform level).  Returns NULL on invalid input. */
void* orc_create(int lat, int model, const int* n, const int* lo, const int* hi, double tau_c,
                 double sigma) {
  if (lat != LAT_D2Q9 && lat != LAT_D3Q19) return NULL;
  if (model < 0 || model > 2 || !(tau_c > 0.5)) return NULL;
  ogrid* g = (ogrid*)calloc(1, sizeof(ogrid));
  lattice_init(lat, &g->L);
  g->lat = lat;
  g->model = model;
  g->D = g->L.D;
  g->Q = g->L.Q;
  g->tau_c = tau_c;
  g->tau_f = orc_tau_fine(tau_c);
  g->sigma = sigma;
  g->has_fine = 0;
  for (int d = 0; d < 3; ++d) {
    g->n[d] = (d < g->D) ? n[d] : 1;
    if (g->n[d] < 1) { orc_destroy(g); return NULL; }
    g->a[d] = 0; g->m[d] = 0; g->nf[d] = 1;
  }
  for (int d = 0; d < g->D; ++d)
    if (hi[d] != lo[d]) g->has_fine = 1;
  if (g->has_fine) {
    for (int d = 0; d < g->D; ++d) {
      g->a[d] = lo[d];
      g->m[d] = hi[d] - lo[d];
      if (g->m[d] < 4 || lo[d] < 2 || hi[d] > g->n[d] - 3) { orc_destroy(g); return NULL; }
      g->nf[d] = 2 * g->m[d] + 1;
    }
  }
  const int Q = g->Q;
  g->Nc = (long)g->n[0] * g->n[1] * g->n[2];
  g->Nf = g->has_fine ? (long)g->nf[0] * g->nf[1] * g->nf[2] : 0;
  g->fc = calloc((size_t)Q * g->Nc, sizeof(double));
  g->fc_pre = calloc((size_t)Q * g->Nc, sizeof(double));
  g->rho_c = calloc((size_t)g->Nc, sizeof(double));
  g->u_c = calloc((size_t)3 * g->Nc, sizeof(double));
  g->u_c_prev = calloc((size_t)3 * g->Nc, sizeof(double));
  g->dyn_c = calloc((size_t)4 * g->Nc, sizeof(double));
  g->dyn_mask_c = calloc((size_t)g->Nc, 1);
  g->cls_c = calloc((size_t)g->Nc, 1);
  for (long i = 0; i < g->Nc; ++i) {
    int c[3];
    cco(g, i, c);
    g->cls_c[i] = (uint8_t)coarse_class(g, c);
  }
  if (!g->has_fine) return g;

  g->ff = calloc((size_t)Q * g->Nf, sizeof(double));
  g->ff_pre = calloc((size_t)Q * g->Nf, sizeof(double));
  g->ff_half = calloc((size_t)Q * g->Nf, sizeof(double));
  g->rho_f = calloc((size_t)g->Nf, sizeof(double));
  g->u_f = calloc((size_t)3 * g->Nf, sizeof(double));
  g->u_f_prev = calloc((size_t)3 * g->Nf, sizeof(double));
  g->dyn_f = calloc((size_t)4 * g->Nf, sizeof(double));
  g->dyn_mask_f = calloc((size_t)g->Nf, 1);
  g->cls_f = calloc((size_t)g->Nf, 1);
  for (long i = 0; i < g->Nf; ++i) {
    int j[3];
    fco(g, i, j);
    g->cls_f[i] = (uint8_t)fine_class(g, j);
  }
  /* History nodes: every coarse vertex lying on a face plane of the patch
   * box and inside [a-1, a+m+1]^D.  These are TF^c plus the coarse nodes
   * one step beyond the box along each face, which the cubic stencils of
   * ring nodes next to an edge or corner reach (Reading: the interpolation
   * runs along the ring line/plane through coarse nodes that exist beyond
   * the patch, so no one-sided stencil is needed). */
  long cap = 0;
  for (long i = 0; i < g->Nc; ++i) {
    int c[3];
    cco(g, i, c);
    int inb = 1, onp = 0;
    for (int d = 0; d < g->D; ++d) {
      if (c[d] < g->a[d] - 1 || c[d] > g->a[d] + g->m[d] + 1) inb = 0;
      if (c[d] == g->a[d] || c[d] == g->a[d] + g->m[d]) onp = 1;
    }
    if (inb && onp) cap++;
  }
  g->NH = cap;
  g->hnode = malloc(sizeof(long) * (size_t)cap);
  long* hof = malloc(sizeof(long) * (size_t)g->Nc);
  long k = 0;
  for (long i = 0; i < g->Nc; ++i) {
    int c[3];
    cco(g, i, c);
    int inb = 1, onp = 0;
    for (int d = 0; d < g->D; ++d) {
      if (c[d] < g->a[d] - 1 || c[d] > g->a[d] + g->m[d] + 1) inb = 0;
      if (c[d] == g->a[d] || c[d] == g->a[d] + g->m[d]) onp = 1;
    }
    hof[i] = -1;
    if (inb && onp) { g->hnode[k] = i; hof[i] = k; k++; }
  }
  for (int s = 0; s < 3; ++s) g->hist[s] = calloc((size_t)NFIELD * g->NH, sizeof(double));
  g->hs[0] = 0; g->hs[1] = 1; g->hs[2] = 2;

  /* ring stencils */
  long nr = 0;
  for (long i = 0; i < g->Nf; ++i)
    if (g->cls_f[i] >= F_TFF && g->cls_f[i] <= F_IEFACE) nr++;
  g->NR = nr;
  g->rnode = malloc(sizeof(long) * (size_t)nr);
  g->rnp = malloc(sizeof(int) * (size_t)nr);
  g->rpt = malloc(sizeof(long) * 16 * (size_t)nr);
  g->rw = malloc(sizeof(double) * 16 * (size_t)nr);
  g->r_rho = malloc(sizeof(double) * (size_t)nr);
  g->r_u = malloc(sizeof(double) * 3 * (size_t)nr);
  g->r_f = malloc(sizeof(double) * MAXQ * (size_t)nr);
  g->r_S = malloc(sizeof(double) * 9 * (size_t)nr);
  double cw[4];
  orc_cubic_weights(cw);
  long r = 0;
  for (long i = 0; i < g->Nf; ++i) {
    int cl = g->cls_f[i];
    if (cl < F_TFF || cl > F_IEFACE) continue;
    int j[3];
    fco(g, i, j);
    int oddax[2], no = 0;
    int base[3];
    for (int d = 0; d < 3; ++d) {
      if (d < g->D && (j[d] & 1)) { oddax[no++] = d; base[d] = 0; }
      else base[d] = (d < g->D) ? g->a[d] + j[d] / 2 : 0;
    }
    g->rnode[r] = i;
    int np = 0;
    if (no == 0) {
      g->rpt[16 * r] = hof[cidx(g, base[0], base[1], base[2])];
      g->rw[16 * r] = 1.0;
      np = 1;
    } else if (no == 1) {
      int e = oddax[0];
      for (int s = 0; s < 4; ++s) {
        int c[3] = {base[0], base[1], base[2]};
        c[e] = g->a[e] + (j[e] - 3) / 2 + s;
        g->rpt[16 * r + s] = hof[cidx(g, c[0], c[1], c[2])];
        g->rw[16 * r + s] = cw[s];
      }
      np = 4;
    } else {
      int e0 = oddax[0], e1 = oddax[1];
      int j0 = j[e0], j1 = j[e1];
      if (g_mut == MUT_FACE_AXES) { j0 = j[e1]; j1 = j[e0]; }
      for (int s1 = 0; s1 < 4; ++s1)
        for (int s0 = 0; s0 < 4; ++s0) {
          int c[3] = {base[0], base[1], base[2]};
          c[e0] = g->a[e0] + (j0 - 3) / 2 + s0;
          c[e1] = g->a[e1] + (j1 - 3) / 2 + s1;
          g->rpt[16 * r + 4 * s1 + s0] = hof[cidx(g, c[0], c[1], c[2])];
          g->rw[16 * r + 4 * s1 + s0] = cw[s0] * cw[s1];
        }
      np = 16;
    }
    g->rnp[r] = np;
    for (int s = 0; s < np; ++s)
      if (g->rpt[16 * r + s] < 0) { free(hof); orc_destroy(g); return NULL; }
    r++;
  }
  free(hof);
  long nt = 0;
  for (long i = 0; i < g->Nf; ++i) nt += (g->cls_f[i] == F_TNF);
  g->NT = nt;
  g->tn_f = malloc(sizeof(long) * (size_t)nt);
  g->tn_c = malloc(sizeof(long) * (size_t)nt);
  g->S_tn = calloc((size_t)9 * nt, sizeof(double));
  long t = 0;
  for (long i = 0; i < g->Nf; ++i) {
    if (g->cls_f[i] != F_TNF) continue;
    int j[3];
    fco(g, i, j);
    int c[3] = {0, 0, 0};
    for (int d = 0; d < g->D; ++d) c[d] = g->a[d] + j[d] / 2;
    g->tn_f[t] = i;
    g->tn_c[t] = cidx(g, c[0], c[1], c[2]);
    t++;
  }
  return g;
}

/* A grid of three nested levels: the coarse grid and patch of orc_create,
 * and a patch of the fine level given by lo2/hi2 in fine-level vertices
 * (the same rules: at least 4 cells, 2 nodes from the fine ring).  The
 * fine level's pair has tau = 2 tau_f - 1/2 (eq rescTau, applied to each
 * pair).  NULL on invalid input. */
void* orc_create_nested(int lat, int model, const int* n, const int* lo, const int* hi, const int* lo2,
                        const int* hi2, double tau_c, double sigma) {
  ogrid* g = (ogrid*)orc_create(lat, model, n, lo, hi, tau_c, sigma);
  if (!g) return NULL;
  if (!g->has_fine) { orc_destroy(g); return NULL; }
  int any = 0;
  for (int d = 0; d < g->D; ++d) any |= (hi2[d] != lo2[d]);
  ogrid* c = any ? (ogrid*)orc_create(lat, model, g->nf, lo2, hi2, g->tau_f, sigma) : NULL;
  if (!c) { orc_destroy(g); return NULL; }
  g->child = c;
  return g;
}
/* The child pair of a nested grid (its coarse level is the fine level). */
void* orc_child(void* hp) { return ((ogrid*)hp)->child; }

int orc_level_dims(void* hp, int level, int* dims) {
  ogrid* g = (ogrid*)hp;
  for (int d = 0; d < 3; ++d) dims[d] = level == 0 ? g->n[d] : g->nf[d];
  if (level == 1 && !g->has_fine) return -1;
  return 0;
}
int orc_class_map(void* hp, int level, uint8_t* out) {
  ogrid* g = (ogrid*)hp;
  if (level == 0) memcpy(out, g->cls_c, (size_t)g->Nc);
  else if (g->has_fine) memcpy(out, g->cls_f, (size_t)g->Nf);
  else return -1;
  return 0;
}
long orc_count(void* hp, int what) {
  ogrid* g = (ogrid*)hp;
  switch (what) {
    case 0: return g->NH;
    case 1: return g->NR;
    case 2: return g->NT;
    default: return -1;
  }
}
/* history node list and ring stencils, exported for the bit-exact checks */
int orc_history_nodes(void* hp, int64_t* out) {
  ogrid* g = (ogrid*)hp;
  for (long h = 0; h < g->NH; ++h) out[h] = g->hnode[h];
  return 0;
}
int orc_ring_stencils(void* hp, int64_t* node, int32_t* np, int64_t* pts, double* w) {
  ogrid* g = (ogrid*)hp;
  for (long r = 0; r < g->NR; ++r) {
    node[r] = g->rnode[r];
    np[r] = g->rnp[r];
    for (int s = 0; s < 16; ++s) {
      pts[16 * r + s] = s < g->rnp[r] ? g->rpt[16 * r + s] : -1;
      w[16 * r + s] = s < g->rnp[r] ? g->rw[16 * r + s] : 0.0;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Finite differences: second-order centred, in the level's lattice units
 * (Sec. 3.3).  S_ab = (d_a u_b + d_b u_a) / 2.  Reading: the full symmetric
 * strain rate (trace included) is used, as in Appendix A.                 */
static void strain_from(int D, const double up[3][3], const double um[3][3], double* S, double gout[3][3]) {
  /* up[a][b]: u_b at x + e_a;  um[a][b]: u_b at x - e_a */
  double gr[3][3] = {{0}};
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      gr[a][b] = (up[a][b] - um[a][b]) / 2.0;
      if (g_mut == MUT_FD_SIGN) gr[a][b] = -gr[a][b];
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) S[3 * a + b] = (a < D && b < D) ? 0.5 * (gr[a][b] + gr[b][a]) : 0.0;
  if (gout)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) gout[a][b] = gr[a][b];
}
static void strain_coarse_g(const ogrid* g, long i, double* S, double gout[3][3]) {
  int c[3];
  double up[3][3], um[3][3];
  cco(g, i, c);
  for (int a = 0; a < g->D; ++a) {
    int p[3] = {c[0], c[1], c[2]}, q[3] = {c[0], c[1], c[2]};
    p[a]++;
    q[a]--;
    long ip = cidx(g, p[0], p[1], p[2]), iq = cidx(g, q[0], q[1], q[2]);
    for (int b = 0; b < 3; ++b) {
      up[a][b] = g->u_c[b * g->Nc + ip];
      um[a][b] = g->u_c[b * g->Nc + iq];
    }
  }
  strain_from(g->D, up, um, S, gout);
}
static void strain_coarse(const ogrid* g, long i, double* S) { strain_coarse_g(g, i, S, NULL); }
static void strain_fine_g(const ogrid* g, long i, double* S, double gout[3][3]) {
  int j[3];
  double up[3][3], um[3][3];
  fco(g, i, j);
  for (int a = 0; a < g->D; ++a) {
    int p[3] = {j[0], j[1], j[2]}, q[3] = {j[0], j[1], j[2]};
    p[a]++;
    q[a]--;
    long ip = fidx(g, p[0], p[1], p[2]), iq = fidx(g, q[0], q[1], q[2]);
    for (int b = 0; b < 3; ++b) {
      up[a][b] = g->u_f[b * g->Nf + ip];
      um[a][b] = g->u_f[b * g->Nf + iq];
    }
  }
  strain_from(g->D, up, um, S, gout);
}
static void strain_fine(const ogrid* g, long i, double* S) { strain_fine_g(g, i, S, NULL); }

/* Dynamic sigma (an H-RR variant the paper suggests in Sec. 9.3 and Sec. 11
 * without defining it).  Reading: at each bulk H-RR collision of a node, the
 * SpuriousAc and SpuriousS tests of Sec. 7 (eqs sensorSpuriousAc,
 * sensorSpuriousS) compare the divergence and the curl of the velocity
 * gradient this collision uses (gr[a][b] = d_a u_b) with those of the node's
 * previous bulk collision on its level (zero before the first); a product
 * below -thr (3D curl: dot product; thr = 0 is the paper's tie-break, a
 * small thr keeps products of rounding noise from switching) takes
 * sigma_dyn, otherwise the grid's sigma.  The new divergence and curl
 * replace the stored ones.  Interface collisions (ring nodes, TN^c) keep the
 * grid's sigma. */
static double dyn_sigma(const ogrid* g, double* prev, uint8_t* mask, long N, long i, const double gr[3][3]) {
  double dv = 0.0, c[3] = {0.0, 0.0, 0.0};
  int nc = 1;
  for (int a = 0; a < g->D; ++a) dv += gr[a][a];
  if (g->D == 2) {
    c[0] = gr[0][1] - gr[1][0];
  } else {
    c[0] = gr[1][2] - gr[2][1];
    c[1] = gr[2][0] - gr[0][2];
    c[2] = gr[0][1] - gr[1][0];
    nc = 3;
  }
  const double pd = prev[i] * dv;
  double pc = 0.0;
  for (int k = 0; k < nc; ++k) pc += prev[(1 + k) * N + i] * c[k];
  prev[i] = dv;
  for (int k = 0; k < nc; ++k) prev[(1 + k) * N + i] = c[k];
  mask[i] = (uint8_t)(pd < -g->dyn_thr || pc < -g->dyn_thr);
  return mask[i] ? g->sigma_dyn : g->sigma;
}

/* Switches dynamic sigma on (with the sigma taken where the sensors fire and
 * the threshold of the products) or off; switching on forgets the stored
 * divergences and curls.  Returns -1 for a model other than H-RR, sigma_dyn
 * outside [0, 1] or a negative threshold. */
int orc_set_dynamic_sigma(void* hp, int on, double sigma_dyn, double thr) {
  ogrid* g = (ogrid*)hp;
  if (on && (g->model != MOD_HRR || !(sigma_dyn >= 0.0 && sigma_dyn <= 1.0) || !(thr >= 0.0))) return -1;
  g->dyn = on ? 1 : 0;
  g->sigma_dyn = sigma_dyn;
  g->dyn_thr = thr;
  memset(g->dyn_c, 0, sizeof(double) * 4 * (size_t)g->Nc);
  memset(g->dyn_mask_c, 0, (size_t)g->Nc);
  if (g->has_fine) {
    memset(g->dyn_f, 0, sizeof(double) * 4 * (size_t)g->Nf);
    memset(g->dyn_mask_f, 0, (size_t)g->Nf);
  }
  return 0;
}

/* Which nodes of a level took sigma_dyn in their last bulk collision. */
int orc_dynamic_mask(void* hp, int level, uint8_t* out) {
  ogrid* g = (ogrid*)hp;
  if (level == 1 && !g->has_fine) return -1;
  memcpy(out, level == 0 ? g->dyn_mask_c : g->dyn_mask_f, (size_t)(level == 0 ? g->Nc : g->Nf));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* State setting.                                                           */

/* History at t=0.  Reading: the state given at t=0 is an equilibrium state
 * with known (rho, u); the pre-collision non-equilibrium part is taken as
 * zero and S as the centred difference of the given u.  Both missing time
 * levels t-1 and t are filled with these values. */
static void init_history(ogrid* g) {
  if (!g->has_fine) return;
  for (int s = 0; s < 3; ++s) {
    double* H = g->hist[s];
    for (long h = 0; h < g->NH; ++h) {
      long i = g->hnode[h];
      H[F_RHO * g->NH + h] = g->rho_c[i];
      for (int d = 0; d < 3; ++d) H[(F_U + d) * g->NH + h] = g->u_c[d * g->Nc + i];
      for (int q = 0; q < MAXQ; ++q) H[(F_F1 + q) * g->NH + h] = 0.0;
      double S[9];
      strain_coarse(g, i, S);
      for (int k = 0; k < 9; ++k) H[(F_S + k) * g->NH + h] = S[k];
    }
  }
  g->hs[0] = 0; g->hs[1] = 1; g->hs[2] = 2;
}

/* Sets the post-collision state of a level to f = f0(rho, u) (Reading: the
 * step starts with propagation, and "all distribution functions known" at
 * the reference state means equilibrium populations of the given fields).
 * rho[N], u[D][N], x fastest. */
int orc_set_state(void* hp, int level, const double* rho, const double* u) {
  ogrid* g = (ogrid*)hp;
  if (level == 1 && !g->has_fine) return -1;
  long N = level == 0 ? g->Nc : g->Nf;
  double* f = level == 0 ? g->fc : g->ff;
  double* R = level == 0 ? g->rho_c : g->rho_f;
  double* U = level == 0 ? g->u_c : g->u_f;
  for (long i = 0; i < N; ++i) {
    double uu[3] = {0, 0, 0}, fe[MAXQ];
    for (int d = 0; d < g->D; ++d) uu[d] = u[d * N + i];
    feq_L(&g->L, rho[i], uu, fe);
    for (int q = 0; q < g->Q; ++q) f[q * N + i] = fe[q];
    R[i] = rho[i];
    for (int d = 0; d < 3; ++d) U[d * N + i] = uu[d];
  }
  if (level == 0) init_history(g);
  g->steps = 0;
  return 0;
}

/* Sets post-collision populations directly, f[Q][N].  On the coarse level
 * the history is re-initialised from their moments as in init_history. */
int orc_set_populations(void* hp, int level, const double* f) {
  ogrid* g = (ogrid*)hp;
  if (level == 1 && !g->has_fine) return -1;
  long N = level == 0 ? g->Nc : g->Nf;
  double* F = level == 0 ? g->fc : g->ff;
  memcpy(F, f, sizeof(double) * (size_t)g->Q * N);
  double* R = level == 0 ? g->rho_c : g->rho_f;
  double* U = level == 0 ? g->u_c : g->u_f;
  for (long i = 0; i < N; ++i) {
    double r, uu[3];
    moments_L(&g->L, F + i, N, &r, uu);
    R[i] = r;
    for (int d = 0; d < 3; ++d) U[d * N + i] = uu[d];
  }
  if (level == 0) init_history(g);
  return 0;
}
int orc_get_populations(void* hp, int level, double* f) {
  ogrid* g = (ogrid*)hp;
  if (level == 1 && !g->has_fine) return -1;
  long N = level == 0 ? g->Nc : g->Nf;
  memcpy(f, level == 0 ? g->fc : g->ff, sizeof(double) * (size_t)g->Q * N);
  return 0;
}

/* Moments of the current post-collision state.  Covered coarse nodes take
 * the values of the co-located fine node (output only; they do not evolve). */
int orc_get_macros(void* hp, int level, double* rho, double* u) {
  ogrid* g = (ogrid*)hp;
  if (level == 1 && !g->has_fine) return -1;
  long N = level == 0 ? g->Nc : g->Nf;
  const double* F = level == 0 ? g->fc : g->ff;
  for (long i = 0; i < N; ++i) {
    const double* src = F;
    long ii = i, NN = N;
    if (level == 0 && g->cls_c[i] == C_COVERED) {
      int c[3], j[3] = {0, 0, 0};
      cco(g, i, c);
      for (int d = 0; d < g->D; ++d) j[d] = 2 * (c[d] - g->a[d]);
      ii = fidx(g, j[0], j[1], j[2]);
      src = g->ff;
      NN = g->Nf;
    }
    double r, uu[3];
    moments_L(&g->L, src + ii, NN, &r, uu);
    rho[i] = r;
    for (int d = 0; d < g->D; ++d) u[d * N + i] = uu[d];
  }
  return 0;
}

/* Sums of rho and rho u over the evolving nodes of each level (coarse:
 * every node but the covered ones; fine: every node), in node order. */
int orc_totals(void* hp, double* mass, double* mom) {
  ogrid* g = (ogrid*)hp;
  for (int lv = 0; lv < 2; ++lv) {
    mass[lv] = 0.0;
    for (int d = 0; d < 3; ++d) mom[3 * lv + d] = 0.0;
    if (lv == 1 && !g->has_fine) continue;
    long N = lv == 0 ? g->Nc : g->Nf;
    const double* F = lv == 0 ? g->fc : g->ff;
    for (long i = 0; i < N; ++i) {
      if (lv == 0 && g->cls_c[i] == C_COVERED) continue;
      for (int q = 0; q < g->Q; ++q) {
        double fi = F[q * N + i];
        mass[lv] += fi;
        for (int d = 0; d < 3; ++d) mom[3 * lv + d] += g->L.xi[q][d] * fi;
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One coarse time step.                                                    */

/* Propagation, eq LBMequation: f_i(x, t+1) = f*_i(x - xi_i, t). */
static void stream_coarse_node(ogrid* g, long i) {
  int c[3];
  cco(g, i, c);
  for (int q = 0; q < g->Q; ++q) {
    int s = (g_mut == MUT_STREAM_PUSH) ? 1 : -1;
    long src = cidx(g, c[0] + s * g->L.xi[q][0], c[1] + s * g->L.xi[q][1], c[2] + s * g->L.xi[q][2]);
    g->fc_pre[q * g->Nc + i] = g->fc[q * g->Nc + src];
  }
  double r, uu[3];
  moments_L(&g->L, g->fc_pre + i, g->Nc, &r, uu);
  g->rho_c[i] = r;
  for (int d = 0; d < 3; ++d) g->u_c[d * g->Nc + i] = uu[d];
}
static void stream_fine_node(ogrid* g, const double* src_f, long i) {
  int j[3];
  fco(g, i, j);
  for (int q = 0; q < g->Q; ++q) {
    int s = (g_mut == MUT_STREAM_PUSH) ? 1 : -1;
    long src = fidx(g, j[0] + s * g->L.xi[q][0], j[1] + s * g->L.xi[q][1], j[2] + s * g->L.xi[q][2]);
    g->ff_pre[q * g->Nf + i] = src_f[q * g->Nf + src];
  }
  double r, uu[3];
  moments_L(&g->L, g->ff_pre + i, g->Nf, &r, uu);
  g->rho_f[i] = r;
  for (int d = 0; d < 3; ++d) g->u_f[d * g->Nf + i] = uu[d];
}

/* Value of history field fld at ring node r: temporal interpolation at each
 * stencil point (weights c over t-1, t, t+1), then the spatial weights. */
static double ring_field(const ogrid* g, long r, int fld, const double* c) {
  const double* Hm = g->hist[g->hs[0]];
  const double* H0 = g->hist[g->hs[1]];
  const double* Hp = g->hist[g->hs[2]];
  double v = 0.0;
  for (int s = 0; s < g->rnp[r]; ++s) {
    long h = g->rpt[16 * r + s];
    long k = (long)fld * g->NH + h;
    double gt = c[0] * Hm[k] + c[1] * H0[k] + c[2] * Hp[k];
    v += g->rw[16 * r + s] * gt;
  }
  return v;
}

/* Ring macroscopic fields at the current fine time (eqs TempInt, spaceInt) */
static void ring_macros(ogrid* g, int half) {
  double c[3];
  orc_temporal_weights(half, c);
#pragma omp parallel for schedule(static)
  for (long r = 0; r < g->NR; ++r) {
    long i = g->rnode[r];
    double rho = ring_field(g, r, F_RHO, c);
    g->r_rho[r] = rho;
    g->rho_f[i] = rho;
    for (int d = 0; d < 3; ++d) {
      double ud = d < g->D ? ring_field(g, r, F_U + d, c) : 0.0;
      g->r_u[3 * r + d] = ud;
      g->u_f[d * g->Nf + i] = ud;
    }
  }
}

/* Ring populations and strain rate (eqs TempInt, spaceInt, rescff, PijResc),
 * then the ring collision, written into dst.  Reading: rho, u and the coarse
 * non-equilibrium part are interpolated separately and the populations are
 * rebuilt as f0(rho, u) + tau_f/(2 tau_c) f1 (all Q populations). */
static void ring_reconstruct_collide(ogrid* g, int half, double* dst) {
  double c[3];
  orc_temporal_weights(half, c);
  const double kf = orc_rescale_c2f(g->tau_c, g->tau_f);
  const double ks = 1.0 / orc_strain_f2c();
#pragma omp parallel for schedule(static)
  for (long r = 0; r < g->NR; ++r) {
    long i = g->rnode[r];
    double f[MAXQ], f0[MAXQ], S[9], out[MAXQ];
    feq_L(&g->L, g->r_rho[r], g->r_u + 3 * r, f0);
    for (int q = 0; q < g->Q; ++q) f[q] = f0[q] + kf * ring_field(g, r, F_F1 + q, c);
    for (int k = 0; k < 9; ++k) S[k] = (g->model == MOD_HRR) ? ks * ring_field(g, r, F_S + k, c) : 0.0;
    collide_L(&g->L, g->model, g->tau_f, g->sigma, f, 1, S, out, 1);
    for (int q = 0; q < g->Q; ++q) dst[q * g->Nf + i] = out[q];
  }
}

static void uniform_step(ogrid* g) {
  long N = g->Nc;
  memcpy(g->u_c_prev, g->u_c, sizeof(double) * 3 * (size_t)N);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) stream_coarse_node(g, i);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double S[9] = {0}, gr[3][3] = {{0}}, sg = g->sigma;
    if (g->model == MOD_HRR) strain_coarse_g(g, i, S, gr);
    if (g->dyn) sg = dyn_sigma(g, g->dyn_c, g->dyn_mask_c, N, i, gr);
    collide_L(&g->L, g->model, g->tau_c, sg, g->fc_pre + i, N, S, g->fc + i, N);
  }
}

/* The phases of one coarse step (Sec. 4.3), shared by the two-level step and
 * the nested step below. */

/* Coarse propagation (every node but TN^c and the covered ones) and the
 * history at t+1: pre-collision rho, u and f1 = f - f0. */
static void coarse_stream_history(ogrid* g) {
  const int Q = g->Q;
  const long Nc = g->Nc, NH = g->NH;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < Nc; ++i)
    if (g->cls_c[i] == C_MIDDLE || g->cls_c[i] == C_TFC) stream_coarse_node(g, i);
  if (g_mut != MUT_NEST_INJ)
    for (long r = 0; r < g->n_inj; ++r) {
      long i = g->inj_node[r];
      g->rho_c[i] = g->inj_rho[r];
      for (int d = 0; d < 3; ++d) g->u_c[d * Nc + i] = g->inj_u[3 * r + d];
    }
  double* Hp = g->hist[g->hs[2]];
#pragma omp parallel for schedule(static)
  for (long h = 0; h < NH; ++h) {
    long i = g->hnode[h];
    double f0[MAXQ], uu[3];
    for (int d = 0; d < 3; ++d) uu[d] = g->u_c[d * Nc + i];
    feq_L(&g->L, g->rho_c[i], uu, f0);
    Hp[F_RHO * NH + h] = g->rho_c[i];
    for (int d = 0; d < 3; ++d) Hp[(F_U + d) * NH + h] = uu[d];
    for (int q = 0; q < MAXQ; ++q)
      Hp[(F_F1 + q) * NH + h] = q < Q ? g->fc_pre[q * Nc + i] - f0[q] : 0.0;
  }
}

/* Filtered fine -> coarse reconstruction at TN (eqs filterFneq, rescfc,
 * PijResc) from the fine pre-collision state at t+1.  Reading: rho and u at
 * TN^c are those of the co-located fine node (unfiltered); the filter acts
 * on the non-equilibrium part only. */
static void coalesce_tn(ogrid* g) {
  const int Q = g->Q;
  const long Nc = g->Nc, Nf = g->Nf;
  const int hrr = (g->model == MOD_HRR);
  const double kc = orc_rescale_f2c(g->tau_c, g->tau_f);
  const double ks = orc_strain_f2c();
  const int D = g->D;
  const int nst = (D == 2) ? 9 : 27;
#pragma omp parallel for schedule(static)
  for (long t = 0; t < g->NT; ++t) {
    int j[3];
    long i = g->tn_f[t];
    fco(g, i, j);
    double ft[MAXQ] = {0};
    for (int s = 0; s < nst; ++s) {
      int o[3] = {s % 3 - 1, (s / 3) % 3 - 1, D == 3 ? s / 9 - 1 : 0};
      int zs = (g_mut == MUT_FILTER_ZOFF && D == 3) ? 1 : 0;
      long k = fidx(g, j[0] + o[0], j[1] + o[1], j[2] + o[2] + zs);
      double f0[MAXQ], uu[3];
      for (int d = 0; d < 3; ++d) uu[d] = g->u_f[d * Nf + k];
      feq_L(&g->L, g->rho_f[k], uu, f0);
      double wgt = orc_filter_weight(D, o);
      for (int q = 0; q < Q; ++q) ft[q] += wgt * (g->ff_pre[q * Nf + k] - f0[q]);
    }
    double f0[MAXQ], uu[3];
    for (int d = 0; d < 3; ++d) uu[d] = g->u_f[d * Nf + i];
    feq_L(&g->L, g->rho_f[i], uu, f0);
    long ic = g->tn_c[t];
    for (int q = 0; q < Q; ++q) g->fc_pre[q * Nc + ic] = f0[q] + kc * ft[q];
    g->rho_c[ic] = g->rho_f[i];
    for (int d = 0; d < 3; ++d) g->u_c[d * Nc + ic] = uu[d];
    double S[9] = {0};
    if (hrr) strain_fine(g, i, S);
    for (int k = 0; k < 9; ++k) g->S_tn[9 * t + k] = ks * S[k];
  }
}

/* Collision of the coarse nodes (middle and TF^c, then TN^c with the strain
 * rate handed over by the fine level), then the time levels move on: t+1
 * becomes t, t becomes t-1. */
static void coarse_collide_advance(ogrid* g) {
  const long Nc = g->Nc;
  const int hrr = (g->model == MOD_HRR);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < Nc; ++i) {
    if (g->cls_c[i] != C_MIDDLE && g->cls_c[i] != C_TFC) continue;
    double S[9] = {0}, gr[3][3] = {{0}}, sg = g->sigma;
    if (hrr) strain_coarse_g(g, i, S, gr);
    if (g->dyn) sg = dyn_sigma(g, g->dyn_c, g->dyn_mask_c, Nc, i, gr);
    collide_L(&g->L, g->model, g->tau_c, sg, g->fc_pre + i, Nc, S, g->fc + i, Nc);
  }
#pragma omp parallel for schedule(static)
  for (long t = 0; t < g->NT; ++t) {
    long ic = g->tn_c[t];
    collide_L(&g->L, g->model, g->tau_c, g->sigma, g->fc_pre + ic, Nc, g->S_tn + 9 * t, g->fc + ic, Nc);
  }
  int old = g->hs[0];
  g->hs[0] = g->hs[1];
  g->hs[1] = g->hs[2];
  g->hs[2] = old;
}

/* H-RR, after the fine collision at t+1/2 (Sec. 4.3 with the strain rate of
 * eq stressT): (e) fictitious propagation of the fine post-collision state
 * onto TN^f gives u(TN^c, t+1); (f) the coarse strain rate at t+1 on the
 * history nodes, which the ring interpolates. */
static void hrr_tn_strain(ogrid* g) {
  const int Q = g->Q;
  const long Nc = g->Nc, Nf = g->Nf, NH = g->NH;
#pragma omp parallel for schedule(static)
  for (long t = 0; t < g->NT; ++t) {
    int j[3];
    long i = g->tn_f[t];
    fco(g, i, j);
    double f[MAXQ], r, uu[3];
    for (int q = 0; q < Q; ++q)
      f[q] = g->ff_half[q * Nf + fidx(g, j[0] - g->L.xi[q][0], j[1] - g->L.xi[q][1], j[2] - g->L.xi[q][2])];
    moments_L(&g->L, f, 1, &r, uu);
    long ic = g->tn_c[t];
    g->rho_c[ic] = r;
    for (int d = 0; d < 3; ++d) g->u_c[d * Nc + ic] = uu[d];
  }
  double* Hp = g->hist[g->hs[2]];
#pragma omp parallel for schedule(static)
  for (long h = 0; h < NH; ++h) {
    double S[9];
    strain_coarse(g, g->hnode[h], S);
    for (int k = 0; k < 9; ++k) Hp[(F_S + k) * NH + h] = S[k];
  }
}

static void two_level_step(ogrid* g) {
  const long Nc = g->Nc, Nf = g->Nf;
  const int hrr = (g->model == MOD_HRR);

  /* velocities of the coarse iteration t, kept for the NH sensors */
  memcpy(g->u_c_prev, g->u_c, sizeof(double) * 3 * (size_t)Nc);
  /* Asynchronous iteration: fine t -> t+1/2, coarse t -> t+1. */
  /* (a) propagation of the coarse nodes other than TN^c (and covered),
   * history at t+1 */
  coarse_stream_history(g);
  /* (a) propagation of the fine middle nodes */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < Nf; ++i)
    if (g->cls_f[i] == F_MIDDLE || g->cls_f[i] == F_TNF) stream_fine_node(g, g->ff, i);
  /* (b, c) rho, u on TF^f (temporal) and IE (spatial) */
  ring_macros(g, 1);
  /* (d) collision of the fine middle nodes */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < Nf; ++i) {
    if (g->cls_f[i] != F_MIDDLE && g->cls_f[i] != F_TNF) continue;
    double S[9] = {0}, gr[3][3] = {{0}}, sg = g->sigma;
    if (hrr) strain_fine_g(g, i, S, gr);
    if (g->dyn) sg = dyn_sigma(g, g->dyn_f, g->dyn_mask_f, Nf, i, gr);
    collide_L(&g->L, g->model, g->tau_f, sg, g->ff_pre + i, Nf, S, g->ff_half + i, Nf);
  }
  if (hrr) hrr_tn_strain(g);
  /* (g, h, i) ring populations and strain rate at t+1/2, ring collision */
  ring_reconstruct_collide(g, 1, g->ff_half);

  /* velocities of the fine iteration t+1/2 (ring included), kept for the
   * NH sensors */
  memcpy(g->u_f_prev, g->u_f, sizeof(double) * 3 * (size_t)Nf);
  /* Synchronous iteration: fine t+1/2 -> t+1. */
  /* (a) propagation of the fine middle nodes */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < Nf; ++i)
    if (g->cls_f[i] == F_MIDDLE || g->cls_f[i] == F_TNF) stream_fine_node(g, g->ff_half, i);
  /* (b, c) ring at t+1 by direct transfer / spatial interpolation */
  ring_macros(g, 0);
  /* (d) filtered fine -> coarse reconstruction at TN */
  coalesce_tn(g);
  /* (e) collision of all nodes */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < Nf; ++i) {
    if (g->cls_f[i] != F_MIDDLE && g->cls_f[i] != F_TNF) continue;
    double S[9] = {0}, gr[3][3] = {{0}}, sg = g->sigma;
    if (hrr) strain_fine_g(g, i, S, gr);
    if (g->dyn) sg = dyn_sigma(g, g->dyn_f, g->dyn_mask_f, Nf, i, gr);
    collide_L(&g->L, g->model, g->tau_f, sg, g->ff_pre + i, Nf, S, g->ff + i, Nf);
  }
  ring_reconstruct_collide(g, 0, g->ff);
  coarse_collide_advance(g);
}

/* Nested refinement (more than two levels; the cylinder case of Sec. 10 nests
 * several refinement domains).  Reading: the two-level step of Sec. 4.3 is
 * applied recursively -- each substep of the fine level is one whole step of
 * the pair (fine level, its own patch), so a level of depth l advances 2^l
 * times per coarse step and every interface keeps the rules of Sec. 4.2 with
 * its own pair's relaxation times.  Here the fine level's substeps are the
 * child's steps: the fine state (ring included) is handed to the child's
 * coarse level, the child steps, and its coarse level comes back; the ring
 * and the transfer to TN^c are this grid's, as in the two-level step.  The
 * ring's rho and u at the child's time (t+1/2, then t+1) are computed before
 * the child steps and given to it: with H-RR its collision of the nodes next
 * to the ring takes the centred differences of eq stressT across them. */
static void level_to_child(ogrid* g, const double* f) {
  ogrid* c = g->child;
  memcpy(c->fc, f, sizeof(double) * (size_t)g->Q * g->Nf);
  c->inj_node = g->rnode;
  c->inj_rho = g->r_rho;
  c->inj_u = g->r_u;
  c->n_inj = g->NR;
}
static void child_to_level(ogrid* g, double* f, int pre) {
  ogrid* c = g->child;
  memcpy(f, c->fc, sizeof(double) * (size_t)g->Q * g->Nf);
  if (pre) {
    memcpy(g->ff_pre, c->fc_pre, sizeof(double) * (size_t)g->Q * g->Nf);
    memcpy(g->rho_f, c->rho_c, sizeof(double) * (size_t)g->Nf);
    memcpy(g->u_f, c->u_c, sizeof(double) * 3 * (size_t)g->Nf);
  }
}
static void level_step(ogrid* g);
static void nested_step(ogrid* g) {
  memcpy(g->u_c_prev, g->u_c, sizeof(double) * 3 * (size_t)g->Nc);
  /* Asynchronous iteration: coarse t -> t+1 (propagation, history), fine
   * t -> t+1/2 as one step of the child from the fine state at t */
  coarse_stream_history(g);
  ring_macros(g, 1);
  level_to_child(g, g->ff);
  level_step(g->child);
  child_to_level(g, g->ff_half, 0);
  /* H-RR: u(TN^c, t+1) and the strain rate on the history nodes */
  if (g->model == MOD_HRR) hrr_tn_strain(g);
  /* ring at t+1/2 */
  if (g_mut != MUT_NEST_RING) ring_reconstruct_collide(g, 1, g->ff_half);
  /* Synchronous iteration: fine t+1/2 -> t+1, one more child step */
  ring_macros(g, 0);
  level_to_child(g, g_mut == MUT_NEST_SYNC ? g->ff : g->ff_half);
  level_step(g->child);
  child_to_level(g, g->ff, 1);
  /* transfer to TN^c from the fine pre-collision state at t+1, ring at t+1 */
  coalesce_tn(g);
  ring_reconstruct_collide(g, 0, g->ff);
  coarse_collide_advance(g);
}
static void level_step(ogrid* g) {
  if (g->child) nested_step(g);
  else if (g->has_fine) two_level_step(g);
  else uniform_step(g);
  g->steps++;
}

int orc_step(void* hp, int nsteps) {
  ogrid* g = (ogrid*)hp;
  for (int s = 0; s < nsteps; ++s) {
    level_step(g);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Non-hydrodynamic-mode sensors of Sec. 7, evaluated on the last iteration
 * of a level after a step (coarse: t+1 against t; fine: t+1 against t+1/2;
 * uniform grid: t+1 against t).
 *   bit 0, SpuriousAc (eq sensorSpuriousAc): div u(previous) * div u(last) < 0
 *   bit 1, SpuriousS  (eq sensorSpuriousS):  curl u(previous) . curl u(last) < 0
 *          Reading: in 3D the product of the two curl vectors is their dot
 *          product; in 2D the curl is the scalar d_x u_y - d_y u_x.
 *   bit 2, SpuriousG  (eqs fneqSplit, reguProceduref1S, sensorSpuriousG):
 *          ||f1 - f1,S|| > thr and neither bit above, with f1 = f - f0(rho, u)
 *          of the pre-collision populations of the last iteration and f1,S
 *          their projection on the second-order Hermite polynomials.
 *          Reading: the paper's "> 0" is taken as "> thr", a threshold the
 *          caller states above the rounding of the populations.
 * A product exactly zero gives 0 (the paper's ">= 0 -> 0").  Derivatives
 * are centred differences in the level's lattice units.  Nodes whose
 * stencil or pre-collision state is not part of the level's evolution get
 * 0: coarse TN^c and covered nodes (their neighbours include covered
 * nodes) and the fine ring (rebuilt by interpolation, not streamed).
 * The previous iteration's velocities exist once a step has been taken. */
static void div_curl(int D, const double* u, long N, const long* nb, double* div, double* curl) {
  /* nb[2a], nb[2a+1]: node indices at x + e_a, x - e_a */
  double gr[3][3] = {{0}};
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) gr[a][b] = (u[b * N + nb[2 * a]] - u[b * N + nb[2 * a + 1]]) / 2.0;
  *div = 0.0;
  for (int a = 0; a < D; ++a) *div += gr[a][a];
  if (D == 2) {
    curl[0] = gr[0][1] - gr[1][0];
    curl[1] = curl[2] = 0.0;
  } else {
    curl[0] = gr[1][2] - gr[2][1];
    curl[1] = gr[2][0] - gr[0][2];
    curl[2] = gr[0][1] - gr[1][0];
  }
}

int orc_sensors(void* hp, int level, double thr, uint8_t* flags, double* div_prod, double* curl_prod,
                double* g_norm) {
  ogrid* g = (ogrid*)hp;
  if (level == 1 && !g->has_fine) return -1;
  if (g->steps == 0) return -2;
  const int D = g->D, Q = g->Q;
  const long N = level == 0 ? g->Nc : g->Nf;
  const double* up = level == 0 ? g->u_c_prev : g->u_f_prev;
  const double* uc = level == 0 ? g->u_c : g->u_f;
  const double* fp = level == 0 ? g->fc_pre : g->ff_pre;
  const double* fpost = level == 0 ? g->fc : g->ff;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    flags[i] = 0;
    if (div_prod) div_prod[i] = 0.0;
    if (curl_prod) curl_prod[i] = 0.0;
    if (g_norm) g_norm[i] = 0.0;
    int c[3];
    long nb[6] = {i, i, i, i, i, i};
    if (level == 0) {
      if (g->has_fine && g->cls_c[i] != C_MIDDLE && g->cls_c[i] != C_TFC) continue;
      cco(g, i, c);
      for (int a = 0; a < D; ++a) {
        int p[3] = {c[0], c[1], c[2]}, q[3] = {c[0], c[1], c[2]};
        p[a]++;
        q[a]--;
        nb[2 * a] = cidx(g, p[0], p[1], p[2]);
        nb[2 * a + 1] = cidx(g, q[0], q[1], q[2]);
      }
    } else {
      if (g->cls_f[i] != F_MIDDLE && g->cls_f[i] != F_TNF) continue;
      fco(g, i, c);
      for (int a = 0; a < D; ++a) {
        int p[3] = {c[0], c[1], c[2]}, q[3] = {c[0], c[1], c[2]};
        p[a]++;
        q[a]--;
        nb[2 * a] = fidx(g, p[0], p[1], p[2]);
        nb[2 * a + 1] = fidx(g, q[0], q[1], q[2]);
      }
    }
    double dp, dc, cp[3], cc[3];
    div_curl(D, up, N, nb, &dp, cp);
    div_curl(D, uc, N, nb, &dc, cc);
    const double pd = dp * dc;
    const double pc = cp[0] * cc[0] + cp[1] * cc[1] + cp[2] * cc[2];
    const int ac = pd < 0.0, sp = pc < 0.0;
    /* pre-collision populations of the last iteration: the streamed state
     * (uniform grid: the post-collision state of the step before is not
     * kept, so the pre-collision one is fc_pre as well) */
    (void)fpost;
    double f[MAXQ], f0[MAXQ], r, uu[3];
    for (int q = 0; q < Q; ++q) f[q] = fp[q * N + i];
    moments_L(&g->L, f, 1, &r, uu);
    feq_L(&g->L, r, uu, f0);
    double f1[MAXQ], a2[3][3] = {{0}};
    for (int q = 0; q < Q; ++q) f1[q] = f[q] - f0[q];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        for (int q = 0; q < Q; ++q) a2[a][b] += g->L.H2[q][a][b] * f1[q];
    double nrm = 0.0;
    for (int q = 0; q < Q; ++q) {
      double hs = 0.0;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) hs += g->L.H2[q][a][b] * a2[a][b];
      const double f1s = g->L.w[q] * hs / (2.0 * CS2 * CS2);
      const double gq = f1[q] - f1s;
      nrm += gq * gq;
    }
    nrm = sqrt(nrm);
    const int gs = (nrm > thr) && !ac && !sp;
    flags[i] = (uint8_t)(ac | (sp << 1) | (gs << 2));
    if (div_prod) div_prod[i] = pd;
    if (curl_prod) curl_prod[i] = pc;
    if (g_norm) g_norm[i] = nrm;
  }
  return 0;
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
