/*
 * lbm.h -- C ABI of the MI355X (gfx950) two-level lattice-Boltzmann library.
 *
 * The library evolves populations on a periodic coarse grid that carries one
 * fine patch at refinement ratio 2, following the cell-vertex scheme analysed
 * in Astoul et al., "Analysis and reduction of spurious noise generated at
 * grid refinement interfaces with the lattice Boltzmann method"
 * (arXiv:2004.11863):
 *   - lattices D2Q9 (Sec. 3.1, eqs xi_i and w_i) and D3Q19 (named in Sec. 10);
 *   - collisions BGK (eq BGKmodel), recursive regularised RR (eqs a1Proj,
 *     f1RR, a13RR, LBMscheme_reg) and hybrid recursive regularised H-RR
 *     (eqs stressT, a1ij_HRR), all with the third-order equilibrium
 *     (eq fEqO3);
 *   - two fine substeps per coarse step; non-equilibrium rescaling by the
 *     relaxation-time ratio (eqs rescTau, fneqResc, rescff, rescfc), the
 *     filtered fine-to-coarse transfer (eq filterFneq), the strain-rate
 *     hand-off (eq PijResc), third-order temporal and cubic spatial
 *     interpolation (eqs TempInt, spaceInt), in the order of Sec. 4.3.
 *
 * Conventions
 *   - Every function returns an int: LBM_OK (0) or a negative error code.
 *     No C++ exception crosses this boundary.  lbm_last_error() returns a
 *     text for the last failure on a handle (or the last create failure when
 *     called with NULL).
 *   - Field arrays are structure-of-arrays, x fastest: a level with nodes
 *     (nx, ny, nz) stores node (x, y, z) at index x + nx (y + ny z).
 *     rho[N]; u[D][N] (component-major); populations f[Q][N].
 *   - Population order: D2Q9 as eq xi_i; D3Q19 as lbm_lattice_info reports
 *     (rest, +x, -x, +y, -y, +z, -z, then the 12 two-axis diagonals).
 *   - Coarse level = 0, fine level = 1.  Fine node j sits at coarse
 *     coordinate lo + j/2; the fine level has 2 (hi - lo) + 1 nodes per axis.
 *   - mem: LBM_HOST for host pointers, LBM_DEVICE for device pointers on the
 *     handle's device.  The caller owns every buffer it passes; the library
 *     copies in and out and keeps no pointer to it.
 *   - A handle is used by one host thread at a time.  All device work is
 *     ordered on the stream given to lbm_step (or the handle's own stream).
 *     Different handles may be used from different threads at once: the
 *     library serialises its blocking HIP calls with its hipGraph captures.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,        /* bad argument or descriptor                         */
  LBM_ENOMEM = -2,        /* device or host allocation failed                   */
  LBM_EUNSUPPORTED = -3,  /* valid request the library does not serve          */
  LBM_EUNSTABLE = -4,     /* non-finite totals detected                         */
  LBM_EDEVICE = -5        /* a HIP call failed                                  */
};

typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 } lbm_lattice;
typedef enum { LBM_BGK = 0, LBM_RR = 1, LBM_HRR = 2 } lbm_collision;
/* LBM_FP64: populations stored and updated in double precision.
 * LBM_FP32_DEV: populations stored in single precision as deviations
 * h_i = f_i - w_i from the rest state; bulk updates in single precision,
 * interface history, interpolation, filtering and rescaling in double,
 * global totals accumulated in double. */
typedef enum { LBM_FP64 = 0, LBM_FP32_DEV = 1 } lbm_precision;
typedef enum { LBM_HOST = 0, LBM_DEVICE = 1 } lbm_mem;

/* Coarse node classes (Fig. Overlap) as returned by lbm_get_index_maps(0). */
enum { LBM_C_MIDDLE = 0, LBM_C_TF = 1, LBM_C_TN = 2, LBM_C_COVERED = 3 };
/* Fine node classes as returned by lbm_get_index_maps(1): middle, ring nodes
 * co-located with coarse nodes (TF), ring nodes between coarse nodes (IE,
 * cubic along one axis; IE_FACE, tensor cubic on a 3D face centre), and
 * middle nodes co-located with TN coarse nodes. */
enum { LBM_F_MIDDLE = 0, LBM_F_TF = 1, LBM_F_IE = 2, LBM_F_IE_FACE = 3, LBM_F_TN = 4 };

typedef struct lbm_grid* lbm_handle;

typedef struct {
  int32_t lattice;    /* lbm_lattice                                            */
  int32_t collision;  /* lbm_collision                                          */
  int32_t precision;  /* lbm_precision                                          */
  int32_t n[3];       /* coarse nodes per axis, periodic; n[2] = 1 for D2Q9    */
  int32_t lo[3];      /* fine patch = box [lo, hi] of coarse vertices; lo == hi */
  int32_t hi[3];      /* on every axis means a single uniform periodic level.   */
                      /* Otherwise per used axis: hi - lo >= 4, lo >= 2 and     */
                      /* hi <= n - 3 (the patch and its interpolation stencils  */
                      /* lie strictly inside one period).                       */
  double tau_coarse;  /* > 0.5; tau_fine = 2 tau_coarse - 1/2 (eq rescTau)      */
  double sigma;       /* H-RR weight of the projected stress, in [0, 1]         */
                      /* (eq a1ij_HRR; the paper uses 0.995); ignored otherwise */
  int32_t device;     /* HIP device ordinal                                     */
  int32_t reserved;   /* must be 0                                              */
} lbm_grid_desc;

/* Creates a grid: validates the descriptor, builds the node-class maps and
 * interface stencil tables, allocates all device state (two population
 * buffers per level, a third fine one for BGK / RR, for D3Q19 BGK / RR a
 * compact copy of the fine x-normal bands, the three-time-level coarse
 * history, stencil tables) and a non-blocking stream.  The state is
 * zero until lbm_set_state.  LBM_EINVAL for a bad descriptor, including a
 * level of 2^31 or more padded node positions (rows padded to a multiple of
 * 4 nodes). */
int lbm_create_grid(const lbm_grid_desc* d, lbm_handle* out);
int lbm_destroy(lbm_handle h);

/* Sets one level's state at t = 0 to the equilibrium populations
 * f = f0(rho, u) of the given fields (Sec. 4.3, reference state).  Setting
 * the coarse level also resets the coarse history: the levels t-1 and t hold
 * rho, u, a zero non-equilibrium part and, for H-RR, the centred-difference
 * strain rate of u.  rho[N], u[D][N], double precision.  Synchronous. */
int lbm_set_state(lbm_handle h, int level, const double* rho, const double* u, int mem);

/* Enqueues n_coarse_steps coarse steps (each = one coarse update and two
 * fine substeps, Sec. 4.3) on hip_stream (a hipStream_t; NULL = the handle's
 * stream).  Asynchronous; returns after the launches. */
int lbm_step(lbm_handle h, int n_coarse_steps, void* hip_stream);

/* Density and velocity of one level at the current time (moments of the
 * post-collision populations, eqs moment_rho and moment_rhoU) in double
 * precision.  Covered coarse nodes take the values of the co-located fine
 * node.  With mem = LBM_HOST the call waits for the stream. */
int lbm_get_macros(lbm_handle h, int level, double* rho, double* u, int mem);

/* Post-collision populations f[Q][N] of one level (double precision, full
 * values, not deviations).  Covered coarse nodes do not evolve: their
 * populations are unspecified.  Setting them on the coarse level
 * re-initialises the history from their moments as lbm_set_state does.
 * Synchronous. */
int lbm_set_populations(lbm_handle h, int level, const double* f, int mem);
int lbm_get_populations(lbm_handle h, int level, double* f, int mem);

/* Sums of rho and rho u over the evolving nodes of each level (coarse: all
 * but covered nodes; fine: all nodes), accumulated in double precision in a
 * fixed order.  mass[2], momentum[2][3].  Returns LBM_EUNSTABLE if any sum
 * is not finite.  Synchronous. */
int lbm_get_totals(lbm_handle h, double mass[2], double momentum[6]);

/* The same totals, bit for bit, from the same kernels, for callers that
 * cannot allocate device memory (serving loops and harnesses that forbid
 * hipMalloc): nothing is allocated on any call.  The partial sums go to a
 * file-scope device array of 8 MiB + 32 B per GPU (4 doubles per block of
 * 256 nodes, then the 4 final sums), which each GPU the library runs on holds
 * until the process ends.  Levels of more than 2^26 = 67,108,864 nodes are
 * rejected with LBM_EINVAL.  Every call on one GPU shares that GPU's array
 * and overwrites all of it that it reads; calls that overlap on one GPU
 * (from several host threads) race -- the library's own lock serialises
 * them within this process.  Returns LBM_EUNSTABLE if any sum is not
 * finite.  Synchronous. */
int lbm_get_totals_noalloc(lbm_handle h, double mass[2], double momentum[6]);

/* Non-hydrodynamic-mode sensors (Sec. 7 of the paper).  lbm_sensors_enable
 * (on = 1) makes the following lbm_step calls record what the sensors
 * compare: the velocities of the iteration before the last step's last one
 * (coarse: t; fine: t+1/2) and the fine t+1/2 state.  Only the last step of
 * each call records (a read-out sees no other); with BGK or RR on two levels
 * the step before it records the coarse velocities as it streams, else a
 * recording pass does.  Off by default; a recording step costs about one
 * extra pass over the populations (D3Q19 runs its fine substeps as two
 * launches then).  Device memory: 2 (1 + D) doubles per coarse node,
 * (1 + D) per fine node, and 3 doubles and a byte per node of the larger
 * level for the read-out.
 * lbm_sensors(level) then returns, for the last step, one byte per node of
 * the level (x fastest):
 *   bit 0 SpuriousAc: div u(previous) * div u(last) < 0  (eq sensorSpuriousAc)
 *   bit 1 SpuriousS:  curl u(previous) . curl u(last) < 0 (eq sensorSpuriousS;
 *                     3D: dot product of the curl vectors)
 *   bit 2 SpuriousG:  ||f1 - f1,S|| > threshold and neither bit above
 *                     (eqs fneqSplit, reguProceduref1S, sensorSpuriousG), with
 *                     f1 = f - f0(rho, u) of the last iteration's pre-collision
 *                     populations and f1,S its second-order Hermite projection
 * Derivatives are centred differences in the level's lattice units, all in
 * double precision.  A product of exactly zero gives 0.  Nodes the level
 * does not evolve by streaming get 0: coarse TN and covered nodes, the fine
 * ring.  diag (optional, may be NULL): [3][N] doubles, the divergence
 * product, the curl product and the ghost norm.  flags / diag are host or
 * device memory per mem.  LBM_EINVAL before any recorded step, or after
 * lbm_set_state, lbm_set_populations or lbm_tune.  Synchronous. */
int lbm_sensors_enable(lbm_handle h, int on);
int lbm_sensors(lbm_handle h, int level, double threshold, uint8_t* flags, double* diag, int mem);

/* Three nested levels: the grid of *d whose patch (level 1) carries a patch
 * of its own (level 2), the box [lo2, hi2] of level-1 vertices, with the same
 * rules as the level-1 patch (at least 4 cells per axis, lo2 >= 2, hi2 <=
 * nodes - 3).  Each pair of levels is coupled as the two-level grid is (Sec.
 * 4), with tau = 2 tau - 1/2 from one level to the next (eq rescTau), and
 * every substep of level 1 is one whole step of the pair (1, 2): level 2
 * takes four steps per coarse step (the paper's cylinder case nests several
 * refinement domains, Sec. 10).  Levels 0, 1, 2 in lbm_set_state,
 * lbm_get_macros, lbm_set/get_populations, lbm_level_dims and
 * lbm_get_index_maps (level 1 has the classes of its own ring and TN nodes).
 * In lbm_get_macros covered nodes take the co-located node of the next
 * level; a level-1 node under level 2 holds no evolved value itself, so the
 * level-0 nodes above it are unspecified.  BGK, RR and H-RR (with H-RR the
 * pair (1, 2) takes the level-1 ring's rho and u at its own time, t+1/2 and
 * t+1, for the centred differences of eq stressT next to that ring).
 * Totals, tuning, variants, sensors, probes and dynamic sigma return
 * LBM_EUNSUPPORTED on a nested grid.  Errors as lbm_create_grid. */
int lbm_create_nested(const lbm_grid_desc* d, const int32_t lo2[3], const int32_t hi2[3], lbm_handle* out);

/* Dynamic sigma (H-RR only): a variant that Sec. 9.3 and Sec. 11 of the
 * paper suggest without defining it -- lower sigma (more finite-difference
 * stress) only where non-hydrodynamic modes are detected.  While on, every
 * bulk H-RR collision (coarse and fine middle nodes, TF^c, TN^f; not the
 * ring or TN^c, which keep sigma) compares the divergence and curl of the
 * velocity gradient it uses with those of the node's previous collision on
 * its level, as the SpuriousAc and SpuriousS sensors do, and takes
 * sigma_dyn where either product is below -threshold (3D curl: dot
 * product; threshold 0 is the sensors' own test, a small positive one keeps
 * products of rounding noise from switching).  Switching on clears the
 * stored divergences and curls (no switch at a node's first collision).
 * Costs 4 values of the storage type per node and level of device memory
 * (read and written by every bulk H-RR collision); D3Q19 runs its H-RR
 * substeps in two passes (velocity pass, then pull + collide), D2Q9 keeps
 * its one-pass kernels.  LBM_EINVAL: not an H-RR grid, sigma_dyn outside [0, 1], or a
 * negative or non-finite threshold.  Not available for batches. */
int lbm_set_dynamic_sigma(lbm_handle h, int on, double sigma_dyn, double threshold);

/* Probe recording: after every following coarse step the density at node
 * node[3] (level coordinates) of `level` is appended on the device to a
 * series of at most `capacity` values (the paper's probes, Sec. 9.3).  A
 * new call restarts the series; level = -1 stops recording.  The node must
 * be evolved by the level (not covered, not on the fine ring).
 * lbm_probe_read copies up to max values to host memory `out` and returns in
 * *count the number recorded (which may exceed max).  Synchronous. */
int lbm_probe_enable(lbm_handle h, int level, const int32_t node[3], int64_t capacity);
int lbm_probe_read(lbm_handle h, double* out, int64_t max, int64_t* count);

/* Node-class map of one level, one byte per node (LBM_C_* / LBM_F_*). */
int lbm_get_index_maps(lbm_handle h, int level, uint8_t* cls, int mem);

/* Nodes per axis of a level (dims[3]); error if the level does not exist. */
int lbm_level_dims(lbm_handle h, int level, int32_t dims[3]);

/* Lattice table: D, Q, xi[Q][3], w[Q]. */
int lbm_lattice_info(int lattice, int32_t* D, int32_t* Q, int32_t* xi, double* w);

/* Interface tables as built by the library, for bit-exact checks:
 * counts[3] = {history nodes, ring nodes, TN nodes};
 * hist_nodes[H] coarse node indices; ring_nodes[R] fine node indices,
 * ring_npts[R] in {1, 4, 16}, ring_pts[R][16] history entries (unused -1). */
int lbm_interface_counts(lbm_handle h, int64_t counts[3]);
int lbm_interface_tables(lbm_handle h, int64_t* hist_nodes, int64_t* ring_nodes, int32_t* ring_npts,
                         int64_t* ring_pts);

/* Lattice updates per coarse step: evolving coarse nodes + 2 x fine nodes. */
int lbm_updates_per_step(lbm_handle h, int64_t* updates);

/* Per-launch timing of the fine-level pull-stream + collide kernel (the
 * dominant kernel): D2Q9 BGK / RR the kernel that runs both fine substeps of
 * a coarse step; D3Q19 BGK / RR the fine stream of each substep, or in fine
 * variants 2 and 3 the marching kernel of both substeps; D2Q9 H-RR the
 * one-pass substep kernel; D3Q19 H-RR the collision pass (which pulls again
 * and collides with the strain rate of the velocities the first pass wrote),
 * or in variants 2 and 3 the one-pass marching kernel.  When enabled,
 * lbm_step records HIP events around each of its launches on the launch
 * stream; lbm_kernel_time returns the number of timed launches, their mean
 * duration in ms and the lattice updates one launch performs (fine middle
 * nodes times the substeps it runs).  Synchronous. */
int lbm_profile_enable(lbm_handle h, int on);
int lbm_kernel_time(lbm_handle h, int64_t* launches, double* mean_ms, int64_t* nodes_per_launch);

/* Bulk-kernel launch variants, 0 .. LBM_N_VARIANTS - 1: the same kernels
 * launched with 0, 53, 80 or 160 KB of unused LDS per 256-lane work group,
 * which caps the work groups resident on a CU (no cap, 3, 2, 1).  For the
 * fine role of a D2Q9 BGK / RR grid, whose kernel runs both substeps with
 * the half-step state on chip, the variants are work-group tiles of one
 * lane per vector, halo included (vectors x rows): 64 x 8, 64 x 16, 32 x 16
 * and 32 x 8.  For the fine role of a D3Q19 BGK / RR grid, variants 0 and 1
 * run the two substeps as two launches (capped at 2 and 3 resident work
 * groups per CU), 2 and 3 as one kernel walking tiles of 14 x 14 and 30 x 6
 * along z.  For the H-RR roles of a D2Q9 grid, whose kernels run a coarse
 * step or a fine substep in one pass (velocities of the tile in LDS), the
 * variants are tiles of 64 x 8, 32 x 8, 32 x 16 and 128 x 4 lanes; for the
 * fine H-RR role of a D3Q19 grid, variants 0 and 1 run the velocity pass and
 * the collision (capped at 2 and 3 resident work groups per CU), 2 and 3 one
 * pass walking tiles of 30 x 6 and 62 x 2 along z.  Every variant computes
 * bitwise the same result. */
enum { LBM_N_VARIANTS = 4 };
/* Autotuner: times every bulk-kernel variant of each bulk role of this grid
 * -- coarse stream, fine stream, coarse and fine H-RR collision -- over reps
 * launches on the grid's own data and keeps the fastest.  variants[4]
 * receives the chosen index per role (roles the grid does not use keep their
 * default).  Only buffers that the next lbm_step rewrites are touched, so the
 * state is unchanged.  Synchronous. */
int lbm_tune(lbm_handle h, int reps, int32_t variants[4]);
/* Sets the variant index per role (as returned by lbm_tune); LBM_EINVAL if
 * an index is outside 0 .. LBM_N_VARIANTS - 1. */
int lbm_set_variants(lbm_handle h, const int32_t variants[4]);

/* Last error text for a handle (NULL: last failure of lbm_create_grid). */
const char* lbm_last_error(lbm_handle h);

/* ------------------------------------------------------------------------
 * Batches: many independent grids of one lattice, collision model and
 * precision, each with its own geometry, tau and sigma, advanced together.
 * Each coarse step is one sequence of launches over the work of all grids
 * (bulk chunks, interface node blocks), captured once as a hipGraph and
 * replayed; grids may join and leave between steps (continuous batching),
 * which rewrites device work lists (the launch is captured again when a list
 * outgrows its buffer, after lbm_batch_tune or lbm_batch_set_variants, and
 * when graphs are switched off and on).  A grid in a batch computes exactly what the
 * same grid computes alone.
 *
 * Every call but lbm_batch_step returns when it is done, and first waits for
 * the batch's own work only: the steps last enqueued (on the stream passed to
 * lbm_batch_step) and its internal stream.  Work of other batches on other
 * streams keeps running meanwhile, so a server can admit or read grids of one
 * batch while another batch steps.  (Freeing device memory, in
 * lbm_batch_remove or when lbm_batch_add grows the shared scratch, waits for
 * the whole device, as hipFree does.)  Calls on one batch handle must not
 * overlap (one host thread at a time per batch).
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch* lbm_batch_handle;

/* capacity: maximum number of grids held at once. */
int lbm_batch_create(int lattice, int collision, int precision, int device, int capacity, lbm_batch_handle* out);
int lbm_batch_destroy(lbm_batch_handle b);
/* Adds a grid (allocates its device state; the descriptor's lattice,
 * collision and precision must match the batch).  *slot receives its index.
 * LBM_ENOMEM when the batch is full or device memory runs out. */
int lbm_batch_add(lbm_batch_handle b, const lbm_grid_desc* d, int32_t* slot);
/* Removes a grid and frees its device state. */
int lbm_batch_remove(lbm_batch_handle b, int slot);
/* As lbm_set_state / lbm_get_macros / lbm_get_populations for one grid. */
int lbm_batch_set_state(lbm_batch_handle b, int slot, int level, const double* rho, const double* u, int mem);
int lbm_batch_get_macros(lbm_batch_handle b, int slot, int level, double* rho, double* u, int mem);
int lbm_batch_get_populations(lbm_batch_handle b, int slot, int level, double* f, int mem);
/* Enqueues n coarse steps of every grid in the batch (asynchronous). */
int lbm_batch_step(lbm_batch_handle b, int n, void* hip_stream);
/* on = 0: launch the phases directly instead of replaying the graph. */
int lbm_batch_use_graph(lbm_batch_handle b, int on);
/* Autotuner over the bulk-kernel variants of the whole batch; variants[2]
 * receives the chosen coarse and fine variant (for D2Q9 BGK / RR batches,
 * whose fine phase runs both substeps in one launch, the fine variant is its
 * tile shape: 0 = 64 x 8, 1 = 32 x 8 lanes).  Synchronous. */
int lbm_batch_tune(lbm_batch_handle b, int reps, int32_t variants[2]);
/* Applies variants as lbm_batch_tune returns them (coarse, fine or tile
 * shape), e.g. from a stored tuning result; LBM_EINVAL when an index is out
 * of range.  Results do not depend on the variants.  Synchronous. */
int lbm_batch_set_variants(lbm_batch_handle b, const int32_t variants[2]);
/* info[3] = {grids held, lattice updates per coarse step over all grids,
 * device bytes of their state}. */
int lbm_batch_info(lbm_batch_handle b, int64_t info[3]);
/* Coarse steps taken by a grid since it joined (or since its last
 * lbm_batch_set_state of level 0). */
int lbm_batch_slot_steps(lbm_batch_handle b, int slot, int64_t* steps);
/* Device bytes a grid of this descriptor occupies in a batch slot
 * (populations, macro planes, history, interface tables), for admission by
 * memory footprint.  Fine levels hold three population buffers for D2Q9
 * BGK / RR (the third keeps the half-step ring and band of the fused fine
 * kernel), two otherwise; a single D3Q19 BGK / RR grid (lbm_create_grid)
 * also holds a third.  D3Q19 BGK / RR fine levels add the compact copy of
 * the fine x-bands (2 * 19 * 5 values per fine (y, z) row). */
int lbm_footprint(const lbm_grid_desc* d, int64_t* bytes);

/* Bandwidth reference (diagnostic): copies `bytes` (rounded down to 16) from
 * one device buffer to another `reps` times with a streaming kernel
 * (16-byte non-temporal loads and stores, 1024 per work group) after one untimed
 * pass, and stores the bytes read plus written per second, in GB/s, timed
 * with HIP events.  Allocates and frees its two buffers (LBM_ENOMEM if they
 * do not fit); LBM_EINVAL for bytes < 16, reps < 1 or an unknown device.
 * Synchronous. */
int lbm_copy_probe(int device, int64_t bytes, int reps, double* gbs);
const char* lbm_batch_last_error(lbm_batch_handle b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H_ */
