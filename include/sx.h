/*
 * sx.h -- C ABI of libsx: SimpleX2 direction-conserving photon transport
 * fused with hydrogen photo-ionisation chemistry, on an AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Paardekooper, Kruip & Icke (2010), "SimpleX2: radiative transfer on
 * an unstructured, dynamic grid", A&A, arXiv:0912.4273.
 *   - photons move along Delaunay edges, one edge per step, and interact at
 *     the vertex they reach (Sects. 2.2, 4.6);
 *   - direction-conserving transport (Sect. 2.2.3): each vertex keeps its
 *     photons in K global direction bins and hands every bin to the (up to)
 *     three neighbours most aligned with that bin's direction, never
 *     backwards (cosine > 0);
 *   - sources send their photons to all neighbours (Sects. 2.2, 4.3), filed
 *     in the bin closest to each edge (Sect. 2.2.4);
 *   - interaction exp(-n_HI sigma dL) (Eqs. optical_depth, intensity_absorbed,
 *     intensity_out) with the rate equation subcycled at constant incoming
 *     flux (Eqs. rate_eq, rate_eq_subcycle, phot_ion_rate_subcycle).
 *
 * Conventions
 *   - CGS units.  Vertex ids, neighbour rows and bins are in the caller's
 *     order on every call; the library may reorder internally but never
 *     exposes that order.
 *   - Every pointer argument is a HOST pointer unless stated otherwise.
 *     The library copies what it needs during the call and never keeps a
 *     caller pointer.
 *   - Return value: SX_OK (0) or a negative SX_E* code.  sx_last_error()
 *     gives a message for the most recent failure on that context.
 *   - One context per host thread.  Work is enqueued on the context's HIP
 *     stream; sx_step is asynchronous, every other call is synchronous.
 */
#ifndef SX_H
#define SX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SX_ABI_VERSION 2

/* ---- return codes ---------------------------------------------------- */
#define SX_OK 0
#define SX_EINVAL (-1)     /* malformed argument or grid                  */
#define SX_ENOMEM (-2)     /* device memory budget or allocation exceeded */
#define SX_EDEVICE (-3)    /* HIP runtime / kernel failure; ctx poisoned  */
#define SX_ENOTFOUND (-4)  /* unknown grid id                             */
#define SX_ENOTSUP (-5)    /* valid request outside the supported limits  */
#define SX_EAGAIN (-6)     /* nothing finished within the wait (serving)  */

/* ---- precision ------------------------------------------------------- */
#define SX_FP64 0            /* photons and chemistry in double            */
#define SX_FP32_TRANSPORT 1  /* photons in float (scaled units, see below),
                                neutral fraction, chemistry and tallies in
                                double                                     */

/* ---- limits ---------------------------------------------------------- */
#define SX_MAX_BINS_FP32 96   /* K <= 96 in SX_FP32_TRANSPORT              */
#define SX_MAX_BINS_FP64 96   /* K <= 96  in SX_FP64                       */
#define SX_MAX_DEGREE 127     /* Delaunay degree of any vertex             */
#define SX_MAX_PER_BIN 3      /* neighbours per bin (the paper's p = d = 3) */
#define SX_MAX_HOPS 1024      /* hops per step of a multi-hop grid          */

/* Transport modes (Sect. 2.2).  SX_TRANSPORT_DCT: direction-conserving
 * transport everywhere (Sect. 2.2.3).  SX_TRANSPORT_COMBINED: combined
 * transport (Sect. 2.2.4): at the start of every step each vertex whose
 * optical depth y tau (tau = n_H sigma dL, y its neutral fraction then) is
 * at least tau_switch uses ballistic transport (Sect. 2.2.2): it holds the
 * photons it received per incoming edge and sends each packet on, split
 * equally, to the <= max_per_bin neighbours most aligned with the edge it
 * came along (cosine > cos_min, ties to the lower id, like the bins).  The
 * other vertices use direction-conserving transport.  Photons reaching a
 * ballistic vertex are filed under the edge they came along; photons sent by
 * a ballistic vertex or a source to a direction-conserving one are filed in
 * the bin of the edge.  tau_switch <= 0 makes every vertex ballistic; the
 * paper uses 1. */
#define SX_TRANSPORT_DCT 0
#define SX_TRANSPORT_COMBINED 1

/* Reference direction of the bin selection of direction-conserving
 * transport.  SX_DCT_REF_BIN: the bin's own direction u_k (Sect. 2.2.3).
 * SX_DCT_REF_EDGE: the reading of the caption of the paper's figure of the
 * three transport modes: the bin is first tied to the vertex's Delaunay edge
 * closest to u_k (largest cosine, > cos_min, ties to the lower id; none:
 * the bin has no neighbour), and goes to the <= max_per_bin neighbours most
 * aligned with that edge. */
#define SX_DCT_REF_BIN 0
#define SX_DCT_REF_EDGE 1

typedef struct sx_ctx sx_ctx;
typedef int64_t sx_grid_id;

/* Device-memory hooks: alloc(bytes, user) returns a device pointer or NULL;
 * free(ptr, user).  Both NULL => hipMalloc / hipFree. */
typedef void *(*sx_alloc_fn)(size_t bytes, void *user);
typedef void (*sx_free_fn)(void *ptr, void *user);

typedef struct sx_ctx_opts {
    int32_t device;        /* HIP device ordinal                             */
    int32_t reserved0;
    uint64_t hbm_budget;   /* bytes the context may hold; 0 = 90% of free   */
    void *stream;          /* hipStream_t to enqueue on; NULL = own stream  */
    sx_alloc_fn alloc;     /* optional device allocator                      */
    sx_free_fn free;
    void *alloc_user;
} sx_ctx_opts;

/* One grid and one solve's physics.  All arrays are host pointers in the
 * caller's vertex order and are only read during sx_grid_upload. */
typedef struct sx_grid_desc {
    int64_t n_vertices;          /* N >= 1                                   */
    const double *pos;           /* [3N] vertex positions (cm)               */
    const int64_t *nbr_ptr;      /* [N+1] CSR row offsets, nbr_ptr[0] = 0    */
    const int32_t *nbr_idx;      /* [E] Delaunay neighbours: symmetric, no
                                    self-loops, no duplicates, deg <= 127    */
    const double *n_H;           /* [N] hydrogen number density (cm^-3)      */
    const double *volume;        /* [N] cell volume (cm^3), > 0              */
    const double *dL;            /* [N] path length through each cell, or
                                    NULL: kappa * mean incident edge length  */
    double kappa;                /* global path-length correction, Sect 2.2.3*/
    const double *x_init;        /* [N] initial ionised fraction or NULL (0) */
    int32_t n_bins;              /* K                                        */
    int32_t max_per_bin;         /* neighbours per bin, 1..3 (paper: 3)      */
    const double *bin_dirs;      /* [3K] unit vectors (|u| = 1 within 1e-12) */
    double cos_min;              /* eligibility: cosine > cos_min (paper: 0) */
    int32_t n_src;               /* number of sources                        */
    int32_t n_subcycles;         /* chemistry substeps per step, >= 1        */
    const int32_t *src_vertex;   /* [n_src] source vertex ids                */
    const double *src_rate;      /* [n_src] ionising photons per second      */
    const double *src_dir;       /* [3 n_src] or NULL.  A zero row means an
                                    isotropic source (all neighbours); a unit
                                    row makes a beam along that direction    */
    double sigma;                /* photo-ionisation cross-section (cm^2)    */
    double alpha_B;              /* case-B recombination coefficient         */
    double dt;                   /* radiative-transfer time step (s)         */
    int32_t precision;           /* SX_FP64 or SX_FP32_TRANSPORT             */
    int32_t transport;           /* SX_TRANSPORT_DCT (0) or _COMBINED        */
    int32_t dct_reference;       /* SX_DCT_REF_BIN (0) or SX_DCT_REF_EDGE    */
    double tau_switch;           /* combined transport: ballistic where
                                    y tau >= tau_switch (not NaN; +inf =
                                    never)                                   */
    double alpha_A;              /* 0: on the spot (alpha_B).  > 0 (>=
                                    alpha_B): diffuse recombination
                                    radiation, Sects. 2.2.1, 4.2: the rate
                                    equation recombines with alpha_A, and a
                                    vertex's recombinations straight to the
                                    ground level in a step, (alpha_A -
                                    alpha_B) / alpha_A of all, become photons
                                    it sends at the next step, equally to
                                    all its neighbours, filed like those of
                                    a source.  They count as emitted when
                                    made and in flight until sent            */
    int32_t hops;                /* multi-hop steps (Sect. 4.6): edges
                                    photons cross per step, 0 or 1 = one (the
                                    paper's tests).  With H > 1 every sweep
                                    is one hop of a step of dt: sources emit
                                    N_dot dt / H per hop, each vertex absorbs
                                    1 - exp(-y tau) of each hop's photons at
                                    its y of the start of the step, capped by
                                    the atoms it had neutral, and its y is
                                    updated once, after the step's last hop,
                                    from the photons it absorbed.  Direction-
                                    conserving transport with on-the-spot
                                    recombination only (else SX_ENOTSUP);
                                    at most SX_MAX_HOPS                      */
} sx_grid_desc;

/* Cumulative photon accounting of one grid (photons, double). */
typedef struct sx_tally {
    double sweeps;       /* steps done                                      */
    double emitted;      /* photons sent out by the sources                  */
    double absorbed;     /* photons absorbed (= photo-ionisations)           */
    double escaped;      /* photons that left the domain                     */
    double in_flight;    /* photons held in the outgoing field now           */
} sx_tally;

/* State read-back; every pointer is nullable (host memory, caller-owned).
 *   x, y      [N]    ionised and neutral fraction
 *   photons   [N*K]  double: O[i][k], the photons each selected neighbour of
 *                    vertex i receives in bin k at the next step (row-major,
 *                    caller's vertex order).  Bin k of vertex i holds
 *                    m(i,k) * O[i][k] photons in total.
 *   nin       [N]    photons that reached each vertex in the last step
 *   tally     accounting above                                            */
typedef struct sx_state_out {
    double *x;
    double *y;
    double *photons;
    double *nin;
    sx_tally *tally;
} sx_state_out;

/* Checkpoint restore: nullable host arrays in the layout of sx_state_out. */
typedef struct sx_state_in {
    const double *y;
    const double *photons;
    const sx_tally *tally;
} sx_state_in;

/* Create a context on opts->device (NULL opts = device 0, defaults).  The
 * context holds, besides the grids, a table of grid slots and a completion
 * counter in device memory and a 3 KiB pinned host buffer (the staging of
 * the routing rebuilds); sx_finalize frees them.
 * Errors: SX_EINVAL (bad opts), SX_EDEVICE (no such device / HIP failure).*/
int sx_init(sx_ctx **out, const sx_ctx_opts *opts);

/* Release every grid and the context.  NULL is accepted. */
int sx_finalize(sx_ctx *ctx);

/* Device bytes a grid with this description would hold (no allocation).
 * Used for admission control.  Errors: SX_EINVAL. */
int sx_grid_bytes(const sx_grid_desc *d, uint64_t *bytes);

/* Validate, reorder for locality, copy to the device, build the bin
 * selection tables and the gather lists, and initialise the state.
 * Errors: SX_EINVAL (asymmetric or malformed graph, non-finite values,
 * non-unit bins, bad source ids, unknown transport or bin reference, NaN
 * tau_switch, alpha_A neither 0 nor >= alpha_B), SX_ENOTSUP (K or degree
 * over the limits, or N K max_per_bin >= 2^31 with combined transport or
 * diffuse radiation), SX_ENOMEM (budget; nothing stays allocated),
 * SX_EDEVICE. */
int sx_grid_upload(sx_ctx *ctx, const sx_grid_desc *d, sx_grid_id *out);

/* Recompute the bin -> neighbour tables and gather lists on the device
 * (direction-conserving transport recomputes them whenever the bins
 * change, Sect. 2.2.3) and reset the state to the upload's initial one:
 * y = 1 - x_init, no photons in flight, tallies zero.  Asynchronous. */
int sx_grid_reset(sx_ctx *ctx, sx_grid_id id);

/* Restore y, photons and tallies (checkpoint).  Synchronous.  A multi-hop
 * grid (hops > 1) restarts at the beginning of a step: its steps done (from
 * the tally, or as they are) must be a multiple of hops, else SX_EINVAL. */
int sx_grid_restore(sx_ctx *ctx, sx_grid_id id, const sx_state_in *in);

/* Release one grid. */
int sx_grid_free(sx_ctx *ctx, sx_grid_id id);

/* Enqueue n_sweeps steps on each of the n grids: per step one launch for
 * each precision and transport class present among them (the class of a
 * grid with diffuse radiation is the combined-transport one), all tiles of
 * those grids in it.  Asynchronous on the context stream.
 * Errors: SX_ENOTFOUND, SX_EINVAL, SX_EDEVICE. */
int sx_step(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, int32_t n_sweeps);

/* sx_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, kernels and results (bit for bit) as sx_step, but it calls no
 * hipMalloc, hipFree or other allocating routine: its launch tables (tile
 * maps, grids to advance) and completion counter live in one static device
 * array per GPU (8 bytes per tile of SX_NOALLOC_MAX_TILES plus 8 KiB, about
 * 1 MiB; its address is looked up at sx_init and the array is held until
 * the process ends), filled by a kernel at every call, and
 * each step is one plain kernel launch per launch class (no graph).  Limits:
 * n <= SX_NOALLOC_MAX_GRIDS grids and at most SX_NOALLOC_MAX_TILES tiles of
 * 64 vertices over all of them (8.4M vertices); beyond either it returns
 * SX_EINVAL and launches nothing.  Every call on one GPU uses that GPU's
 * array: calls from different contexts or streams that overlap in time on
 * one GPU race (calls on one stream are ordered and safe).  Asynchronous on
 * the context stream.  Errors: SX_ENOTFOUND, SX_EINVAL, SX_ENOMEM (grid left
 * unusable by a rotation), SX_EDEVICE. */
#define SX_NOALLOC_MAX_GRIDS 256
#define SX_NOALLOC_MAX_TILES 131072
int sx_step_noalloc(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, int32_t n_sweeps);

/* Run grid ids[i] for n_sweeps[i] steps (grids finish independently and
 * drop out of the batch), then wait for the device. */
int sx_solve(sx_ctx *ctx, const sx_grid_id *ids, int32_t n,
             const int32_t *n_sweeps);

/* Wait for all work enqueued on the context. */
int sx_sync(sx_ctx *ctx);

/* Copy the state of one grid to host memory (synchronous). */
int sx_read_state(sx_ctx *ctx, sx_grid_id id, const sx_state_out *out);

/* Selection tables in the caller's order (synchronous), all nullable:
 *   sel_nbr  [N*K*3] neighbour ids chosen for each (vertex, bin), best
 *            first, -1 padding
 *   sel_m    [N*K]   how many were chosen
 *   edge_bin [E]     bin of each directed edge, caller's CSR order
 *   dL, tau  [N]     path length and neutral optical depth n_H sigma dL */
int sx_read_tables(sx_ctx *ctx, sx_grid_id id, int32_t *sel_nbr,
                   int32_t *sel_m, int32_t *edge_bin, double *dL,
                   double *tau);

/* Grid facts: N, K, edges, precision, the photon unit S (photons per stored
 * unit, a power of two), device bytes held. Any pointer nullable. */
int sx_grid_info(sx_ctx *ctx, sx_grid_id id, int64_t *n, int32_t *k,
                 int64_t *n_edges, int32_t *precision, double *photon_unit,
                 uint64_t *bytes);

/* Device bytes held by the context and its budget. */
int sx_mem_info(sx_ctx *ctx, uint64_t *used, uint64_t *budget);

/* The hipStream_t the context enqueues on. */
void *sx_stream(sx_ctx *ctx);

/* Kernel timing.  With enable != 0, every sweep-kernel launch made singly,
 * and every graph replay (graph_sweeps sweeps back to back), is bracketed by
 * a pair of HIP events on the context stream; sx_profile_read waits for them
 * and returns the number of sweep launches timed since the last read, their
 * total time, and the shortest and longest time per launch (a replay counts
 * as its launches, each at the replay's average, which includes the gaps
 * between its kernels) in milliseconds, then starts a new count.  Any
 * out-pointer may be NULL. */
int sx_profile(sx_ctx *ctx, int32_t enable);
int sx_profile_read(sx_ctx *ctx, int64_t *launches, double *total_ms,
                    double *min_ms, double *max_ms);

/* Rotate the direction bins of a grid to R u_k, u_k the bins given at
 * upload (R: row-major 3x3, orthonormal within 1e-9, determinant +1).  The
 * method rotates its bins over random angles between transport steps
 * against preferential directions (Sect. 2.2.3); the caller draws the
 * rotations.  The routing (selection, edge bins, bins of the source shares,
 * gather lists) is rebuilt on the device.  Photons in flight keep their
 * direction as closely as the rotated bins allow (the paper's small
 * numerical diffusion per rotation, Sect. 5.2): what a vertex holds in an
 * old bin moves to the rotated bin closest to that bin's previous direction
 * (largest cosine, ties to the lower bin; holdings that meet in one bin add
 * up in ascending old bin), is split over the neighbours selected for it
 * (kept as it is where one old bin with the same number selected feeds it),
 * and escapes where none is selected (tallied as escaped).  sx_grid_reset
 * restores the given bins.  With combined transport or diffuse radiation
 * the bin of each incoming edge and the per-edge bin lists are rebuilt too
 * (ballistic routing does not depend on the bins; what ballistic vertices
 * hold is untouched).  Synchronous.  Errors: SX_EINVAL (not a rotation),
 * SX_ENOTFOUND, SX_ENOMEM, SX_EDEVICE.  SX_ENOMEM from the per-edge bin
 * lists (their pool could not grow within the budget) leaves the grid
 * unusable: sx_step and sx_solve refuse it with SX_ENOMEM, launching
 * nothing, until sx_grid_reset rebuilds its tables (or it is freed). */
int sx_rotate_bins(sx_ctx *ctx, sx_grid_id id, const double *R);

/* ---- combined transport -------------------------------------------------
 * Per-edge state of a grid uploaded with SX_TRANSPORT_COMBINED (host
 * memory, caller-owned, nullable):
 *   photons_e [E] for edge slot p of vertex j (caller's CSR order, the edge
 *             j -> nbr_idx[p]): photons each chosen neighbour of j receives
 *             at the next step from the packet that came into j along that
 *             edge (ballistic vertices; 0 elsewhere)
 *   layout    [N] 1 where the vertex holds its photons per incoming edge
 *             (it was ballistic in the last step), 0 where it holds bins;
 *             sx_read_state reports 0 photons in the bins of layout-1
 *             vertices.
 * Synchronous.  Errors: SX_ENOTFOUND, SX_EINVAL (not a combined grid). */
int sx_read_edge_state(sx_ctx *ctx, sx_grid_id id, double *photons_e,
                       uint8_t *layout);

/* Checkpoint restore of the per-edge state in the layout above (after
 * sx_grid_restore, which restores y, bins and tallies and leaves every
 * vertex holding bins).  Synchronous.  Errors: SX_EINVAL (not a combined
 * grid, negative or non-finite photons, layout not 0/1), SX_ENOTFOUND. */
int sx_grid_restore_edges(sx_ctx *ctx, sx_grid_id id, const double *photons_e,
                          const uint8_t *layout);

/* ---- dynamic grid (Sect. 2.1.4) --------------------------------------------
 * Between solves a caller may thin the grid where the optical depth has
 * dropped: choose the vertices to remove, triangulate the rest (on the
 * host), upload the new grid with the same bins and move the state over.
 *
 * sx_grid_select_removal: vertex i is a candidate when its optical depth
 * y tau (neutral fraction now, tau = n_H sigma dL) is below tau_remove,
 * its path length dL is below min_spacing (the grid there is finer than the
 * minimum resolution) and it holds no source.  Candidates are taken in
 * ascending optical depth (ties: lower id) and kept out when a neighbour
 * has already been taken, so no two removed vertices are neighbours.
 * remove [N] (caller's order) receives 1 for removed vertices; n_removed
 * (nullable) their number.  Synchronous.  Errors: SX_EINVAL (NaN
 * thresholds), SX_ENOTFOUND. */
int sx_grid_select_removal(sx_ctx *ctx, sx_grid_id id, double tau_remove,
                           double min_spacing, uint8_t *remove, int64_t *n_removed);

/* Move the state of grid `from` onto grid `to` (the same transport, the
 * same recombination radiation, one hop per step, the same unrotated bins):
 * new_of_old [N_from] gives each old vertex's index in `to`, or -1 for a
 * removed one; every vertex of `to` must be hit once.  Kept vertices keep
 * y.  What a vertex holds in a bin, m O, stays in that bin with the vertex
 * it maps to (a removed vertex's goes to its nearest kept former neighbour,
 * ties to the lower id) and is split over that vertex's selection on the
 * new grid; where none is selected (or a removed vertex has no kept
 * neighbour) it is counted as escaped.  Combined transport: a vertex that
 * holds its photons per incoming edge first files each packet, bm O_e in
 * all, in the bin of the edge it came along (i -> j), the bin a
 * direction-conserving vertex takes it in (Sect. 2.2.4); every vertex of
 * `to` starts holding bins.  Diffuse recombination radiation: the photons
 * a vertex still has to send (sx_read_diffuse) move the same way and are
 * sent from there at the next step.  Tallies carry over (in_flight counts
 * what was moved, escaped what was not).  Synchronous.  Errors: SX_EINVAL
 * (bad map, different transport, radiation or bins), SX_ENOTSUP
 * (multi-hop steps), SX_ENOTFOUND. */
int sx_grid_remap(sx_ctx *ctx, sx_grid_id from, sx_grid_id to, const int32_t *new_of_old);

/* Diffuse recombination radiation: the photons each vertex made in the last
 * step and sends at the next one [N] (caller's order; zeros without diffuse
 * radiation).  sx_grid_restore clears them.  Synchronous. */
int sx_read_diffuse(sx_ctx *ctx, sx_grid_id id, double *pending);

/* Ballistic tables in the caller's order (nullable): bsel [E*3] the
 * neighbour ids chosen for the packet that arrives along each edge slot
 * (best first, -1 padding), bm [E] how many.  Errors as above. */
int sx_read_ballistic(sx_ctx *ctx, sx_grid_id id, int32_t *bsel, int32_t *bm);

/* ---- upload in two parts ---------------------------------------------
 * sx_grid_upload = sx_grid_prepare + sx_grid_commit.  The host part (all
 * validation, the Hilbert reorder, neighbour rows, edge geometry, tile
 * halos, per-vertex coefficients, source lists) needs no context and no
 * device and may run on any thread, concurrently; the device part runs on
 * the context's thread.  A request loop prepares on worker threads while the
 * GPU sweeps. */
typedef struct sx_prepared sx_prepared;

/* Prepare a grid on the host.  On failure returns the SX_E* code of
 * sx_grid_upload and, if err is not NULL, a message in err[0..err_len). */
int sx_grid_prepare(const sx_grid_desc *d, sx_prepared **out, char *err, size_t err_len);

/* Device bytes the prepared grid is expected to take (admission control). */
int sx_prepared_bytes(const sx_prepared *p, uint64_t *bytes);

/* Upload a prepared grid.  p is consumed on success (it may then only be
 * freed).  When the budget check refuses it (SX_ENOMEM, nothing allocated)
 * it stays usable and may be committed later; sx_prepared_bytes tells
 * (SX_EINVAL once p is consumed).  Errors: as sx_grid_upload. */
int sx_grid_commit(sx_ctx *ctx, sx_prepared *p, sx_grid_id *out);

/* Release a prepared grid (committed or not).  NULL is accepted. */
int sx_prepared_free(sx_prepared *p);

/* ---- sweep schedule --------------------------------------------------
 * How the sweeps of a step are launched.  A schedule only changes the order
 * in which independent 64-vertex tiles run (each tile's arithmetic and every
 * sum order are fixed), so results are bitwise the same under every
 * schedule.
 *   tiles_per_group  tiles per workgroup: 1, 2 or 4
 *   work_split       waves per tile: 1, 2 or 4, with tiles_per_group x
 *                    work_split <= 4 (0 reads as 1).  The waves of a tile
 *                    split its direction bins into contiguous ranges and
 *                    one of them runs the chemistry; more, shorter waves
 *                    fill the GPU better when a launch has few tiles.
 *                    Combined-transport launches always use 1.
 *   order            SX_ORDER_GRID: grid by grid, each in its internal
 *                    (Hilbert) order; SX_ORDER_DIRECT_FIRST: tiles too large
 *                    for LDS staging first, then the rest
 *   xcd_contiguous   1: each of the 8 XCDs runs a contiguous eighth of the
 *                    tile list (its L2 sees one neighbourhood); 0: the
 *                    hardware's round-robin
 *   graph_sweeps     > 0: sweeps are launched as replays of one HIP graph of
 *                    that many sweeps (the rest singly); 0: one launch per
 *                    sweep and precision
 * Default {4, SX_ORDER_GRID, 1, 50, 1}. */
#define SX_ORDER_GRID 0
#define SX_ORDER_DIRECT_FIRST 1
#define SX_MAX_GRAPH_SWEEPS 4096
typedef struct sx_schedule {
    int32_t tiles_per_group;
    int32_t order;
    int32_t xcd_contiguous;
    int32_t graph_sweeps;
    int32_t work_split;
} sx_schedule;

/* Schedule for steps over exactly this list of grids, in this order (n = 0:
 * the default for every list without its own).  Synchronous.  Errors:
 * SX_EINVAL (invalid schedule), SX_ENOTFOUND. */
int sx_set_schedule(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, const sx_schedule *s);

/* The schedule a step over this list uses (n = 0: the default), and the
 * autotuner's time per sweep in microseconds for it (0 if not tuned);
 * us_per_sweep may be NULL. */
int sx_get_schedule(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, sx_schedule *out,
                    double *us_per_sweep);

/* trials > 0 turns the autotuner on: the first sx_step / sx_solve over a grid
 * list that has no schedule of its own, if it asks for at least 4 x trials x
 * (number of candidates) sweeps, runs `trials` of those sweeps under each
 * candidate schedule, timed with HIP events, in two stages: the launch shape
 * (tiles per group 1, 2, 4 and work split 1, 2, 4, at most 4 waves per
 * group; 6 candidates) in XCD-contiguous grid order, then for the fastest
 * shape the other tile orders (XCD round-robin, and direct tiles first when
 * the list has any; 1 or 3 candidates), and
 * keeps the fastest for that list (graph_sweeps is kept from the default).
 * The sweeps count toward the step; the step synchronises the stream while
 * tuning.  trials = 0 turns it off.  Errors: SX_EINVAL (trials outside
 * [0, 64]). */
int sx_autotune(sx_ctx *ctx, int32_t trials);

/* ---- serving ----------------------------------------------------------
 * A request loop with continuous batching over one context.  Requests
 * (sx_serve_submit, any thread) are copied, prepared on prep_threads host
 * threads, and admitted in arrival order between rounds as the HBM budget
 * (hbm_budget, 0 = the context's) and max_active allow.  A round runs up to
 * round_sweeps sweeps over every resident grid as one batch (each grid only
 * the sweeps it still needs, under the context's schedule); grids that are
 * done are read back into the server and freed, making room for the next
 * admissions.  Each result equals the result of solving that grid alone.
 * While serving, the context belongs to the server's thread: the caller must
 * not use it until sx_serve_stop returns. */
typedef struct sx_server sx_server;

typedef struct sx_serve_opts {
    int32_t round_sweeps;   /* sweeps per round; 0 = 50                       */
    int32_t max_active;     /* grids resident at once; 0 = 64 (<= 1024)        */
    int32_t prep_threads;   /* host threads preparing uploads; 0 = 4 (<= 64)   */
    int32_t reserved;
    uint64_t hbm_budget;    /* admission limit in bytes; 0 = context budget    */
} sx_serve_opts;

typedef struct sx_serve_result {
    int64_t ticket;
    int32_t status;         /* SX_OK or the request's error                   */
    int32_t n_bins;
    int64_t n_vertices;
    int32_t n_sweeps;
    int32_t reserved;
    double t_submit, t_prepared, t_admit, t_done;  /* s since sx_serve_start */
    sx_tally tally;
} sx_serve_result;

typedef struct sx_serve_stats {
    int64_t finished, failed, rounds;
    int32_t peak_active, reserved;
    double updates;         /* vertex-direction updates of finished requests  */
    double span_s;          /* first admission to last completion             */
    double round_s;         /* time inside rounds (GPU sweeps + their sync)   */
    double latency_p50_s, latency_p99_s, latency_max_s;  /* submit -> done   */
} sx_serve_stats;

/* Start the loop on ctx.  Errors: SX_EINVAL. */
int sx_serve_start(sx_ctx *ctx, const sx_serve_opts *opts, sx_server **out);

/* Queue a request: the description is copied during the call.  *ticket
 * identifies it.  Errors: SX_EINVAL (malformed, or the server is
 * stopping).  Validation errors of the grid itself come back as the
 * result's status. */
int sx_serve_submit(sx_server *s, const sx_grid_desc *d, int32_t n_sweeps, int64_t *ticket);

/* Wait up to timeout_s seconds for the next finished request (in completion
 * order) and describe it in *res.  Returns SX_OK or SX_EAGAIN. */
int sx_serve_poll(sx_server *s, double timeout_s, sx_serve_result *res);

/* Copy a polled request's x and y [N] (caller order; either may be NULL)
 * and release them.  Errors: SX_ENOTFOUND (not polled, or already taken). */
int sx_serve_take(sx_server *s, int64_t ticket, double *x, double *y);

/* Finish every queued request, stop the threads, fill *st (nullable), and
 * release the server; results not taken are dropped.  NULL is accepted. */
int sx_serve_stop(sx_server *s, sx_serve_stats *st);

const char *sx_strerror(int code);
const char *sx_last_error(const sx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* SX_H */
