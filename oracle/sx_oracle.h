/*
 * sx_oracle.h -- CPU reference ("oracle") for SimpleX2 direction-conserving
 * photon transport with on-the-spot hydrogen photo-ionisation chemistry.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential FP64
 * implementation written to be checked against the paper by eye.  It is
 * called by the test-suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark; the product library never links or calls it, and it shares
 * no code, header or table with the GPU library.
 *
 * Paper: Paardekooper, Kruip & Icke (2010), "SimpleX2: radiative transfer on
 * an unstructured, dynamic grid", A&A (arXiv:0912.4273).
 *
 * Conventions: vertices, neighbour rows and bins are used in the order the
 * caller gives them.  Units are CGS.  All arithmetic is IEEE double.
 */
#ifndef SX_ORACLE_H
#define SX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_grid ora_grid;

/* Build the oracle state for one grid.  Arrays are copied.  src_dir may be
 * NULL (every source isotropic); a row of zeros also means isotropic.
 * dL may be NULL (then dL_i = kappa * mean incident edge length).
 * x_init may be NULL (then x = 0, fully neutral).  Returns NULL on invalid
 * input (message in ora_last_error()). */
ora_grid *ora_create(int64_t n, const double *pos, const int64_t *nbr_ptr,
                     const int32_t *nbr_idx, const double *n_H,
                     const double *volume, const double *dL, double kappa,
                     const double *x_init, int32_t n_bins,
                     const double *bin_dirs, int32_t max_per_bin,
                     double cos_min, int32_t n_src, const int32_t *src_vertex,
                     const double *src_rate, const double *src_dir,
                     double sigma, double alpha_B, double dt,
                     int32_t n_subcycles);

/* Run n_sweeps sweeps.  history (nullable, [n_sweeps*4]) receives the
 * cumulative tallies emitted, absorbed, escaped, in_flight after each sweep. */
int ora_run(ora_grid *g, int32_t n_sweeps, double *history);

/* Timing only (the CPU baseline on all cores): the same sweeps of
 * direction-conserving transport with on-the-spot chemistry as ora_run, in
 * pull form over `threads` OpenMP threads; fields as ora_run, the tallies
 * summed in another order.  Returns -1 for combined transport or diffuse
 * radiation. */
int ora_run_threads(ora_grid *g, int32_t n_sweeps, int32_t threads);

/* Copy out the state.  Any pointer may be NULL.
 *   y, x        [N]   neutral and ionised fraction
 *   photons     [N*K] outgoing photons per selected neighbour, O[j][k]
 *   nin         [N]   photons that entered each vertex in the last sweep
 *   tallies     [5]   sweeps, emitted, absorbed, escaped, in_flight */
void ora_get_state(const ora_grid *g, double *y, double *x, double *photons,
                   double *nin, double *tallies);

/* Replace y (neutral fraction) and O (photons, [N*K]) -- checkpoint restore.
 * Either may be NULL. tallies (nullable, [5]) restores the counters. */
void ora_set_state(ora_grid *g, const double *y, const double *photons,
                   const double *tallies);

/* Rotate the direction bins to R u_k (u_k as given at creation; R a
 * row-major 3x3 rotation) and recompute the routing.  The photons each
 * vertex holds in a bin move to the rotated bin nearest that bin's previous
 * direction (summed where several arrive) and are split over its new
 * selection (escaping where none is selected). */
int ora_rotate(ora_grid *g, const double *R);

/* Selection tables.  sel_nbr [N*K*max_per_bin] neighbour vertex ids (best
 * first, -1 padding), sel_m [N*K], edge_bin [E] (bin of each directed edge
 * in the caller's CSR order), dL [N], tau [N] (n_H sigma dL).  Nullable. */
void ora_get_tables(const ora_grid *g, int32_t *sel_nbr, int32_t *sel_m,
                    int32_t *edge_bin, double *dL, double *tau);

/* Diffuse recombination radiation (Sects. 2.2.1, 4.2).  alpha_A > 0
 * (>= alpha_B): the rate equation recombines with alpha_A, and each sweep's
 * recombinations straight to the ground level, (alpha_A - alpha_B)/alpha_A
 * of all, become photons that the vertex sends at the next sweep, equally
 * to all its neighbours (filed like those of a source).  They count as
 * emitted when produced and in flight until sent.  alpha_A = 0: on the spot
 * (alpha_B, no diffuse photons).  Returns 0, or -1 for a bad argument. */
int ora_set_diffuse(ora_grid *g, double alpha_A);

/* Recombination photons produced in the last sweep, to be sent in the next
 * one [N] (zeros while off); and their restore. */
void ora_get_diffuse(const ora_grid *g, double *pending);
void ora_set_diffuse_pending(ora_grid *g, const double *pending);

/* Reference direction of the bin selection: edge = 0 (default) the bin's
 * own direction u_k; edge = 1 the vertex's Delaunay edge closest to u_k
 * (largest cosine, > cos_min, ties to the lower id): the bin then goes to
 * the neighbours most aligned with that edge.  Rebuilds the routing; call
 * before the first sweep.  Returns 0, or -1 for a bad argument. */
/* Multi-hop steps (Sect. 4.6): hops per step, >= 1 (1: one edge per step,
 * the paper's tests).  With hops H > 1 every sweep is one hop; sources emit
 * N_dot dt / H per hop; each vertex absorbs at the neutral fraction of the
 * start of the step, capped by the atoms it had neutral, and its neutral
 * fraction is updated once, after the step's last hop, from the photons it
 * absorbed (ionisations = absorbed photons).  Direction-conserving,
 * on-the-spot grids only.  Returns 0, or -1 (ora_last_error). */
int ora_set_hops(ora_grid *g, int32_t hops);

int ora_set_dct_reference(ora_grid *g, int32_t edge);

/* Combined transport (Sects. 2.2.2-2.2.4).  combined = 1: from the next
 * sweep on, every vertex whose optical depth y tau is at least tau_switch at
 * the start of a sweep uses ballistic transport (photons held per incoming
 * edge, sent on to the <= max_per_bin neighbours most aligned with that
 * edge), the others direction-conserving transport; tau_switch <= 0 makes
 * every vertex ballistic.  combined = 0: direction-conserving everywhere.
 * Returns 0, or -1 for a bad argument. */
int ora_set_transport(ora_grid *g, int32_t combined, double tau_switch);

/* Per-edge state of combined transport (nothing happens while combined is
 * 0).  photons_e [E]: for edge slot e of vertex j (caller's CSR order), the
 * photons each chosen neighbour of j receives next step from the packet that
 * came into j along that edge; layout [N]: 0 = the vertex holds bins
 * (photons of ora_get_state), 1 = edges. */
void ora_get_edge_state(const ora_grid *g, double *photons_e, int8_t *layout);
void ora_set_edge_state(ora_grid *g, const double *photons_e, const int8_t *layout);

/* Ballistic tables: bsel [E*max_per_bin] the neighbour ids chosen for the
 * packet arriving along each edge slot (best first, -1 padding), bm [E] how
 * many. */
void ora_get_ballistic(const ora_grid *g, int32_t *bsel, int32_t *bm);

void ora_free(ora_grid *g);

/* One vertex, one radiative-transfer step of length dt: n_sub backward-Euler
 * subcycles of the rate equation with a constant incoming photon flux
 * n_in/dt.  nHV = n_H * V (atoms in the cell), tau = n_H sigma dL (optical
 * depth of the fully neutral cell), b = alpha_B n_H.  Returns the new neutral
 * fraction; *absorbed and *transmitted receive the photons absorbed and
 * passed on. */
double ora_chem_cell(double y, double n_in, double dt, double nHV, double tau,
                     double b, int32_t n_sub, double *absorbed,
                     double *transmitted);

const char *ora_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
