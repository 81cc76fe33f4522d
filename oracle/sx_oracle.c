/*
 * sx_oracle.c -- CPU reference ("oracle") for SimpleX2 direction-conserving
 * transport with on-the-spot hydrogen chemistry.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  The product library never uses it.
 *
 * Plain sequential FP64, compiled with -ffp-contract=off.  Every loop runs in
 * a fixed order: vertex ascending, bin ascending, neighbour slot ascending,
 * source ascending.  Each step cites the passage of Paardekooper, Kruip &
 * Icke (2010) it follows; where the paper leaves a detail open the chosen
 * reading is stated next to the code.
 */
#include "sx_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[256];
const char *ora_last_error(void) { return g_err; }

struct ora_grid {
    int64_t n;
    int64_t n_edges;
    int32_t K, mpb;
    double cos_min, sigma, alpha_B, dt;
    int32_t n_sub;
    int64_t *ptr;        /* [N+1] */
    int32_t *nbr;        /* [E]   */
    double *edir;        /* [E*3] unit edge vectors (Sect. 2.2) */
    double *elen;        /* [E]   edge lengths */
    double *bins;        /* [K*3] current bin directions */
    double *bins0;       /* [K*3] bin directions given at creation */
    double *nH, *vol, *dL, *tau; /* [N] */
    int32_t *sel;        /* [N*K*mpb] selected neighbour ids, best first */
    int32_t *m;          /* [N*K] number selected */
    int32_t *ebin;       /* [E] bin of each directed edge */
    int32_t n_src;
    int32_t *src_v;
    double *src_rate;
    double *src_dir;     /* [S*3], zero row = isotropic */
    double *y;           /* [N] neutral fraction */
    double *O;           /* [N*K] outgoing photons per selected neighbour */
    double *I;           /* [N*K] scratch: incoming photons */
    double *nin;         /* [N] last sweep's incoming photons */
    double sweeps, emitted, absorbed, escaped, in_flight;
    /* Combined transport (Sect. 2.2.4); unused while combined == 0. */
    int32_t combined;
    double tau_switch;   /* ballistic where y tau >= tau_switch */
    int32_t *rev;        /* [E] slot of i in the row of j, for edge i -> j */
    int32_t *bsel;       /* [E*mpb] ballistic choice for the packet that came
                            into the row's vertex along the slot's edge */
    int32_t *bm;         /* [E] number chosen */
    double *Oe;          /* [E] outgoing photons per chosen neighbour of each
                            incoming packet of a ballistic vertex */
    double *Ie;          /* [E] scratch: photons in, per incoming edge */
    int8_t *layout;      /* [N] 0: vertex holds bins (O), 1: edges (Oe) */
    int8_t *mode;        /* [N] scratch: this sweep's mode */
    int32_t dct_ref;     /* 0: bins go by their own direction; 1: by the
                            vertex's edge closest to the bin */
    /* Diffuse recombination radiation (Sects. 2.2.1, 4.2); off while
     * alpha_A == 0 (on the spot). */
    double alpha_A;
    double *D;           /* [N] recombination photons to send next sweep */
    /* Multi-hop steps (Sect. 4.6); one hop per step while hops <= 1. */
    int32_t hops;
    double *habs;        /* [N] photons absorbed so far in the current step */
    double *hnin;        /* [N] photons that arrived so far in the step */
    /* Timing-only pull form (ora_run_threads): senders of each receiver,
     * built on first use from the current routing; NULL when stale. */
    int64_t *pull_ptr;
    int32_t *pull_from, *pull_bin;
};

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    return p;
}

/* ---------------------------------------------------------------------- */
/* Direction cosine of a unit edge vector with a unit direction: the
 * "straightforwardness" used to rank neighbours (Sect. 2.2.2-2.2.3).
 * Evaluated as ((ex*ux + ey*uy) + ez*uz) with no fused multiply-add. */
static double cosine(const double *e, const double *u) {
    double a = e[0] * u[0];
    double b = e[1] * u[1];
    double c = e[2] * u[2];
    return (a + b) + c;
}

/* The <= mpb neighbours of vertex i most aligned with direction u, keeping
 * only those with cosine > cos_min (photons never travel backwards: the 90
 * degree cone of Sect. 2.2.2).  Ties go to the lower neighbour id.  Writes
 * the chosen slots (row positions) into out, returns how many. */
static int select_slots(const ora_grid *g, int64_t i, const double *u,
                        int32_t *out) {
    int64_t b = g->ptr[i], deg = g->ptr[i + 1] - g->ptr[i];
    int cnt = 0;
    for (int r = 0; r < g->mpb; r++) {
        int64_t best = -1;
        double cb = 0.0;
        for (int64_t s = 0; s < deg; s++) {
            double c = cosine(&g->edir[3 * (b + s)], u);
            if (!(c > g->cos_min)) continue;
            int taken = 0;
            for (int q = 0; q < cnt; q++) if (out[q] == s) taken = 1;
            if (taken) continue;
            if (best < 0 || c > cb ||
                (c == cb && g->nbr[b + s] < g->nbr[b + best])) {
                best = s;
                cb = c;
            }
        }
        if (best < 0) break;
        out[cnt++] = (int32_t)best;
    }
    return cnt;
}

/* The bin whose direction is closest to the unit direction d (largest
 * cosine, ties to the lower bin): where photons of a known direction of
 * travel are filed (Sect. 2.2.4 for photons arriving along an edge; a beam's
 * photons travel along the beam). */
static int32_t nearest_bin(const ora_grid *g, const double *d) {
    int32_t best = 0;
    double cb = cosine(d, &g->bins[0]);
    for (int32_t k = 1; k < g->K; k++) {
        double c = cosine(d, &g->bins[3 * k]);
        if (c > cb) { cb = c; best = k; }
    }
    return best;
}

/* ---------------------------------------------------------------------- */
/* Chemistry of one vertex over one transport step (Sect. 4.5).
 *
 * The rate equation dn_HII/dt = n_HI Gamma - n_e n_HII alpha_B (Eq. rate_eq,
 * on-the-spot, pure hydrogen so n_e = n_HII, no collisional ionisation) is
 * subcycled with the photo-ionisation rate rescaled so that the incoming
 * photon flux n_in/dt stays constant over the step (Eqs. rate_eq_subcycle,
 * phot_ion_rate_subcycle).  With y the neutral fraction and tau the optical
 * depth of the fully neutral cell, the ionisations per atom per second are
 * a (1 - exp(-y tau)) with a = n_in / (dt n_H V), recombinations per atom per
 * second are b (1 - y)^2 with b = alpha_B n_H.
 *
 * Reading of the subcycle step (the paper fixes neither the step nor the
 * integrator): n_sub equal substeps h = dt/n_sub, each backward Euler in y,
 *     y' = y - h a (1 - exp(-y' tau)) + h b (1 - y')^2 ,
 * which is stable for any h, keeps the equilibrium points of the rate
 * equation, and absorbs exactly as many photons as it ionises atoms.  The
 * substep equation G(y') = 0 is monotone decreasing in y' on [0,1] with
 * G(0) >= 0 >= G(1); it is solved by Newton's method from y' = y inside that
 * bracket, falling back to bisection when a Newton step leaves it. */
static double be_substep(double y0, double ha, double hb, double tau) {
    double lo = 0.0, hi = 1.0, yn = y0;
    for (int it = 0; it < 200; it++) {
        double ion = -expm1(-yn * tau);          /* 1 - exp(-y tau) */
        double x = 1.0 - yn;
        double g = (y0 - yn) - ha * ion + hb * (x * x);
        if (g == 0.0) return yn;
        if (g > 0.0) lo = yn; else hi = yn;
        double gp = -1.0 - ha * tau * exp(-yn * tau) - 2.0 * hb * x;
        double d = g / gp;
        /* Newton has converged when its step is within rounding of y */
        if (fabs(d) <= 4.0e-16 * yn) {
            double yc = yn - d;
            return yc < 0.0 ? 0.0 : (yc > 1.0 ? 1.0 : yc);
        }
        double yc = yn - d;
        if (!(yc > lo && yc < hi)) yc = 0.5 * (lo + hi);
        yn = yc;
        if (hi - lo <= 4.0e-16 * hi) break;
    }
    return yn;
}

/* Returns the new y; *A = photons absorbed (= atoms ionised, summed over the
 * substeps), *T = fraction of the incoming photons passed on, the mean over
 * the substeps of exp(-y' tau) (Eqs. intensity_absorbed, intensity_out, with
 * the optical depth of Eq. optical_depth re-evaluated every substep). */
static double chem(double y, double n_in, double dt, double nHV, double tau,
                   double b, int n_sub, double *A, double *T, double *Rsum) {
    double h = dt / (double)n_sub;
    double a = n_in / (dt * nHV);
    double ha = h * a, hb = h * b;
    double abs_sum = 0.0, tr_sum = 0.0, rec_sum = 0.0;
    double share = n_in / (double)n_sub;
    for (int s = 0; s < n_sub; s++) {
        y = be_substep(y, ha, hb, tau);
        abs_sum += share * (-expm1(-y * tau));
        tr_sum += exp(-y * tau);
        /* recombinations per atom in the substep, the b term of the
         * backward-Euler update */
        double x = 1.0 - y;
        rec_sum += hb * (x * x);
    }
    *A = abs_sum;
    *T = (n_in > 0.0) ? tr_sum / (double)n_sub : 1.0;
    if (Rsum) *Rsum = rec_sum;
    return y;
}

/* Multi-hop steps (Sect. 4.6: the subcycled chemistry allows a radiative
 * transfer step in which photons cross more than one Delaunay edge; the
 * paper's tests do not do it and the paper does not fix the scheme).
 * Reading: a step of dt is H hops.  Photons move one edge per hop, sources
 * emit N_dot dt / H per hop, and the neutral fraction y of a vertex is
 * updated once, after the last hop.  During the step a vertex absorbs from
 * each hop's photons the fraction 1 - exp(-y tau) of Eq. intensity_absorbed
 * with y frozen at its value at the start of the step, but never more atoms
 * than it had neutral at the start (n_H V y, less what it absorbed in the
 * earlier hops of the step); the rest goes on (Eq. intensity_out).  After
 * the last hop the absorbed photons ionise exactly as many atoms, spread
 * evenly over the n_sub substeps, and the recombinations are taken backward
 * Euler per substep:
 *     y' = y - i + h b (1 - y')^2,  i = A / (n_H V n_sub),
 * whose root in [0, 1] is y' = 1 - z with z = 2c / (1 + sqrt(1 + 4 h b c)),
 * c = 1 - y + i (z = c when h b = 0).  Photons are conserved exactly
 * (absorbed = ionisations), and y' >= 0 since A <= n_H V y. */
static double chem_fixed(double y, double ion, double hb, int n_sub) {
    double is = ion / (double)n_sub;
    for (int s = 0; s < n_sub; s++) {
        double c = (1.0 - y) + is;
        double z = hb > 0.0 ? (2.0 * c) / (1.0 + sqrt(1.0 + 4.0 * hb * c)) : c;
        y = 1.0 - z;
        if (y < 0.0) y = 0.0;
    }
    return y;
}

double ora_chem_cell(double y, double n_in, double dt, double nHV, double tau,
                     double b, int32_t n_sub, double *absorbed,
                     double *transmitted) {
    double A, T;
    double yn = chem(y, n_in, dt, nHV, tau, b, n_sub, &A, &T, NULL);
    if (absorbed) *absorbed = A;
    if (transmitted) *transmitted = n_in * T;
    return yn;
}

/* ---------------------------------------------------------------------- */
/* The routing of direction-conserving transport for the current bins:
 * which neighbours each bin of each vertex goes to, and the bin of every
 * directed edge. */
static void drop_pull(ora_grid *g) {
    free(g->pull_ptr); free(g->pull_from); free(g->pull_bin);
    g->pull_ptr = NULL; g->pull_from = NULL; g->pull_bin = NULL;
}

static void build_routing(ora_grid *g) {
    int64_t n = g->n, K = g->K, E = g->n_edges;
    drop_pull(g);
    int max_per_bin = g->mpb;
    /* Direction-bin -> neighbour selection of direction-conserving transport
     * (Sect. 2.2.3): every bin goes to the mpb (= dimension d = 3) most
     * straightforward neighbours w.r.t. the bin's own direction, or (the
     * reading of the caption of the figure of the three transport modes)
     * w.r.t. the vertex's Delaunay edge closest to the bin: the edge with
     * the largest cosine to u_k, which must exceed cos_min, ties to the
     * lower neighbour id. */
    for (int64_t i = 0; i < n; i++) {
        for (int64_t k = 0; k < K; k++) {
            int32_t slots[16];
            const double *ref = &g->bins[3 * k];
            int c = 0;
            if (g->dct_ref) {
                int64_t b = g->ptr[i], best = -1;
                double cb = g->cos_min;
                for (int64_t s = 0; s < g->ptr[i + 1] - b; s++) {
                    double cs = cosine(&g->edir[3 * (b + s)], ref);
                    if (cs > cb || (best >= 0 && cs == cb && g->nbr[b + s] < g->nbr[b + best])) {
                        cb = cs;
                        best = s;
                    }
                }
                if (best >= 0) c = select_slots(g, i, &g->edir[3 * (b + best)], slots);
            } else {
                c = select_slots(g, i, ref, slots);
            }
            int32_t *dst = &g->sel[(i * K + k) * max_per_bin];
            for (int r = 0; r < max_per_bin; r++)
                dst[r] = r < c ? g->nbr[g->ptr[i] + slots[r]] : -1;
            g->m[i * K + k] = c;
        }
    }

    /* Bin of each directed edge: photons sent along an edge are filed in
     * the solid angle whose direction is closest to the edge (Sect. 2.2.4);
     * ties go to the lower bin. */
    for (int64_t e = 0; e < E; e++) g->ebin[e] = nearest_bin(g, &g->edir[3 * e]);
}

ora_grid *ora_create(int64_t n, const double *pos, const int64_t *nbr_ptr,
                     const int32_t *nbr_idx, const double *n_H,
                     const double *volume, const double *dL, double kappa,
                     const double *x_init, int32_t n_bins,
                     const double *bin_dirs, int32_t max_per_bin,
                     double cos_min, int32_t n_src, const int32_t *src_vertex,
                     const double *src_rate, const double *src_dir,
                     double sigma, double alpha_B, double dt,
                     int32_t n_subcycles) {
    g_err[0] = 0;
    if (n <= 0 || n_bins <= 0 || max_per_bin <= 0 || n_subcycles <= 0 ||
        !(dt > 0.0) || n_src < 0) {
        snprintf(g_err, sizeof g_err, "bad sizes");
        return NULL;
    }
    ora_grid *g = (ora_grid *)xcalloc(1, sizeof *g);
    g->n = n;
    g->n_edges = nbr_ptr[n];
    g->K = n_bins;
    g->mpb = max_per_bin;
    g->cos_min = cos_min;
    g->sigma = sigma;
    g->alpha_B = alpha_B;
    g->dt = dt;
    g->n_sub = n_subcycles;
    int64_t E = g->n_edges, K = n_bins;
    g->ptr = (int64_t *)xcalloc(n + 1, sizeof(int64_t));
    memcpy(g->ptr, nbr_ptr, (n + 1) * sizeof(int64_t));
    g->nbr = (int32_t *)xcalloc(E, sizeof(int32_t));
    memcpy(g->nbr, nbr_idx, E * sizeof(int32_t));
    g->bins = (double *)xcalloc(K * 3, sizeof(double));
    memcpy(g->bins, bin_dirs, K * 3 * sizeof(double));
    g->bins0 = (double *)xcalloc(K * 3, sizeof(double));
    memcpy(g->bins0, bin_dirs, K * 3 * sizeof(double));
    g->nH = (double *)xcalloc(n, sizeof(double));
    g->vol = (double *)xcalloc(n, sizeof(double));
    memcpy(g->nH, n_H, n * sizeof(double));
    memcpy(g->vol, volume, n * sizeof(double));
    g->dL = (double *)xcalloc(n, sizeof(double));
    g->tau = (double *)xcalloc(n, sizeof(double));
    g->edir = (double *)xcalloc(E * 3, sizeof(double));
    g->elen = (double *)xcalloc(E, sizeof(double));
    g->sel = (int32_t *)xcalloc(n * K * max_per_bin, sizeof(int32_t));
    g->m = (int32_t *)xcalloc(n * K, sizeof(int32_t));
    g->ebin = (int32_t *)xcalloc(E, sizeof(int32_t));
    g->y = (double *)xcalloc(n, sizeof(double));
    g->O = (double *)xcalloc(n * K, sizeof(double));
    g->I = (double *)xcalloc(n * K, sizeof(double));
    g->nin = (double *)xcalloc(n, sizeof(double));
    g->n_src = n_src;
    g->src_v = (int32_t *)xcalloc(n_src, sizeof(int32_t));
    g->src_rate = (double *)xcalloc(n_src, sizeof(double));
    g->src_dir = (double *)xcalloc(n_src * 3, sizeof(double));
    if (n_src) {
        memcpy(g->src_v, src_vertex, n_src * sizeof(int32_t));
        memcpy(g->src_rate, src_rate, n_src * sizeof(double));
        if (src_dir) memcpy(g->src_dir, src_dir, n_src * 3 * sizeof(double));
    }

    /* Edge geometry: unit vector and length of every directed Delaunay edge
     * i -> j (Sect. 2.2: photons travel along the edges). */
    for (int64_t i = 0; i < n; i++) {
        double sum = 0.0;
        int64_t deg = g->ptr[i + 1] - g->ptr[i];
        for (int64_t e = g->ptr[i]; e < g->ptr[i + 1]; e++) {
            int32_t j = g->nbr[e];
            double dx = pos[3 * j + 0] - pos[3 * i + 0];
            double dy = pos[3 * j + 1] - pos[3 * i + 1];
            double dz = pos[3 * j + 2] - pos[3 * i + 2];
            double xx = dx * dx, yy = dy * dy, zz = dz * dz;
            double len = sqrt((xx + yy) + zz);
            g->edir[3 * e + 0] = dx / len;
            g->edir[3 * e + 1] = dy / len;
            g->edir[3 * e + 2] = dz / len;
            g->elen[e] = len;
            sum += len;
        }
        /* Path length through the cell (Sect. 4.4, Eq. optical_depth): a
         * grid property fixed when the grid is made.  Reading: the mean
         * length of the incident Delaunay edges times the global path-length
         * correction factor kappa of Sect. 2.2.3, unless given. */
        if (dL) g->dL[i] = dL[i];
        else g->dL[i] = deg > 0 ? kappa * (sum / (double)deg) : 0.0;
        /* Optical depth of the fully neutral cell, n_H sigma dL; the
         * printed second form of Eq. optical_depth omits sigma. */
        g->tau[i] = (g->nH[i] * sigma) * g->dL[i];
        g->y[i] = x_init ? 1.0 - x_init[i] : 1.0;
    }

    build_routing(g);
    return g;
}

/* ---------------------------------------------------------------------- */
/* Diffuse recombination radiation (Sects. 2.2.1, 4.2).  Off the spot, the
 * rate equation recombines with alpha_A (all levels); the recombinations
 * straight to the ground level, the share (alpha_A - alpha_B) / alpha_A of
 * them, emit ionising photons.  A vertex's such photons of one step leave it
 * in the next step, split equally over all its neighbours (isotropic
 * re-emission), and are filed by the receivers like those of a source.  They
 * count as emitted when produced and as in flight until sent. */
static double recomb_coeff(const ora_grid *g) {
    return g->alpha_A > 0.0 ? g->alpha_A : g->alpha_B;
}

/* Photons produced by the recombinations of vertex j in this sweep (Rsum:
 * recombinations per atom). */
static void diffuse_made(ora_grid *g, int64_t j, double Rsum) {
    if (g->alpha_A <= 0.0) return;
    double Dj = (g->nH[j] * g->vol[j]) * Rsum * ((g->alpha_A - g->alpha_B) / g->alpha_A);
    g->D[j] = Dj;
    g->emitted += Dj;
}

static void deliver(ora_grid *g, int64_t e, int32_t b, double v);

/* Send last sweep's recombination photons: each vertex to all neighbours. */
static void diffuse_send(ora_grid *g) {
    if (g->alpha_A <= 0.0) return;
    for (int64_t i = 0; i < g->n; i++) {
        double Di = g->D[i];
        if (Di == 0.0) continue;
        g->D[i] = 0.0;
        int64_t b = g->ptr[i], deg = g->ptr[i + 1] - g->ptr[i];
        if (deg == 0) { g->escaped += Di; continue; }
        double share = Di / (double)deg;
        for (int64_t e = b; e < b + deg; e++) {
            if (g->combined) deliver(g, e, g->ebin[e], share);
            else g->I[(int64_t)g->nbr[e] * g->K + g->ebin[e]] += share;
        }
    }
}

static double pending_diffuse(const ora_grid *g) {
    double f = 0.0;
    if (g->alpha_A > 0.0)
        for (int64_t j = 0; j < g->n; j++) f += g->D[j];
    return f;
}

/* ---------------------------------------------------------------------- */
/* One radiative-transfer time step: photons move one Delaunay edge and
 * interact once, at the vertex they arrive at (Sect. 4.6). */
static void sweep(ora_grid *g) {
    int64_t n = g->n, K = g->K;
    int mpb = g->mpb;
    memset(g->I, 0, (size_t)(n * K) * sizeof(double));

    /* Transport: every bin of every vertex is handed to its selected
     * neighbours, keeping its bin (direction-conserving transport).  O
     * already holds the share of each selected neighbour. */
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = 0; k < K; k++) {
            int32_t mm = g->m[i * K + k];
            double v = g->O[i * K + k];
            const int32_t *s = &g->sel[(i * K + k) * mpb];
            for (int t = 0; t < mm; t++) g->I[(int64_t)s[t] * K + k] += v;
        }

    /* Sources: a source is a vertex that sends its photons N_dot dt to all
     * its neighbours (Sects. 2.2, 4.3); each receiver files them in the bin
     * of the edge they came along (Sect. 2.2.4).  The source itself does
     * not absorb them.  A source with a direction emits a beam instead: the
     * photons are split over the neighbours selected for that direction by
     * the rule used for bins (used for a plane-parallel front), and every
     * receiver files them in the bin closest to the beam's direction, the
     * direction they travel in (reading: the bin of the edge would turn a
     * collimated beam into a fan of edge directions). */
    /* which hop of the step this sweep is (multi-hop steps) */
    int32_t H = g->hops > 1 ? g->hops : 1;
    int32_t hop = (int32_t)fmod(g->sweeps, (double)H);
    for (int32_t s = 0; s < g->n_src; s++) {
        int64_t v = g->src_v[s];
        double E = g->src_rate[s] * g->dt;
        if (H > 1) E = E / (double)H;
        g->emitted += E;
        const double *d = &g->src_dir[3 * s];
        int64_t b = g->ptr[v], deg = g->ptr[v + 1] - g->ptr[v];
        if (d[0] == 0.0 && d[1] == 0.0 && d[2] == 0.0) {
            if (deg == 0) { g->escaped += E; continue; }
            double share = E / (double)deg;
            for (int64_t e = b; e < b + deg; e++)
                g->I[(int64_t)g->nbr[e] * K + g->ebin[e]] += share;
        } else {
            int32_t slots[16];
            int c = select_slots(g, v, d, slots);
            if (c == 0) { g->escaped += E; continue; }
            double share = E / (double)c;
            int32_t kb = nearest_bin(g, d);
            for (int t = 0; t < c; t++) {
                int64_t e = b + slots[t];
                g->I[(int64_t)g->nbr[e] * K + kb] += share;
            }
        }
    }
    diffuse_send(g);

    /* Interaction and chemistry at every vertex, then the outgoing photons
     * of every bin are split equally over its selected neighbours; a bin
     * with no neighbour in its forward cone leaves the domain. */
    for (int64_t j = 0; j < n; j++) {
        double nin = 0.0;
        for (int64_t k = 0; k < K; k++) nin += g->I[j * K + k];
        double A, T, R;
        if (H > 1) {
            /* a hop of a multi-hop step: absorption at the frozen y, capped
             * by the atoms left; the chemistry after the last hop */
            double nHV = g->nH[j] * g->vol[j];
            double y0 = g->y[j];
            double cap = nHV * y0 - g->habs[j];
            if (cap < 0.0) cap = 0.0;
            /* passed on: exp(-y tau) of the photons, or all beyond the cap */
            T = exp(-y0 * g->tau[j]);
            double a = nin - nin * T;
            if (a > cap) {
                a = cap;
                T = (nin - a) / nin;
            }
            g->habs[j] += a;
            g->hnin[j] += nin;
            A = a;
            if (hop == H - 1) {
                double hb = (g->dt / (double)g->n_sub) * (g->alpha_B * g->nH[j]);
                g->y[j] = chem_fixed(y0, g->habs[j] / nHV, hb, g->n_sub);
                g->nin[j] = g->hnin[j];
                g->habs[j] = 0.0;
                g->hnin[j] = 0.0;
            }
            g->absorbed += A;
        } else {
            g->nin[j] = nin;
            g->y[j] = chem(g->y[j], nin, g->dt, g->nH[j] * g->vol[j], g->tau[j],
                           recomb_coeff(g) * g->nH[j], g->n_sub, &A, &T, &R);
            g->absorbed += A;
            diffuse_made(g, j, R);
        }
        for (int64_t k = 0; k < K; k++) {
            double out = g->I[j * K + k] * T;
            int32_t mm = g->m[j * K + k];
            if (mm > 0) {
                g->O[j * K + k] = out / (double)mm;
            } else {
                g->escaped += out;
                g->O[j * K + k] = 0.0;
            }
        }
    }

    /* Photons still travelling. */
    double f = 0.0;
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = 0; k < K; k++)
            f += g->O[j * K + k] * (double)g->m[j * K + k];
    g->in_flight = f + pending_diffuse(g);
    g->sweeps += 1.0;
}

/* ---------------------------------------------------------------------- */
/* Combined transport (Sects. 2.2.2-2.2.4, 5.1.3).
 *
 * Ballistic transport: photons that came into vertex j along the edge from
 * i keep travelling in the direction of that edge, i -> j; they are split
 * equally over the mpb (= d = 3) neighbours of j most aligned with it,
 * excluding any outside the forward 90 degree cone, with the selection rule
 * of the bins.  These tables depend on the grid alone.
 *
 * Mode of a vertex: ballistic where its optical depth y tau (Eq.
 * optical_depth with the neutral fraction at the start of the step) is at
 * least tau_switch, direction-conserving elsewhere.  A ballistic vertex
 * holds its photons per incoming edge, a direction-conserving one per bin.
 * Conversion at the receiver: photons that reach a ballistic vertex are
 * filed under the edge they came along (whatever bin they were in); photons
 * sent by a ballistic vertex (and photons of sources) that reach a
 * direction-conserving vertex are filed in the bin of the edge they came
 * along. */

/* Index of the directed edge i -> j in the row of i. */
static int64_t edge_index(const ora_grid *g, int64_t i, int32_t j) {
    for (int64_t e = g->ptr[i]; e < g->ptr[i + 1]; e++)
        if (g->nbr[e] == j) return e;
    return -1;
}

static void build_ballistic(ora_grid *g) {
    int64_t n = g->n;
    int mpb = g->mpb;
    for (int64_t j = 0; j < n; j++) {
        for (int64_t e = g->ptr[j]; e < g->ptr[j + 1]; e++) {
            /* the packet arrived along nbr[e] -> j: the direction opposite
             * to the unit vector of the edge j -> nbr[e] */
            double u[3] = {-g->edir[3 * e + 0], -g->edir[3 * e + 1],
                           -g->edir[3 * e + 2]};
            int32_t slots[16];
            int c = select_slots(g, j, u, slots);
            for (int r = 0; r < mpb; r++)
                g->bsel[e * mpb + r] = r < c ? g->nbr[g->ptr[j] + slots[r]] : -1;
            g->bm[e] = c;
            /* the edge j -> nbr[e] is the incoming edge nbr[e] -> j seen
             * from the other end: its slot in the row of nbr[e] */
            int64_t back = edge_index(g, g->nbr[e], (int32_t)j);
            g->rev[e] = (int32_t)(back - g->ptr[g->nbr[e]]);
        }
    }
}

/* Photons v travel along the edge e (i -> j) carrying bin b; file them at j
 * by j's mode in this step. */
static void deliver(ora_grid *g, int64_t e, int32_t b, double v) {
    int32_t j = g->nbr[e];
    if (g->mode[j] == 0)
        g->I[(int64_t)j * g->K + b] += v;
    else
        g->Ie[g->ptr[j] + g->rev[e]] += v;
}

static void sweep_combined(ora_grid *g) {
    int64_t n = g->n, K = g->K, E = g->n_edges;
    int mpb = g->mpb;
    for (int64_t j = 0; j < n; j++)
        g->mode[j] = (g->y[j] * g->tau[j] >= g->tau_switch) ? 1 : 0;
    memset(g->I, 0, (size_t)(n * K) * sizeof(double));
    memset(g->Ie, 0, (size_t)E * sizeof(double));

    /* Transport from what every vertex held after the previous step. */
    for (int64_t i = 0; i < n; i++) {
        if (g->layout[i] == 0) {
            for (int64_t k = 0; k < K; k++) {
                int32_t mm = g->m[i * K + k];
                double v = g->O[i * K + k];
                const int32_t *s = &g->sel[(i * K + k) * mpb];
                for (int t = 0; t < mm; t++)
                    deliver(g, edge_index(g, i, s[t]), (int32_t)k, v);
            }
        } else {
            for (int64_t ein = g->ptr[i]; ein < g->ptr[i + 1]; ein++) {
                double v = g->Oe[ein];
                for (int t = 0; t < g->bm[ein]; t++) {
                    int64_t e = edge_index(g, i, g->bsel[ein * mpb + t]);
                    deliver(g, e, g->ebin[e], v);
                }
            }
        }
    }

    /* Sources, as in direction-conserving transport, filed by the mode of
     * each receiver. */
    for (int32_t s = 0; s < g->n_src; s++) {
        int64_t v = g->src_v[s];
        double En = g->src_rate[s] * g->dt;
        g->emitted += En;
        const double *d = &g->src_dir[3 * s];
        int64_t b = g->ptr[v], deg = g->ptr[v + 1] - g->ptr[v];
        if (d[0] == 0.0 && d[1] == 0.0 && d[2] == 0.0) {
            if (deg == 0) { g->escaped += En; continue; }
            double share = En / (double)deg;
            for (int64_t e = b; e < b + deg; e++) deliver(g, e, g->ebin[e], share);
        } else {
            int32_t slots[16];
            int c = select_slots(g, v, d, slots);
            if (c == 0) { g->escaped += En; continue; }
            double share = En / (double)c;
            int32_t kb = nearest_bin(g, d);
            for (int t = 0; t < c; t++) deliver(g, b + slots[t], kb, share);
        }
    }
    diffuse_send(g);

    /* Interaction, then the outgoing photons in the vertex's mode. */
    for (int64_t j = 0; j < n; j++) {
        double nin = 0.0;
        if (g->mode[j] == 0)
            for (int64_t k = 0; k < K; k++) nin += g->I[j * K + k];
        else
            for (int64_t e = g->ptr[j]; e < g->ptr[j + 1]; e++) nin += g->Ie[e];
        g->nin[j] = nin;
        double A, T, R;
        g->y[j] = chem(g->y[j], nin, g->dt, g->nH[j] * g->vol[j], g->tau[j],
                       recomb_coeff(g) * g->nH[j], g->n_sub, &A, &T, &R);
        g->absorbed += A;
        diffuse_made(g, j, R);
        for (int64_t k = 0; k < K; k++) g->O[j * K + k] = 0.0;
        for (int64_t e = g->ptr[j]; e < g->ptr[j + 1]; e++) g->Oe[e] = 0.0;
        if (g->mode[j] == 0) {
            for (int64_t k = 0; k < K; k++) {
                double out = g->I[j * K + k] * T;
                int32_t mm = g->m[j * K + k];
                if (mm > 0) g->O[j * K + k] = out / (double)mm;
                else g->escaped += out;
            }
        } else {
            for (int64_t e = g->ptr[j]; e < g->ptr[j + 1]; e++) {
                double out = g->Ie[e] * T;
                if (g->bm[e] > 0) g->Oe[e] = out / (double)g->bm[e];
                else g->escaped += out;
            }
        }
        g->layout[j] = g->mode[j];
    }

    double f = 0.0;
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = 0; k < K; k++)
            f += g->O[j * K + k] * (double)g->m[j * K + k];
    for (int64_t e = 0; e < E; e++) f += g->Oe[e] * (double)g->bm[e];
    g->in_flight = f + pending_diffuse(g);
    g->sweeps += 1.0;
}

int ora_set_diffuse(ora_grid *g, double alpha_A) {
    g_err[0] = 0;
    if (!(alpha_A == 0.0 || alpha_A >= g->alpha_B)) {
        snprintf(g_err, sizeof g_err, "alpha_A must be 0 or >= alpha_B");
        return -1;
    }
    if (alpha_A > 0.0 && g->hops > 1) {
        snprintf(g_err, sizeof g_err, "diffuse radiation takes one hop per step");
        return -1;
    }
    g->alpha_A = alpha_A;
    if (alpha_A > 0.0 && !g->D) g->D = (double *)xcalloc(g->n, sizeof(double));
    return 0;
}

void ora_get_diffuse(const ora_grid *g, double *pending) {
    if (!pending) return;
    for (int64_t j = 0; j < g->n; j++) pending[j] = g->D ? g->D[j] : 0.0;
}

void ora_set_diffuse_pending(ora_grid *g, const double *pending) {
    if (!g->D || !pending) return;
    memcpy(g->D, pending, (size_t)g->n * sizeof(double));
}

/* Hops per step (multi-hop steps, see chem_fixed); 1 is the paper's one
 * hop per step.  Direction-conserving, on-the-spot grids only; the next
 * sweep starts a step. */
int ora_set_hops(ora_grid *g, int32_t hops) {
    g_err[0] = 0;
    if (hops < 1 || (hops > 1 && (g->combined || g->alpha_A > 0.0))) {
        snprintf(g_err, sizeof g_err,
                 "hops must be >= 1, and 1 with combined transport or diffuse radiation");
        return -1;
    }
    g->hops = hops;
    if (hops > 1 && !g->habs) {
        g->habs = (double *)xcalloc(g->n, sizeof(double));
        g->hnin = (double *)xcalloc(g->n, sizeof(double));
    }
    if (g->habs) {
        memset(g->habs, 0, (size_t)g->n * sizeof(double));
        memset(g->hnin, 0, (size_t)g->n * sizeof(double));
    }
    return 0;
}

int ora_set_dct_reference(ora_grid *g, int32_t edge) {
    g_err[0] = 0;
    if (edge != 0 && edge != 1) {
        snprintf(g_err, sizeof g_err, "bad reference");
        return -1;
    }
    g->dct_ref = edge;
    build_routing(g);
    return 0;
}

int ora_set_transport(ora_grid *g, int32_t combined, double tau_switch) {
    g_err[0] = 0;
    if (combined != 0 && combined != 1) {
        snprintf(g_err, sizeof g_err, "bad transport");
        return -1;
    }
    if (combined && g->hops > 1) {
        snprintf(g_err, sizeof g_err, "combined transport takes one hop per step");
        return -1;
    }
    g->combined = combined;
    g->tau_switch = tau_switch;
    if (combined && !g->bsel) {
        int64_t E = g->n_edges;
        g->rev = (int32_t *)xcalloc(E, sizeof(int32_t));
        g->bsel = (int32_t *)xcalloc(E * g->mpb, sizeof(int32_t));
        g->bm = (int32_t *)xcalloc(E, sizeof(int32_t));
        g->Oe = (double *)xcalloc(E, sizeof(double));
        g->Ie = (double *)xcalloc(E, sizeof(double));
        g->layout = (int8_t *)xcalloc(g->n, sizeof(int8_t));
        g->mode = (int8_t *)xcalloc(g->n, sizeof(int8_t));
        build_ballistic(g);
    }
    return 0;
}

void ora_get_edge_state(const ora_grid *g, double *photons_e, int8_t *layout) {
    if (!g->combined) return;
    if (photons_e) memcpy(photons_e, g->Oe, (size_t)g->n_edges * sizeof(double));
    if (layout) memcpy(layout, g->layout, (size_t)g->n * sizeof(int8_t));
}

void ora_set_edge_state(ora_grid *g, const double *photons_e, const int8_t *layout) {
    if (!g->combined) return;
    if (photons_e) memcpy(g->Oe, photons_e, (size_t)g->n_edges * sizeof(double));
    if (layout) memcpy(g->layout, layout, (size_t)g->n * sizeof(int8_t));
}

void ora_get_ballistic(const ora_grid *g, int32_t *bsel, int32_t *bm) {
    if (!g->combined) return;
    if (bsel) memcpy(bsel, g->bsel, (size_t)(g->n_edges * g->mpb) * sizeof(int32_t));
    if (bm) memcpy(bm, g->bm, (size_t)g->n_edges * sizeof(int32_t));
}

/* ---------------------------------------------------------------------- */
/* Timing only: the CPU baseline on all cores.  The same sweeps of
 * direction-conserving transport with on-the-spot chemistry as sweep(), in
 * pull form so that every vertex is written by one thread: each receiver j
 * sums, for every bin, what its senders hand it, in ascending sender id (the
 * order sweep() adds them in), then its source shares, then takes its
 * chemistry and outgoing step.  Only the tallies are summed in another order
 * (per thread, then over threads).  Combined transport and diffuse radiation
 * are not covered (returns -1). */
typedef struct {
    int64_t *ptr;    /* [N+1] */
    int32_t *from;   /* sender */
    int32_t *bin;    /* bin */
} ora_inlist;

static ora_inlist build_inlist(const ora_grid *g) {
    ora_inlist L;
    int64_t n = g->n, K = g->K;
    L.ptr = (int64_t *)xcalloc(n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = 0; k < K; k++)
            for (int t = 0; t < g->m[i * K + k]; t++)
                L.ptr[g->sel[(i * K + k) * g->mpb + t] + 1]++;
    for (int64_t j = 0; j < n; j++) L.ptr[j + 1] += L.ptr[j];
    int64_t *fill = (int64_t *)xcalloc(n, sizeof(int64_t));
    L.from = (int32_t *)xcalloc(L.ptr[n], sizeof(int32_t));
    L.bin = (int32_t *)xcalloc(L.ptr[n], sizeof(int32_t));
    /* senders in ascending id, so each (j, k) sums in sweep()'s order */
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = 0; k < K; k++)
            for (int t = 0; t < g->m[i * K + k]; t++) {
                int32_t j = g->sel[(i * K + k) * g->mpb + t];
                int64_t q = L.ptr[j] + fill[j]++;
                L.from[q] = (int32_t)i;
                L.bin[q] = (int32_t)k;
            }
    free(fill);
    return L;
}

int ora_run_threads(ora_grid *g, int32_t n_sweeps, int32_t threads) {
    if (g->combined || g->alpha_A > 0.0 || g->hops > 1 || threads < 1) return -1;
    int64_t n = g->n, K = g->K;
    if (!g->pull_ptr) {
        ora_inlist B = build_inlist(g);
        g->pull_ptr = B.ptr; g->pull_from = B.from; g->pull_bin = B.bin;
    }
    ora_inlist L = {g->pull_ptr, g->pull_from, g->pull_bin};
    /* source shares per receiver: (bin, amount), in source order */
    int64_t *sp = (int64_t *)xcalloc(n + 1, sizeof(int64_t));
    for (int32_t s = 0; s < g->n_src; s++) {
        int64_t v = g->src_v[s], b = g->ptr[v], deg = g->ptr[v + 1] - b;
        const double *d = &g->src_dir[3 * s];
        if (d[0] == 0.0 && d[1] == 0.0 && d[2] == 0.0) {
            for (int64_t e = b; e < b + deg; e++) sp[g->nbr[e] + 1]++;
        } else {
            int32_t slots[16];
            int c = select_slots(g, v, d, slots);
            for (int t = 0; t < c; t++) sp[g->nbr[b + slots[t]] + 1]++;
        }
    }
    for (int64_t j = 0; j < n; j++) sp[j + 1] += sp[j];
    int64_t *sf = (int64_t *)xcalloc(n, sizeof(int64_t));
    int32_t *sk = (int32_t *)xcalloc(sp[n] + 1, sizeof(int32_t));
    double *sa = (double *)xcalloc(sp[n] + 1, sizeof(double));
    double esc_src = 0.0;
    for (int32_t s = 0; s < g->n_src; s++) {
        int64_t v = g->src_v[s], b = g->ptr[v], deg = g->ptr[v + 1] - b;
        double E = g->src_rate[s] * g->dt;
        const double *d = &g->src_dir[3 * s];
        if (d[0] == 0.0 && d[1] == 0.0 && d[2] == 0.0) {
            if (deg == 0) { esc_src += E; continue; }
            for (int64_t e = b; e < b + deg; e++) {
                int64_t q = sp[g->nbr[e]] + sf[g->nbr[e]]++;
                sk[q] = g->ebin[e];
                sa[q] = E / (double)deg;
            }
        } else {
            int32_t slots[16];
            int c = select_slots(g, v, d, slots);
            if (c == 0) { esc_src += E; continue; }
            int32_t kb = nearest_bin(g, d);
            for (int t = 0; t < c; t++) {
                int32_t j = g->nbr[b + slots[t]];
                int64_t q = sp[j] + sf[j]++;
                sk[q] = kb;
                sa[q] = E / (double)c;
            }
        }
    }
    double e_sweep = 0.0;
    for (int32_t s = 0; s < g->n_src; s++) e_sweep += g->src_rate[s] * g->dt;
    double *On = (double *)xcalloc(n * K, sizeof(double));
    for (int32_t s = 0; s < n_sweeps; s++) {
        double absorbed = 0.0, escaped = 0.0, fly = 0.0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : absorbed, escaped, fly)
        for (int64_t j = 0; j < n; j++) {
            double *I = &g->I[j * K];
            for (int64_t k = 0; k < K; k++) I[k] = 0.0;
            for (int64_t q = L.ptr[j]; q < L.ptr[j + 1]; q++)
                I[L.bin[q]] += g->O[(int64_t)L.from[q] * K + L.bin[q]];
            for (int64_t q = sp[j]; q < sp[j + 1]; q++) I[sk[q]] += sa[q];
            double nin = 0.0;
            for (int64_t k = 0; k < K; k++) nin += I[k];
            g->nin[j] = nin;
            double A, T, R;
            g->y[j] = chem(g->y[j], nin, g->dt, g->nH[j] * g->vol[j], g->tau[j],
                           g->alpha_B * g->nH[j], g->n_sub, &A, &T, &R);
            absorbed += A;
            for (int64_t k = 0; k < K; k++) {
                double out = I[k] * T;
                int32_t mm = g->m[j * K + k];
                if (mm > 0) {
                    On[j * K + k] = out / (double)mm;
                    fly += out;
                } else {
                    On[j * K + k] = 0.0;
                    escaped += out;
                }
            }
        }
        double *t = g->O; g->O = On; On = t;
        g->emitted += e_sweep;
        g->absorbed += absorbed;
        g->escaped += escaped + esc_src;
        g->in_flight = fly;
        g->sweeps += 1.0;
    }
    free(On); free(sp); free(sf); free(sk); free(sa);
    return 0;
}

int ora_run(ora_grid *g, int32_t n_sweeps, double *history) {
    for (int32_t s = 0; s < n_sweeps; s++) {
        if (g->combined) sweep_combined(g);
        else sweep(g);
        if (history) {
            history[4 * s + 0] = g->emitted;
            history[4 * s + 1] = g->absorbed;
            history[4 * s + 2] = g->escaped;
            history[4 * s + 3] = g->in_flight;
        }
    }
    return 0;
}

void ora_get_state(const ora_grid *g, double *y, double *x, double *photons,
                   double *nin, double *tallies) {
    int64_t n = g->n, K = g->K;
    if (y) memcpy(y, g->y, n * sizeof(double));
    if (x) for (int64_t i = 0; i < n; i++) x[i] = 1.0 - g->y[i];
    if (photons) memcpy(photons, g->O, (size_t)(n * K) * sizeof(double));
    if (nin) memcpy(nin, g->nin, n * sizeof(double));
    if (tallies) {
        tallies[0] = g->sweeps;
        tallies[1] = g->emitted;
        tallies[2] = g->absorbed;
        tallies[3] = g->escaped;
        tallies[4] = g->in_flight;
    }
}

void ora_set_state(ora_grid *g, const double *y, const double *photons,
                   const double *tallies) {
    int64_t n = g->n, K = g->K;
    if (y) memcpy(g->y, y, n * sizeof(double));
    if (photons) memcpy(g->O, photons, (size_t)(n * K) * sizeof(double));
    if (tallies) {
        g->sweeps = tallies[0];
        g->emitted = tallies[1];
        g->absorbed = tallies[2];
        g->escaped = tallies[3];
        g->in_flight = tallies[4];
    }
}

/* Random rotation of the direction bins between transport steps, against
 * preferential directions (Sect. 2.2.3): the bins become R u_k of the bins
 * given at creation (R row-major, applied as ((R_r0 u_x + R_r1 u_y) +
 * R_r2 u_z) with no fused multiply-add) and the routing is recomputed.
 * What happens to the photons in flight is not spelled out; the paper notes
 * that every rotation brings a small amount of numerical diffusion, which
 * grows with the number of rotations a photon undergoes and shrinks with
 * more bins (Sect. 5.2).  Reading: photons keep their direction as closely
 * as the rotated bins allow.  The photons a vertex holds in old bin k, O m,
 * move to the rotated bin closest in direction to old bin k (largest cosine,
 * ties to the lower bin); what several old bins bring to one new bin adds up
 * in ascending old bin; it is split equally over the neighbours selected for
 * the new bin, and leaves the domain where none is selected.  A new bin fed
 * by exactly one old bin with the same number of selected neighbours keeps
 * that bin's share as it is. */
int ora_rotate(ora_grid *g, const double *R) {
    int64_t n = g->n, K = g->K;
    int32_t *m_old = (int32_t *)xcalloc(n * K, sizeof(int32_t));
    double *O_old = (double *)xcalloc(n * K, sizeof(double));
    double *b_old = (double *)xcalloc(3 * K, sizeof(double));
    int32_t *to = (int32_t *)xcalloc(K, sizeof(int32_t));
    int32_t *feeds = (int32_t *)xcalloc(K, sizeof(int32_t));
    int32_t *from = (int32_t *)xcalloc(K, sizeof(int32_t));
    memcpy(m_old, g->m, (size_t)(n * K) * sizeof(int32_t));
    memcpy(O_old, g->O, (size_t)(n * K) * sizeof(double));
    memcpy(b_old, g->bins, (size_t)(3 * K) * sizeof(double));
    for (int64_t k = 0; k < K; k++) {
        const double *u = &g->bins0[3 * k];
        for (int r = 0; r < 3; r++) {
            double a = R[3 * r + 0] * u[0];
            double b = R[3 * r + 1] * u[1];
            double c = R[3 * r + 2] * u[2];
            g->bins[3 * k + r] = (a + b) + c;
        }
    }
    build_routing(g);
    /* old bin k -> the new bin nearest its direction */
    for (int64_t k = 0; k < K; k++) {
        to[k] = nearest_bin(g, &b_old[3 * k]);
        feeds[to[k]] += 1;
        from[to[k]] = (int32_t)k;
    }
    for (int64_t i = 0; i < n; i++) {
        for (int64_t kn = 0; kn < K; kn++) {
            int32_t mn = g->m[i * K + kn];
            if (feeds[kn] == 1 && mn == m_old[i * K + from[kn]] && mn > 0) {
                g->O[i * K + kn] = O_old[i * K + from[kn]];
                continue;
            }
            double held = 0.0;
            for (int64_t k = 0; k < K; k++)
                if (to[k] == kn) held += O_old[i * K + k] * (double)m_old[i * K + k];
            if (mn == 0) {
                g->escaped += held;
                g->in_flight -= held;
                g->O[i * K + kn] = 0.0;
            } else {
                g->O[i * K + kn] = held / (double)mn;
            }
        }
    }
    free(m_old); free(O_old); free(b_old); free(to); free(feeds); free(from);
    return 0;
}

void ora_get_tables(const ora_grid *g, int32_t *sel_nbr, int32_t *sel_m,
                    int32_t *edge_bin, double *dL, double *tau) {
    int64_t n = g->n, K = g->K;
    if (sel_nbr) memcpy(sel_nbr, g->sel, (size_t)(n * K * g->mpb) * sizeof(int32_t));
    if (sel_m) memcpy(sel_m, g->m, (size_t)(n * K) * sizeof(int32_t));
    if (edge_bin) memcpy(edge_bin, g->ebin, (size_t)g->n_edges * sizeof(int32_t));
    if (dL) memcpy(dL, g->dL, n * sizeof(double));
    if (tau) memcpy(tau, g->tau, n * sizeof(double));
}

void ora_free(ora_grid *g) {
    if (!g) return;
    free(g->ptr); free(g->nbr); free(g->edir); free(g->elen); free(g->bins); free(g->bins0);
    free(g->nH); free(g->vol); free(g->dL); free(g->tau); free(g->sel);
    free(g->m); free(g->ebin); free(g->src_v); free(g->src_rate);
    free(g->src_dir); free(g->y); free(g->O); free(g->I); free(g->nin);
    free(g->rev); free(g->bsel); free(g->bm); free(g->Oe); free(g->Ie);
    free(g->layout); free(g->mode); free(g->D);
    free(g->habs); free(g->hnin);
    drop_pull(g);
    free(g);
}
