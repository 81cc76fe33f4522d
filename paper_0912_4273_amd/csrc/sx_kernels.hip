// sx_kernels.hip -- HIP kernels of libsx for gfx950 (MI355X).
//
// SimpleX2 direction-conserving transport (Paardekooper, Kruip & Icke 2010,
// Sect. 2.2.3) fused with the subcycled hydrogen rate equation (Sect. 4.5).
//
// Layout (one grid):
//   vertices reordered along a Hilbert curve, tiles of 64 consecutive
//   vertices = one wavefront, lane = vertex;
//   photon field O in bin-major planes [K][npad] (fp32 or fp64), double
//   buffered; a lane reads and writes one element per plane, so every store
//   and the in-word / m-bit loads are fully coalesced, and the gathers of a
//   wave hit the few cache lines of the tile's Hilbert neighbourhood;
//   gather lists per (vertex, bin) as 32-bit in-words [tile][K][64].
#include "sx_internal.h"

namespace sx {

// --------------------------------------------------------------- helpers --

// Direction cosine of a unit edge vector with a unit bin direction, rounded
// step by step as ((ex*ux + ey*uy) + ez*uz) with no fused multiply-add, so
// that the neighbour ranking is bit-identical to a plain IEEE evaluation on
// any host.
__device__ __forceinline__ double cosine3(const double *e, const double *u) {
#pragma clang fp contract(off)
  const double a = e[0] * u[0];
  const double b = e[1] * u[1];
  const double c = e[2] * u[2];
  const double ab = a + b;
  return ab + c;
}

__device__ __forceinline__ bool fwd_selects(uint32_t f, uint32_t slot) {
  return ((f & 127u) == slot) | (((f >> 7) & 127u) == slot) |
         (((f >> 14) & 127u) == slot);
}

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <typename T>
static hipError_t fill(T *p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v,
                     n);
  return hipGetLastError();
}

// -------------------------------------------------------- bin selection --
// For every (vertex, bin): the <= mpb neighbours with the largest cosine
// between edge and bin direction, cosine > cos_min (photons never go
// backwards), ties to the lower original neighbour id.  Rows are sorted by
// original id, so "lower slot" is "lower id".  One lane per pair.
__global__ void k_select(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int K = g.k;
  if (p >= (int64_t)g.npad * K) return;
  const int i = (int)(p / K);
  const int k = (int)(p - (int64_t)i * K);
  uint32_t s0 = kEmptySlot, s1 = kEmptySlot, s2 = kEmptySlot, cnt = 0;
  if (i < g.n) {
    const double u[3] = {g.bins[3 * k], g.bins[3 * k + 1], g.bins[3 * k + 2]};
    const int rb = g.row_ptr[i], re = g.row_ptr[i + 1];
    double c0 = -3.0, c1 = -3.0, c2 = -3.0;
    for (int e = rb; e < re; ++e) {
      const double c = cosine3(&g.edir[3 * (int64_t)e], u);
      if (!(c > g.cos_min)) continue;
      const uint32_t s = (uint32_t)(e - rb);
      if (c > c0) {
        c2 = c1; s2 = s1; c1 = c0; s1 = s0; c0 = c; s0 = s;
      } else if (c > c1) {
        c2 = c1; s2 = s1; c1 = c; s1 = s;
      } else if (c > c2) {
        c2 = c; s2 = s;
      }
      ++cnt;
    }
    if (cnt > (uint32_t)g.mpb) cnt = (uint32_t)g.mpb;
    if (g.mpb < 3) s2 = kEmptySlot;
    if (g.mpb < 2) s1 = kEmptySlot;
  }
  g.fwd[p] = s0 | (s1 << 7) | (s2 << 14) | (cnt << 21);
}

// Bin of each directed edge: the bin whose direction is closest to the edge
// (Sect. 2.2.4), ties to the lower bin.  One lane per edge.
__global__ void k_edge_bins(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.n_edges) return;
  const double *ed = &g.edir[3 * e];
  int best = 0;
  double cb = cosine3(ed, &g.bins[0]);
  for (int k = 1; k < g.k; ++k) {
    const double c = cosine3(ed, &g.bins[3 * k]);
    if (c > cb) { cb = c; best = k; }
  }
  g.ebin[e] = (uint8_t)best;
}

// ------------------------------------------------------- gather lists ---
// The receiver side of the selection: neighbour t of j sends bin k to j iff
// j is among the selected slots of (nbr_t, k).  Entries are kept in
// ascending slot order.  Pass 1 counts, per vertex, the entries beyond the
// four an in-word holds; pass 2 (after a scan) writes in-words, packed m
// and the overflow entries.
__global__ void k_inlist_count(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.npad) return;
  int extras = 0;
  if (j < g.n) {
    const int rb = g.row_ptr[j], re = g.row_ptr[j + 1];
    const int K = g.k;
    for (int k = 0; k < K; ++k) {
      int c = 0;
      for (int e = rb; e < re; ++e)
        c += fwd_selects(g.fwd[(int64_t)g.nbr[e] * K + k], g.rev[e]) ? 1 : 0;
      extras += c > 4 ? c - 4 : 0;
    }
  }
  g.ovf_cnt[j] = extras;
}

__global__ void k_inlist_fill(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.npad) return;
  const int tile = j >> 6, lane = j & 63;
  const int K = g.k;
  const bool valid = j < g.n;
  const int rb = g.row_ptr[j], re = g.row_ptr[j + 1];
  int64_t op = g.ovf_ptr[j];
  uint32_t mword = 0;
  for (int k = 0; k < K; ++k) {
    uint32_t w = 0, c = 0, m = 0;
    if (valid) {
      for (int e = rb; e < re; ++e) {
        if (!fwd_selects(g.fwd[(int64_t)g.nbr[e] * K + k], g.rev[e])) continue;
        const uint32_t t = (uint32_t)(e - rb);
        if (c < 4) {
          w |= t << (4 + 7 * c);
        } else if (op < g.ovf_cap) {
          g.ovf[op] = (uint16_t)(((uint32_t)k << 7) | t);
          ++op;
        }
        ++c;
      }
      w |= (c < 4 ? c : 4u) | (c > 4 ? 8u : 0u);
      m = (g.fwd[(int64_t)j * K + k] >> 21) & 3u;
    }
    g.inword[((int64_t)tile * K + k) * 64 + lane] = w;
    mword |= m << (2 * (k & 15));
    if ((k & 15) == 15 || k == K - 1) {
      g.mbits[((int64_t)tile * g.kw + (k >> 4)) * 64 + lane] = mword;
      mword = 0;
    }
  }
}

// Exclusive scan of n counts into ptr[0..n] by one workgroup.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ cnt,
                                               int32_t *__restrict__ ptr,
                                               int32_t n) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = ((int64_t)n + 1023) / 1024;
  const int64_t b = t * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = b; i < e; ++i) {
    ptr[i] = (int32_t)run;
    run += cnt[i];
  }
  if (t == 1023) ptr[n] = (int32_t)part[1023];
}

// ---------------------------------------------------------- chemistry ---
// One backward-Euler substep of the rate equation for the neutral fraction
// (Eqs. rate_eq, rate_eq_subcycle, phot_ion_rate_subcycle; on the spot,
// n_e = n_HII):  y' = y - ha (1 - exp(-y' tau)) + hb (1 - y')^2, solved by
// safeguarded Newton inside the bracket [0, 1].
__device__ __forceinline__ double be_substep(double y0, double ha, double hb,
                                             double tau) {
  double lo = 0.0, hi = 1.0, yn = y0;
  for (int it = 0; it < 200; ++it) {
    const double ion = -expm1(-yn * tau);
    const double x = 1.0 - yn;
    const double g = (y0 - yn) - ha * ion + hb * (x * x);
    if (g == 0.0) break;
    if (g > 0.0) lo = yn; else hi = yn;
    const double gp = -1.0 - ha * tau * (1.0 - ion) - 2.0 * hb * x;
    double yc = yn - g / gp;
    if (!(yc > lo && yc < hi)) yc = 0.5 * (lo + hi);
    const double step = fabs(yc - yn);
    yn = yc;
    if (step <= 4.0e-16 * yn || hi - lo <= 4.0e-16 * hi) break;
  }
  return yn;
}

// n_sub substeps at constant incoming flux; returns y, absorbed photons A
// and the transmitted fraction T (mean over substeps of exp(-y tau)).
__device__ __forceinline__ double chem_step(double y, double nin, double dt,
                                            double dtnhv, double tau, double b,
                                            int n_sub, double &A, double &T) {
  const double h = dt / (double)n_sub;
  const double a = nin / dtnhv;
  const double ha = h * a, hb = h * b;
  const double share = nin / (double)n_sub;
  double abs_sum = 0.0, tr_sum = 0.0;
  for (int s = 0; s < n_sub; ++s) {
    y = be_substep(y, ha, hb, tau);
    abs_sum += share * (-expm1(-y * tau));
    tr_sum += exp(-y * tau);
  }
  A = abs_sum;
  T = nin > 0.0 ? tr_sum / (double)n_sub : 1.0;
  return y;
}

// -------------------------------------------------------------- sweep ---
// One radiative-transfer step of every active grid in the batch (Sect. 4.6:
// photons move one edge, interact once).  Lane = vertex of a 64-vertex tile:
//   1. gather: I[k] = sum over the in-word (+ overflow) entries of the
//      senders' O[k]; plus this vertex's share of source emission;
//   2. N_in = sum_k I[k];
//   3. chemistry in fp64 -> y, absorbed A, transmitted fraction T;
//   4. O'[k] = I[k] T / m(j,k), or escape when m = 0;
//   5. per-tile photon accounting in fp64, fixed-order wave reduction.
template <typename P, int KMAX>
__global__ __launch_bounds__(256) void k_sweep(
    const GridDev *__restrict__ grids, const int2 *__restrict__ tile_map,
    int32_t n_tiles) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Workgroups are dealt round-robin to the 8 XCDs; renumber them so each
  // XCD runs a contiguous range of tiles and its L2 sees the neighbourhood.
  const uint32_t nb = gridDim.x;   // a multiple of 8
  const uint32_t b = blockIdx.x;
  const uint32_t lb = (b & 7u) * (nb >> 3) + (b >> 3);
  const int gt = (int)lb * kTilesPerBlock + wave;
  if (gt >= n_tiles) return;
  int gi = 0, tile = gt;
  if (tile_map) {
    const int2 tm = tile_map[gt];
    gi = __builtin_amdgcn_readfirstlane(tm.x);
    tile = __builtin_amdgcn_readfirstlane(tm.y);
  }
  const GridDev *__restrict__ G = grids + gi;
  if (G->remaining <= 0) return;

  const int K = G->k;
  const int64_t plane = G->plane;
  const int j = tile * kTile + lane;
  const bool valid = j < G->n;
  const int par = G->parity;
  const P *__restrict__ oin = (const P *)G->o[par];
  P *__restrict__ oout = (P *)G->o[par ^ 1];
  const int32_t *__restrict__ nbr = G->nbr;
  const int rb = G->row_ptr[j];
  const uint32_t *__restrict__ iw = G->inword + (int64_t)tile * K * 64 + lane;
  const uint16_t *__restrict__ ovf = G->ovf;
  int op = G->ovf_ptr[j];
  const int oe = G->ovf_ptr[j + 1];

  P I[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    P acc = P(0);
    if (k < K) {
      const uint32_t w = iw[(int64_t)k * 64];
      const uint32_t nm = w & 7u;
      const P *__restrict__ pk = oin + (int64_t)k * plane;
      if (nm > 0) acc += pk[nbr[rb + ((w >> 4) & 127u)]];
      if (nm > 1) acc += pk[nbr[rb + ((w >> 11) & 127u)]];
      if (nm > 2) acc += pk[nbr[rb + ((w >> 18) & 127u)]];
      if (nm > 3) acc += pk[nbr[rb + ((w >> 25) & 127u)]];
      if (w & 8u) {
        while (op < oe) {
          const uint32_t v = ovf[op];
          if ((int)(v >> 7) != k) break;
          acc += pk[nbr[rb + (v & 127u)]];
          ++op;
        }
      }
    }
    I[k] = acc;
  }

  // Sources: this vertex's share of each neighbouring source's photons,
  // in source order, filed in the bin of the edge they come along.
  {
    int ep = G->em_ptr[j];
    const int ee = G->em_ptr[j + 1];
    for (; ep < ee; ++ep) {
      const int kk = G->em_k[ep];
      const P amt = (P)G->em_amt[ep];
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k == kk) I[k] += amt;
    }
  }

  P sum = P(0);
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < K) sum += I[k];

  double A = 0.0, T = 1.0;
  if (valid) {
    const double nin = (double)sum * G->unit;
    const double y0 = G->y[j];
    if (!(nin == 0.0 && y0 == 1.0)) {
      const double yn = chem_step(y0, nin, G->dt, G->dtnhv[j], G->tau[j],
                                  G->bcoef[j], G->n_sub, A, T);
      G->y[j] = yn;
    }
    G->nin[j] = nin;
  }
  A /= G->unit;   // tallies in stored units; scaled back on read

  const double t2 = T * 0.5;
  const double t3 = T / 3.0;
  double esc = 0.0, fly = 0.0;
  const uint32_t *__restrict__ mb = G->mbits + (int64_t)tile * G->kw * 64 + lane;
  uint32_t mw = 0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      if ((k & 15) == 0) mw = mb[(int64_t)(k >> 4) * 64];
      const uint32_t m = (mw >> (2 * (k & 15))) & 3u;
      const double it = (double)I[k] * T;
      double o;
      if (m == 0u) {
        esc += it;
        o = 0.0;
      } else if (m == 1u) {
        o = it;
      } else if (m == 2u) {
        o = (double)I[k] * t2;
      } else if constexpr (sizeof(P) == 8) {
        o = it / 3.0;   // same rounding as (I T) / 3 on the host
      } else {
        o = (double)I[k] * t3;
      }
      const P os = (P)o;
      fly += (double)os * (double)m;
      if (valid) oout[(int64_t)k * plane + j] = os;
    }
  }

  // Fixed butterfly: every lane ends with the same, order-determined sum.
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    A += __shfl_xor(A, off);
    esc += __shfl_xor(esc, off);
    fly += __shfl_xor(fly, off);
  }
  if (lane == 0) {
    double *t = G->tally + (int64_t)tile * 3;
    t[0] += A;
    t[1] += esc;
    t[2] = fly;
  }
}

struct SlotVals {
  int32_t slot[120];
  int32_t v[120];
};

// After a step: every listed grid that ran flips its buffers.
__global__ void k_advance(GridDev *table, SlotVals sv, int32_t n) {
  const int i = threadIdx.x;
  if (i >= n) return;
  GridDev &g = table[sv.slot[i]];
  if (g.remaining > 0) {
    g.parity ^= 1;
    g.remaining -= 1;
    g.sweeps += 1;
  }
}

__global__ void k_set_remaining(GridDev *table, SlotVals sv, int32_t n,
                                int32_t add) {
  const int i = threadIdx.x;
  if (i >= n) return;
  GridDev &g = table[sv.slot[i]];
  g.remaining = add ? g.remaining + sv.v[i] : sv.v[i];
}

__global__ void k_reset(GridDev *__restrict__ gp, const double *__restrict__ y0) {
  const GridDev &g = *gp;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.npad) return;
  g.y[j] = y0[j];
  g.nin[j] = 0.0;
}

__global__ void k_reset_ctl(GridDev *gp) {
  gp->parity = 0;
  gp->remaining = 0;
  gp->sweeps = 0;
}

// ----------------------------------------------------------- launchers ---
static inline unsigned blocks_for(int64_t n, int t) {
  return (unsigned)((n + t - 1) / t);
}

hipError_t launch_select(const GridDev *dg, const GridDev &hg, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(blocks_for((int64_t)hg.npad * hg.k, 256)),
                     dim3(256), 0, s, dg);
  return hipGetLastError();
}

hipError_t launch_edge_bins(const GridDev *dg, const GridDev &hg,
                            hipStream_t s) {
  if (hg.n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_bins, dim3(blocks_for(hg.n_edges, 256)), dim3(256),
                     0, s, dg);
  return hipGetLastError();
}

hipError_t launch_inlist_count(const GridDev *dg, const GridDev &hg,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_inlist_count, dim3(blocks_for(hg.npad, 256)), dim3(256),
                     0, s, dg);
  return hipGetLastError();
}

hipError_t launch_scan(int32_t *cnt, int32_t *ptr, int32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cnt, ptr, n);
  return hipGetLastError();
}

hipError_t launch_inlist_fill(const GridDev *dg, const GridDev &hg,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_inlist_fill, dim3(blocks_for(hg.npad, 256)), dim3(256),
                     0, s, dg);
  return hipGetLastError();
}

hipError_t launch_reset_state(GridDev *dg, const GridDev &hg, const double *y0,
                              hipStream_t s) {
  hipError_t e;
  const int64_t nk = (int64_t)hg.k * hg.plane;
  for (int b = 0; b < 2; ++b) {
    if (hg.precision == 0)
      e = fill<double>((double *)hg.o[b], 0.0, nk, s);
    else
      e = fill<float>((float *)hg.o[b], 0.0f, nk, s);
    if (e != hipSuccess) return e;
  }
  e = fill<double>(hg.tally, 0.0, (int64_t)hg.ntiles * 3, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reset, dim3(blocks_for(hg.npad, 256)), dim3(256), 0, s,
                     dg, y0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(1), 0, s, dg);
  return hipGetLastError();
}

int kmax_bucket(int k, int precision) {
  (void)precision;
  static const int b[] = {8, 16, 32, 42, 48, 64, 84, 96};
  for (int v : b)
    if (k <= v) return v;
  return 0;
}

template <typename P>
static hipError_t sweep_p(const GridDev *grids, const int2 *tile_map,
                          int32_t n_tiles, int kmax, hipStream_t s) {
  unsigned nb = blocks_for(n_tiles, kTilesPerBlock);
  nb = (nb + 7u) & ~7u;
  dim3 g(nb), t(64 * kTilesPerBlock);
  switch (kmax) {
#define SX_CASE(KM)                                                         \
  case KM:                                                                  \
    hipLaunchKernelGGL((k_sweep<P, KM>), g, t, 0, s, grids, tile_map,       \
                       n_tiles);                                            \
    break;
    SX_CASE(8)
    SX_CASE(16)
    SX_CASE(32)
    SX_CASE(42)
    SX_CASE(48)
    SX_CASE(64)
    SX_CASE(84)
    SX_CASE(96)
#undef SX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sweep(const GridDev *grids, const int2 *tile_map,
                        int32_t n_tiles, int32_t kmax, int32_t precision,
                        hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (precision == 0) return sweep_p<double>(grids, tile_map, n_tiles, kmax, s);
  return sweep_p<float>(grids, tile_map, n_tiles, kmax, s);
}

hipError_t launch_advance(GridDev *table, const int32_t *slots, int32_t n,
                          hipStream_t s) {
  for (int32_t base = 0; base < n; base += 120) {
    SlotVals v;
    const int32_t m = n - base < 120 ? n - base : 120;
    for (int32_t i = 0; i < m; ++i) { v.slot[i] = slots[base + i]; v.v[i] = 0; }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(128), 0, s, table, v, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_set_remaining(GridDev *table, const int32_t *slots,
                                const int32_t *values, int32_t n, int32_t add,
                                hipStream_t s) {
  for (int32_t base = 0; base < n; base += 120) {
    SlotVals v;
    const int32_t m = n - base < 120 ? n - base : 120;
    for (int32_t i = 0; i < m; ++i) {
      v.slot[i] = slots[base + i];
      v.v[i] = values[base + i];
    }
    hipLaunchKernelGGL(k_set_remaining, dim3(1), dim3(128), 0, s, table, v, m,
                       add);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sx
