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
#include <mutex>
#include <utility>

#include "sx.h"
#include "sx_internal.h"

namespace sx {

// Pointers read from a GridDev are generic to the compiler; casting them to
// the global address space makes it emit global (not flat) loads and stores,
// which do not share the LDS wait counter.
#define SX_G __attribute__((address_space(1)))
// LDS pointers carry their address space explicitly: volatile accesses
// through a generic pointer would be emitted as FLAT instructions.
#define SX_L __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ const SX_G T *gld(const T *p) {
  return (const SX_G T *)p;
}
template <typename T>
__device__ __forceinline__ SX_G T *gst(T *p) {
  return (SX_G T *)p;
}

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1, so
// per-bin register arrays are indexed by constants (never spilled).
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f,
                                                std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

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

// A product that is rounded on its own (never fused into a following add),
// so that staged and direct gathers round a sender's outgoing photons alike.
template <typename P>
__device__ __forceinline__ P mul_rn(P a, P b) {
#pragma clang fp contract(off)
  return a * b;
}

// DPP lane moves (GFX9 controls): row_shr:n within rows of 16 lanes, the
// broadcast of lane 15 (31) of a row to the next rows, and a shift of the
// whole wave by one lane towards lane 0.  Lanes with no source (or outside
// row_mask) keep `old`.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114,
              kDppRowShr8 = 0x118, kDppBcast15 = 0x142, kDppBcast31 = 0x143,
              kDppWaveShl1 = 0x130;
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS, typename P>
__device__ __forceinline__ P dpp_val(P v) {
  if constexpr (sizeof(P) == 8) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)dpp_i32<CTRL, ROWS>(0, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)dpp_i32<CTRL, ROWS>(0, (int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(P, ((uint64_t)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(P, dpp_i32<CTRL, ROWS>(0, __builtin_bit_cast(int, v)));
  }
}
// Inclusive scan of v over runs of equal key (keys ascending along the
// lanes, so a run is contiguous): row-local steps 1, 2, 4, 8, then the rows'
// last lanes carried into the following rows.  A lane adds a source only
// when the source lane carries the same key, so sums never cross runs.
template <typename P>
__device__ __forceinline__ void seg_scan(P &v, int key) {
  auto step = [&](auto ctrl, auto rows) {
    constexpr int C = decltype(ctrl)::value, R = decltype(rows)::value;
    const int ks = dpp_i32<C, R>(-2000, key);
    const P vs = dpp_val<C, R>(v);
    if (ks == key) v += vs;
  };
  step(std::integral_constant<int, kDppRowShr1>{}, std::integral_constant<int, 0xF>{});
  step(std::integral_constant<int, kDppRowShr2>{}, std::integral_constant<int, 0xF>{});
  step(std::integral_constant<int, kDppRowShr4>{}, std::integral_constant<int, 0xF>{});
  step(std::integral_constant<int, kDppRowShr8>{}, std::integral_constant<int, 0xF>{});
  step(std::integral_constant<int, kDppBcast15>{}, std::integral_constant<int, 0xA>{});
  step(std::integral_constant<int, kDppBcast31>{}, std::integral_constant<int, 0xC>{});
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

// The reverse of every directed edge: e in j's row points at i = nbr[e],
// and j sits in slot rev[e] of i's row.  One lane per edge, once per upload.
__global__ void k_erev(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.n_edges) return;
  g.erev[e] = g.row_ptr[g.nbr[e]] + g.rev[e];
}

// -------------------------------------------------------- bin selection --
// For every (vertex, bin): the <= mpb neighbours with the largest cosine
// between edge and bin direction, cosine > cos_min (photons never go
// backwards), ties to the lower original neighbour id.  Rows are sorted by
// original id, so "lower slot" is "lower id".  With dct_ref the reference
// direction is the vertex's edge closest to the bin (largest cosine over
// cos_min, ties to the lower id) in place of the bin.  A vertex's edge
// directions are staged in LDS once and its bins run over them in row
// order.
// The three largest cosines so far, c0 >= c1 >= c2, all above cos_min (an
// empty place holds cos_min and kEmptySlot, so "c > c2" also tests the
// cone).  A candidate is tested against the third place first: most fail
// there once the places are full.  Strict comparisons keep the earlier
// (lower) slot on ties.
struct Top3 {
  double c0, c1, c2;
  uint32_t s0 = kEmptySlot, s1 = kEmptySlot, s2 = kEmptySlot;
  __device__ __forceinline__ explicit Top3(double cos_min) : c0(cos_min), c1(cos_min), c2(cos_min) {}
  __device__ __forceinline__ void add(double c, uint32_t s) {
    if (c > c2) {
      if (c > c1) {
        c2 = c1; s2 = s1;
        if (c > c0) {
          c1 = c0; s1 = s0; c0 = c; s0 = s;
        } else {
          c1 = c; s1 = s;
        }
      } else {
        c2 = c; s2 = s;
      }
    }
  }
  __device__ __forceinline__ uint32_t word(int mpb) const {
    const uint32_t filled = (s0 != (uint32_t)kEmptySlot) + (s1 != (uint32_t)kEmptySlot) +
                            (s2 != (uint32_t)kEmptySlot);
    const uint32_t n = filled > (uint32_t)mpb ? (uint32_t)mpb : filled;
    const uint32_t t2 = mpb < 3 ? (uint32_t)kEmptySlot : s2;
    const uint32_t t1 = mpb < 2 ? (uint32_t)kEmptySlot : s1;
    return s0 | (t1 << 7) | (t2 << 14) | (n << 21);
  }
};

// the reference direction of bin u under dct_ref: the closest edge in the
// forward cone; returns the number of edges to consider (0 if none)
__device__ __forceinline__ int ref_edge(const SX_L double *ed, int deg, double cos_min,
                                        double u[3]) {
  int best = -1;
  double cb = cos_min;
  for (int t = 0; t < deg; ++t) {
    const double d[3] = {ed[3 * t], ed[3 * t + 1], ed[3 * t + 2]};
    const double c = cosine3(d, u);
    if (c > cb) { cb = c; best = t; }
  }
  if (best < 0) return 0;
  u[0] = ed[3 * best];
  u[1] = ed[3 * best + 1];
  u[2] = ed[3 * best + 2];
  return deg;
}

// The forward word of (vertex, bin k) over the vertex's n staged edge
// directions, and the bits of its selected slots in the vertex's masks.
__device__ __forceinline__ void select_bin(const GridDev &g, int64_t i, int k,
                                           const SX_L double *ed, SX_L uint32_t *ms,
                                           SX_L uint32_t *mw, int n) {
  double u[3] = {g.bins[3 * k], g.bins[3 * k + 1], g.bins[3 * k + 2]};
  if (g.dct_ref) n = ref_edge(ed, n, g.cos_min, u);
  Top3 a(g.cos_min);
  for (int t = 0; t < n; ++t) {
    const double d[3] = {ed[3 * t], ed[3 * t + 1], ed[3 * t + 2]};
    a.add(cosine3(d, u), (uint32_t)t);
  }
  const uint32_t word = a.word(g.mpb);
  g.fwd[i * g.k + k] = word;
  // each selected slot gets the bit of bin k's storage position in its
  // out-edge's mask (an OR, so the order of the lanes does not matter)
  const int p = g.bpos[k];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint32_t s = (word >> (7 * q)) & 127u;
    if (s != (uint32_t)kEmptySlot) atomicOr((uint32_t *)&ms[4 * s + (p >> 5)], 1u << (p & 31));
  }
  // and m at bits 2 (p mod 16) of the vertex's m word p / 16
  const uint32_t m = (word >> 21) & 3u;
  if (m) atomicOr((uint32_t *)&mw[p >> 4], m << (2 * (p & 15)));
}

// One wave per two vertices: bins 0..63 of the first vertex, then of the
// second, then bins 64..95 of both at once (lanes 0..31 the first, 32..63
// the second), so that with K = 84 few lanes idle.
static_assert(SX_MAX_BINS_FP32 <= 96 && SX_MAX_BINS_FP64 <= 96,
              "k_select covers bins 0..95: a larger bin limit needs another pass");
// LDS of k_select per workgroup (8 vertices), sized by the grid's largest
// degree: the edge directions, the selection masks, then 6 m words per vertex
constexpr int kSelMWords = 6;
static_assert((SX_MAX_BINS_FP32 + 15) / 16 <= kSelMWords && (SX_MAX_BINS_FP64 + 15) / 16 <= kSelMWords,
              "k_select keeps at most 6 m words per vertex");
__host__ __device__ constexpr int64_t select_lds_bytes(int max_deg) {
  return 8 * (3 * 8 + 4 * 4) * (int64_t)max_deg + 8 * kSelMWords * 4;
}

// 8 waves per SIMD: the compiler then fits the kernel in 48 VGPRs without
// spilling (88 by default, 5 waves), and the FP64 chains hide each other
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_select(
    const GridDev *__restrict__ gp, uint32_t *__restrict__ mout) {
  const GridDev &g = *gp;
  extern __shared__ __attribute__((aligned(16))) double sel_lds[];
  const int md = g.max_deg;
  // vertex slot s: edge directions at sd(s), masks (4 words per out-edge) at sm(s)
  auto sd = [&](int s) { return sel_lds + (int64_t)s * 3 * md; };
  auto sm = [&](int s) { return (uint32_t *)(sel_lds + (int64_t)8 * 3 * md) + (int64_t)s * 4 * md; };
  // m words of vertex slot s
  auto smw = [&](int s) {
    return (uint32_t *)(sel_lds + (int64_t)8 * 3 * md) + (int64_t)8 * 4 * md + s * kSelMWords;
  };
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + w) * 2;   // npad is even
  const bool live = i0 < g.npad;   // the block's barriers are reached by all
  const int K = g.k;
  int rb[2], deg[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    rb[v] = 0;
    deg[v] = 0;
    if (i0 + v < g.n) {
      rb[v] = g.row_ptr[i0 + v];
      deg[v] = g.row_ptr[i0 + v + 1] - rb[v];
    }
    SX_L double *ed = (SX_L double *)sd(2 * w + v);
    SX_L uint32_t *ms = (SX_L uint32_t *)sm(2 * w + v);
    for (int q = lane; q < 3 * deg[v]; q += 64) ed[q] = g.edir[3 * (int64_t)rb[v] + q];
    for (int q = lane; q < 4 * deg[v]; q += 64) ms[q] = 0u;
    if (lane < kSelMWords) ((SX_L uint32_t *)smw(2 * w + v))[lane] = 0u;
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int v = 0; v < 2; ++v)
      if (lane < K)
        select_bin(g, i0 + v, lane, (const SX_L double *)sd(2 * w + v),
                   (SX_L uint32_t *)sm(2 * w + v), (SX_L uint32_t *)smw(2 * w + v), deg[v]);
    const int v = lane >> 5, k = 64 + (lane & 31);
    if (k < K)
      select_bin(g, i0 + v, k, (const SX_L double *)sd(2 * w + v), (SX_L uint32_t *)sm(2 * w + v),
                 (SX_L uint32_t *)smw(2 * w + v), v == 0 ? deg[0] : deg[1]);
  }
  __syncthreads();
  // the m words, tile-major ([tile][word][lane]); padding vertices get zeros
  if (live && lane < g.kw) {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int64_t i = i0 + v;
      mout[((i >> 6) * g.kw + lane) * 64 + (i & 63)] = ((const SX_L uint32_t *)smw(2 * w + v))[lane];
    }
  }
  // out-edge (i, t) is the receiver's in-edge erev[rb + t]; the masks are
  // four planes of E + 1 words (word q of edge e at q (E + 1) + e)
  typedef uint32_t U4 __attribute__((ext_vector_type(4)));
  const int64_t pl = g.n_edges + 1;
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const SX_L uint32_t *ms = (const SX_L uint32_t *)sm(2 * w + v);
    for (int t = lane; t < deg[v]; t += 64) {
      const U4 m = *(const SX_L U4 *)(ms + 4 * t);
      const int64_t e = g.erev[rb[v] + t];
      g.smask[e] = m.x;
      g.smask[pl + e] = m.y;
      g.smask[2 * pl + e] = m.z;
      g.smask[3 * pl + e] = m.w;
    }
  }
}

// Bin of each directed edge: the bin whose direction is closest to the edge
// (Sect. 2.2.4), ties to the lower bin.  One lane per edge.
__global__ __launch_bounds__(256) void k_edge_bins(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  // the bin directions, read by every lane in the same order
  __shared__ double sb[3 * SX_MAX_BINS_FP32];
  const int K = g.k;
  for (int q = threadIdx.x; q < 3 * K; q += blockDim.x) sb[q] = g.bins[q];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.n_edges) return;
  const double ed[3] = {g.edir[3 * e], g.edir[3 * e + 1], g.edir[3 * e + 2]};
  // two independent chains, even and odd bins, each keeping its first
  // largest cosine; the larger wins, a tie goes to the lower bin
  int ba = 0, bo = -1;
  double ca = cosine3(ed, &sb[0]), co = 0.0;
  if (K > 1) {
    co = cosine3(ed, &sb[3]);
    bo = 1;
  }
#pragma unroll 2
  for (int k = 2; k < K; k += 2) {
    const double c = cosine3(ed, &sb[3 * k]);
    if (c > ca) { ca = c; ba = k; }
    if (k + 1 < K) {
      const double d = cosine3(ed, &sb[3 * (k + 1)]);
      if (d > co) { co = d; bo = k + 1; }
    }
  }
  const int best = (bo >= 0 && (co > ca || (co == ca && bo < ba))) ? bo : ba;
  g.ebin[e] = (uint8_t)best;
}

// ------------------------------------------------------- gather lists ---
// The receiver side of the selection: neighbour t of j sends bin k to j iff
// j is among the selected slots of (nbr_t, k).  The gather-list kernels read
// it from the receiving side: one mask per in-edge e of j (bit p % 32 of
// word e of plane p / 32 set iff the bin at storage position p of sender
// nbr[e] selects j), written by the selection kernel.
__device__ __forceinline__ int sender_index(const GridDev &g, bool direct,
                                            int e, int rb) {
  return direct ? e - rb : (int)g.edge_hidx[e];
}

constexpr uint32_t kRecEmission = 1u << kRecIdxBits;
constexpr uint32_t kRecIdxMask = (1u << kRecIdxBits) - 1u;

static_assert(SX_MAX_BINS_FP32 <= 128 && SX_MAX_BINS_FP64 <= 128 &&
                  SX_MAX_BINS_FP64 <= SX_MAX_BINS_FP32,
              "selection masks hold 128 bins; edge bins stage up to "
              "SX_MAX_BINS_FP32 directions");

// One wave per (tile, group of 16 bin positions), lane = receiver j: the
// lane walks j's in-edges once, in row order, reading the 16 bits of each
// mask that cover the group (blocks kq KQ .. kq KQ + KQ - 1, KQ = 16 / BB).
// A sender with bins in a block takes the block's next in-word entry while
// there is one (and its slot fits), otherwise it becomes records, one per
// bin; j's source shares of those bins come after.  Counts and offsets are
// kept per (tile, position, group of kRecGroupLanes receivers), so the
// records of a (tile, position) come out sorted by lane; a lane's place in
// its group comes from a shuffle scan of the counts.  Pass 1 counts the
// records (per group for the scan, and per lane as bytes for pass 2), pass
// 2 (after a scan) writes in-words and records.  Pass 2 walks again only
// in a wave where a lane's count reached 255.
constexpr int kInlistBins = 16;   // bin positions per wave of the gather-list build
static_assert(kRecGroupLanes == 8, "the record scan below works on groups of 8 lanes");

template <bool FILL, int BB>
__global__ __launch_bounds__(256) void k_inlist(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int K = g.k, KB = g.kb;
  constexpr int KQ = kInlistBins / BB;
  const int nkq = (K + kInlistBins - 1) / kInlistBins;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(t & 63);
  const int64_t tk = t >> 6;
  if (tk >= (int64_t)g.ntiles * nkq) return;   // whole waves
  const int kq = (int)(tk % nkq), tile = (int)(tk / nkq);
  const int grp = lane / kRecGroupLanes;
  const int p0 = kq * kInlistBins;
  const bool direct = g.tile_direct[tile] != 0;
  const int eb = inw_entry_bits(BB);
  const int cap = g.inw_cap;
  const int j = tile * kTile + lane;
  const bool valid = j < g.n;
  const int rb = valid ? g.row_ptr[j] : 0;
  const int re = valid ? g.row_ptr[j + 1] : 0;
  const uint32_t *mw = g.smask + (int64_t)(p0 >> 5) * (g.n_edges + 1);
  const int sh = p0 & 31;
  // records per bin position of the group: this lane's count, then (fill)
  // where its next record goes
  int rc[kInlistBins];
#pragma unroll
  for (int b = 0; b < kInlistBins; ++b) rc[b] = 0;
  uint64_t w[KQ];
  int c[KQ];
  uint32_t flag = 0;
  auto walk = [&](bool write) {
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      w[q] = 0;
      c[q] = 0;
    }
    flag = 0;
#pragma unroll 4
    for (int e = rb; e < re; ++e) {
      const uint32_t m16 = (mw[e] >> sh) & 0xFFFFu;
      if (m16 == 0u) continue;
      const int s = e - rb;
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const uint32_t nib = (m16 >> (q * BB)) & ((1u << BB) - 1u);
        if (nib == 0u) continue;
        if (c[q] < cap && s < kSlotRows) {
          w[q] |= (uint64_t)((uint32_t)s | (nib << 5)) << (eb * c[q]);
          ++c[q];
        } else {
          flag |= 1u << q;
          const uint32_t idx = (uint32_t)sender_index(g, direct, e, rb);
#pragma unroll
          for (int b = 0; b < BB; ++b) {
            if (!((nib >> b) & 1u)) continue;
            const int pb = q * BB + b;
            if (!write) ++rc[pb];
            else if (rc[pb] < g.rec_cap)
              g.rec[rc[pb]++] = ((uint32_t)lane << 26) | ((uint32_t)b << 24) | idx;
          }
        }
      }
    }
    // source shares come after the transported photons of the bin
    if (valid) {
      for (int qq = g.em_ptr[j]; qq < g.em_ptr[j + 1]; ++qq) {
        const int pe = (int)g.bpos[g.em_k[qq]] - p0;
        if (pe < 0 || pe >= kInlistBins) continue;
        flag |= 1u << (pe / BB);
        // the counter by a compile-time index (no indexed register array)
#pragma unroll
        for (int pb = 0; pb < kInlistBins; ++pb) {
          if (pb != pe) continue;
          if (!write) ++rc[pb];
          else if (rc[pb] < g.rec_cap)
            g.rec[rc[pb]++] = ((uint32_t)lane << 26) | ((uint32_t)(pb % BB) << 24) |
                              kRecEmission | (uint32_t)qq;
        }
      }
    }
  };
  uint8_t *rl = g.rec_lane + (int64_t)tile * K * kTile + lane;
  if (!FILL) {
    walk(false);
    // sum over the 8 lanes of the group; its first lane writes
#pragma unroll
    for (int b = 0; b < kInlistBins; ++b) {
      int v = rc[b];
      const int p = p0 + b;
      if (p < K) rl[p * kTile] = (uint8_t)(v < 255 ? v : 255);
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      if ((lane & 7) == 0 && p < K) g.rec_cnt[((int64_t)tile * K + p) * kRecGroups + grp] = v;
    }
    return;
  }
  // this lane's counts from pass 1
  bool sat = false;
#pragma unroll
  for (int b = 0; b < kInlistBins; ++b) {
    const int p = p0 + b;
    rc[b] = p < K ? (int)rl[p * kTile] : 0;
    sat |= rc[b] == 255;
  }
  if (__ballot(sat)) {
#pragma unroll
    for (int b = 0; b < kInlistBins; ++b) rc[b] = 0;
    walk(false);
  }
  // this lane's first record per bin: the group's offset plus the counts of
  // the group's lower lanes (inclusive scan over 8 lanes, minus its own)
#pragma unroll
  for (int b = 0; b < kInlistBins; ++b) {
    const int own = rc[b];
    int v = own;
#pragma unroll
    for (int d = 1; d < 8; d <<= 1) {
      const int u = __shfl_up(v, d, 8);
      if ((lane & 7) >= d) v += u;
    }
    const int p = p0 + b;
    rc[b] = p < K ? g.rec_ptr[((int64_t)tile * K + p) * kRecGroups + grp] + (v - own) : 0;
  }
  walk(true);
  // in-words of the group's blocks; bit 63: the (vertex, block) has records
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int kb = kq * KQ + q;
    if (kb >= KB) break;
    uint64_t x = valid ? w[q] : 0ull;
    if (valid && ((flag >> q) & 1u)) x |= 1ull << 63;
    g.inw[((int64_t)tile * KB + kb) * kTile + lane] = x;
  }
}

// Combined transport: the bin of each in-edge (j, slot of i), which is the
// bin of the edge i -> j.  One lane per in-edge.
__global__ void k_ebin_in(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.n_edges) return;
  const int i = g.nbr[e];
  g.ebin_in[e] = g.ebin[g.row_ptr[i] + g.rev[e]];
}

// Combined transport: the bins of sender i whose selection holds receiver
// j, for every in-edge e = (j, slot of i): the set bits of the in-edge's
// selection mask (a bin with m = 0 selects no slot), as storage positions,
// ascending.  One lane per in-edge; pass 1 counts, pass 2 (after a scan)
// writes each list.
__global__ void k_kl_count(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e > g.n_edges) return;
  if (e == g.n_edges) {   // the scan's total slot
    g.kl_cnt[e] = 0;
    return;
  }
  const int64_t pl = g.n_edges + 1;
  const uint32_t *m = g.smask + e;
  g.kl_cnt[e] = __popc(m[0]) + __popc(m[pl]) + __popc(m[2 * pl]) + __popc(m[3 * pl]);
}

// A workgroup's 256 lists are contiguous in the pool: they are built in
// LDS and written out as aligned words (the partial words at either end,
// shared with the neighbouring workgroups, byte by byte).  A range longer
// than the LDS buffer is written directly.
constexpr int kKlStage = 16384;

__global__ __launch_bounds__(256) void k_kl_fill(const GridDev *__restrict__ gp) {
  const GridDev &g = *gp;
  __shared__ __attribute__((aligned(16))) uint8_t st[kKlStage];
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t e = e0 + threadIdx.x;
  const int64_t e1 = e0 + blockDim.x < g.n_edges ? e0 + blockDim.x : g.n_edges;
  const int64_t base = g.kl_ptr[e0], end = g.kl_ptr[e1];
  const bool staged = end - base <= kKlStage;   // the same for the whole block
  if (e < g.n_edges) {
    const uint32_t *m = g.smask + e;
    const int64_t pl = g.n_edges + 1;
    int64_t p = g.kl_ptr[e];
    for (int q = 0; q < 4; ++q) {
      uint32_t w = m[q * pl];
      while (w) {
        const int bit = __ffs(w) - 1;
        const uint8_t k = (uint8_t)(32 * q + bit);   // the bin's storage position
        if (staged) st[p - base] = k;
        else g.kl[p] = k;
        ++p;
        w &= w - 1u;
      }
    }
  }
  if (!staged) return;
  __syncthreads();
  const int64_t a = (base + 3) & ~(int64_t)3, b = end & ~(int64_t)3;
  if (a < b) {
    uint32_t *dst = (uint32_t *)(g.kl + a);
    for (int64_t q = threadIdx.x; q < (b - a) / 4; q += blockDim.x) {
      const int64_t o = a - base + 4 * q;
      dst[q] = (uint32_t)st[o] | ((uint32_t)st[o + 1] << 8) | ((uint32_t)st[o + 2] << 16) |
               ((uint32_t)st[o + 3] << 24);
    }
    for (int64_t q = base + threadIdx.x; q < a; q += blockDim.x) g.kl[q] = st[q - base];
    for (int64_t q = b + threadIdx.x; q < end; q += blockDim.x) g.kl[q] = st[q - base];
  } else {
    for (int64_t q = base + threadIdx.x; q < end; q += blockDim.x) g.kl[q] = st[q - base];
  }
}

// Bin of each source share: the bin closest to the direction its photons
// travel in, the edge from the source (the edge-bin rule) or, for a beam
// share, the beam's direction.
__global__ void k_em_bins(GridDev *__restrict__ gp, int64_t n_em) {
  GridDev &g = *gp;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_em) return;
  const int32_t bs = g.em_beam ? g.em_beam[q] : -1;
  const double *ed = bs >= 0 ? &g.beam_dir[3 * (int64_t)bs] : &g.edir[3 * (int64_t)g.em_edge[q]];
  int best = 0;
  double cb = cosine3(ed, &g.bins[0]);
  for (int k = 1; k < g.k; ++k) {
    const double c = cosine3(ed, &g.bins[3 * k]);
    if (c > cb) { cb = c; best = k; }
  }
  g.em_k[q] = best;
}

// Re-binning after a rotation of the bins.  Photons keep their direction as
// closely as the rotated bins allow: what vertex j holds in old bin k (m_old
// Ipre, times T_j) moves to the new bin whose direction is closest to old
// bin k's.  The map gives, for every new bin (by storage position), the old
// bins it takes (ascending); their holdings add up in that order and are split over the
// new bin's m_new selected neighbours, or leave the domain (escape tally)
// where m_new = 0.  A new bin fed by one old bin with the same m keeps its
// Ipre as it is.  Thread = vertex, tile = wave; the new field is written to
// the other photon buffer (the one the next sweep would overwrite), with T
// and any per-step state of combined transport and diffuse radiation copied
// across, and k_flip then makes it current.  A workgroup is one tile: it
// stages the tile's old field in LDS first (one 16-byte load per lane and
// block, all in flight together) and the map beside it, so the walk over
// the new bins reads only LDS.  The tile's escapes are summed by a
// butterfly.
constexpr int kRebinChunk = 12;   // 16-byte loads per lane in flight
template <typename P>
__host__ __device__ constexpr int64_t rebin_lds_bytes(int kb) {
  // old holdings by storage position, then the old m words
  return (int64_t)kb * (kBlockBytes / sizeof(P)) * 64 * sizeof(P) + 6 * 64 * 4;
}
template <typename P>
__global__ __launch_bounds__(64) void k_rebin(GridDev *__restrict__ gp, RebinMap map) {
  constexpr int BB = kBlockBytes / sizeof(P);
  typedef P V __attribute__((ext_vector_type(BB)));
  extern __shared__ __attribute__((aligned(16))) unsigned char rebin_lds[];
  __shared__ uint8_t mptr[132], mlist[128];
  const int tile = (int)blockIdx.x, lane = (int)threadIdx.x;
  const int j = tile * 64 + lane;
  // everything the walk needs, read once
  const int K = gp->k, KB = gp->kb, kw = gp->kw;
  const int par = gp->parity;
  const SX_G V *__restrict__ oin = gld((const V *)gp->o[par]) + (int64_t)tile * KB * 64 + lane;
  SX_G V *__restrict__ oout = gst((V *)gp->o[par ^ 1]) + (int64_t)tile * KB * 64 + lane;
  SX_G uint32_t *__restrict__ mb = gst(gp->mbits) + (int64_t)tile * kw * 64 + lane;
  const SX_G uint32_t *__restrict__ mb2 = gld(gp->mbits2) + (int64_t)tile * kw * 64 + lane;
  P *ro = (P *)rebin_lds;                                            // [p * 64 + lane]
  uint32_t *mol = (uint32_t *)(rebin_lds + (int64_t)KB * BB * 64 * sizeof(P));   // [q * 64 + lane]
  for (int i = lane; i < 132; i += 64) mptr[i] = map.ptr[i];
  for (int i = lane; i < 128; i += 64) mlist[i] = map.list[i];
  for (int c = 0; c < KB; c += kRebinChunk) {
    V v[kRebinChunk];
#pragma unroll
    for (int i = 0; i < kRebinChunk; ++i)
      if (c + i < KB) v[i] = oin[(c + i) * 64];
#pragma unroll
    for (int i = 0; i < kRebinChunk; ++i)
      if (c + i < KB) {
#pragma unroll
        for (int b = 0; b < BB; ++b) ro[((c + i) * BB + b) * 64 + lane] = v[i][b];
      }
  }
  // old and new m, 16 bins per word in storage order; the old words go to
  // LDS before the new ones replace them
  uint32_t mw[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    mw[q] = q < kw ? mb2[q * 64] : 0u;
    if (q < kw) mol[q * 64 + lane] = mb[q * 64];
  }
  const P Tp = gld((const P *)gp->t[par])[j];
  const double T = (double)Tp;
  __syncthreads();
  auto m_old = [&](int po) -> uint32_t {
    return (mol[(po >> 4) * 64 + lane] >> (2 * (po & 15))) & 3u;
  };
  double esc = 0.0;
  uint32_t mword = 0, cw = mw[0];
  V out = V(0);
  // new bins in storage order; every lane takes the same map entries
#pragma unroll 4
  for (int p = 0; p < K; ++p) {
    if ((p & 15) == 0 && p > 0) {
      const int q = p >> 4;
      cw = q == 1 ? mw[1] : q == 2 ? mw[2] : q == 3 ? mw[3] : q == 4 ? mw[4] : mw[5];
    }
    const uint32_t mn = (cw >> (2 * (p & 15))) & 3u;
    const int q0 = mptr[p], q1 = mptr[p + 1];
    // holdings m_old Ipre of the old bins, added in the map's order; the
    // first one's Ipre and m kept for the one-to-one case
    double h = 0.0;
    P first = P(0);
    uint32_t mfirst = 0;
    for (int q = q0; q < q1; ++q) {
      const int po = mlist[q];
      const P v = ro[po * 64 + lane];
      const uint32_t mo = m_old(po);
      if (q == q0) {
        first = v;
        mfirst = mo;
      }
      h += (double)v * (double)mo;
    }
    const bool keep = q1 - q0 == 1 && mn > 0u && mn == mfirst;
    esc += mn == 0u ? h * T : 0.0;
    const P val = keep ? first : (mn == 0u ? P(0) : (P)(h / (double)mn));
    out[p % BB] = val;
    if (p % BB == BB - 1 || p == K - 1) {
      oout[(p / BB) * 64] = out;
      out = V(0);
    }
    mword |= mn << (2 * (p & 15));
    if ((p & 15) == 15 || p == K - 1) {
      mb[(p / 16) * 64] = mword;
      mword = 0;
    }
  }
  gst((P *)gp->t[par ^ 1])[j] = Tp;
  if (gp->lay[0]) gp->lay[par ^ 1][j] = gp->lay[par][j];
  if (gp->oe[0])
    for (int e = gp->row_ptr[j]; e < gp->row_ptr[j + 1]; ++e)
      ((P *)gp->oe[par ^ 1])[e] = ((const P *)gp->oe[par])[e];
  if (gp->dsh[0]) ((P *)gp->dsh[par ^ 1])[j] = ((const P *)gp->dsh[par])[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) esc += __shfl_xor(esc, off);
  if (lane == 0) {
    gp->tally[(int64_t)tile * 3 + 1] += esc;
    gp->tally[(int64_t)tile * 3 + 2] -= esc;
  }
}

// After a re-binning: the other photon buffer becomes current.
__global__ void k_flip(GridDev *gp) { gp->parity ^= 1; }

// Exclusive scan of n counts into ptr[0..n] (ptr[n] = total) in three
// passes: each workgroup of 1024 scans its part and leaves its total in
// part[], one workgroup scans the totals, each part adds its offset.
__global__ __launch_bounds__(1024) void k_scan_part(const int32_t *__restrict__ cnt,
                                                    int32_t *__restrict__ ptr,
                                                    int64_t *__restrict__ part, int32_t n) {
  __shared__ int64_t ws[16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * 1024 + t;
  const int64_t v = i < n ? cnt[i] : 0;
  int64_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) ws[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int64_t z = lane < 16 ? ws[lane] : 0;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int64_t y = __shfl_up(z, off);
      if (lane >= off) z += y;
    }
    if (lane < 16) ws[lane] = z;
  }
  __syncthreads();
  if (i < n) ptr[i] = (int32_t)(x - v + (wave > 0 ? ws[wave - 1] : 0));
  if (t == 0) part[blockIdx.x] = ws[15];
}

// Exclusive scan of the nb part totals in place (part[nb] = total), one
// workgroup, any nb.
__global__ __launch_bounds__(1024) void k_scan_top(int64_t *__restrict__ part, int32_t nb) {
  __shared__ int64_t acc[1024];
  const int t = threadIdx.x;
  const int64_t chunk = ((int64_t)nb + 1023) / 1024;
  const int64_t b = t * chunk;
  const int64_t e = b + chunk < nb ? b + chunk : nb;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += part[i];
  acc[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? acc[t - off] : 0;
    __syncthreads();
    acc[t] += v;
    __syncthreads();
  }
  int64_t run = acc[t] - s;
  for (int64_t i = b; i < e; ++i) {
    const int64_t c = part[i];
    part[i] = run;
    run += c;
  }
  if (t == 1023) part[nb] = acc[1023];
}

__global__ __launch_bounds__(1024) void k_scan_add(int32_t *__restrict__ ptr,
                                                   const int64_t *__restrict__ part,
                                                   int32_t n, int32_t nb) {
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < n) ptr[i] += (int32_t)part[blockIdx.x];
  if (i == 0) ptr[n] = (int32_t)part[nb];
}

// ---------------------------------------------------------- chemistry ---
// One backward-Euler substep of the rate equation for the neutral fraction
// (Eqs. rate_eq, rate_eq_subcycle, phot_ion_rate_subcycle; on the spot,
// n_e = n_HII):  y' = y - ha (1 - exp(-y' tau)) + hb (1 - y')^2, solved by
// safeguarded Newton inside the bracket [0, 1].
// Also returns 1 - exp(-y tau) at the root (from the last Newton
// evaluation when the final step is within rounding of y).
__device__ __forceinline__ double be_substep(double y0, double ha, double hb,
                                             double tau, double &ion_root) {
  double lo = 0.0, hi = 1.0, yn = y0;
  for (int it = 0; it < 200; ++it) {
    const double ion = -expm1(-yn * tau);
    const double x = 1.0 - yn;
    const double g = (y0 - yn) - ha * ion + hb * (x * x);
    if (g == 0.0) {
      ion_root = ion;
      return yn;
    }
    if (g > 0.0) lo = yn; else hi = yn;
    const double gp = -1.0 - ha * tau * (1.0 - ion) - 2.0 * hb * x;
    const double d = g / gp;
    if (fabs(d) <= 4.0e-16 * yn) {   // Newton step within rounding of y
      const double yc = yn - d;
      ion_root = ion;
      return yc < 0.0 ? 0.0 : (yc > 1.0 ? 1.0 : yc);
    }
    double yc = yn - d;
    if (!(yc > lo && yc < hi)) yc = 0.5 * (lo + hi);
    yn = yc;
    if (hi - lo <= 4.0e-16 * hi) break;
  }
  ion_root = -expm1(-yn * tau);
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
    double ion;
    y = be_substep(y, ha, hb, tau, ion);
    abs_sum += share * ion;
    // exp(-y tau): 1 - ion where that loses nothing; in a thick cell ion
    // rounds towards 1 and the difference would cancel to 0
    tr_sum += ion < 0.5 ? 1.0 - ion : exp(-y * tau);
  }
  A = abs_sum;
  T = nin > 0.0 ? tr_sum / (double)n_sub : 1.0;
  return y;
}

// The same with the recombinations per atom of the step, R = sum over the
// substeps of h b (1 - y')^2 (the b term of each backward-Euler update).
__device__ __forceinline__ double chem_step_r(double y, double nin, double dt,
                                              double dtnhv, double tau, double b,
                                              int n_sub, double &A, double &T,
                                              double &R) {
  const double h = dt / (double)n_sub;
  const double a = nin / dtnhv;
  const double ha = h * a, hb = h * b;
  const double share = nin / (double)n_sub;
  double abs_sum = 0.0, tr_sum = 0.0, rec_sum = 0.0;
  for (int s = 0; s < n_sub; ++s) {
    double ion;
    y = be_substep(y, ha, hb, tau, ion);
    abs_sum += share * ion;
    tr_sum += ion < 0.5 ? 1.0 - ion : exp(-y * tau);
    const double x = 1.0 - y;
    rec_sum += hb * (x * x);
  }
  A = abs_sum;
  T = nin > 0.0 ? tr_sum / (double)n_sub : 1.0;
  R = rec_sum;
  return y;
}

// After the last hop of a multi-hop step: the photons a vertex absorbed
// over the step (ion per atom, at most y) ionise exactly as many atoms,
// spread evenly over the substeps; each substep takes the recombinations
// backward Euler, y' = y - i + hb (1 - y')^2, whose root in [0, 1] is
// y' = 1 - z, z = 2c / (1 + sqrt(1 + 4 hb c)), c = 1 - y + i (z = c when
// hb = 0).
__device__ __forceinline__ double chem_fixed(double y, double ion, double hb, int n_sub) {
  const double is = ion / (double)n_sub;
  for (int s = 0; s < n_sub; ++s) {
    const double c = (1.0 - y) + is;
    const double z = hb > 0.0 ? (2.0 * c) / (1.0 + sqrt(1.0 + 4.0 * hb * c)) : c;
    y = 1.0 - z;
    if (y < 0.0) y = 0.0;
  }
  return y;
}

// -------------------------------------------------------------- sweep ---
// State between steps: for every vertex i and bin k, Ipre[k][i] = I/m, the
// photons that entered i in bin k divided over its m selected neighbours,
// and per vertex the fraction T_i it passed on.  A neighbour receives
// Ipre * T_i from i, which is the outgoing share I T / m of the method.
// Keeping T apart lets a step write each bin the moment it is gathered.
//
// One radiative-transfer step of one tile (Sect. 4.6: photons move one edge
// and interact once).  Lane = receiver j of the 64-vertex tile.
// 1. Per bin k: I = photons arriving at j in bin k, summed over its senders
//    in ascending sender id, then its source shares.  A staged tile copies
//    the bin's Ipre * T of its whole halo into LDS (kStageQ coalesced loads
//    per lane); each lane then reads its seven in-word senders from LDS
//    (slot kZeroSlot holds 0, so every read is unconditional).  Loads for
//    bin k + 2 are in flight while bin k is summed.  Records (senders beyond
//    the seventh, source shares) go lane-parallel: record r to lane r, runs
//    of records for one receiver summed by a segmented scan (only when a
//    receiver has two), sums handed over through LDS.
//    Ipre'[k][j] = I / m(j,k) is stored at once; N_in and the photons of
//    bins with no forward neighbour (m = 0, they leave the domain) add up.
// 2. Chemistry in fp64 -> y, absorbed A, transmitted fraction T' of j.
// 3. Per-tile photon accounting in fp64, fixed-order wave reduction.
// LDS of one wave of the tile code: the staged halo block (vertex-major, one
// 16-byte block per halo vertex; entry kHaloMax reads 0), the halo index of
// every row slot of every lane (row s at s * 64 + lane), and the hand-over
// slots of the records.
// Orders this wave's LDS accesses at this point: the wave barrier keeps the
// hardware's issue order, the empty asm with a memory clobber stops the
// compiler from moving a memory access across it.  Between two of these, a
// wave may read LDS through plain pointers, so that its loads batch.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// a + v where bit b of x is set, else a + 0 (the same bits as skipping the
// add: the sums are never -0); branch-free, by masking v's bits
// a + v where bit `pos` (0..63, a constant once unrolled) of w is set, else
// a + 0: the bit is extended to a mask of all ones or zeros (one bit-field
// extract, no compare and select) and ANDed into v.
__device__ __forceinline__ int bit_mask(uint64_t w, int pos) {
  return pos < 32 ? __builtin_amdgcn_sbfe((int)(uint32_t)w, pos, 1)
                  : __builtin_amdgcn_sbfe((int)(uint32_t)(w >> 32), pos - 32, 1);
}
__device__ __forceinline__ float add_if_bit(float a, float v, uint64_t w, int pos) {
  return a + __int_as_float(__float_as_int(v) & bit_mask(w, pos));
}
__device__ __forceinline__ double add_if_bit(double a, double v, uint64_t w, int pos) {
  return a + __longlong_as_double(__double_as_longlong(v) & (long long)bit_mask(w, pos));
}

template <typename P>
struct __attribute__((aligned(16))) TileLds {
  static constexpr int BB = kBlockBytes / sizeof(P);
  P h[(kHaloMax + 1) * BB];
  uint16_t slot[kSlotRows * kTile];
  P x[kTile * BB];
};

// What a combined-transport step hands the tile code (CT = true): whether
// this lane's vertex is ballistic (then its bins are written as zeros and
// its N_in and escapes come from the per-edge sums), and for a
// direction-conserving vertex the bins that receive photons from ballistic
// senders: their sums wait in xin (element (j, k) in the layout of o[]),
// flagged per block in xmask, and are added and cleared there.
template <typename P>
struct CtIn {
  bool bal = false;
  double y0 = 1.0;
  P nin_b = P(0), esc_b = P(0);
  uint64_t xmask = 0;   // one bit per 16-byte block (up to 48)
  P *xin = nullptr;
};

// End of a combined-transport (or diffuse) step for one lane: chemistry,
// the recombination photons it sends next step, the tile's accounting.
template <typename P>
__device__ __forceinline__ void ct_finish(const GridDev *__restrict__ G, int tile, int lane,
                                          bool valid, double y0, P nin_p, P esc_p) {
  const int j = tile * kTile + lane;
  const int par = G->parity;
  double A = 0.0, T = 1.0, R = 0.0;
  const double nin = (double)nin_p;
  double made = 0.0, lost = 0.0;   // recombination photons / unit
  if (valid) {
    if (!(nin == 0.0 && y0 == 1.0)) {
      double yn;
      if (G->diffuse)
        yn = chem_step_r(y0, nin * G->unit, G->dt, gld(G->dtnhv)[j], gld(G->tau)[j],
                         gld(G->bcoef)[j], G->n_sub, A, T, R);
      else
        yn = chem_step(y0, nin * G->unit, G->dt, gld(G->dtnhv)[j], gld(G->tau)[j],
                       gld(G->bcoef)[j], G->n_sub, A, T);
      gst(G->y)[j] = yn;
    }
    gst(G->nin)[j] = nin * G->unit;
    gst((P *)G->t[par ^ 1])[j] = (P)T;
    if (G->diffuse) {
      made = ((gld(G->nhv)[j] * R) * G->dfrac) / G->unit;
      const int deg = gld(G->row_ptr)[j + 1] - gld(G->row_ptr)[j];
      // a vertex with no neighbour: what it made last step leaves now
      if (deg == 0) lost = (double)gld((const P *)G->dsh[par])[j];
      gst((P *)G->dsh[par ^ 1])[j] = deg > 0 ? (P)(made / (double)deg) : (P)made;
    }
  }
  A /= G->unit;
  double esc = (double)esc_p * T + lost;
  double fly = (nin - (double)esc_p) * T + made;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    A += __shfl_xor(A, off);
    esc += __shfl_xor(esc, off);
    fly += __shfl_xor(fly, off);
    made += __shfl_xor(made, off);
  }
  if (lane == 0) {
    SX_G double *t = gst(G->tally) + (int64_t)tile * 3;
    t[0] += A;
    t[1] += esc;
    t[2] = fly;
    if (G->diffuse) gst(G->dtally)[tile] += made;
  }
}

// A lane's N_in and escaping photons, summed over the bins in an order that
// does not depend on how the tile's bin blocks are split over waves: the
// blocks fall into four groups (group g holds blocks [g KB / 4, (g + 1) KB /
// 4)), each group is summed bin by bin, and the group sums are added left to
// right.  A wave that runs groups [g0, g1) keeps the running total of its
// groups and the sums of its first two (to hand over to the wave that adds
// them to its own).
template <typename P>
struct BinSums {
  P tot_n = P(0), tot_e = P(0);
  P cur_n = P(0), cur_e = P(0);
  P hn0 = P(0), hn1 = P(0), he0 = P(0), he1 = P(0);
  int g = 0, gi = 0;
  __device__ __forceinline__ void close() {
    tot_n += cur_n;
    tot_e += cur_e;
    if (gi == 0) {
      hn0 = cur_n;
      he0 = cur_e;
    } else {
      hn1 = cur_n;
      he1 = cur_e;
    }
    cur_n = P(0);
    cur_e = P(0);
    ++g;
    ++gi;
  }
};

// Chemistry and accounting of one lane of a direction-conserving tile after
// its bins: the backward-Euler update from N_in, T for the next sweep, and
// the tile's tallies by a fixed butterfly.
template <typename P>
__device__ __forceinline__ void dct_finish(const GridDev *__restrict__ G, int tile, int lane,
                                           P nin_p, P esc_p) {
  const int j = tile * kTile + lane;
  const int par = G->parity;
  double A = 0.0, T = 1.0;
  const double nin = (double)nin_p;
  if (j < G->n) {
    SX_G double *__restrict__ yv = gst(G->y);
    const double y0 = yv[j];
    if (G->hops > 1) {
      // one hop of a multi-hop step: absorb 1 - exp(-y tau) of the photons
      // at the y of the start of the step, capped by the atoms left
      const double nph = nin * G->unit;
      const double nhv = gld(G->nhv)[j];
      SX_G double *__restrict__ ha = gst(G->habs);
      SX_G double *__restrict__ hn = gst(G->hnin);
      double hab = ha[j];
      double cap = nhv * y0 - hab;
      if (cap < 0.0) cap = 0.0;
      T = exp(-y0 * gld(G->tau)[j]);
      double a = nph - nph * T;
      if (a > cap) {
        a = cap;
        T = (nph - a) / nph;
      }
      A = a;
      hab += a;
      const double hin = hn[j] + nph;
      if (G->sweeps % G->hops == G->hops - 1) {
        // the step's last hop: the neutral fraction from what was absorbed
        const double hb = (G->dt / (double)G->n_sub) * gld(G->bcoef)[j];
        yv[j] = chem_fixed(y0, hab / nhv, hb, G->n_sub);
        gst(G->nin)[j] = hin;
        ha[j] = 0.0;
        hn[j] = 0.0;
      } else {
        ha[j] = hab;
        hn[j] = hin;
      }
    } else {
      if (!(nin == 0.0 && y0 == 1.0)) {
        const double yn = chem_step(y0, nin * G->unit, G->dt, gld(G->dtnhv)[j],
                                    gld(G->tau)[j], gld(G->bcoef)[j], G->n_sub, A, T);
        yv[j] = yn;
      }
      gst(G->nin)[j] = nin * G->unit;
    }
    gst((P *)G->t[par ^ 1])[j] = (P)T;
  }
  A /= G->unit;   // tallies in stored units; scaled back on read
  double esc = (double)esc_p * T;
  double fly = (nin - (double)esc_p) * T;

  // Fixed butterfly: every lane ends with the same, order-determined sum.
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    A += __shfl_xor(A, off);
    esc += __shfl_xor(esc, off);
    fly += __shfl_xor(fly, off);
  }
  if (lane == 0) {
    SX_G double *t = gst(G->tally) + (int64_t)tile * 3;
    t[0] += A;
    t[1] += esc;
    t[2] = fly;
  }
}

// The bins of one tile in blocks [kb0, kb1) (groups [g0, g1) of BinSums):
// gather, overflow records, outgoing photons; the sums go to bs.
template <typename P, bool DIRECT, bool CT = false, bool NT = false>
__device__ __forceinline__ void sweep_bins(const GridDev *__restrict__ G, int tile,
                                           int lane, SX_L TileLds<P> *L, const CtIn<P> &ci,
                                           int kb0, int kb1, int g0, int g1,
                                           BinSums<P> &bs) {
  // The LDS carries data between lanes of this wave.  The accesses are
  // volatile so that the compiler keeps every store and load in program
  // order (it may not forward a lane's own store past another lane's); LDS
  // executes a wave's operations in issue order.
  constexpr int BB = kBlockBytes / sizeof(P);
  typedef P V __attribute__((ext_vector_type(BB)));
  constexpr int NQ = DIRECT ? 1 : kStageQ;
  constexpr int EB = inw_entry_bits(BB);
  constexpr int NE = inw_entries(BB);
  constexpr uint32_t EM = (1u << EB) - 1u;
  volatile SX_L V *hl = (volatile SX_L V *)L->h;
  volatile SX_L uint16_t *stab = (volatile SX_L uint16_t *)L->slot;
  volatile SX_L P *xchg = (volatile SX_L P *)L->x;
  const int K = G->k;
  const int KB = G->kb;
  const int j = tile * kTile + lane;
  const bool valid = j < G->n;
  const int par = G->parity;
  const SX_G V *__restrict__ oin = gld((const V *)G->o[par]);
  const SX_G P *__restrict__ tin = gld((const P *)G->t[par]);
  SX_G V *__restrict__ oout = gst((V *)G->o[par ^ 1]);
  const SX_G int32_t *__restrict__ nbr = gld(G->nbr);
  const SX_G int32_t *__restrict__ rowp = gld(G->row_ptr);
  const int rb = rowp[j];
  const SX_G uint64_t *__restrict__ iw = gld(G->inw + (int64_t)tile * KB * kTile + lane);
  const SX_G int32_t *__restrict__ rptr = gld(G->rec_ptr) + (int64_t)tile * K * kRecGroups;
  const SX_G uint32_t *__restrict__ rec = gld(G->rec);
  // first record of every block of the range, lane l holding block kb0 + l's
  // (KB < 64), so that no load inside the block loop waits on another
  const int kl_ = kb0 + lane;
  const int rpl = kl_ <= kb1 ? rptr[(kl_ * BB < K ? kl_ * BB : K) * kRecGroups] : 0;
  const SX_G double *__restrict__ ema = gld(G->em_amt);
  // block of (vertex v, block kb)
  auto blk = [&](uint32_t v, int kb) -> uint32_t {
    return ((v >> 6) * (uint32_t)KB + (uint32_t)kb) * 64u + (v & 63u);
  };

  // halo of the tile and its senders' T (once per step), and the halo index
  // of every row slot an in-word entry can name; hb: the block index of each
  // staged halo vertex's block 0 (block kb is 64 kb further on)
  uint32_t hv[NQ], hb[NQ];
  P th[NQ];
  if constexpr (!DIRECT) {
    const SX_G int32_t *__restrict__ hptr = gld(G->halo_ptr);
    const int hp = hptr[tile];
    const int hlen = hptr[tile + 1] - hp;
    const SX_G int32_t *__restrict__ hvid = gld(G->halo_vid);
    const uint32_t zero = (uint32_t)G->npad;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = 64 * q + lane;
      hv[q] = idx < hlen ? (uint32_t)hvid[hp + idx] : zero;
      th[q] = tin[hv[q]];
      hb[q] = ((hv[q] >> 6) * (uint32_t)KB) * 64u + (hv[q] & 63u);
    }
    if (lane == 0) hl[kHaloMax] = V(0);
    const int deg = valid ? rowp[j + 1] - rb : 0;
    const SX_G uint16_t *__restrict__ eh = gld(G->edge_hidx) + rb;
#pragma unroll
    for (int s = 0; s < kSlotRows; ++s) {
      uint16_t h = (uint16_t)kHaloMax;
      if (s < deg) h = eh[s];
      stab[s * kTile + lane] = h;
    }
  }
  // packed m(j, k), 16 bins per word, consumed 2 bits at a time from the
  // range's first bin
  const int k0 = kb0 * BB;
  const SX_G uint32_t *__restrict__ mbp =
      gld(G->mbits) + ((int64_t)tile * G->kw + (k0 >> 4)) * 64 + lane;
  uint32_t mwv[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) mwv[q] = (k0 >> 4) + q < G->kw ? mbp[q * 64] : 0u;
  mwv[0] >>= 2 * (k0 & 15);

  // ring of loads in flight, slot = block mod 2
  V st[2][NQ];
  uint64_t wq[2];
  uint32_t rq[2];   // this lane's first record of the block (if lane < rn)
  int rn[2];        // records of the block
  int rs[2];        // index of the block's first record
  auto issue = [&](int kb, int slot) {
    if constexpr (!DIRECT) {
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        st[slot][q] = oin[hb[q] + (uint32_t)kb * 64u];
    }
    // in-words are read once per sweep.  With NT (the launch's photon planes
    // fit in the last-level cache) they are loaded non-temporal, so that they
    // do not displace the planes the next sweep reads back.
    if constexpr (NT)
      wq[slot] = __builtin_nontemporal_load(&iw[(int64_t)kb * kTile]);
    else
      wq[slot] = iw[(int64_t)kb * kTile];
    const int r0 = __builtin_amdgcn_readlane(rpl, kb - kb0);
    const int nr = __builtin_amdgcn_readlane(rpl, kb - kb0 + 1) - r0;
    rn[slot] = nr;
    rs[slot] = r0;
    // unconditional and in bounds (the pool holds one spare entry); lanes
    // past the block's records are masked where the value is used
    rq[slot] = rec[r0 + (lane < nr ? lane : (nr > 0 ? nr - 1 : 0))];
  };

  bs.g = g0;
  auto block = [&](int kb, int slot) {
    // always issued (the last block re-reads itself from L2): a load that
    // is skipped on some path leaves the wait counts conservative, and the
    // wave would stall on the loads it has just issued
    issue(kb + 1 < kb1 ? kb + 1 : kb, slot ^ 1);
    while (((bs.g + 1) * KB >> 2) <= kb) bs.close();
    const uint64_t w = wq[slot];
    P acc[BB];
#pragma unroll
    for (int b = 0; b < BB; ++b) acc[b] = P(0);
    if constexpr (!DIRECT) {
      // the halo's block, attenuated by each sender's T, one 16-byte entry
      // per halo vertex
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const V v = st[slot][q];
        V a;
#pragma unroll
        for (int b = 0; b < BB; ++b) a[b] = mul_rn(v[b], th[q]);
        hl[64 * q + lane] = a;
      }
      wave_sync();
      // every entry: its sender's block from LDS, added to the bins it
      // sends (an entry without bins adds zeros); the slot-table reads of
      // all entries go out together, then the halo reads
      const SX_L uint16_t *stn = (const SX_L uint16_t *)L->slot + lane;
      const SX_L V *hln = (const SX_L V *)L->h;
      uint32_t hx[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) hx[e] = stn[((uint32_t)(w >> (EB * e)) & 31u) * kTile];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const V v = hln[hx[e]];
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] = add_if_bit(acc[b], v[b], w, EB * e + 5 + b);
      }
    } else {
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const uint32_t x = (uint32_t)(w >> (EB * e)) & EM;
        const uint32_t nib = x >> 5;
        if (nib != 0u) {
          const uint32_t src = (uint32_t)nbr[rb + (int)(x & 31u)];
          const V v = oin[blk(src, kb)];
          const P t = tin[src];
#pragma unroll
          for (int b = 0; b < BB; ++b)
            if ((nib >> b) & 1u) acc[b] += mul_rn(v[b], t);
        }
      }
    }
    // The block's records (senders beyond the in-word's entries, then source
    // shares), sorted by bin then receiver: lane r fetches record r's
    // photons, runs of one receiver and bin are summed by a segmented scan
    // across lanes (DPP, no LDS), and the last lane of each run hands the
    // sum over through LDS.  Receivers whose in-word flags records (bit 63)
    // clear their hand-over slots first and read them back after.
    const int nrec = __builtin_amdgcn_readfirstlane(rn[slot]);
    const bool fl = (w >> 63) != 0ull;
    for (int c0 = 0; c0 < nrec; c0 += 64) {
      const uint32_t r = lane >= nrec - c0 ? ~0u
                         : (c0 == 0 ? rq[slot] : rec[rs[slot] + c0 + lane]);
      const bool has = r != ~0u;
      // key = bin-in-block * 64 + receiver lane; records are sorted by key
      const int key = has ? (int)(((r >> 24) & 3u) * 64u + (r >> 26)) : -1 - lane;
      const uint32_t idx = r & kRecIdxMask;
      const int rb_ = (int)((r >> 24) & 3u);
      P v = P(0);
      if (has) {
        if (r & kRecEmission) {
          v = (P)ema[idx];
        } else if constexpr (!DIRECT) {
          v = ((volatile SX_L P *)hl)[idx * BB + rb_];
        } else {
          const uint32_t src = (uint32_t)nbr[rowp[tile * kTile + (int)(r >> 26)] + idx];
          v = mul_rn(((const SX_G P *)oin)[blk(src, kb) * BB + rb_], tin[src]);
        }
      }
      const int knext = dpp_i32<kDppWaveShl1, 0xF>(-3000, key);
      if (__ballot(has && knext == key)) seg_scan<P>(v, key);
      // with more than 64 records every lane takes part in every round
      const bool take = fl || nrec > 64;
      if (take) *(volatile SX_L V *)(xchg + lane * BB) = V(0);
      wave_sync();
      if (has && knext != key) xchg[(int)(r >> 26) * BB + rb_] = v;
      wave_sync();
      if (take) {
        const V got = *(volatile SX_L V *)(xchg + lane * BB);
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] += got[b];
      }
      wave_sync();
    }
    wave_sync();
    if constexpr (CT) {
      if ((ci.xmask >> kb) & 1ull) {
        SX_G V *xp = (SX_G V *)ci.xin + blk((uint32_t)j, kb);
        const V xv = *xp;
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] += xv[b];
        *xp = V(0);
      }
    }
    V out;
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      const int k = kb * BB + b;
      P ipre = P(0);
      if (k < K) {
        const uint32_t m = mwv[0] & 3u;
        mwv[0] >>= 2;
        if ((k & 15) == 15) {
#pragma unroll
          for (int q = 0; q < 5; ++q) mwv[q] = mwv[q + 1];
        }
        bs.cur_n += acc[b];
        if constexpr (sizeof(P) == 8) {
          bs.cur_e += m == 0u ? acc[b] : P(0);
          ipre = m == 0u ? 0.0 : (m == 1u ? acc[b] : (m == 2u ? acc[b] * 0.5 : acc[b] / 3.0));
        } else {
          // no branches: the escape share through a mask that is all ones
          // iff m = 0, and 1/m for m = 0..3 as m (85 + m (11 m - 60)) / 36
          // (0, 1, 1/2 and 1/3 rounded to float; 0 where nothing is chosen)
          const int em = ((int)m - 1) >> 31;
          bs.cur_e += __int_as_float(__float_as_int(acc[b]) & em);
          const int mi = (int)m;
          const float fm = (float)(mi * (85 + mi * (11 * mi - 60))) * (1.0f / 36.0f);
          ipre = acc[b] * fm;
        }
      }
      out[b] = ipre;
    }
    if constexpr (CT) {
      if (ci.bal) out = V(0);
    }
    if (valid) oout[blk((uint32_t)j, kb)] = out;
  };

  if (kb0 < kb1) issue(kb0, 0);
  for (int kb = kb0; kb < kb1; kb += 2) {
    block(kb, 0);
    if (kb + 1 < kb1) block(kb + 1, 1);
  }
  while (bs.g < g1) bs.close();
}

// One whole direction-conserving tile (every bin, then chemistry); with CT,
// the direction-conserving part of a combined-transport tile.
template <typename P, bool DIRECT, bool CT = false, bool NT = false>
__device__ __forceinline__ void sweep_tile(const GridDev *__restrict__ G, int tile,
                                           int lane, SX_L TileLds<P> *L,
                                           const CtIn<P> &ci = CtIn<P>()) {
  BinSums<P> bs;
  sweep_bins<P, DIRECT, CT, NT>(G, tile, lane, L, ci, 0, G->kb, 0, 4, bs);
  if constexpr (CT) {
    P nin_p = bs.tot_n, esc_p = bs.tot_e;
    if (ci.bal) {
      nin_p = ci.nin_b;
      esc_p = ci.esc_b;
    }
    ct_finish<P>(G, tile, lane, tile * kTile + lane < G->n, ci.y0, nin_p, esc_p);
    return;
  }
  dct_finish<P>(G, tile, lane, bs.tot_n, bs.tot_e);
}

// One sweep over a list of tiles (a batch of grids, or one grid when
// tile_map is null): workgroups of TPB waves, S waves per tile (TPB / S
// tiles per workgroup).  The S waves of a tile split its bin blocks into S
// contiguous ranges (S = 1, 2 or 4: one, two or one of the four BinSums
// groups each); the first adds the others' group sums to its own in group
// order after a barrier and runs the chemistry, so the results are bitwise
// the same for every S.  With xcd_remap, workgroup numbers are rearranged
// so that each XCD (workgroups are dealt to the 8 XCDs round-robin) runs a
// contiguous eighth of the tile list and its L2 sees one neighbourhood.
// The workgroup that finishes last flips the buffers of the listed grids and
// clears the completion counter, so consecutive launches are identical and
// need no kernel between them.
template <typename P, int TPB, int S, bool NT>
__global__ __launch_bounds__(64 * TPB, 4) void k_sweep(
    GridDev *__restrict__ grids, const int2 *__restrict__ tile_map,
    int32_t n_tiles, const int32_t *__restrict__ adv, int32_t n_adv,
    uint32_t *__restrict__ done, int32_t xcd_remap) {
  static_assert((S == 1 || S == 2 || S == 4) && TPB % S == 0, "split");
  constexpr int GPW = 4 / S;   // BinSums groups per wave
  __shared__ TileLds<P> lds[TPB];
  __shared__ int last;
  const int lane = threadIdx.x & 63;
  const int wave = TPB == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int part = wave % S;
  const uint32_t nb = gridDim.x;   // a multiple of 8
  const uint32_t b = blockIdx.x;
  const uint32_t grp = xcd_remap ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  const int gt = ((int)grp * TPB + wave) / S;
  const GridDev *__restrict__ G = grids;
  int tile = gt;
  bool act = false;
  BinSums<P> bs;
  if (gt < n_tiles) {
    int gi = 0;
    if (tile_map) {
      const int2 tm = tile_map[gt];
      gi = __builtin_amdgcn_readfirstlane(tm.x);
      tile = __builtin_amdgcn_readfirstlane(tm.y);
    }
    G = grids + gi;
    if (G->remaining > 0) {
      act = true;
      SX_L TileLds<P> *L = (SX_L TileLds<P> *)&lds[wave];
      volatile SX_L P *hl = (volatile SX_L P *)L->h;
      const int KB = G->kb;
      const int kb0 = part * KB / S, kb1 = (part + 1) * KB / S;
      if (gld(G->tile_direct)[tile] != 0)
        sweep_bins<P, true, false, NT>(G, tile, lane, L, CtIn<P>(), kb0, kb1,
                                       part * GPW, (part + 1) * GPW, bs);
      else
        sweep_bins<P, false, false, NT>(G, tile, lane, L, CtIn<P>(), kb0, kb1,
                                        part * GPW, (part + 1) * GPW, bs);
      if constexpr (S > 1) {
        // hand the group sums over in this wave's halo block (its last
        // block has read it)
        if (part > 0) {
          hl[lane] = bs.hn0;
          hl[128 + lane] = bs.he0;
          if constexpr (GPW > 1) {
            hl[64 + lane] = bs.hn1;
            hl[192 + lane] = bs.he1;
          }
        }
      }
    }
  }
  if constexpr (S > 1) __syncthreads();
  if (act && part == 0) {
    if constexpr (S > 1) {
#pragma unroll
      for (int q = 1; q < S; ++q) {
        const volatile SX_L P *o = (const volatile SX_L P *)lds[wave + q].h;
#pragma unroll
        for (int g = 0; g < GPW; ++g) {
          bs.tot_n += o[64 * g + lane];
          bs.tot_e += o[128 + 64 * g + lane];
        }
      }
    }
    dct_finish<P>(G, tile, lane, bs.tot_n, bs.tot_e);
  }
  // completion count; the last workgroup advances the grids
  __syncthreads();
  if (threadIdx.x == 0)
    last = atomicAdd(done, 1u) == nb - 1u;
  __syncthreads();
  if (!last) return;
  for (int i = threadIdx.x; i < n_adv; i += 64 * TPB) {
    GridDev &g = grids[adv ? adv[i] : i];
    if (g.remaining > 0) {
      g.parity ^= 1;
      g.remaining -= 1;
      g.sweeps += 1;
    }
  }
  if (threadIdx.x == 0) atomicExch(done, 0u);
}

// ------------------------------------------------- combined transport ---
// One step of combined transport (Sects. 2.2.2-2.2.4) for one tile; lane =
// receiver j.  j is ballistic in this step when its optical depth y tau at
// the start of the step is at least tau_switch.  Each sender i holds what it
// received in the previous step either per bin (layout 0: Ipre = I/m in
// o[], as in direction-conserving transport) or per incoming edge (layout 1:
// Ipre = I/bm in oe[]), and passes on Ipre * T_i.  What arrives along the
// edge i -> j:
//  - from a sender holding bins: the bins whose selection holds j (kl), each
//    in its own bin;
//  - from a sender holding edges: the packets whose ballistic choice holds j
//    (bl), in the bin of the edge i -> j;
//  - source shares, in the bin of the edge from the source.
// A ballistic j stores I / bm per incoming edge; a direction-conserving j
// stores I / m per bin.  Chemistry and accounting as in direction-conserving
// transport.
//
// A vertex holding edges keeps zeros in its bins (it clears them in the two
// steps after it turns ballistic, and writes zeros while it is in a tile
// that runs the bin code), so the bin gathers of the direction-conserving
// tile code read 0 from it, and only what it sends along edges is added
// apart.  Per tile:
//  1. every receiver direction-conserving and every halo sender holding
//     bins (the ionised interior): the tile code of k_sweep as it is;
//  2. otherwise the tile's incoming edges are summed one edge per lane,
//     rounds of 64 over the tile's CSR range (the static per-edge data read
//     coalesced): for a ballistic receiver everything that arrives along the
//     edge (stored at once as I / bm), for a direction-conserving one what a
//     ballistic sender sends; the sums wait in LDS.  Each receiver then adds
//     its row in order: a ballistic one its N_in and escapes, a
//     direction-conserving one files the ballistic senders' photons in xin
//     under the bin of the edge;
//  3. a tile of ballistic receivers only ends there (chemistry, tallies);
//     any other runs the tile code with those hand-overs.
constexpr int kVeCap = 1536;   // incoming edges of a tile summed through LDS

template <typename P>
__device__ __forceinline__ P div_m(P v, uint32_t m) {
  if constexpr (sizeof(P) == 8) {
    return m == 0u ? 0.0 : (m == 1u ? v : (m == 2u ? v * 0.5 : v / 3.0));
  } else {
    const float fm = (float)(int)(m * m - 6u * m + 11u) * (1.0f / 6.0f);
    return m == 0u ? 0.0f : v * fm;
  }
}

template <typename P, bool NT>
__device__ __forceinline__ void sweep_tile_ct(const GridDev *__restrict__ G, int tile,
                                              int lane, SX_L P *veb, SX_L TileLds<P> *L) {
  constexpr int BB = kBlockBytes / sizeof(P);
  typedef P V __attribute__((ext_vector_type(BB)));
  const int KB = G->kb;
  const int j = tile * kTile + lane;
  const bool valid = j < G->n;
  const int par = G->parity;
  const SX_G P *__restrict__ oin = gld((const P *)G->o[par]);
  const SX_G P *__restrict__ tin = gld((const P *)G->t[par]);
  const SX_G P *__restrict__ ein = gld((const P *)G->oe[par]);
  SX_G P *__restrict__ eout = gst((P *)G->oe[par ^ 1]);
  const SX_G uint8_t *__restrict__ lin = gld((const uint8_t *)G->lay[par]);
  SX_G uint8_t *__restrict__ lout = gst(G->lay[par ^ 1]);
  const SX_G int32_t *__restrict__ rowp = gld(G->row_ptr);
  const SX_G int32_t *__restrict__ nbr = gld(G->nbr);
  const SX_G uint8_t *__restrict__ rev = gld(G->rev);
  const SX_G uint8_t *__restrict__ ebin_in = gld(G->ebin_in);
  const SX_G int32_t *__restrict__ klp = gld(G->kl_ptr);
  const SX_G uint8_t *__restrict__ kl = gld(G->kl);
  const SX_G int32_t *__restrict__ blp = gld(G->bl_ptr);
  const SX_G int32_t *__restrict__ bl = gld(G->bl);
  const SX_G uint8_t *__restrict__ bmv = gld(G->bm);
  const SX_G uint8_t *__restrict__ elane = gld(G->elane);
  typedef int I4 __attribute__((ext_vector_type(4)));
  const SX_G I4 *__restrict__ bl4 = (const SX_G I4 *)G->bl4;
  const SX_G int32_t *__restrict__ emp = gld(G->em_ptr);
  const SX_G double *__restrict__ ema = gld(G->em_amt);
  const SX_G int32_t *__restrict__ eme = gld(G->em_edge);
  SX_G P *__restrict__ xin = gst((P *)G->xin);
  const SX_G P *__restrict__ dshin = gld((const P *)G->dsh[par]);
  const bool diffuse = G->diffuse != 0;
  // element (v, bin at storage position p) of the bin field
  auto at = [&](uint32_t v, int p) -> uint32_t {
    return (((v >> 6) * (uint32_t)KB + (uint32_t)(p / BB)) * 64u + (v & 63u)) * BB +
           (uint32_t)(p % BB);
  };
  const bool direct = gld(G->tile_direct)[tile] != 0;

  double y0 = 1.0;
  bool bal = false;
  if (valid) {
    y0 = gld(G->y)[j];
    bal = y0 * gld(G->tau)[j] >= G->tau_switch;
  }
  const uint64_t balmask = __ballot(bal);
  const uint64_t validmask = __ballot(valid);

  // 1. direction-conserving transport proper
  if (balmask == 0 && !direct && !diffuse) {
    const SX_G int32_t *__restrict__ hptr = gld(G->halo_ptr);
    const int hp = hptr[tile];
    const int hlen = hptr[tile + 1] - hp;
    const SX_G int32_t *__restrict__ hvid = gld(G->halo_vid);
    bool edges = false;
#pragma unroll
    for (int q = 0; q < kStageQ; ++q) {
      const int idx = 64 * q + lane;
      if (idx < hlen && lin[hvid[hp + idx]] != 0) edges = true;
    }
    if (__ballot(edges) == 0) {
      sweep_tile<P, false, false, NT>(G, tile, lane, L);
      if (valid) lout[j] = 0;
      return;
    }
  }

  // 2. per incoming edge e (receiver lane r): everything that arrives at a
  // ballistic receiver (stored as I / bm), or what a ballistic sender sends
  // a direction-conserving one
  // which lanes receive source shares (so the others skip the search)
  const uint64_t emmask = __ballot(valid && emp[j] < emp[j + 1]);
  auto edge_in = [&](int e, int r, bool rbal) -> P {
    const int i = nbr[e];
    // the first four packets of a ballistic sender, read before its layout
    // is known (the indices are valid edges either way; padding reads edge 0)
    const I4 b4 = bl4[e];
    const P p0 = ein[b4.x < 0 ? 0 : b4.x], p1 = ein[b4.y < 0 ? 0 : b4.y];
    const P p2 = ein[b4.z < 0 ? 0 : b4.z], p3 = ein[b4.w < 0 ? 0 : b4.w];
    const bool iedges = lin[i] != 0;
    // the sender's recombination photons of last step, its share per edge
    P ve = diffuse ? dshin[i] : P(0);
    if (!rbal && !iedges) return ve;
    const P ti = tin[i];
    if (!iedges) {
      // the sender's bins, eight gathers in flight at a time, added in order
      int q = klp[e];
      const int q1 = klp[e + 1];
      for (; q + 8 <= q1; q += 8) {
        P a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = oin[at((uint32_t)i, kl[q + u])];
#pragma unroll
        for (int u = 0; u < 8; ++u) ve += mul_rn(a[u], ti);
      }
      for (; q + 4 <= q1; q += 4) {
        const P a0 = oin[at((uint32_t)i, kl[q])], a1 = oin[at((uint32_t)i, kl[q + 1])];
        const P a2 = oin[at((uint32_t)i, kl[q + 2])], a3 = oin[at((uint32_t)i, kl[q + 3])];
        ve += mul_rn(a0, ti);
        ve += mul_rn(a1, ti);
        ve += mul_rn(a2, ti);
        ve += mul_rn(a3, ti);
      }
      for (; q < q1; ++q) ve += mul_rn(oin[at((uint32_t)i, kl[q])], ti);
    } else {
      if (b4.x >= 0) ve += mul_rn(p0, ti);
      if (b4.y >= 0) ve += mul_rn(p1, ti);
      if (b4.z >= 0) ve += mul_rn(p2, ti);
      if (b4.w >= 0) {
        ve += mul_rn(p3, ti);
        const int q1 = blp[e + 1];
        for (int q = blp[e] + 4; q < q1; ++q) ve += mul_rn(ein[bl[q]], ti);
      }
    }
    if (rbal) {
      if ((emmask >> r) & 1ull) {
        const int jr = tile * kTile + r;
        const int e0 = emp[jr], e1 = emp[jr + 1];
        const int rbj = rowp[jr];
        for (int q = e0; q < e1; ++q)
          if (rbj + (int)rev[eme[q]] == e) ve += (P)ema[q];
      }
      eout[e] = div_m(ve, (uint32_t)bmv[e]);
    }
    return ve;
  };
  const int E0 = rowp[tile * kTile];
  const int ne = rowp[tile * kTile + kTile] - E0;
  const bool edge_par = ne <= kVeCap;
  if (edge_par) {
    for (int base = 0; base < ne; base += 2 * kTile) {
      const int l0 = base + lane, l1 = base + kTile + lane;
      P v0 = P(0), v1 = P(0);
      if (l0 < ne) {
        const int r = elane[E0 + l0];
        v0 = edge_in(E0 + l0, r, (balmask >> r) & 1ull);
      }
      if (l1 < ne) {
        const int r = elane[E0 + l1];
        v1 = edge_in(E0 + l1, r, (balmask >> r) & 1ull);
      }
      if (l0 < ne) veb[l0] = v0;
      if (l1 < ne) veb[l1] = v1;
    }
    __syncthreads();
  }
  CtIn<P> ci;
  ci.bal = bal;
  ci.y0 = y0;
  ci.xin = (P *)G->xin;
  if (valid) {
    const int rb = rowp[j], re = rowp[j + 1];
    for (int e = rb; e < re; ++e) {
      const P ve = edge_par ? veb[e - E0] : edge_in(e, lane, bal);
      if (bal) {
        ci.nin_b += ve;
        ci.esc_b += bmv[e] == 0 ? ve : P(0);
      } else if (ve != P(0)) {
        const int p = G->bpos[ebin_in[e]];
        xin[at((uint32_t)j, p)] += ve;
        ci.xmask |= 1ull << (p / BB);
      }
    }
  }
  // the per-edge sums are dead from here on: their LDS becomes the halo
  // planes of the tile code
  __syncthreads();

  // 3. ballistic receivers only: no bins to gather
  if (balmask == validmask) {
    if (valid && lout[j] == 0) {
      // the buffer about to be written still holds the bins of two steps
      // ago: clear them
      SX_G V *__restrict__ oout = gst((V *)G->o[par ^ 1]);
      for (int kb = 0; kb < KB; ++kb)
        oout[((uint32_t)tile * (uint32_t)KB + (uint32_t)kb) * 64u + (uint32_t)lane] = V(0);
    }
    ct_finish<P>(G, tile, lane, valid, y0, ci.nin_b, ci.esc_b);
    if (valid) lout[j] = 1;
    return;
  }
  if (direct)
    sweep_tile<P, true, true, NT>(G, tile, lane, L, ci);
  else
    sweep_tile<P, false, true, NT>(G, tile, lane, L, ci);
  if (valid) lout[j] = bal ? 1 : 0;
}

// LDS of one combined-transport workgroup: the per-edge sums of the edge
// phase share their space with the tile code's LDS (the sums are read
// before the tile code writes its slot table and stages its first block,
// with a barrier between).
template <typename P>
union CtLds {
  TileLds<P> t;
  P ve[kVeCap];
};

// One combined-transport step over a tile list: one tile per workgroup of
// one wave, the same tile lists, XCD numbering and completion as k_sweep.
template <typename P, bool NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_ct(
    GridDev *__restrict__ grids, const int2 *__restrict__ tile_map,
    int32_t n_tiles, const int32_t *__restrict__ adv, int32_t n_adv,
    uint32_t *__restrict__ done, int32_t xcd_remap) {
  __shared__ CtLds<P> lds;
  __shared__ int last;
  const int lane = threadIdx.x & 63;
  const uint32_t nb = gridDim.x;   // a multiple of 8
  const uint32_t b = blockIdx.x;
  const uint32_t gt = xcd_remap ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  if ((int)gt < n_tiles) {
    int gi = 0, tile = (int)gt;
    if (tile_map) {
      const int2 tm = tile_map[gt];
      gi = __builtin_amdgcn_readfirstlane(tm.x);
      tile = __builtin_amdgcn_readfirstlane(tm.y);
    }
    const GridDev *__restrict__ G = grids + gi;
    if (G->remaining > 0)
      sweep_tile_ct<P, NT>(G, tile, lane, (SX_L P *)lds.ve, (SX_L TileLds<P> *)&lds.t);
  }
  __syncthreads();
  if (threadIdx.x == 0)
    last = atomicAdd(done, 1u) == nb - 1u;
  __syncthreads();
  if (!last) return;
  for (int i = threadIdx.x; i < n_adv; i += 64) {
    GridDev &g = grids[adv ? adv[i] : i];
    if (g.remaining > 0) {
      g.parity ^= 1;
      g.remaining -= 1;
      g.sweeps += 1;
    }
  }
  if (threadIdx.x == 0) atomicExch(done, 0u);
}

struct SlotVals {
  int32_t slot[120];
  int32_t v[120];
};

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
  if (g.habs) {
    g.habs[j] = 0.0;
    g.hnin[j] = 0.0;
  }
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

// ------------------------------------------------ no-allocation steps ---
// sx_step_noalloc keeps its launch tables (per launch class: the tile map
// and the list of grids to advance) and its completion counter in one
// file-scope device array, so that a step allocates nothing.  Each device
// holds its own copy of the array; host code never passes `scratch` itself
// to a kernel, only the device address looked up once per device.
constexpr int64_t kScratchBytes = kNoAllocMapOffset + 8 * (int64_t)SX_NOALLOC_MAX_TILES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device, void **out) {
  if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// The tile map of one launch class in the scratch array: tile t of the
// list goes to grid slot[g], tile t - first[g], for first[g] <= t <
// first[g+1] (grids in the caller's order); the first n threads also write
// the list of grids to advance, and thread 0 clears the completion counter
// when asked (once per call, before the first sweep).
__global__ void k_noalloc_tables(uint8_t *__restrict__ base, NoAllocList L) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int2 *map = (int2 *)(base + kNoAllocMapOffset) + L.map_first;
  int32_t *adv = (int32_t *)(base + kNoAllocAdvOffset) + (int64_t)L.cls * SX_NOALLOC_MAX_GRIDS;
  if (t == 0 && L.clear_done) *(uint32_t *)base = 0u;
  if (t < L.n) adv[t] = L.slot[t];
  if (t >= L.first[L.n]) return;
  int lo = 0, hi = L.n - 1;   // last g with first[g] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.first[mid] <= t) lo = mid; else hi = mid - 1;
  }
  map[t] = make_int2(L.slot[lo], (int)(t - L.first[lo]));
}

hipError_t launch_noalloc_tables(uint8_t *base, const NoAllocList &L, hipStream_t s) {
  const int64_t n = L.first[L.n] > L.n ? L.first[L.n] : L.n;
  hipLaunchKernelGGL(k_noalloc_tables, dim3(blocks_for(n > 0 ? n : 1, 256)), dim3(256), 0, s,
                     base, L);
  return hipGetLastError();
}


hipError_t launch_erev(const GridDev *dg, const GridDev &hg, hipStream_t s) {
  if (hg.n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL(k_erev, dim3(blocks_for(hg.n_edges, 256)), dim3(256), 0, s, dg);
  return hipGetLastError();
}

hipError_t launch_select(const GridDev *dg, const GridDev &hg, uint32_t *mout, hipStream_t s) {
  // one wave per two vertices, four waves per workgroup
  hipLaunchKernelGGL(k_select, dim3(blocks_for((int64_t)hg.npad * 32, 256)),
                     dim3(256), (unsigned)select_lds_bytes(hg.max_deg), s, dg, mout);
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
  // one wave per (tile, group of 16 bin positions)
  const int64_t waves = (int64_t)hg.ntiles * ((hg.k + kInlistBins - 1) / kInlistBins);
  if (hg.bb == 4)
    hipLaunchKernelGGL((k_inlist<false, 4>), dim3(blocks_for(waves * 64, 256)), dim3(256), 0, s, dg);
  else
    hipLaunchKernelGGL((k_inlist<false, 2>), dim3(blocks_for(waves * 64, 256)), dim3(256), 0, s, dg);
  return hipGetLastError();
}

hipError_t launch_clear_inw(const GridDev &hg, hipStream_t s) {
  return fill<uint64_t>(hg.inw, 0ull, (int64_t)hg.ntiles * hg.kb * kTile, s);
}

hipError_t launch_rebin(GridDev *dg, const GridDev &hg, const RebinMap &map, hipStream_t s) {
  // one workgroup per tile (npad is a multiple of 64)
  if (hg.precision == 0)
    hipLaunchKernelGGL(k_rebin<double>, dim3((unsigned)hg.ntiles), dim3(64),
                       (size_t)rebin_lds_bytes<double>(hg.kb), s, dg, map);
  else
    hipLaunchKernelGGL(k_rebin<float>, dim3((unsigned)hg.ntiles), dim3(64),
                       (size_t)rebin_lds_bytes<float>(hg.kb), s, dg, map);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_flip, dim3(1), dim3(1), 0, s, dg);
  return hipGetLastError();
}
hipError_t launch_em_bins(GridDev *dg, const GridDev &hg, int64_t n_em, hipStream_t s) {
  (void)hg;
  if (n_em <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_em_bins, dim3(blocks_for(n_em, 256)), dim3(256), 0, s, dg, n_em);
  return hipGetLastError();
}

hipError_t launch_ebin_in(const GridDev *dg, const GridDev &hg, hipStream_t s) {
  if (hg.n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ebin_in, dim3(blocks_for(hg.n_edges, 256)), dim3(256), 0, s, dg);
  return hipGetLastError();
}

hipError_t launch_kl_count(const GridDev *dg, const GridDev &hg, hipStream_t s) {
  hipLaunchKernelGGL(k_kl_count, dim3(blocks_for(hg.n_edges + 1, 256)), dim3(256), 0, s, dg);
  return hipGetLastError();
}

hipError_t launch_kl_fill(const GridDev *dg, const GridDev &hg, hipStream_t s) {
  if (hg.n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kl_fill, dim3(blocks_for(hg.n_edges, 256)), dim3(256), 0, s, dg);
  return hipGetLastError();
}

hipError_t launch_scan(int32_t *cnt, int32_t *ptr, int64_t *part, int32_t n,
                       hipStream_t s) {
  const unsigned nb = blocks_for(n, 1024);
  if (nb > 0)
    hipLaunchKernelGGL(k_scan_part, dim3(nb), dim3(1024), 0, s, cnt, ptr, part, n);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, part, (int32_t)nb);
  hipLaunchKernelGGL(k_scan_add, dim3(nb > 0 ? nb : 1), dim3(1024), 0, s, ptr, part, n,
                     (int32_t)nb);
  return hipGetLastError();
}

hipError_t launch_inlist_fill(const GridDev *dg, const GridDev &hg,
                              hipStream_t s) {
  const int64_t waves = (int64_t)hg.ntiles * ((hg.k + kInlistBins - 1) / kInlistBins);
  if (hg.bb == 4)
    hipLaunchKernelGGL((k_inlist<true, 4>), dim3(blocks_for(waves * 64, 256)), dim3(256), 0, s, dg);
  else
    hipLaunchKernelGGL((k_inlist<true, 2>), dim3(blocks_for(waves * 64, 256)), dim3(256), 0, s, dg);
  return hipGetLastError();
}


hipError_t launch_reset_state(GridDev *dg, const GridDev &hg, const double *y0,
                              hipStream_t s) {
  hipError_t e;
  // photon blocks of all tiles plus the zero tile, in photon words
  const int64_t nk = ((int64_t)hg.ntiles + 1) * hg.kb * kTile * hg.bb;
  for (int b = 0; b < 2; ++b) {
    if (hg.precision == 0) {
      e = fill<double>((double *)hg.o[b], 0.0, nk, s);
      if (e == hipSuccess) e = fill<double>((double *)hg.t[b], 1.0, hg.plane, s);
    } else {
      e = fill<float>((float *)hg.o[b], 0.0f, nk, s);
      if (e == hipSuccess) e = fill<float>((float *)hg.t[b], 1.0f, hg.plane, s);
    }
    if (e != hipSuccess) return e;
  }
  e = fill<double>(hg.tally, 0.0, (int64_t)hg.ntiles * 3, s);
  if (e != hipSuccess) return e;
  if (hg.transport != 0) {
    for (int b = 0; b < 2; ++b) {
      if (hg.precision == 0) e = fill<double>((double *)hg.oe[b], 0.0, hg.n_edges, s);
      else e = fill<float>((float *)hg.oe[b], 0.0f, hg.n_edges, s);
      if (e == hipSuccess) e = fill<uint8_t>(hg.lay[b], (uint8_t)0, hg.npad, s);
      if (e != hipSuccess) return e;
    }
    if (hg.precision == 0) e = fill<double>((double *)hg.xin, 0.0, nk, s);
    else e = fill<float>((float *)hg.xin, 0.0f, nk, s);
    if (e != hipSuccess) return e;
  }
  if (hg.diffuse != 0) {
    for (int b = 0; b < 2; ++b) {
      if (hg.precision == 0) e = fill<double>((double *)hg.dsh[b], 0.0, hg.plane, s);
      else e = fill<float>((float *)hg.dsh[b], 0.0f, hg.plane, s);
      if (e != hipSuccess) return e;
    }
    e = fill<double>(hg.dtally, 0.0, (int64_t)hg.ntiles, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reset, dim3(blocks_for(hg.npad, 256)), dim3(256), 0, s,
                     dg, y0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(1), 0, s, dg);
  return hipGetLastError();
}

template <typename P, bool NT>
static const void *sweep_fn(int tpb, int split) {
  switch (tpb * 8 + split) {
    case 1 * 8 + 1: return (const void *)k_sweep<P, 1, 1, NT>;
    case 2 * 8 + 1: return (const void *)k_sweep<P, 2, 1, NT>;
    case 4 * 8 + 1: return (const void *)k_sweep<P, 4, 1, NT>;
    case 2 * 8 + 2: return (const void *)k_sweep<P, 2, 2, NT>;
    case 4 * 8 + 2: return (const void *)k_sweep<P, 4, 2, NT>;
    case 4 * 8 + 4: return (const void *)k_sweep<P, 4, 4, NT>;
  }
  return nullptr;
}

static hipError_t sweep_shape(const SweepLaunch &l, const void **fn, dim3 *grid,
                              dim3 *block) {
  if (l.transport != 0) {
    if (l.n_tiles <= 0 || !l.done) return hipErrorInvalidValue;
    *fn = l.precision == 0
              ? (l.nt ? (const void *)k_sweep_ct<double, true> : (const void *)k_sweep_ct<double, false>)
              : (l.nt ? (const void *)k_sweep_ct<float, true> : (const void *)k_sweep_ct<float, false>);
    *grid = dim3(((unsigned)l.n_tiles + 7u) & ~7u);
    *block = dim3(64u);
    return hipSuccess;
  }
  const int split = l.split > 1 ? l.split : 1;
  const void *f = l.precision == 0
                      ? (l.nt ? sweep_fn<double, true>(l.tpb, split)
                              : sweep_fn<double, false>(l.tpb, split))
                      : (l.nt ? sweep_fn<float, true>(l.tpb, split)
                              : sweep_fn<float, false>(l.tpb, split));
  if (!f || l.n_tiles <= 0 || !l.done) return hipErrorInvalidValue;
  *fn = f;
  // one workgroup per tpb / split tiles, rounded up to a multiple of 8
  const unsigned tpg = (unsigned)(l.tpb / split);
  *grid = dim3((((unsigned)l.n_tiles + tpg - 1) / tpg + 7u) & ~7u);
  *block = dim3(64u * (unsigned)l.tpb);
  return hipSuccess;
}

hipError_t launch_sweep(const SweepLaunch &l, hipStream_t s) {
  const void *fn;
  dim3 g, t;
  hipError_t e = sweep_shape(l, &fn, &g, &t);
  if (e != hipSuccess) return e;
  SweepLaunch a = l;
  void *args[] = {&a.grids, &a.map, &a.n_tiles, &a.adv, &a.n_adv, &a.done, &a.xcd_remap};
  return hipLaunchKernel(fn, g, t, args, 0, s);
}

hipError_t add_sweep_node(hipGraph_t graph, const SweepLaunch &l,
                          hipGraphNode_t *prev) {
  const void *fn;
  dim3 g, t;
  hipError_t e = sweep_shape(l, &fn, &g, &t);
  if (e != hipSuccess) return e;
  SweepLaunch a = l;
  void *args[] = {&a.grids, &a.map, &a.n_tiles, &a.adv, &a.n_adv, &a.done, &a.xcd_remap};
  hipKernelNodeParams kp = {};
  kp.func = const_cast<void *>(fn);
  kp.gridDim = g;
  kp.blockDim = t;
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  hipGraphNode_t node;
  e = hipGraphAddKernelNode(&node, graph, *prev ? prev : nullptr, *prev ? 1 : 0, &kp);
  if (e == hipSuccess) *prev = node;
  return e;
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
