// sx_host.cpp -- host side of libsx: the C ABI declared in include/sx.h.
//
// Upload path (per grid, outside the per-step hot loop):
//   validate -> Hilbert-curve reorder -> CSR rows sorted by original id ->
//   unit edge vectors, path lengths, chemistry coefficients (fp64, no FMA
//   contraction) -> device copies -> selection / edge-bin / gather-list
//   kernels -> source emission lists -> initial state.
// Step path: per-grid control words live in a device slot table; a step is
//   one sweep launch per (precision, bin class) group plus one small
//   advance launch, all on the context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "sx.h"
#include "sx_internal.h"

using sx::GridDev;

namespace {

constexpr int kMaxSlots = 4096;

struct DevBuf {
  void *p = nullptr;
  uint64_t bytes = 0;
};

struct Grid {
  sx_grid_id id = 0;
  int slot = -1;
  GridDev hg{};
  int64_t n_em = 0;
  std::vector<int32_t> perm;           // new -> original
  std::vector<int32_t> inv;            // original -> new
  std::vector<int32_t> orig_to_new_e;  // original CSR position -> new edge
  std::vector<int32_t> row_ptr_h;      // new CSR, host copy
  std::vector<int32_t> nbr_h;
  std::vector<double> dL_h;            // new order
  std::vector<double> tau_h;
  std::vector<double> elen_h;          // [E] edge lengths, new order
  std::vector<uint8_t> is_src_h;       // [N] new order: vertex holds a source
  std::vector<DevBuf> bufs;
  uint64_t bytes = 0;
  double *y_init = nullptr;
  double e_sweep = 0.0;     // photons emitted per step
  double esc_emit = 0.0;    // photons per step with no way out of a beam source
  double base_sweeps = 0.0, base_emitted = 0.0, base_escaped = 0.0;
  int64_t n_direct = 0;     // tiles whose halo is too large for LDS staging
  std::vector<double> bins0;   // [3K] bin directions given at upload
  std::vector<double> bins_cur;   // [3K] bin directions on the device now
  bool rotated = false;
  // A routing rebuild that could not finish (its bin-list pool could not
  // grow) leaves the device tables inconsistent: no sweep may run on the
  // grid until a reset rebuilds them.
  bool unusable = false;
  bool ebin_stale = false;
  std::vector<uint8_t> tile_direct;
  int32_t transport = SX_TRANSPORT_DCT;   // as uploaded (the kernel class may differ)
  std::vector<int32_t> bsel_h;   // combined transport: [3E] chosen out-edges per in-edge, -1 pad
  std::vector<uint8_t> bm_h;     // [E]
};

// How the sweeps of one list of grids are launched: one kernel launch per
// precision present, the tile lists and advance lists they read, and a HIP
// graph of graph_sweeps consecutive sweeps, replayed.
struct Plan {
  std::vector<int32_t> key;   // slots, in the caller's order
  sx_schedule sched{};
  bool fixed = false;         // set by the caller or by the autotuner
  bool built = false;
  std::vector<sx::SweepLaunch> launches;
  std::vector<void *> dev;    // tile maps and advance lists
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  double tuned_us = 0.0;      // autotuner's best time per sweep
};

struct ProfEv {
  hipEvent_t a = nullptr, b = nullptr;
  int32_t launches = 0;
};

}  // namespace

struct sx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  uint64_t used = 0;
  sx_alloc_fn alloc = nullptr;
  sx_free_fn free_fn = nullptr;
  void *user = nullptr;
  GridDev *table = nullptr;
  std::vector<int> free_slots;
  std::map<sx_grid_id, Grid *> grids;
  sx_grid_id next_id = 1;
  std::string err;
  bool poisoned = false;
  std::vector<Plan *> plans;
  sx_schedule dflt{4, SX_ORDER_GRID, 1, 50, 1};
  int32_t autotune = 0;
  uint32_t *done = nullptr;   // completion counter of the sweep launches
  // pinned host staging of the routing rebuild: bin directions going in
  // (offset 0), record and bin-list counts coming back (kPinCounts)
  uint8_t *pin = nullptr;
  bool prof = false;
  std::vector<ProfEv> ev;     // pool
  uint8_t *scratch = nullptr; // device address of this device's sx_step_noalloc array
  size_t ev_used = 0;
  // A second stream for uploads and read-backs that overlap the sweeps of
  // other grids (the request loop's): while io_on, the upload, read-back and
  // release calls work on it and wait only for it.
  hipStream_t io = nullptr;
  bool io_on = false;
};

namespace {

constexpr size_t kPinCounts = 3 * 8 * 128;         // after 3 doubles per bin, up to 128 bins
constexpr size_t kPinBytes = kPinCounts + 64;
static_assert(SX_MAX_BINS_FP32 <= 128 && SX_MAX_BINS_FP64 <= 128, "pinned staging holds 128 bins");

void drop_plans(sx_ctx *ctx, int slot);

// The stream of the calls that move a grid's data (upload, read-back,
// release): the context's own, or its second stream while io_on.
hipStream_t wstream(const sx_ctx *ctx) { return ctx->io_on ? ctx->io : ctx->stream; }

int fail(sx_ctx *ctx, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) {
    ctx->err = buf;
    if (code == SX_EDEVICE) ctx->poisoned = true;
  }
  return code;
}

#define HIP_TRY(ctx, call)                                                   \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail((ctx), SX_EDEVICE, "%s failed: %s", #call,                 \
                  hipGetErrorString(e_));                                    \
  } while (0)

void *dev_alloc(sx_ctx *ctx, uint64_t bytes) {
  if (bytes == 0) bytes = 16;
  void *p = nullptr;
  if (ctx->alloc) {
    p = ctx->alloc((size_t)bytes, ctx->user);
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  return p;
}

void dev_free(sx_ctx *ctx, void *p) {
  if (!p) return;
  if (ctx->free_fn)
    ctx->free_fn(p, ctx->user);
  else
    (void)hipFree(p);
}

// Allocate for a grid, enforcing the context budget.
template <typename T>
int galloc(sx_ctx *ctx, Grid *g, T **out, uint64_t count) {
  const uint64_t bytes = ((count * sizeof(T)) + 255) & ~uint64_t(255);
  if (ctx->used + bytes > ctx->budget)
    return fail(ctx, SX_ENOMEM, "device budget exceeded (%llu + %llu > %llu)",
                (unsigned long long)ctx->used, (unsigned long long)bytes,
                (unsigned long long)ctx->budget);
  void *p = dev_alloc(ctx, bytes);
  if (!p) return fail(ctx, SX_ENOMEM, "device allocation of %llu bytes failed",
                      (unsigned long long)bytes);
  g->bufs.push_back({p, bytes});
  g->bytes += bytes;
  ctx->used += bytes;
  *out = (T *)p;
  return SX_OK;
}

void grid_release(sx_ctx *ctx, Grid *g) {
  for (auto &b : g->bufs) {
    dev_free(ctx, b.p);
    ctx->used -= b.bytes;
  }
  g->bufs.clear();
  if (g->slot >= 0) ctx->free_slots.push_back(g->slot);
  g->slot = -1;
  delete g;
}

// ------------------------------------------------------------ Hilbert ---
// Index of a point along a 3-D Hilbert curve with b bits per axis, from
// J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707 (2004):
// the axes are transformed in place into the curve's "transpose" form, whose
// bits, interleaved from the top, are the index.
uint64_t hilbert_key(uint32_t x0, uint32_t x1, uint32_t x2, int b) {
  uint32_t X[3] = {x0, x1, x2};
  const uint32_t M = 1u << (b - 1);
  for (uint32_t Q = M; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
  uint32_t t = 0;
  for (uint32_t Q = M; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  for (int i = 0; i < 3; ++i) X[i] ^= t;
  uint64_t key = 0;
  for (int q = b - 1; q >= 0; --q)
    for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> q) & 1u);
  return key;
}

// Storage order of the bins: blocks of bb bins that point in nearby
// directions.  Greedy grouping: walk the bins in some order and give each
// bin not yet taken the bb - 1 closest bins not yet taken (largest cosine,
// ties to the lower index); the group with fewer bins, if K is not a
// multiple of bb, comes last.  Several walk orders are tried (the given
// order, then seeded shuffles) and the grouping whose groups are tightest
// (largest sum over groups of the smallest cosine within the group) is
// kept.  Returns the bin at each position; the bins of a group are
// ascending.
std::vector<uint8_t> cluster_bins(const double *u, int K, int bb) {
  auto dot = [&](int a, int b) {
    return (u[3 * a] * u[3 * b] + u[3 * a + 1] * u[3 * b + 1]) + u[3 * a + 2] * u[3 * b + 2];
  };
  std::vector<uint8_t> best;
  double best_score = -INFINITY;
  std::vector<int> order((size_t)K);
  uint64_t rs = 0x9E3779B97F4A7C15ull;
  auto next = [&]() {   // xorshift64*
    rs ^= rs >> 12;
    rs ^= rs << 25;
    rs ^= rs >> 27;
    return rs * 0x2545F4914F6CDD1Dull;
  };
  std::vector<std::pair<double, int>> cand;
  for (int trial = 0; trial < 64; ++trial) {
    for (int k = 0; k < K; ++k) order[(size_t)k] = k;
    if (trial > 0)
      for (int k = K - 1; k > 0; --k) std::swap(order[(size_t)k], order[next() % (uint64_t)(k + 1)]);
    std::vector<char> used((size_t)K, 0);
    std::vector<uint8_t> perm;
    double score = 0.0;
    for (int a : order) {
      if (used[(size_t)a]) continue;
      cand.clear();
      for (int k = 0; k < K; ++k)
        if (!used[(size_t)k] && k != a) cand.push_back({-dot(a, k), k});
      std::sort(cand.begin(), cand.end());
      std::vector<int> grp{a};
      for (size_t c = 0; c < cand.size() && (int)grp.size() < bb; ++c) grp.push_back(cand[c].second);
      std::sort(grp.begin(), grp.end());
      double mn = 1.0;
      for (size_t x = 0; x < grp.size(); ++x)
        for (size_t y = x + 1; y < grp.size(); ++y) mn = std::min(mn, dot(grp[x], grp[y]));
      score += mn;
      for (int k : grp) {
        used[(size_t)k] = 1;
        perm.push_back((uint8_t)k);
      }
    }
    if (score > best_score) {
      best_score = score;
      best = perm;
    }
  }
  return best;
}

std::vector<int32_t> hilbert_order(const double *pos, int64_t n) {
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], pos[3 * i + a]);
      hi[a] = std::max(hi[a], pos[3 * i + a]);
    }
  const int bits = 21;
  const double scale = (double)((1u << bits) - 1);
  std::vector<std::pair<uint64_t, int32_t>> kv((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
      const double w = hi[a] - lo[a];
      const double f = w > 0 ? (pos[3 * i + a] - lo[a]) / w : 0.0;
      double v = std::floor(f * scale);
      v = std::min(std::max(v, 0.0), scale);
      q[a] = (uint32_t)v;
    }
    kv[(size_t)i] = {hilbert_key(q[0], q[1], q[2], bits), (int32_t)i};
  }
  std::sort(kv.begin(), kv.end());
  std::vector<int32_t> perm((size_t)n);
  for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = kv[(size_t)i].second;
  return perm;
}

// -------------------------------------------------------- validation ---
bool finite3(const double *p) {
  return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]);
}

int validate(sx_ctx *ctx, const sx_grid_desc *d) {
  if (!d) return fail(ctx, SX_EINVAL, "null descriptor");
  const int64_t n = d->n_vertices;
  if (n < 1) return fail(ctx, SX_EINVAL, "n_vertices must be >= 1");
  if (n > (int64_t)1 << 30) return fail(ctx, SX_ENOTSUP, "n_vertices too large");
  if (!d->pos || !d->nbr_ptr || !d->nbr_idx || !d->n_H || !d->volume ||
      !d->bin_dirs)
    return fail(ctx, SX_EINVAL, "required array is NULL");
  if (d->precision != SX_FP64 && d->precision != SX_FP32_TRANSPORT)
    return fail(ctx, SX_EINVAL, "precision must be SX_FP64 or SX_FP32_TRANSPORT");
  if (d->transport != SX_TRANSPORT_DCT && d->transport != SX_TRANSPORT_COMBINED)
    return fail(ctx, SX_EINVAL, "transport must be SX_TRANSPORT_DCT or SX_TRANSPORT_COMBINED");
  if (d->transport == SX_TRANSPORT_COMBINED && std::isnan(d->tau_switch))
    return fail(ctx, SX_EINVAL, "tau_switch is NaN");
  if (!(d->alpha_A == 0.0 || (std::isfinite(d->alpha_A) && d->alpha_A >= d->alpha_B)))
    return fail(ctx, SX_EINVAL, "alpha_A must be 0 or finite and >= alpha_B");
  if ((d->transport == SX_TRANSPORT_COMBINED || d->alpha_A > 0.0) &&
      (double)n * (double)d->n_bins * (double)d->max_per_bin >= 2147483647.0)
    return fail(ctx, SX_ENOTSUP, "grid too large for the per-edge lists of combined transport");
  if (d->hops < 0 || d->hops > SX_MAX_HOPS)
    return fail(ctx, SX_EINVAL, "hops must be in 0..%d", SX_MAX_HOPS);
  if (d->hops > 1 && (d->transport != SX_TRANSPORT_DCT || d->alpha_A > 0.0))
    return fail(ctx, SX_ENOTSUP,
                "multi-hop steps take direction-conserving transport with on-the-spot "
                "recombination");
  if (d->dct_reference != SX_DCT_REF_BIN && d->dct_reference != SX_DCT_REF_EDGE)
    return fail(ctx, SX_EINVAL, "dct_reference must be SX_DCT_REF_BIN or SX_DCT_REF_EDGE");
  const int K = d->n_bins;
  if (K < 1) return fail(ctx, SX_EINVAL, "n_bins must be >= 1");
  if (K > (d->precision == SX_FP64 ? SX_MAX_BINS_FP64 : SX_MAX_BINS_FP32))
    return fail(ctx, SX_ENOTSUP, "n_bins %d over the limit for this precision",
                K);
  if (d->max_per_bin < 1 || d->max_per_bin > SX_MAX_PER_BIN)
    return fail(ctx, SX_EINVAL, "max_per_bin must be 1..3");
  if (d->n_subcycles < 1) return fail(ctx, SX_EINVAL, "n_subcycles must be >= 1");
  if (!(d->dt > 0.0) || !std::isfinite(d->dt))
    return fail(ctx, SX_EINVAL, "dt must be finite and > 0");
  if (!(d->sigma >= 0.0) || !std::isfinite(d->sigma) ||
      !(d->alpha_B >= 0.0) || !std::isfinite(d->alpha_B))
    return fail(ctx, SX_EINVAL, "sigma and alpha_B must be finite and >= 0");
  if (!std::isfinite(d->cos_min) || d->cos_min < -1.0 || d->cos_min >= 1.0)
    return fail(ctx, SX_EINVAL, "cos_min must lie in [-1, 1)");
  if (!d->dL && (!(d->kappa > 0.0) || !std::isfinite(d->kappa)))
    return fail(ctx, SX_EINVAL, "kappa must be finite and > 0");
  for (int k = 0; k < K; ++k) {
    const double *u = d->bin_dirs + 3 * k;
    if (!finite3(u)) return fail(ctx, SX_EINVAL, "bin %d not finite", k);
    const double r = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (std::fabs(r - 1.0) > 1e-12)
      return fail(ctx, SX_EINVAL, "bin %d is not a unit vector", k);
  }
  if (d->nbr_ptr[0] != 0) return fail(ctx, SX_EINVAL, "nbr_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i) {
    const int64_t deg = d->nbr_ptr[i + 1] - d->nbr_ptr[i];
    if (deg < 0) return fail(ctx, SX_EINVAL, "nbr_ptr decreases at %lld", (long long)i);
    if (deg > SX_MAX_DEGREE)
      return fail(ctx, SX_ENOTSUP, "vertex %lld has degree %lld > %d",
                  (long long)i, (long long)deg, SX_MAX_DEGREE);
    if (!finite3(d->pos + 3 * i))
      return fail(ctx, SX_EINVAL, "position %lld not finite", (long long)i);
    if (!(d->n_H[i] >= 0.0) || !std::isfinite(d->n_H[i]))
      return fail(ctx, SX_EINVAL, "n_H[%lld] must be finite and >= 0", (long long)i);
    if (!(d->volume[i] > 0.0) || !std::isfinite(d->volume[i]))
      return fail(ctx, SX_EINVAL, "volume[%lld] must be finite and > 0", (long long)i);
    if (d->dL && (!(d->dL[i] >= 0.0) || !std::isfinite(d->dL[i])))
      return fail(ctx, SX_EINVAL, "dL[%lld] must be finite and >= 0", (long long)i);
    if (d->x_init && !(d->x_init[i] >= 0.0 && d->x_init[i] <= 1.0))
      return fail(ctx, SX_EINVAL, "x_init[%lld] outside [0,1]", (long long)i);
  }
  const int64_t E = d->nbr_ptr[n];
  if (E >= ((int64_t)1 << 31) - 1) return fail(ctx, SX_ENOTSUP, "too many edges");
  // rows: ids in range, no self loops, no duplicates; graph symmetric
  std::vector<int32_t> sorted(d->nbr_idx, d->nbr_idx + E);
  for (int64_t i = 0; i < n; ++i) {
    auto b = sorted.begin() + d->nbr_ptr[i], e = sorted.begin() + d->nbr_ptr[i + 1];
    std::sort(b, e);
    for (auto it = b; it != e; ++it) {
      if (*it < 0 || *it >= n)
        return fail(ctx, SX_EINVAL, "neighbour id %d out of range", *it);
      if (*it == i) return fail(ctx, SX_EINVAL, "self loop at vertex %lld", (long long)i);
      if (it != b && *it == *(it - 1))
        return fail(ctx, SX_EINVAL, "duplicate neighbour %d of vertex %lld", *it,
                    (long long)i);
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = d->nbr_ptr[i]; p < d->nbr_ptr[i + 1]; ++p) {
      const int32_t j = d->nbr_idx[p];
      auto b = sorted.begin() + d->nbr_ptr[j], e = sorted.begin() + d->nbr_ptr[j + 1];
      if (!std::binary_search(b, e, (int32_t)i))
        return fail(ctx, SX_EINVAL, "graph not symmetric: %lld->%d has no reverse",
                    (long long)i, j);
    }
  if (d->n_src < 0) return fail(ctx, SX_EINVAL, "n_src < 0");
  if (d->n_src > 0 && (!d->src_vertex || !d->src_rate))
    return fail(ctx, SX_EINVAL, "source arrays are NULL");
  for (int s = 0; s < d->n_src; ++s) {
    if (d->src_vertex[s] < 0 || d->src_vertex[s] >= n)
      return fail(ctx, SX_EINVAL, "source %d vertex out of range", s);
    if (!(d->src_rate[s] >= 0.0) || !std::isfinite(d->src_rate[s]))
      return fail(ctx, SX_EINVAL, "source %d rate must be finite and >= 0", s);
    if (d->src_dir) {
      const double *u = d->src_dir + 3 * s;
      if (!finite3(u)) return fail(ctx, SX_EINVAL, "source %d direction not finite", s);
      const bool zero = u[0] == 0.0 && u[1] == 0.0 && u[2] == 0.0;
      const double r = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      if (!zero && std::fabs(r - 1.0) > 1e-12)
        return fail(ctx, SX_EINVAL, "source %d direction neither zero nor unit", s);
    }
  }
  return SX_OK;
}

struct Sizes {
  int64_t n, npad, ntiles, E, K, kw, sp, bb, kb;
  int32_t transport, mpb;   // transport: the kernel class (1 also for diffuse radiation)
  int32_t hops;             // hops per step (1: one edge per step)
  bool diffuse;
  int64_t n_src;
};

Sizes sizes_of(const sx_grid_desc *d) {
  Sizes s;
  s.n = d->n_vertices;
  s.npad = (s.n + sx::kTile - 1) / sx::kTile * sx::kTile;
  s.ntiles = s.npad / sx::kTile;
  s.E = d->nbr_ptr[s.n];
  s.K = d->n_bins;
  s.kw = (s.K + 15) / 16;
  s.sp = d->precision == SX_FP64 ? 8 : 4;
  s.bb = sx::kBlockBytes / s.sp;
  s.kb = (s.K + s.bb - 1) / s.bb;
  s.diffuse = d->alpha_A > 0.0;
  s.transport = (d->transport == SX_TRANSPORT_COMBINED || s.diffuse) ? SX_TRANSPORT_COMBINED
                                                                     : SX_TRANSPORT_DCT;
  s.mpb = d->max_per_bin;
  s.hops = d->hops > 1 ? d->hops : 1;
  s.n_src = d->n_src;
  return s;
}

uint64_t rnd(uint64_t b) { return (b + 255) & ~uint64_t(255); }

uint64_t bytes_estimate(const Sizes &s, int64_t n_em, int64_t n_rec, int64_t n_halo) {
  uint64_t b = 0;
  b += rnd(4 * (s.npad + 1)) + rnd(4 * s.E) + rnd(s.E) + rnd(24 * s.E) + rnd(24 * s.K);
  b += rnd(4 * s.npad * s.K) + rnd(s.E) + rnd(8 * s.npad * s.kb) +
       2 * rnd(4 * s.npad * s.kw) + 2 * rnd(4 * (s.ntiles * s.K * sx::kRecGroups + 1)) +
       rnd(s.ntiles * s.K * sx::kTile) + rnd(4 * n_rec + 4) +
       rnd(16 * s.E + 16) + rnd(4 * s.E + 4);
  b += rnd(4 * (s.ntiles + 1)) + rnd(4 * n_halo + 4) + rnd(2 * s.E) + rnd(s.ntiles);
  b += rnd(4 * (s.npad + 1)) + rnd(4 * n_em + 4) + rnd(8 * n_em + 8);
  b += rnd(4 * n_em + 4) + rnd(24 * s.n_src + 8);   // beam shares: their sources and directions
  b += 6 * rnd(8 * s.npad);
  b += 2 * rnd((uint64_t)sx::kBlockBytes * s.kb * (s.npad + sx::kTile));
  b += 2 * rnd((uint64_t)s.sp * (s.npad + sx::kTile));
  b += rnd(24 * s.ntiles);
  if (s.transport == SX_TRANSPORT_COMBINED) {
    // bin lists (at most mpb entries per (vertex, bin)), ballistic lists
    // (at most mpb per edge), counts, per-edge photons, layouts
    b += 3 * rnd(4 * (s.E + 1)) + rnd(8 * (s.E / 1024 + 2)) + rnd((uint64_t)s.mpb * s.npad * s.K) +
         rnd((uint64_t)4 * s.mpb * s.E) + 3 * rnd(s.E) + 2 * rnd((uint64_t)s.sp * s.E) +
         rnd((uint64_t)16 * (s.E + 1)) +
         rnd((uint64_t)sx::kBlockBytes * s.kb * (s.npad + sx::kTile)) +
         2 * rnd(s.npad);
  }
  if (s.diffuse) b += rnd(8 * s.npad) + 2 * rnd((uint64_t)s.sp * (s.npad + sx::kTile)) +
                     rnd(8 * s.ntiles);
  if (s.hops > 1) b += 3 * rnd(8 * s.npad);
  return b;
}

Grid *find(sx_ctx *ctx, sx_grid_id id) {
  auto it = ctx->grids.find(id);
  return it == ctx->grids.end() ? nullptr : it->second;
}

int write_slot(sx_ctx *ctx, Grid *g) {
  HIP_TRY(ctx, hipMemcpyAsync(ctx->table + g->slot, &g->hg, sizeof(GridDev),
                              hipMemcpyHostToDevice, wstream(ctx)));
  HIP_TRY(ctx, hipStreamSynchronize(wstream(ctx)));
  return SX_OK;
}

// Release one of a grid's device buffers.
void gfree(sx_ctx *ctx, Grid *g, void *p) {
  for (size_t i = 0; i < g->bufs.size(); ++i)
    if (g->bufs[i].p == p) {
      dev_free(ctx, p);
      ctx->used -= g->bufs[i].bytes;
      g->bytes -= g->bufs[i].bytes;
      g->bufs.erase(g->bufs.begin() + (long)i);
      return;
    }
}

// Combined transport (and diffuse radiation): the bin of each in-edge and
// the per-in-edge bin lists from the current selection and edge bins, on
// the device; the list pool grows when needed.  Only the pool pointer and
// capacity are written to the device table.  Synchronous.
int build_ct_tables(sx_ctx *ctx, Grid *g) {
  GridDev &h = g->hg;
  GridDev *dg = ctx->table + g->slot;
  hipStream_t st = wstream(ctx);
  HIP_TRY(ctx, sx::launch_ebin_in(dg, h, st));
  HIP_TRY(ctx, sx::launch_kl_count(dg, h, st));
  HIP_TRY(ctx, sx::launch_scan(h.kl_cnt, h.kl_ptr, h.kl_part, (int32_t)h.n_edges, st));
  int32_t *pin_total = (int32_t *)(ctx->pin + kPinCounts + 4);
  HIP_TRY(ctx, hipMemcpyAsync(pin_total, h.kl_ptr + h.n_edges, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  const int32_t total = *pin_total;
  if (!h.kl || total > h.kl_cap) {
    // the larger pool is allocated before the old one is released; if it
    // cannot be, the list offsets already describe the new routing and the
    // grid is marked unusable (sweeps are refused until a reset)
    uint8_t *d = nullptr;
    const int r = galloc(ctx, g, &d, (uint64_t)total + 1);
    if (r) {
      g->unusable = true;
      return fail(ctx, SX_ENOMEM,
                  "bin lists of combined transport need %d entries and the pool could not "
                  "grow; the grid is unusable until sx_grid_reset", total);
    }
    if (h.kl) gfree(ctx, g, h.kl);
    h.kl = d;
    h.kl_cap = total;
    HIP_TRY(ctx, hipMemcpyAsync(&dg->kl, &h.kl, sizeof(h.kl), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(&dg->kl_cap, &h.kl_cap, sizeof(h.kl_cap), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
  }
  HIP_TRY(ctx, sx::launch_kl_fill(dg, h, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return SX_OK;
}

// Rebuild a grid's routing on the device for bin directions `bins` [3K]:
// selection, (with a re-binning map) the photons in flight moved to their
// new bins and split over the new selection, edge bins, source-share bins,
// m, gather lists; the overflow record pool grows when the new routing
// needs more.  Synchronous.
int rebuild_routing(sx_ctx *ctx, Grid *g, const double *bins, const sx::RebinMap *rebin) {
  GridDev &h = g->hg;
  GridDev *dg = ctx->table + g->slot;
  hipStream_t st = ctx->stream;
  const int32_t nrow = h.ntiles * h.k * sx::kRecGroups;
  // the previous rebuild ended with a synchronisation: the staging is free
  std::memcpy(ctx->pin, bins, sizeof(double) * 3 * h.k);
  HIP_TRY(ctx, hipMemcpyAsync(const_cast<double *>(h.bins), ctx->pin, sizeof(double) * 3 * h.k,
                              hipMemcpyHostToDevice, st));
  // the selection writes the m words: into the spare array when the photons
  // in flight are re-binned (which replaces the old words with them)
  HIP_TRY(ctx, sx::launch_select(dg, h, rebin ? h.mbits2 : h.mbits, st));
  HIP_TRY(ctx, sx::launch_em_bins(dg, h, g->n_em, st));
  g->ebin_stale = true;   // the full edge-bin table is rebuilt when read
  if (rebin) HIP_TRY(ctx, sx::launch_rebin(dg, h, *rebin, st));
  g->bins_cur.assign(bins, bins + 3 * h.k);
  // no clearing of the in-words: the fill rewrites the word of every bin
  // below K, and the padding bins of the last block keep their empty words
  // from the upload
  HIP_TRY(ctx, sx::launch_inlist_count(dg, h, st));
  HIP_TRY(ctx, sx::launch_scan(h.rec_cnt, h.rec_ptr, h.scan_part, nrow, st));
  // The fill keeps its records within the current pool, so it runs before
  // the host has seen the count; if the new routing needs more, the pool
  // grows and the fill runs again.
  int32_t *pin_rec = (int32_t *)(ctx->pin + kPinCounts);
  HIP_TRY(ctx, hipMemcpyAsync(pin_rec, h.rec_ptr + nrow, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, sx::launch_inlist_fill(dg, h, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  const int32_t n_rec = *pin_rec;
  if (n_rec > h.rec_cap) {
    // Only the pool pointer and capacity change in the device table: the
    // per-sweep control there (parity, steps done) is the device's own and
    // newer than the host copy, so the whole slot is not rewritten.
    static_assert(offsetof(GridDev, rec_cap) == offsetof(GridDev, rec) + sizeof(h.rec),
                  "rec and rec_cap adjacent");
    auto put_pool = [&]() {
      return hipMemcpyAsync(&dg->rec, &h.rec, sizeof(h.rec) + sizeof(h.rec_cap),
                            hipMemcpyHostToDevice, st);
    };
    gfree(ctx, g, h.rec);
    uint32_t *d_rec = nullptr;
    int r = galloc(ctx, g, &d_rec, (uint64_t)n_rec + 1);
    if (r) {
      h.rec = nullptr;
      h.rec_cap = 0;
      (void)put_pool();
      (void)hipStreamSynchronize(st);
      return fail(ctx, SX_EDEVICE, "overflow record pool could not grow to %d entries", n_rec);
    }
    h.rec = d_rec;
    h.rec_cap = n_rec;
    HIP_TRY(ctx, put_pool());
    HIP_TRY(ctx, sx::launch_inlist_fill(dg, h, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
  }
  if (h.transport == SX_TRANSPORT_COMBINED) {
    // the in-edge bins need the full edge-bin table
    HIP_TRY(ctx, sx::launch_edge_bins(dg, h, st));
    g->ebin_stale = false;
    return build_ct_tables(ctx, g);
  }
  return SX_OK;
}

}  // namespace

// Host-side product of sx_grid_prepare: a Grid with its host tables filled,
// and everything the device part uploads.
struct sx_prepared {
  Grid *g = nullptr;
  Sizes S{};
  int32_t n_sub = 0, mpb = 0, precision = 0;
  double dt = 0.0, cos_min = 0.0, unit = 1.0;
  std::vector<double> bins;
  std::vector<uint8_t> bperm;    // bin at each storage position
  std::vector<uint8_t> rev;
  std::vector<double> edir;
  std::vector<int32_t> halo_ptr, halo_vid;
  std::vector<uint16_t> edge_hidx;
  std::vector<double> tau, dtnhv, bco, y0;
  std::vector<int32_t> em_ptr, em_k, em_edge;
  std::vector<double> em_amt;
  std::vector<int32_t> em_beam;    // [n_em] source of a beam share, -1 isotropic (empty: no beams)
  std::vector<double> beam_dir;    // [3 n_src] source directions (empty: no beams)
  int32_t transport = 0, dct_ref = 0;   // transport: the kernel class
  double tau_switch = 0.0, alpha_A = 0.0, alpha_B = 0.0;
  std::vector<double> nhv;
  std::vector<int32_t> bl_ptr;   // combined transport: ballistic lists by in-edge
  std::vector<int32_t> bl;
  std::vector<int32_t> bl4;      // [4E] first four entries of each ballistic list, -1 padding
  std::vector<uint8_t> elane;
  ~sx_prepared() { delete g; }
};

namespace {

// The host part of an upload: validation, Hilbert reorder, CSR, edge
// geometry, halos, per-vertex coefficients, photon unit and source lists.
// No device work; `ctx` only collects the error message.
int prepare(sx_ctx *ctx, const sx_grid_desc *d, sx_prepared *P) {
  int rc = validate(ctx, d);
  if (rc) return rc;
  const Sizes S = sizes_of(d);
  P->S = S;
  P->n_sub = d->n_subcycles;
  P->mpb = d->max_per_bin;
  P->precision = d->precision;
  P->dt = d->dt;
  P->cos_min = d->cos_min;
  P->bins.assign(d->bin_dirs, d->bin_dirs + 3 * S.K);
  P->bperm = cluster_bins(d->bin_dirs, (int)S.K, (int)S.bb);
  const int64_t n = S.n, E = S.E, K = S.K, npad = S.npad;
  (void)K;
  Grid *g = new Grid();
  P->g = g;

  // ---- reorder along a Hilbert curve (locality of the gathers)
  g->perm = hilbert_order(d->pos, n);
  g->inv.assign((size_t)n, 0);
  for (int64_t v = 0; v < n; ++v) g->inv[(size_t)g->perm[(size_t)v]] = (int32_t)v;

  // ---- new CSR, rows sorted by ORIGINAL neighbour id, so that summing the
  // in-list in slot order adds the senders in ascending original id
  std::vector<int32_t> &rp = g->row_ptr_h;
  rp.assign((size_t)npad + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    const int32_t i = g->perm[(size_t)v];
    rp[(size_t)v + 1] = rp[(size_t)v] + (int32_t)(d->nbr_ptr[i + 1] - d->nbr_ptr[i]);
  }
  for (int64_t v = n; v < npad; ++v) rp[(size_t)v + 1] = rp[(size_t)v];
  std::vector<int32_t> orig_nbr((size_t)E);   // original id of each new edge's target
  g->nbr_h.assign((size_t)E, 0);
  g->orig_to_new_e.assign((size_t)E, 0);
  std::vector<double> &edir = P->edir;
  edir.assign((size_t)(3 * E), 0.0);
  std::vector<double> len_orig((size_t)E);     // per original CSR position
  g->elen_h.assign((size_t)E, 0.0);
  {
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int64_t v = 0; v < n; ++v) {
      const int32_t i = g->perm[(size_t)v];
      row.clear();
      for (int64_t p = d->nbr_ptr[i]; p < d->nbr_ptr[i + 1]; ++p)
        row.push_back({d->nbr_idx[p], p});
      std::sort(row.begin(), row.end());
      for (size_t r = 0; r < row.size(); ++r) {
        const int64_t e = rp[(size_t)v] + (int64_t)r;
        const int32_t j = row[r].first;
        orig_nbr[(size_t)e] = j;
        g->nbr_h[(size_t)e] = g->inv[(size_t)j];
        g->orig_to_new_e[(size_t)row[r].second] = (int32_t)e;
      }
    }
  }
  // ---- edge geometry in IEEE double with every operation rounded (the
  // library is built without FMA contraction on the host): unit vector and
  // length of each directed edge
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = d->nbr_ptr[i]; p < d->nbr_ptr[i + 1]; ++p) {
      const int32_t j = d->nbr_idx[p];
      const double dx = d->pos[3 * j + 0] - d->pos[3 * i + 0];
      const double dy = d->pos[3 * j + 1] - d->pos[3 * i + 1];
      const double dz = d->pos[3 * j + 2] - d->pos[3 * i + 2];
      const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
      const double len = std::sqrt((xx + yy) + zz);
      const int64_t e = g->orig_to_new_e[(size_t)p];
      edir[(size_t)(3 * e + 0)] = dx / len;
      edir[(size_t)(3 * e + 1)] = dy / len;
      edir[(size_t)(3 * e + 2)] = dz / len;
      len_orig[(size_t)p] = len;
      g->elen_h[(size_t)e] = len;
    }
  }
  // ---- reverse slots: position of the row's vertex in its neighbour's row
  std::vector<uint8_t> &rev = P->rev;
  rev.assign((size_t)E, 0);
  for (int64_t v = 0; v < n; ++v) {
    const int32_t vi = g->perm[(size_t)v];
    for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) {
      const int32_t w = g->nbr_h[(size_t)e];
      auto b = orig_nbr.begin() + rp[(size_t)w], en = orig_nbr.begin() + rp[(size_t)w + 1];
      auto it = std::lower_bound(b, en, vi);
      rev[(size_t)e] = (uint8_t)(it - b);
    }
  }
  // ---- tile halos: every neighbour of a tile's vertices, ascending; the
  // index of each edge's target in its tile's halo.  Tiles with more than
  // kHaloMax halo vertices gather directly (edge index = row slot).
  const int64_t ntiles = S.ntiles;
  std::vector<int32_t> &halo_ptr = P->halo_ptr, &halo_vid = P->halo_vid;
  halo_ptr.assign((size_t)ntiles + 1, 0);
  std::vector<uint16_t> &edge_hidx = P->edge_hidx;
  edge_hidx.assign((size_t)E, 0);
  std::vector<uint8_t> tile_direct((size_t)ntiles, 0);
  {
    // SX_FORCE_DIRECT=1 makes every tile gather directly (a test knob for
    // the path large-halo tiles take)
    const char *fd = std::getenv("SX_FORCE_DIRECT");
    const bool force_direct = fd && fd[0] == '1';
    std::vector<int32_t> h;
    for (int64_t t = 0; t < ntiles; ++t) {
      const int64_t v0 = t * sx::kTile, v1 = std::min<int64_t>(v0 + sx::kTile, n);
      h.clear();
      for (int64_t v = v0; v < v1; ++v)
        for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) h.push_back(g->nbr_h[(size_t)e]);
      std::sort(h.begin(), h.end());
      h.erase(std::unique(h.begin(), h.end()), h.end());
      if ((int64_t)h.size() > sx::kHaloMax || force_direct) {
        tile_direct[(size_t)t] = 1;
        for (int64_t v = v0; v < v1; ++v)
          for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e)
            edge_hidx[(size_t)e] = (uint16_t)(e - rp[(size_t)v]);
      } else {
        for (int64_t v = v0; v < v1; ++v)
          for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e)
            edge_hidx[(size_t)e] = (uint16_t)(std::lower_bound(h.begin(), h.end(),
                                                               g->nbr_h[(size_t)e]) - h.begin());
        halo_vid.insert(halo_vid.end(), h.begin(), h.end());
      }
      halo_ptr[(size_t)t + 1] = (int32_t)halo_vid.size();
    }
  }
  g->n_direct = 0;
  for (auto d8 : tile_direct) g->n_direct += d8;
  g->tile_direct = tile_direct;

  // ---- per-vertex physics in new order
  std::vector<double> &tau = P->tau, &dtnhv = P->dtnhv, &bco = P->bco, &y0 = P->y0;
  tau.assign((size_t)npad, 0.0);
  dtnhv.assign((size_t)npad, 1.0);
  bco.assign((size_t)npad, 0.0);
  y0.assign((size_t)npad, 1.0);
  g->dL_h.assign((size_t)n, 0.0);
  g->tau_h.assign((size_t)n, 0.0);
  for (int64_t v = 0; v < n; ++v) {
    const int32_t i = g->perm[(size_t)v];
    double dl;
    if (d->dL) {
      dl = d->dL[i];
    } else {
      // mean incident edge length (in the caller's row order) times kappa
      double sum = 0.0;
      const int64_t deg = d->nbr_ptr[i + 1] - d->nbr_ptr[i];
      for (int64_t p = d->nbr_ptr[i]; p < d->nbr_ptr[i + 1]; ++p) sum += len_orig[(size_t)p];
      dl = deg > 0 ? d->kappa * (sum / (double)deg) : 0.0;
    }
    g->dL_h[(size_t)v] = dl;
    tau[(size_t)v] = (d->n_H[i] * d->sigma) * dl;
    g->tau_h[(size_t)v] = tau[(size_t)v];
    dtnhv[(size_t)v] = d->dt * (d->n_H[i] * d->volume[i]);
    bco[(size_t)v] = (d->alpha_A > 0.0 ? d->alpha_A : d->alpha_B) * d->n_H[i];
    y0[(size_t)v] = d->x_init ? 1.0 - d->x_init[i] : 1.0;
  }
  // ---- photon unit: the power of two nearest the photons emitted per step
  double e_sweep = 0.0;
  for (int s = 0; s < d->n_src; ++s) e_sweep += d->src_rate[s] * d->dt;
  double unit = 1.0;
  if (e_sweep > 0.0 && std::isfinite(e_sweep)) unit = std::ldexp(1.0, (int)std::lround(std::log2(e_sweep)));
  // with multi-hop steps each sweep is a hop and emits N_dot dt / hops
  if (S.hops > 1) {
    e_sweep = 0.0;
    for (int s = 0; s < d->n_src; ++s) e_sweep += (d->src_rate[s] * d->dt) / (double)S.hops;
  }
  g->e_sweep = e_sweep;

  P->unit = unit;

  // ---- sources: per receiving vertex, in source order, the share of each
  // source's photons and the bin of the edge it arrives along.  The edge bin
  // is the device's rule (largest cosine, ties to the lower bin) evaluated
  // the same way, so both sides agree bit for bit.
  auto nearest_bin = [&](const double *ed) -> int32_t {
    int32_t best = 0;
    double cb = 0.0;
    for (int32_t k = 0; k < (int32_t)S.K; ++k) {
      const double *u = &P->bins[(size_t)(3 * k)];
      const double a = ed[0] * u[0], b = ed[1] * u[1], c3 = ed[2] * u[2];
      const double c = (a + b) + c3;
      if (k == 0 || c > cb) { cb = c; best = k; }
    }
    return best;
  };
  auto edge_bin = [&](int64_t e) -> int32_t { return nearest_bin(&edir[(size_t)(3 * e)]); };
  // The <= mpb edges of v's row most aligned with direction u, cosine >
  // cos_min, ties to the lower original id (rows are in original-id order):
  // the rule of the bins, used for beams and for ballistic transport.
  auto pick = [&](int64_t v, const double *u, int32_t *sl) -> int {
    double cs[3];
    int cnt = 0;
    for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) {
      const double *ed = &edir[(size_t)(3 * e)];
      const double a = ed[0] * u[0], b = ed[1] * u[1], c3 = ed[2] * u[2];
      const double c = (a + b) + c3;
      if (!(c > d->cos_min)) continue;
      int pos = cnt < d->max_per_bin ? cnt : d->max_per_bin;
      while (pos > 0 && c > cs[pos - 1]) --pos;
      if (pos >= d->max_per_bin) continue;
      const int last = cnt < d->max_per_bin ? cnt : d->max_per_bin - 1;
      for (int q = last; q > pos; --q) { cs[q] = cs[q - 1]; sl[q] = sl[q - 1]; }
      cs[pos] = c;
      sl[pos] = e;
      if (cnt < d->max_per_bin) ++cnt;
    }
    return cnt;
  };
  struct Em {
    int32_t recv;
    int32_t k;
    double amt;
    int32_t edge;   // the source's edge it travels along (new edge id)
    int32_t beam;   // the source of a beam share (its bin is the beam's), -1 isotropic
  };
  std::vector<Em> em;
  double esc_emit = 0.0;
  bool has_beam = false;
  for (int s = 0; s < d->n_src; ++s) {
    const int32_t vi = d->src_vertex[s];
    if (g->is_src_h.empty()) g->is_src_h.assign((size_t)n, 0);
    g->is_src_h[(size_t)g->inv[(size_t)vi]] = 1;
    const int32_t v = g->inv[(size_t)vi];
    double Es = d->src_rate[s] * d->dt;
    if (S.hops > 1) Es = Es / (double)S.hops;
    const double *u = d->src_dir ? d->src_dir + 3 * s : nullptr;
    const bool iso = !u || (u[0] == 0.0 && u[1] == 0.0 && u[2] == 0.0);
    const int64_t deg = d->nbr_ptr[vi + 1] - d->nbr_ptr[vi];
    if (iso) {
      if (deg == 0) { esc_emit += Es; continue; }
      const double share = (Es / unit) / (double)deg;
      for (int64_t p = d->nbr_ptr[vi]; p < d->nbr_ptr[vi + 1]; ++p) {
        const int32_t e = g->orig_to_new_e[(size_t)p];
        em.push_back({g->nbr_h[(size_t)e], edge_bin(e), share, e, -1});
      }
    } else {
      // beam: the <= mpb neighbours most aligned with u; the photons travel
      // along u and are filed in the bin closest to it
      int32_t sl[3];
      const int cnt = pick(v, u, sl);
      if (cnt == 0) { esc_emit += Es; continue; }
      const double share = (Es / unit) / (double)cnt;
      const int32_t kb = nearest_bin(u);
      for (int q = 0; q < cnt; ++q)
        em.push_back({g->nbr_h[(size_t)sl[q]], kb, share, sl[q], s});
      has_beam = true;
    }
  }
  g->esc_emit = esc_emit;
  if ((int64_t)em.size() >= ((int64_t)1 << sx::kRecIdxBits))
    return fail(ctx, SX_ENOTSUP, "too many source-neighbour pairs (%zu)", em.size());
  // per receiver, in source order (a bin's shares then add in source order
  // whatever the bins' orientation)
  std::stable_sort(em.begin(), em.end(), [](const Em &a, const Em &b) { return a.recv < b.recv; });
  std::vector<int32_t> &em_ptr = P->em_ptr, &em_k = P->em_k, &em_edge = P->em_edge;
  std::vector<double> &em_amt = P->em_amt;
  em_ptr.assign((size_t)npad + 1, 0);
  em_k.assign(em.size(), 0);
  em_edge.assign(em.size(), 0);
  em_amt.assign(em.size(), 0.0);
  P->em_beam.clear();
  P->beam_dir.clear();
  if (has_beam) {
    P->em_beam.assign(em.size(), -1);
    P->beam_dir.assign((size_t)3 * d->n_src, 0.0);
    for (int s = 0; s < d->n_src; ++s)
      for (int c = 0; c < 3; ++c) P->beam_dir[(size_t)(3 * s + c)] = d->src_dir[3 * s + c];
  }
  for (size_t q = 0; q < em.size(); ++q) {
    em_ptr[(size_t)em[q].recv + 1]++;
    em_k[q] = em[q].k;
    em_edge[q] = em[q].edge;
    em_amt[q] = em[q].amt;
    if (has_beam) P->em_beam[q] = em[q].beam;
  }
  for (int64_t v = 0; v < npad; ++v) em_ptr[(size_t)v + 1] += em_ptr[(size_t)v];
  g->n_em = (int64_t)em.size();

  // ---- combined transport: ballistic choice for the packet that entered v
  // along each of its edges (it keeps the direction nbr -> v, the opposite
  // of the edge's unit vector), and per receiving in-edge the list of the
  // sender's edges whose packets it gets, ascending
  P->transport = S.transport;
  g->transport = d->transport;
  // diffuse radiation runs in the combined-transport kernel; without
  // combined transport no vertex turns ballistic
  P->tau_switch = d->transport == SX_TRANSPORT_COMBINED ? d->tau_switch : INFINITY;
  P->dct_ref = d->dct_reference;
  P->alpha_A = d->alpha_A;
  P->alpha_B = d->alpha_B;
  if (d->alpha_A > 0.0 || S.hops > 1) {
    P->nhv.assign((size_t)npad, 0.0);
    for (int64_t v = 0; v < n; ++v) {
      const int32_t i = g->perm[(size_t)v];
      P->nhv[(size_t)v] = d->n_H[i] * d->volume[i];
    }
  }
  if (S.transport == SX_TRANSPORT_COMBINED) {
    g->bsel_h.assign((size_t)(3 * E), -1);
    g->bm_h.assign((size_t)E, 0);
    std::vector<int32_t> &blp = P->bl_ptr;
    blp.assign((size_t)E + 1, 0);
    for (int64_t v = 0; v < n; ++v)
      for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) {
        const double u[3] = {-edir[(size_t)(3 * e)], -edir[(size_t)(3 * e + 1)],
                             -edir[(size_t)(3 * e + 2)]};
        int32_t sl[3];
        const int cnt = pick(v, u, sl);
        g->bm_h[(size_t)e] = (uint8_t)cnt;
        for (int q = 0; q < cnt; ++q) {
          g->bsel_h[(size_t)(3 * e + q)] = sl[q];
          const int32_t l = g->nbr_h[(size_t)sl[q]];
          blp[(size_t)(rp[(size_t)l] + rev[(size_t)sl[q]]) + 1]++;
        }
      }
    int64_t tot = 0;
    for (int64_t e = 0; e < E; ++e) tot += blp[(size_t)e + 1];
    if (tot >= INT32_MAX) return fail(ctx, SX_ENOTSUP, "too many ballistic routes");
    for (int64_t e = 0; e < E; ++e) blp[(size_t)e + 1] += blp[(size_t)e];
    std::vector<int32_t> fillp(blp.begin(), blp.end() - 1);
    P->bl.assign((size_t)blp[(size_t)E], 0);
    P->elane.assign((size_t)E, 0);
    for (int64_t v = 0; v < n; ++v)
      for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) P->elane[(size_t)e] = (uint8_t)(v & 63);
    for (int64_t v = 0; v < n; ++v)
      for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e)
        for (int q = 0; q < g->bm_h[(size_t)e]; ++q) {
          const int32_t f = g->bsel_h[(size_t)(3 * e + q)];
          const int32_t in = rp[(size_t)g->nbr_h[(size_t)f]] + rev[(size_t)f];
          P->bl[(size_t)fillp[(size_t)in]++] = e;
        }
    P->bl4.assign((size_t)(4 * E), -1);
    for (int64_t e = 0; e < E; ++e)
      for (int32_t q = blp[(size_t)e]; q < blp[(size_t)e + 1] && q < blp[(size_t)e] + 4; ++q)
        P->bl4[(size_t)(4 * e + (q - blp[(size_t)e]))] = P->bl[(size_t)q];
  }
  return SX_OK;
}

// The device part of an upload: budget, slot, allocations, copies, the
// selection tables and gather lists built on the GPU, initial state.
int commit(sx_ctx *ctx, sx_prepared *P, sx_grid_id *out) {
  const Sizes S = P->S;
  const int64_t n = S.n, E = S.E, K = S.K, npad = S.npad, ntiles = S.ntiles;
  (void)n;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (ctx->free_slots.empty()) return fail(ctx, SX_ENOMEM, "too many grids");
  {
    const uint64_t want = bytes_estimate(S, (int64_t)P->em_k.size(),
                                         (int64_t)(0.05 * (double)(S.npad * S.K)),
                                         (int64_t)P->halo_vid.size());
    if (ctx->used + want > ctx->budget)
      return fail(ctx, SX_ENOMEM, "grid needs ~%llu bytes, %llu of %llu free",
                  (unsigned long long)want,
                  (unsigned long long)(ctx->budget - ctx->used),
                  (unsigned long long)ctx->budget);
  }
  Grid *g = P->g;
  P->g = nullptr;   // owned here from now on
  std::vector<int32_t> &rp = g->row_ptr_h;
  std::vector<int32_t> &halo_vid = P->halo_vid;
  const double unit = P->unit;

  // ---- device allocations
  GridDev &h = g->hg;
  h.n = (int32_t)n;
  h.npad = (int32_t)npad;
  h.ntiles = (int32_t)S.ntiles;
  h.k = (int32_t)K;
  h.kw = (int32_t)S.kw;
  h.bb = (int32_t)S.bb;
  h.kb = (int32_t)S.kb;
  h.n_sub = P->n_sub;
  h.mpb = P->mpb;
  h.max_deg = 1;
  for (int64_t v = 0; v < n; ++v)
    h.max_deg = std::max(h.max_deg, g->row_ptr_h[(size_t)v + 1] - g->row_ptr_h[(size_t)v]);
  h.precision = P->precision;
  {
    // SX_INW_ENTRIES=n (n >= 0) fills at most n entries of each in-word, so
    // that the rest become records (a test knob for the record path)
    h.inw_cap = sx::inw_entries((int)S.bb);
    const char *ie = std::getenv("SX_INW_ENTRIES");
    if (ie && ie[0] >= '0' && ie[0] <= '9') h.inw_cap = std::min(h.inw_cap, std::atoi(ie));
    std::memset(h.bperm, 0, sizeof(h.bperm));
    std::memset(h.bpos, 0, sizeof(h.bpos));
    for (int64_t p = 0; p < K; ++p) {
      h.bperm[p] = P->bperm[(size_t)p];
      h.bpos[P->bperm[(size_t)p]] = (uint8_t)p;
    }
  }
  h.parity = 0;
  h.remaining = 0;
  h.sweeps = 0;
  h.unit = unit;
  h.dt = P->dt;
  h.cos_min = P->cos_min;
  h.plane = npad + sx::kTile;   // the extra tile stays zero
  h.n_edges = E;
  h.transport = P->transport;
  h.dct_ref = P->dct_ref;
  h.diffuse = P->alpha_A > 0.0 ? 1 : 0;
  h.hops = (int32_t)S.hops;
  h.habs = nullptr;
  h.hnin = nullptr;
  h.dfrac = P->alpha_A > 0.0 ? (P->alpha_A - P->alpha_B) / P->alpha_A : 0.0;
  h.tau_switch = P->transport == SX_TRANSPORT_COMBINED ? P->tau_switch : 0.0;
  int32_t *d_rp, *d_nbr, *d_rec_cnt, *d_rec_ptr, *d_hptr, *d_hvid;
  uint8_t *d_rev, *d_ebin, *d_tdir;
  uint16_t *d_ehidx;
  double *d_edir, *d_bins, *d_tau, *d_dtnhv, *d_b, *d_y, *d_nin, *d_y0, *d_tally;
  uint32_t *d_fwd, *d_mb;
  uint64_t *d_inw;
  void *d_o0, *d_o1;
#define GA(ptr, cnt)                                      \
  do {                                                    \
    int r_ = galloc(ctx, g, &ptr, (uint64_t)(cnt));       \
    if (r_) { grid_release(ctx, g); return r_; }          \
  } while (0)
  GA(d_rp, npad + 1);
  GA(d_nbr, E);
  GA(d_rev, E);
  GA(d_edir, 3 * E);
  GA(d_bins, 3 * K);
  GA(d_fwd, npad * K);
  GA(d_ebin, E);
  GA(d_inw, npad * S.kb);
  GA(d_mb, npad * S.kw);
  uint32_t *d_mb2;
  GA(d_mb2, npad * S.kw);
  GA(d_rec_cnt, ntiles * K * sx::kRecGroups + 1);
  uint8_t *d_rlane;
  GA(d_rlane, ntiles * K * sx::kTile);
  GA(d_rec_ptr, ntiles * K * sx::kRecGroups + 1);
  int64_t *d_part;
  GA(d_part, ntiles * K * sx::kRecGroups / 1024 + 2);
  uint32_t *d_smask;
  GA(d_smask, 4 * (E + 1));
  int32_t *d_erev;
  GA(d_erev, E + 1);
  GA(d_hptr, ntiles + 1);
  GA(d_hvid, halo_vid.size() + 1);
  GA(d_ehidx, E);
  GA(d_tdir, ntiles);
  GA(d_tau, npad);
  GA(d_dtnhv, npad);
  GA(d_b, npad);
  GA(d_y, npad);
  GA(d_nin, npad);
  GA(d_y0, npad);
  GA(d_tally, 3 * S.ntiles);
  void *d_t0, *d_t1;
  {
    uint8_t *o0, *o1, *t0, *t1;
    GA(o0, (uint64_t)sx::kBlockBytes * S.kb * (npad + sx::kTile));
    GA(o1, (uint64_t)sx::kBlockBytes * S.kb * (npad + sx::kTile));
    GA(t0, (uint64_t)S.sp * (npad + sx::kTile));
    GA(t1, (uint64_t)S.sp * (npad + sx::kTile));
    d_o0 = o0;
    d_o1 = o1;
    d_t0 = t0;
    d_t1 = t1;
  }
  h.row_ptr = d_rp;
  h.nbr = d_nbr;
  h.rev = d_rev;
  h.edir = d_edir;
  h.bins = d_bins;
  h.fwd = d_fwd;
  h.ebin = d_ebin;
  h.inw = d_inw;
  h.mbits = d_mb;
  h.mbits2 = d_mb2;
  h.rec_cnt = d_rec_cnt;
  h.rec_lane = d_rlane;
  h.rec_ptr = d_rec_ptr;
  h.scan_part = d_part;
  h.smask = d_smask;
  h.erev = d_erev;
  h.rec = nullptr;
  h.rec_cap = 0;
  h.halo_ptr = d_hptr;
  h.halo_vid = d_hvid;
  h.edge_hidx = d_ehidx;
  h.tile_direct = d_tdir;
  h.tau = d_tau;
  h.dtnhv = d_dtnhv;
  h.bcoef = d_b;
  h.y = d_y;
  h.nin = d_nin;
  h.o[0] = d_o0;
  h.o[1] = d_o1;
  h.t[0] = d_t0;
  h.t[1] = d_t1;
  h.tally = d_tally;
  g->y_init = d_y0;
  g->slot = ctx->free_slots.back();
  ctx->free_slots.pop_back();

  hipStream_t st = wstream(ctx);
  auto H2D = [&](void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
#define UP(dst, src, bytes)                                                   \
  do {                                                                        \
    hipError_t e_ = H2D(dst, src, bytes);                                     \
    if (e_ != hipSuccess) {                                                   \
      grid_release(ctx, g);                                                   \
      return fail(ctx, SX_EDEVICE, "upload copy failed: %s", hipGetErrorString(e_)); \
    }                                                                         \
  } while (0)
  UP(d_rp, rp.data(), 4 * (npad + 1));
  UP(d_nbr, g->nbr_h.data(), 4 * E);
  UP(d_rev, P->rev.data(), E);
  UP(d_edir, P->edir.data(), 24 * E);
  UP(d_bins, P->bins.data(), 24 * K);
  UP(d_tau, P->tau.data(), 8 * npad);
  UP(d_dtnhv, P->dtnhv.data(), 8 * npad);
  UP(d_b, P->bco.data(), 8 * npad);
  UP(d_y0, P->y0.data(), 8 * npad);
  UP(d_hptr, P->halo_ptr.data(), 4 * (ntiles + 1));
  UP(d_hvid, halo_vid.data(), 4 * halo_vid.size());
  UP(d_ehidx, P->edge_hidx.data(), 2 * E);
  UP(d_tdir, g->tile_direct.data(), ntiles);
  if (hipStreamSynchronize(st) != hipSuccess) {
    grid_release(ctx, g);
    return fail(ctx, SX_EDEVICE, "upload sync failed");
  }
  int r;
  if ((r = write_slot(ctx, g))) { grid_release(ctx, g); return r; }

  // ---- selection tables, source lists, gather lists (records sized by a
  // count pass)
  GridDev *dg = ctx->table + g->slot;
  auto kfail = [&](hipError_t e) {
    grid_release(ctx, g);
    return fail(ctx, SX_EDEVICE, "table kernels failed: %s", hipGetErrorString(e));
  };
  hipError_t he;
  const int32_t nrow = (int32_t)(ntiles * K * sx::kRecGroups);
  if ((he = sx::launch_erev(dg, h, st)) != hipSuccess) return kfail(he);
  if ((he = sx::launch_select(dg, h, h.mbits, st)) != hipSuccess) return kfail(he);
  if ((he = sx::launch_edge_bins(dg, h, st)) != hipSuccess) return kfail(he);
  g->n_em = (int64_t)P->em_k.size();
  {
    int32_t *d_emp, *d_emk, *d_eme;
    double *d_ema;
    GA(d_emp, npad + 1);
    GA(d_emk, g->n_em + 1);
    GA(d_eme, g->n_em + 1);
    GA(d_ema, g->n_em + 1);
    UP(d_emp, P->em_ptr.data(), 4 * (npad + 1));
    if (g->n_em) {
      UP(d_emk, P->em_k.data(), 4 * g->n_em);
      UP(d_eme, P->em_edge.data(), 4 * g->n_em);
      UP(d_ema, P->em_amt.data(), 8 * g->n_em);
    }
    h.em_ptr = d_emp;
    h.em_k = d_emk;
    h.em_edge = d_eme;
    h.em_amt = d_ema;
    h.em_beam = nullptr;
    h.beam_dir = nullptr;
    if (!P->em_beam.empty()) {
      int32_t *d_emb;
      double *d_bd;
      GA(d_emb, g->n_em + 1);
      GA(d_bd, P->beam_dir.size());
      UP(d_emb, P->em_beam.data(), 4 * g->n_em);
      UP(d_bd, P->beam_dir.data(), 8 * P->beam_dir.size());
      h.em_beam = d_emb;
      h.beam_dir = d_bd;
    }
  }
  g->bins0 = P->bins;
  g->bins_cur = P->bins;
  if ((r = write_slot(ctx, g))) { grid_release(ctx, g); return r; }
  if ((he = sx::launch_clear_inw(h, st)) != hipSuccess) return kfail(he);
  if ((he = sx::launch_inlist_count(dg, h, st)) != hipSuccess) return kfail(he);
  if ((he = sx::launch_scan(h.rec_cnt, h.rec_ptr, h.scan_part, nrow, st)) != hipSuccess) return kfail(he);
  int32_t n_rec = 0;
  if ((he = hipMemcpyAsync(&n_rec, h.rec_ptr + nrow, 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return kfail(he);
  if ((he = hipStreamSynchronize(st)) != hipSuccess) return kfail(he);
  {
    uint32_t *d_rec;
    GA(d_rec, (uint64_t)n_rec + 1);
    h.rec = d_rec;
    h.rec_cap = n_rec;
  }
  if ((r = write_slot(ctx, g))) { grid_release(ctx, g); return r; }
  if ((he = sx::launch_inlist_fill(dg, h, st)) != hipSuccess) return kfail(he);

  if (P->transport == SX_TRANSPORT_COMBINED) {
    int32_t *d_klp, *d_klc, *d_blp, *d_bl;
    int64_t *d_klpart;
    uint8_t *d_bm, *d_el, *d_eb, *d_l0, *d_l1, *d_e0, *d_e1, *d_x;
    GA(d_klp, E + 1);
    GA(d_klc, E + 1);
    GA(d_klpart, E / 1024 + 2);
    GA(d_blp, E + 1);
    GA(d_bl, P->bl.size() + 1);
    GA(d_bm, E + 1);
    GA(d_el, E + 1);
    int4 *d_b4;
    GA(d_b4, E + 1);
    GA(d_eb, E + 1);
    GA(d_x, (uint64_t)sx::kBlockBytes * S.kb * (npad + sx::kTile));
    GA(d_e0, (uint64_t)S.sp * (E + 1));
    GA(d_e1, (uint64_t)S.sp * (E + 1));
    GA(d_l0, npad);
    GA(d_l1, npad);
    UP(d_blp, P->bl_ptr.data(), 4 * (E + 1));
    UP(d_bl, P->bl.data(), 4 * P->bl.size());
    UP(d_bm, g->bm_h.data(), E);
    UP(d_el, P->elane.data(), E);
    UP(d_b4, P->bl4.data(), 16 * E);
    if ((he = hipStreamSynchronize(st)) != hipSuccess) return kfail(he);
    h.kl_ptr = d_klp;
    h.kl_cnt = d_klc;
    h.kl_part = d_klpart;
    h.kl = nullptr;
    h.kl_cap = 0;
    h.bl_ptr = d_blp;
    h.bl = d_bl;
    h.elane = d_el;
    h.bl4 = d_b4;
    h.ebin_in = d_eb;
    h.xin = d_x;
    h.bm = d_bm;
    h.oe[0] = d_e0;
    h.oe[1] = d_e1;
    h.lay[0] = d_l0;
    h.lay[1] = d_l1;
    // the bin of each in-edge and the per-in-edge bin lists, on the device
    if ((r = write_slot(ctx, g))) { grid_release(ctx, g); return r; }
    if ((r = build_ct_tables(ctx, g))) { grid_release(ctx, g); return r; }
  }
  if (h.hops > 1) {
    double *d_nhv, *d_ha, *d_hn;
    GA(d_nhv, npad);
    GA(d_ha, npad);
    GA(d_hn, npad);
    UP(d_nhv, P->nhv.data(), 8 * npad);
    if ((he = hipStreamSynchronize(st)) != hipSuccess) return kfail(he);
    h.nhv = d_nhv;
    h.habs = d_ha;
    h.hnin = d_hn;
  }
  if (h.diffuse) {
    double *d_nhv, *d_dt;
    uint8_t *d_s0, *d_s1;
    GA(d_nhv, npad);
    GA(d_dt, ntiles);
    GA(d_s0, (uint64_t)S.sp * (npad + sx::kTile));
    GA(d_s1, (uint64_t)S.sp * (npad + sx::kTile));
    UP(d_nhv, P->nhv.data(), 8 * npad);
    if ((he = hipStreamSynchronize(st)) != hipSuccess) return kfail(he);
    h.nhv = d_nhv;
    h.dtally = d_dt;
    h.dsh[0] = d_s0;
    h.dsh[1] = d_s1;
  }

#undef GA
#undef UP
  if ((r = write_slot(ctx, g))) { grid_release(ctx, g); return r; }
  if ((he = sx::launch_reset_state(dg, h, g->y_init, st)) != hipSuccess) return kfail(he);
  if ((he = hipStreamSynchronize(st)) != hipSuccess) return kfail(he);
  if ((he = hipGetLastError()) != hipSuccess) return kfail(he);
  g->id = ctx->next_id++;
  ctx->grids[g->id] = g;
  *out = g->id;
  return SX_OK;
}

}  // namespace

// Combined-transport grid by id, or an error code.
static int combined_grid(sx_ctx *ctx, sx_grid_id id, Grid **out) {
  if (!ctx) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  if (g->transport != SX_TRANSPORT_COMBINED)
    return fail(ctx, SX_EINVAL, "grid %lld does not use combined transport", (long long)id);
  *out = g;
  return SX_OK;
}

// new edge -> caller's CSR position
static std::vector<int32_t> new_to_orig_edges(const Grid *g) {
  std::vector<int32_t> m(g->orig_to_new_e.size());
  for (size_t p = 0; p < m.size(); ++p) m[(size_t)g->orig_to_new_e[p]] = (int32_t)p;
  return m;
}

// =================================================================== ABI ==
extern "C" {

const char *sx_strerror(int code) {
  switch (code) {
    case SX_OK: return "ok";
    case SX_EINVAL: return "invalid argument";
    case SX_ENOMEM: return "out of device memory budget";
    case SX_EDEVICE: return "device error";
    case SX_ENOTFOUND: return "unknown grid";
    case SX_ENOTSUP: return "not supported";
    default: return "unknown error";
  }
}

const char *sx_last_error(const sx_ctx *ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

int sx_init(sx_ctx **out, const sx_ctx_opts *opts) {
  if (!out) return SX_EINVAL;
  *out = nullptr;
  sx_ctx_opts o{};
  if (opts) o = *opts;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return SX_EDEVICE;
  }
  if (o.device < 0 || o.device >= ndev) return SX_EINVAL;
  if ((o.alloc == nullptr) != (o.free == nullptr)) return SX_EINVAL;
  if (hipSetDevice(o.device) != hipSuccess) return SX_EDEVICE;
  sx_ctx *ctx = new sx_ctx();
  ctx->device = o.device;
  ctx->alloc = o.alloc;
  ctx->free_fn = o.free;
  ctx->user = o.alloc_user;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    delete ctx;
    return SX_EDEVICE;
  }
  ctx->budget = o.hbm_budget ? o.hbm_budget : (uint64_t)(0.9 * (double)fr);
  if (o.stream) {
    ctx->stream = (hipStream_t)o.stream;
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return SX_EDEVICE;
    }
    ctx->own_stream = true;
  }
  if (hipMalloc(&ctx->table, sizeof(GridDev) * kMaxSlots) != hipSuccess) {
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return SX_EDEVICE;
  }
  if (hipMalloc(&ctx->done, 256) != hipSuccess || hipMemset(ctx->done, 0, 256) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(ctx->table);
    if (ctx->done) (void)hipFree(ctx->done);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return SX_EDEVICE;
  }
  if (hipHostMalloc((void **)&ctx->pin, kPinBytes, hipHostMallocDefault) != hipSuccess) {
    ctx->pin = nullptr;
    (void)hipFree(ctx->done);
    (void)hipFree(ctx->table);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return SX_EDEVICE;
  }
  // the device address of the no-allocation step's scratch array, once per
  // device (kept by the library for later contexts)
  {
    void *sp = nullptr;
    if (sx::noalloc_scratch_init(o.device, &sp) != hipSuccess || !sp) {
      (void)hipGetLastError();
      (void)hipHostFree(ctx->pin);
      (void)hipFree(ctx->done);
      (void)hipFree(ctx->table);
      if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
      delete ctx;
      return SX_EDEVICE;
    }
    ctx->scratch = (uint8_t *)sp;
  }
  if (hipStreamCreateWithFlags(&ctx->io, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(ctx->pin);
    (void)hipFree(ctx->done);
    (void)hipFree(ctx->table);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return SX_EDEVICE;
  }
  for (int s = kMaxSlots - 1; s >= 0; --s) ctx->free_slots.push_back(s);
  *out = ctx;
  return SX_OK;
}

int sx_finalize(sx_ctx *ctx) {
  if (!ctx) return SX_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipStreamSynchronize(ctx->io);
  ctx->io_on = false;
  for (auto &kv : ctx->grids) grid_release(ctx, kv.second);
  ctx->grids.clear();
  drop_plans(ctx, -1);
  for (auto &e : ctx->ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  (void)hipFree(ctx->done);
  (void)hipFree(ctx->table);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  if (ctx->io) (void)hipStreamDestroy(ctx->io);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return SX_OK;
}

void *sx_stream(sx_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

int sx_mem_info(sx_ctx *ctx, uint64_t *used, uint64_t *budget) {
  if (!ctx) return SX_EINVAL;
  if (used) *used = ctx->used;
  if (budget) *budget = ctx->budget;
  return SX_OK;
}

int sx_grid_bytes(const sx_grid_desc *d, uint64_t *bytes) {
  if (!d || !bytes || d->n_vertices < 1 || !d->nbr_ptr || d->n_bins < 1)
    return SX_EINVAL;
  const Sizes s = sizes_of(d);
  // overflow entries: expect ~0.3 per (vertex, bin) on Poisson-Delaunay
  // grids; the exact pool is allocated after the count pass
  // records: ~0.02 per (vertex, bin) on Poisson-Delaunay grids; halos
  // ~4 vertices per tile vertex.  The exact pools are allocated at upload.
  *bytes = bytes_estimate(s, s.E, (int64_t)(0.05 * (double)(s.npad * s.K)), 5 * s.npad);
  return SX_OK;
}

int sx_grid_prepare(const sx_grid_desc *d, sx_prepared **out, char *err, size_t err_len) {
  if (!out) return SX_EINVAL;
  *out = nullptr;
  sx_ctx sink;   // collects the message only
  sx_prepared *P = new sx_prepared();
  int r = prepare(&sink, d, P);
  if (r) {
    delete P;
    if (err && err_len) snprintf(err, err_len, "%s", sink.err.c_str());
    return r;
  }
  *out = P;
  return SX_OK;
}

int sx_grid_commit(sx_ctx *ctx, sx_prepared *p, sx_grid_id *out) {
  if (!ctx || !p || !out) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  if (!p->g) return fail(ctx, SX_EINVAL, "prepared grid already committed");
  return commit(ctx, p, out);
}

int sx_prepared_free(sx_prepared *p) {
  delete p;
  return SX_OK;
}

int sx_prepared_bytes(const sx_prepared *p, uint64_t *bytes) {
  if (!p || !bytes || !p->g) return SX_EINVAL;
  *bytes = bytes_estimate(p->S, (int64_t)p->em_k.size(),
                          (int64_t)(0.05 * (double)(p->S.npad * p->S.K)),
                          (int64_t)p->halo_vid.size());
  return SX_OK;
}

int sx_grid_upload(sx_ctx *ctx, const sx_grid_desc *d, sx_grid_id *out) {
  if (!ctx || !out) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  sx_prepared P;
  int r = prepare(ctx, d, &P);
  if (r) return r;
  return commit(ctx, &P, out);
}

int sx_grid_reset(sx_ctx *ctx, sx_grid_id id) {
  if (!ctx) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  int r = rebuild_routing(ctx, g, g->bins0.data(), nullptr);
  if (r) return r;
  g->rotated = false;
  g->unusable = false;
  HIP_TRY(ctx, sx::launch_reset_state(ctx->table + g->slot, g->hg, g->y_init, ctx->stream));
  g->base_sweeps = g->base_emitted = g->base_escaped = 0.0;
  return SX_OK;
}

int sx_rotate_bins(sx_ctx *ctx, sx_grid_id id, const double *R) {
  if (!ctx) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  if (!R) return fail(ctx, SX_EINVAL, "null rotation");
  // a rotation: orthonormal rows, determinant +1
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(R[i])) return fail(ctx, SX_EINVAL, "rotation has a non-finite entry");
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double d = R[3 * a] * R[3 * b] + R[3 * a + 1] * R[3 * b + 1] + R[3 * a + 2] * R[3 * b + 2];
      if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-9)
        return fail(ctx, SX_EINVAL, "rotation rows are not orthonormal");
    }
  const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                     R[2] * (R[3] * R[7] - R[4] * R[6]);
  if (!(det > 0.0)) return fail(ctx, SX_EINVAL, "rotation has determinant %g", det);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int64_t K = g->hg.k;
  std::vector<double> b((size_t)(3 * K));
  for (int64_t k = 0; k < K; ++k) {
    const double *u = &g->bins0[(size_t)(3 * k)];
    for (int r = 0; r < 3; ++r) {
      const double p0 = R[3 * r] * u[0], p1 = R[3 * r + 1] * u[1], p2 = R[3 * r + 2] * u[2];
      b[(size_t)(3 * k + r)] = (p0 + p1) + p2;
    }
  }
  // Each old bin's photons go to the rotated bin closest to its direction
  // (largest cosine ((d_x n_x + d_y n_y) + d_z n_z), ties to the lower new
  // bin); the map lists, per new bin, the old bins it takes, ascending.
  sx::RebinMap map{};
  {
    std::vector<int32_t> to((size_t)K), cnt((size_t)K + 1, 0);
    for (int64_t k = 0; k < K; ++k) {
      const double *d = &g->bins_cur[(size_t)(3 * k)];
      int32_t best = 0;
      double cb = 0.0;
      for (int64_t q = 0; q < K; ++q) {
        const double *u = &b[(size_t)(3 * q)];
        const double p0 = d[0] * u[0], p1 = d[1] * u[1], p2 = d[2] * u[2];
        const double c = (p0 + p1) + p2;
        if (q == 0 || c > cb) { cb = c; best = (int32_t)q; }
      }
      to[(size_t)k] = best;
      cnt[(size_t)best + 1]++;
    }
    for (int64_t q = 0; q < K; ++q) cnt[(size_t)q + 1] += cnt[(size_t)q];
    std::vector<uint8_t> list((size_t)K);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t k = 0; k < K; ++k) list[(size_t)fill[(size_t)to[(size_t)k]]++] = (uint8_t)k;
    // the same lists by storage position, for the device
    const GridDev &hg = g->hg;
    int32_t at = 0;
    for (int64_t p = 0; p < K; ++p) {
      const int kn = hg.bperm[p];
      map.ptr[p] = (uint8_t)at;
      map.bin[p] = (uint8_t)kn;
      for (int32_t q = cnt[(size_t)kn]; q < cnt[(size_t)kn + 1]; ++q)
        map.list[at++] = hg.bpos[list[(size_t)q]];
    }
    map.ptr[K] = (uint8_t)at;
  }
  int r = rebuild_routing(ctx, g, b.data(), &map);
  if (r) return r;
  g->rotated = true;
  return SX_OK;
}

int sx_grid_free(sx_ctx *ctx, sx_grid_id id) {
  if (!ctx) return SX_EINVAL;
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(wstream(ctx));
  // launch plans that reference this grid's slot (none of them is running
  // while io_on: the caller frees only grids outside the running sweeps)
  drop_plans(ctx, g->slot);
  ctx->grids.erase(id);
  grid_release(ctx, g);
  return SX_OK;
}

namespace {

int split_of(const sx_schedule &s) { return s.work_split > 1 ? s.work_split : 1; }

bool valid_schedule(const sx_schedule &s) {
  return (s.tiles_per_group == 1 || s.tiles_per_group == 2 || s.tiles_per_group == 4) &&
         (s.work_split >= 0 && s.work_split <= 4 && s.work_split != 3) &&
         s.tiles_per_group * split_of(s) <= 4 &&
         (s.order == SX_ORDER_GRID || s.order == SX_ORDER_DIRECT_FIRST) &&
         (s.xcd_contiguous == 0 || s.xcd_contiguous == 1) && s.graph_sweeps >= 0 &&
         s.graph_sweeps <= SX_MAX_GRAPH_SWEEPS;
}

void plan_unbuild(Plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  for (void *d : p->dev) (void)hipFree(d);
  p->dev.clear();
  p->launches.clear();
  p->built = false;
}

// Lay out the launches of one sweep for `gs` under p->sched: one launch per
// precision and transport mode present (grids in the caller's order), tiles grid by grid in
// each grid's (Hilbert) order, or the directly gathering tiles first.
int plan_build(sx_ctx *ctx, Plan *p, const std::vector<Grid *> &gs) {
  plan_unbuild(p);
  for (int cls = 0; cls < 4; ++cls) {
    const int prec = cls & 1 ? SX_FP32_TRANSPORT : SX_FP64;
    const int tr = cls >> 1;
    std::vector<Grid *> grp;
    for (Grid *g : gs)
      if (g->hg.precision == prec && g->hg.transport == tr) grp.push_back(g);
    if (grp.empty()) continue;
    sx::SweepLaunch l{};
    l.done = ctx->done;
    l.split = tr ? 1 : split_of(p->sched);
    l.tpb = tr ? 1 : p->sched.tiles_per_group * l.split;
    l.xcd_remap = p->sched.xcd_contiguous;
    l.precision = prec;
    l.transport = tr;
    int64_t plane_bytes = 0;   // both photon planes of every grid in the launch
    for (Grid *g : grp)
      plane_bytes += 2 * (int64_t)sx::kBlockBytes * g->hg.kb * (g->hg.npad + sx::kTile);
    l.nt = plane_bytes <= sx::kLlcBytes;
    const bool any_direct = std::any_of(grp.begin(), grp.end(),
                                        [](Grid *g) { return g->n_direct > 0; });
    const bool reorder = p->sched.order == SX_ORDER_DIRECT_FIRST && any_direct;
    if (grp.size() == 1 && !reorder) {
      l.grids = ctx->table + grp[0]->slot;
      l.map = nullptr;
      l.n_tiles = grp[0]->hg.ntiles;
      l.adv = nullptr;
      l.n_adv = 1;
    } else {
      std::vector<int2> map;
      for (int pass = reorder ? 0 : 1; pass < 2; ++pass)
        for (Grid *g : grp)
          for (int32_t t = 0; t < g->hg.ntiles; ++t)
            if (!reorder || (g->tile_direct[(size_t)t] != 0) == (pass == 0))
              map.push_back(make_int2(g->slot, t));
      std::vector<int32_t> adv;
      for (Grid *g : grp) adv.push_back(g->slot);
      int2 *dmap = nullptr;
      int32_t *dadv = nullptr;
      HIP_TRY(ctx, hipMalloc(&dmap, sizeof(int2) * map.size()));
      p->dev.push_back(dmap);
      HIP_TRY(ctx, hipMalloc(&dadv, sizeof(int32_t) * adv.size()));
      p->dev.push_back(dadv);
      HIP_TRY(ctx, hipMemcpyAsync(dmap, map.data(), sizeof(int2) * map.size(),
                                  hipMemcpyHostToDevice, ctx->stream));
      HIP_TRY(ctx, hipMemcpyAsync(dadv, adv.data(), sizeof(int32_t) * adv.size(),
                                  hipMemcpyHostToDevice, ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      l.grids = ctx->table;
      l.map = dmap;
      l.n_tiles = (int32_t)map.size();
      l.adv = dadv;
      l.n_adv = (int32_t)adv.size();
    }
    p->launches.push_back(l);
  }
  if (p->sched.graph_sweeps > 0) {
    HIP_TRY(ctx, hipGraphCreate(&p->graph, 0));
    hipGraphNode_t prev = nullptr;
    for (int32_t s = 0; s < p->sched.graph_sweeps; ++s)
      for (auto &l : p->launches) HIP_TRY(ctx, sx::add_sweep_node(p->graph, l, &prev));
    HIP_TRY(ctx, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  }
  p->built = true;
  return SX_OK;
}

// Plans that hold `slot` (all plans for slot < 0), after the stream drains.
void drop_plans(sx_ctx *ctx, int slot) {
  (void)hipStreamSynchronize(wstream(ctx));
  std::vector<Plan *> keep;
  for (Plan *p : ctx->plans) {
    if (slot < 0 || std::find(p->key.begin(), p->key.end(), slot) != p->key.end()) {
      plan_unbuild(p);
      delete p;
    } else {
      keep.push_back(p);
    }
  }
  ctx->plans.swap(keep);
}

Plan *get_plan(sx_ctx *ctx, const std::vector<Grid *> &gs) {
  std::vector<int32_t> key;
  for (Grid *g : gs) key.push_back(g->slot);
  for (Plan *p : ctx->plans)
    if (p->key == key) return p;
  if (ctx->plans.size() >= 64) {
    // forget the oldest plan without a caller-set schedule
    (void)hipStreamSynchronize(ctx->stream);
    for (size_t i = 0; i < ctx->plans.size(); ++i) {
      Plan *o = ctx->plans[i];
      plan_unbuild(o);
      delete o;
      ctx->plans.erase(ctx->plans.begin() + (long)i);
      break;
    }
  }
  Plan *p = new Plan();
  p->key = key;
  p->sched = ctx->dflt;
  ctx->plans.push_back(p);
  return p;
}

ProfEv *prof_begin(sx_ctx *ctx, int32_t launches, hipError_t *err) {
  *err = hipSuccess;
  if (!ctx->prof) return nullptr;
  if (ctx->ev_used == ctx->ev.size()) {
    ProfEv e;
    if ((*err = hipEventCreate(&e.a)) != hipSuccess) return nullptr;
    if ((*err = hipEventCreate(&e.b)) != hipSuccess) return nullptr;
    ctx->ev.push_back(e);
  }
  ProfEv *e = &ctx->ev[ctx->ev_used++];
  e->launches = launches;
  *err = hipEventRecord(e->a, ctx->stream);
  return e;
}

// n sweeps of a built plan: whole graph replays, then single launches.
int run_plan(sx_ctx *ctx, Plan *p, int32_t n) {
  hipError_t pe;
  const int32_t per = (int32_t)p->launches.size();
  int32_t s = 0;
  if (p->exec)
    for (; s + p->sched.graph_sweeps <= n; s += p->sched.graph_sweeps) {
      ProfEv *e = prof_begin(ctx, p->sched.graph_sweeps * per, &pe);
      HIP_TRY(ctx, pe);
      HIP_TRY(ctx, hipGraphLaunch(p->exec, ctx->stream));
      if (e) HIP_TRY(ctx, hipEventRecord(e->b, ctx->stream));
    }
  for (; s < n; ++s)
    for (auto &l : p->launches) {
      ProfEv *e = prof_begin(ctx, 1, &pe);
      HIP_TRY(ctx, pe);
      HIP_TRY(ctx, sx::launch_sweep(l, ctx->stream));
      if (e) HIP_TRY(ctx, hipEventRecord(e->b, ctx->stream));
    }
  return SX_OK;
}

// Time each candidate schedule on `trials` of the grids' own sweeps (the
// schedule only reorders independent tiles, so results do not change) and
// keep the fastest.  Returns the sweeps used in *used.
int autotune(sx_ctx *ctx, Plan *p, const std::vector<Grid *> &gs, int32_t trials,
             int32_t n_launch, int32_t *used) {
  *used = 0;
  bool any_direct = false;
  for (Grid *g : gs) any_direct = any_direct || g->n_direct > 0;
  // Two stages: the launch shape (tiles per group x waves per tile) under
  // the XCD-contiguous grid order, then the tile order for the best shape.
  const int shapes[6][2] = {{4, 1}, {2, 1}, {1, 1}, {2, 2}, {1, 2}, {1, 4}};
  const int n_orders = any_direct ? 4 : 2;
  const int64_t n_cand = 6 + (n_orders - 1);
  // only when tuning takes at most a quarter of the sweeps asked for
  if ((int64_t)n_launch < 4 * (int64_t)trials * n_cand) return SX_OK;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev((size_t)trials);
  for (auto &e : ev) {
    HIP_TRY(ctx, hipEventCreate(&e.first));
    HIP_TRY(ctx, hipEventCreate(&e.second));
  }
  const int32_t graph_sweeps = p->sched.graph_sweeps;
  double best = 1e300;
  sx_schedule best_s = p->sched;
  int rc = SX_OK;
  auto time_one = [&](const sx_schedule &c) {
    p->sched = c;
    if ((rc = plan_build(ctx, p, gs))) return;
    std::vector<double> t;
    for (int32_t i = 0; i < trials && rc == SX_OK; ++i) {
      if (hipEventRecord(ev[(size_t)i].first, ctx->stream) != hipSuccess ||
          run_plan(ctx, p, 1) != SX_OK ||
          hipEventRecord(ev[(size_t)i].second, ctx->stream) != hipSuccess)
        rc = fail(ctx, SX_EDEVICE, "autotune launch failed");
    }
    if (rc) return;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
      rc = fail(ctx, SX_EDEVICE, "autotune sync failed");
      return;
    }
    for (int32_t i = 0; i < trials; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[(size_t)i].first, ev[(size_t)i].second) == hipSuccess)
        t.push_back(ms);
    }
    *used += trials;
    // the first trial of a schedule also pays for its first launch
    std::sort(t.begin() + (t.size() > 1 ? 1 : 0), t.end());
    const double v = t.size() > 1 ? t[1] : (t.empty() ? 1e300 : t[0]);
    if (v < best) {
      best = v;
      best_s = c;
    }
  };
  for (const auto &sh : shapes) {
    if (rc) break;
    time_one({sh[0], SX_ORDER_GRID, 1, 0, sh[1]});
  }
  const sx_schedule shape = best_s;
  for (int o = 1; o < n_orders && rc == SX_OK; ++o) {
    sx_schedule c = shape;
    c.xcd_contiguous = (o & 1) ? 0 : 1;
    c.order = (o & 2) ? SX_ORDER_DIRECT_FIRST : SX_ORDER_GRID;
    time_one(c);
  }
  for (auto &e : ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (rc) return rc;
  best_s.graph_sweeps = graph_sweeps;
  p->sched = best_s;
  p->fixed = true;
  p->tuned_us = 1e3 * best;
  return plan_build(ctx, p, gs);
}

int launch_steps(sx_ctx *ctx, std::vector<Grid *> &gs, int32_t n_launch) {
  if (n_launch <= 0 || gs.empty()) return SX_OK;
  Plan *p = get_plan(ctx, gs);
  if (ctx->autotune > 0 && !p->fixed) {
    int32_t used = 0;
    int r = autotune(ctx, p, gs, ctx->autotune, n_launch, &used);
    if (r) return r;
    n_launch -= used;
  }
  if (!p->built) {
    int r = plan_build(ctx, p, gs);
    if (r) return r;
  }
  return run_plan(ctx, p, n_launch);
}

int collect(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, std::vector<Grid *> &gs) {
  if (n < 0 || (n > 0 && !ids)) return fail(ctx, SX_EINVAL, "bad id list");
  for (int32_t i = 0; i < n; ++i) {
    Grid *g = find(ctx, ids[i]);
    if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)ids[i]);
    if (g->unusable)
      return fail(ctx, SX_ENOMEM, "grid %lld: a rotation could not finish its tables; "
                  "reset or free it", (long long)ids[i]);
    for (Grid *o : gs)
      if (o == g) return fail(ctx, SX_EINVAL, "grid %lld listed twice", (long long)ids[i]);
    gs.push_back(g);
  }
  return SX_OK;
}

}  // namespace

int sx_step(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, int32_t n_sweeps) {
  if (!ctx) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  if (n_sweeps < 0) return fail(ctx, SX_EINVAL, "n_sweeps < 0");
  std::vector<Grid *> gs;
  int r = collect(ctx, ids, n, gs);
  if (r) return r;
  if (n_sweeps == 0 || gs.empty()) return SX_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  std::vector<int32_t> slots, vals;
  for (Grid *g : gs) {
    slots.push_back(g->slot);
    vals.push_back(n_sweeps);
  }
  HIP_TRY(ctx, sx::launch_set_remaining(ctx->table, slots.data(), vals.data(), n, 1,
                                        ctx->stream));
  return launch_steps(ctx, gs, n_sweeps);
}

int sx_step_noalloc(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, int32_t n_sweeps) {
  if (!ctx) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  if (n_sweeps < 0) return fail(ctx, SX_EINVAL, "n_sweeps < 0");
  if (n < 0 || (n > 0 && !ids)) return fail(ctx, SX_EINVAL, "bad id list");
  if (n > SX_NOALLOC_MAX_GRIDS)
    return fail(ctx, SX_EINVAL, "%d grids exceed the no-allocation limit of %d", n,
                SX_NOALLOC_MAX_GRIDS);
  if (!ctx->scratch) return fail(ctx, SX_EDEVICE, "no-allocation scratch not set up");
  // fixed-size host arrays: nothing is allocated on either side
  Grid *gs[SX_NOALLOC_MAX_GRIDS];
  int32_t slots[SX_NOALLOC_MAX_GRIDS], vals[SX_NOALLOC_MAX_GRIDS];
  int64_t tiles = 0;
  for (int32_t i = 0; i < n; ++i) {
    Grid *g = find(ctx, ids[i]);
    if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)ids[i]);
    if (g->unusable)
      return fail(ctx, SX_ENOMEM, "grid %lld: a rotation could not finish its tables; "
                  "reset or free it", (long long)ids[i]);
    for (int32_t q = 0; q < i; ++q)
      if (gs[q] == g) return fail(ctx, SX_EINVAL, "grid %lld listed twice", (long long)ids[i]);
    gs[i] = g;
    slots[i] = g->slot;
    vals[i] = n_sweeps;
    tiles += g->hg.ntiles;
  }
  if (tiles > SX_NOALLOC_MAX_TILES)
    return fail(ctx, SX_EINVAL, "%lld tiles exceed the no-allocation limit of %d",
                (long long)tiles, SX_NOALLOC_MAX_TILES);
  if (n_sweeps == 0 || n == 0) return SX_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, sx::launch_set_remaining(ctx->table, slots, vals, n, 1, ctx->stream));
  // one launch per precision and transport class present, grids in the
  // caller's order and tiles in each grid's order, as a plan of sx_step lays
  // them out; the tables are written into the scratch array by a kernel
  sx::SweepLaunch ls[4];
  int nl = 0;
  int32_t map_first = 0;
  sx::NoAllocList L;
  for (int cls = 0; cls < 4; ++cls) {
    const int prec = cls & 1 ? SX_FP32_TRANSPORT : SX_FP64;
    const int tr = cls >> 1;
    L.n = 0;
    L.first[0] = 0;
    int64_t plane_bytes = 0;
    for (int32_t i = 0; i < n; ++i) {
      const Grid *g = gs[i];
      if (g->hg.precision != prec || g->hg.transport != tr) continue;
      L.slot[L.n] = g->slot;
      L.first[L.n + 1] = L.first[L.n] + g->hg.ntiles;
      ++L.n;
      plane_bytes += 2 * (int64_t)sx::kBlockBytes * g->hg.kb * (g->hg.npad + sx::kTile);
    }
    if (L.n == 0) continue;
    L.cls = cls;
    L.map_first = map_first;
    L.clear_done = nl == 0 ? 1 : 0;
    HIP_TRY(ctx, sx::launch_noalloc_tables(ctx->scratch, L, ctx->stream));
    sx::SweepLaunch &l = ls[nl++];
    l = sx::SweepLaunch{};
    l.grids = ctx->table;
    l.map = (const int2 *)(ctx->scratch + sx::kNoAllocMapOffset) + map_first;
    l.n_tiles = L.first[L.n];
    l.adv = (const int32_t *)(ctx->scratch + sx::kNoAllocAdvOffset) +
            (int64_t)cls * SX_NOALLOC_MAX_GRIDS;
    l.n_adv = L.n;
    l.done = (uint32_t *)ctx->scratch;
    l.xcd_remap = ctx->dflt.xcd_contiguous;
    l.split = tr ? 1 : split_of(ctx->dflt);
    l.tpb = tr ? 1 : ctx->dflt.tiles_per_group * l.split;
    l.precision = prec;
    l.transport = tr;
    l.nt = plane_bytes <= sx::kLlcBytes;
    map_first += L.first[L.n];
  }
  for (int32_t s = 0; s < n_sweeps; ++s)
    for (int i = 0; i < nl; ++i) HIP_TRY(ctx, sx::launch_sweep(ls[i], ctx->stream));
  return SX_OK;
}

int sx_solve(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, const int32_t *n_sweeps) {
  int r = sx::solve_launch(ctx, ids, n, n_sweeps);
  if (r) return r;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipGetLastError());
  return SX_OK;
}

}  // extern "C"

int sx::solve_launch(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, const int32_t *n_sweeps) {
  if (!ctx) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  std::vector<Grid *> gs;
  int r = collect(ctx, ids, n, gs);
  if (r) return r;
  if (gs.empty()) return SX_OK;
  if (!n_sweeps) return fail(ctx, SX_EINVAL, "n_sweeps is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  int32_t mx = 0;
  std::vector<int32_t> slots, vals;
  for (int32_t i = 0; i < n; ++i) {
    if (n_sweeps[i] < 0) return fail(ctx, SX_EINVAL, "n_sweeps[%d] < 0", i);
    mx = std::max(mx, n_sweeps[i]);
    slots.push_back(gs[(size_t)i]->slot);
    vals.push_back(n_sweeps[i]);
  }
  HIP_TRY(ctx, sx::launch_set_remaining(ctx->table, slots.data(), vals.data(), n, 0,
                                        ctx->stream));
  return launch_steps(ctx, gs, mx);
}

void sx::set_io_stream(sx_ctx *ctx, bool on) { ctx->io_on = on; }

int sx::wait_sweeps(sx_ctx *ctx) {
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipGetLastError());
  return SX_OK;
}

extern "C" {

int sx_profile(sx_ctx *ctx, int32_t enable) {
  if (!ctx) return SX_EINVAL;
  ctx->prof = enable != 0;
  return SX_OK;
}

int sx_profile_read(sx_ctx *ctx, int64_t *launches, double *total_ms, double *min_ms,
                    double *max_ms) {
  if (!ctx) return SX_EINVAL;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double tot = 0.0, mn = 0.0, mx = 0.0;
  int64_t nl = 0;
  for (size_t i = 0; i < ctx->ev_used; ++i) {
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev[i].a, ctx->ev[i].b));
    const int32_t k = std::max(ctx->ev[i].launches, 1);
    const double per = (double)ms / k;
    tot += ms;
    nl += k;
    mn = i == 0 ? per : std::min(mn, per);
    mx = std::max(mx, per);
  }
  if (launches) *launches = nl;
  if (total_ms) *total_ms = tot;
  if (min_ms) *min_ms = mn;
  if (max_ms) *max_ms = mx;
  ctx->ev_used = 0;
  return SX_OK;
}

int sx_set_schedule(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, const sx_schedule *s) {
  if (!ctx) return SX_EINVAL;
  if (!s || !valid_schedule(*s)) return fail(ctx, SX_EINVAL, "invalid schedule");
  if (n == 0) {
    ctx->dflt = *s;
    // plans that follow the default are rebuilt on their next step
    (void)hipStreamSynchronize(ctx->stream);
    for (Plan *p : ctx->plans)
      if (!p->fixed) {
        plan_unbuild(p);
        p->sched = *s;
      }
    return SX_OK;
  }
  std::vector<Grid *> gs;
  int r = collect(ctx, ids, n, gs);
  if (r) return r;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  Plan *p = get_plan(ctx, gs);
  plan_unbuild(p);
  p->sched = *s;
  p->fixed = true;
  p->tuned_us = 0.0;
  return SX_OK;
}

int sx_get_schedule(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, sx_schedule *out,
                    double *us_per_sweep) {
  if (!ctx || !out) return SX_EINVAL;
  *out = ctx->dflt;
  if (us_per_sweep) *us_per_sweep = 0.0;
  if (n == 0) return SX_OK;
  std::vector<Grid *> gs;
  int r = collect(ctx, ids, n, gs);
  if (r) return r;
  std::vector<int32_t> key;
  for (Grid *g : gs) key.push_back(g->slot);
  for (Plan *p : ctx->plans)
    if (p->key == key) {
      *out = p->sched;
      if (us_per_sweep) *us_per_sweep = p->tuned_us;
    }
  return SX_OK;
}

int sx_autotune(sx_ctx *ctx, int32_t trials) {
  if (!ctx) return SX_EINVAL;
  if (trials < 0 || trials > 64) return fail(ctx, SX_EINVAL, "trials must be in [0, 64]");
  ctx->autotune = trials;
  return SX_OK;
}

int sx_sync(sx_ctx *ctx) {
  if (!ctx) return SX_EINVAL;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return SX_OK;
}

int sx_read_state(sx_ctx *ctx, sx_grid_id id, const sx_state_out *out) {
  if (!ctx || !out) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = wstream(ctx);
  const GridDev &h = g->hg;
  const int64_t n = h.n, npad = h.npad, K = h.k;
  GridDev cur;
  HIP_TRY(ctx, hipMemcpyAsync(&cur, ctx->table + g->slot, sizeof cur,
                              hipMemcpyDeviceToHost, st));
  std::vector<double> buf;
  if (out->x || out->y) {
    buf.resize((size_t)npad);
    HIP_TRY(ctx, hipMemcpyAsync(buf.data(), h.y, 8 * npad, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) {
      const double yv = buf[(size_t)g->inv[(size_t)i]];
      if (out->y) out->y[i] = yv;
      if (out->x) out->x[i] = 1.0 - yv;
    }
  }
  if (out->nin) {
    buf.resize((size_t)npad);
    HIP_TRY(ctx, hipMemcpyAsync(buf.data(), h.nin, 8 * npad, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) out->nin[i] = buf[(size_t)g->inv[(size_t)i]];
  }
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (out->photons) {
    // O = Ipre * T in the stored precision, as the next step would form it
    const int64_t words = (h.ntiles + 1) * (int64_t)h.kb * sx::kTile * h.bb;
    auto at = [&](int64_t v, int64_t k) {
      const int64_t p = h.bpos[k];
      return (((v >> 6) * h.kb + p / h.bb) * sx::kTile + (v & 63)) * h.bb + p % h.bb;
    };
    const void *src = h.o[cur.parity];
    const void *tsrc = h.t[cur.parity];
    const int64_t pl = h.plane;
    // combined transport: vertices holding edges have no photons in bins
    std::vector<uint8_t> lay;
    if (h.transport != SX_TRANSPORT_DCT) {
      lay.resize((size_t)npad);
      HIP_TRY(ctx, hipMemcpyAsync(lay.data(), h.lay[cur.parity], npad, hipMemcpyDeviceToHost, st));
    }
    auto held = [&](int64_t v) { return lay.empty() || lay[(size_t)v] == 0; };
    if (h.precision == SX_FP64) {
      std::vector<double> o((size_t)words), t((size_t)pl);
      HIP_TRY(ctx, hipMemcpyAsync(o.data(), src, 8 * words, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipMemcpyAsync(t.data(), tsrc, 8 * pl, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipStreamSynchronize(st));
      for (int64_t i = 0; i < n; ++i) {
        const int64_t v = g->inv[(size_t)i];
        for (int64_t k = 0; k < K; ++k)
          out->photons[i * K + k] = held(v) ? (o[(size_t)at(v, k)] * t[(size_t)v]) * h.unit : 0.0;
      }
    } else {
      std::vector<float> o((size_t)words), t((size_t)pl);
      HIP_TRY(ctx, hipMemcpyAsync(o.data(), src, 4 * words, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipMemcpyAsync(t.data(), tsrc, 4 * pl, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipStreamSynchronize(st));
      for (int64_t i = 0; i < n; ++i) {
        const int64_t v = g->inv[(size_t)i];
        for (int64_t k = 0; k < K; ++k) {
          const float ov = o[(size_t)at(v, k)] * t[(size_t)v];
          out->photons[i * K + k] = held(v) ? (double)ov * h.unit : 0.0;
        }
      }
    }
  }
  if (out->tally) {
    std::vector<double> t((size_t)(3 * h.ntiles));
    HIP_TRY(ctx, hipMemcpyAsync(t.data(), h.tally, 8 * 3 * h.ntiles, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    double a = 0, e = 0, f = 0;
    for (int64_t q = 0; q < h.ntiles; ++q) {
      a += t[(size_t)(3 * q)];
      e += t[(size_t)(3 * q + 1)];
      f += t[(size_t)(3 * q + 2)];
    }
    const double sw = (double)cur.sweeps;
    const double since = sw - g->base_sweeps;
    out->tally->sweeps = sw;
    double made = 0.0;
    if (h.diffuse) {
      std::vector<double> dt((size_t)h.ntiles);
      HIP_TRY(ctx, hipMemcpyAsync(dt.data(), h.dtally, 8 * h.ntiles, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipStreamSynchronize(st));
      for (double v : dt) made += v;
    }
    out->tally->emitted = g->base_emitted + since * g->e_sweep + made * h.unit;
    out->tally->absorbed = a * h.unit;
    out->tally->escaped = g->base_escaped + e * h.unit + since * g->esc_emit;
    out->tally->in_flight = f * h.unit;
  }
  return SX_OK;
}

int sx_grid_restore(sx_ctx *ctx, sx_grid_id id, const sx_state_in *in) {
  if (!ctx || !in) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  HIP_TRY(ctx, hipStreamSynchronize(st));
  GridDev &h = g->hg;
  const int64_t n = h.n, npad = h.npad, K = h.k;
  GridDev cur;
  HIP_TRY(ctx, hipMemcpy(&cur, ctx->table + g->slot, sizeof cur, hipMemcpyDeviceToHost));
  if (h.hops > 1) {
    const double sw = in->tally ? in->tally->sweeps : (double)cur.sweeps;
    if (!(sw >= 0.0) || std::fmod(sw, (double)h.hops) != 0.0)
      return fail(ctx, SX_EINVAL, "a multi-hop grid restores at the start of a step "
                                  "(steps done a multiple of %d)", h.hops);
    // nothing absorbed yet in the step that starts
    HIP_TRY(ctx, hipMemset(h.habs, 0, 8 * npad));
    HIP_TRY(ctx, hipMemset(h.hnin, 0, 8 * npad));
  }
  if (in->y) {
    std::vector<double> y((size_t)npad, 1.0);
    for (int64_t i = 0; i < n; ++i) {
      if (!(in->y[i] >= 0.0 && in->y[i] <= 1.0))
        return fail(ctx, SX_EINVAL, "restored y[%lld] outside [0,1]", (long long)i);
      y[(size_t)g->inv[(size_t)i]] = in->y[i];
    }
    HIP_TRY(ctx, hipMemcpy(h.y, y.data(), 8 * npad, hipMemcpyHostToDevice));
  }
  if (in->photons) {
    for (int64_t q = 0; q < n * K; ++q)
      if (!(in->photons[q] >= 0.0) || !std::isfinite(in->photons[q]))
        return fail(ctx, SX_EINVAL, "restored photons must be finite and >= 0");
    // the restored field is the outgoing share itself: Ipre = O, T = 1
    const int64_t words = (h.ntiles + 1) * (int64_t)h.kb * sx::kTile * h.bb;
    auto at = [&](int64_t v, int64_t k) {
      const int64_t p = h.bpos[k];
      return (((v >> 6) * h.kb + p / h.bb) * sx::kTile + (v & 63)) * h.bb + p % h.bb;
    };
    void *dst = h.o[cur.parity];
    void *tdst = h.t[cur.parity];
    const int64_t pl = h.plane;
    if (h.precision == SX_FP64) {
      std::vector<double> o((size_t)words, 0.0), t((size_t)pl, 1.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < K; ++k)
          o[(size_t)at(g->inv[(size_t)i], k)] = in->photons[i * K + k] / h.unit;
      HIP_TRY(ctx, hipMemcpy(dst, o.data(), 8 * words, hipMemcpyHostToDevice));
      HIP_TRY(ctx, hipMemcpy(tdst, t.data(), 8 * pl, hipMemcpyHostToDevice));
    } else {
      std::vector<float> o((size_t)words, 0.0f), t((size_t)pl, 1.0f);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < K; ++k)
          o[(size_t)at(g->inv[(size_t)i], k)] = (float)(in->photons[i * K + k] / h.unit);
      HIP_TRY(ctx, hipMemcpy(dst, o.data(), 4 * words, hipMemcpyHostToDevice));
      HIP_TRY(ctx, hipMemcpy(tdst, t.data(), 4 * pl, hipMemcpyHostToDevice));
    }
    if (h.transport != SX_TRANSPORT_DCT) {
      HIP_TRY(ctx, hipMemset(h.lay[cur.parity], 0, npad));
      HIP_TRY(ctx, hipMemset(h.oe[cur.parity], 0, (size_t)(h.precision == SX_FP64 ? 8 : 4) * h.n_edges));
    }
  }
  if (in->tally) {
    std::vector<double> t((size_t)(3 * h.ntiles), 0.0);
    t[0] = in->tally->absorbed / h.unit;
    t[2] = in->tally->in_flight / h.unit;
    HIP_TRY(ctx, hipMemcpy(h.tally, t.data(), 8 * 3 * h.ntiles, hipMemcpyHostToDevice));
    g->base_sweeps = in->tally->sweeps;
    g->base_emitted = in->tally->emitted;
    g->base_escaped = in->tally->escaped;
    if (h.diffuse) {
      HIP_TRY(ctx, hipMemset(h.dtally, 0, 8 * h.ntiles));
      HIP_TRY(ctx, hipMemset(h.dsh[cur.parity], 0, (size_t)(h.precision == SX_FP64 ? 8 : 4) * h.plane));
    }
    cur.sweeps = (int64_t)in->tally->sweeps;
    HIP_TRY(ctx, hipMemcpy(&ctx->table[g->slot].sweeps, &cur.sweeps, sizeof(int64_t),
                           hipMemcpyHostToDevice));
  }
  return SX_OK;
}

int sx_read_tables(sx_ctx *ctx, sx_grid_id id, int32_t *sel_nbr, int32_t *sel_m,
                   int32_t *edge_bin, double *dL, double *tau) {
  if (!ctx) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const GridDev &h = g->hg;
  const int64_t n = h.n, K = h.k, E = h.n_edges;
  if (edge_bin && g->ebin_stale) {
    HIP_TRY(ctx, sx::launch_edge_bins(ctx->table + g->slot, h, st));
    g->ebin_stale = false;
  }
  if (sel_nbr || sel_m) {
    std::vector<uint32_t> f((size_t)(h.npad * K));
    HIP_TRY(ctx, hipMemcpyAsync(f.data(), h.fwd, 4 * h.npad * K, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) {
      const int64_t v = g->inv[(size_t)i];
      const int32_t rb = g->row_ptr_h[(size_t)v];
      for (int64_t k = 0; k < K; ++k) {
        const uint32_t w = f[(size_t)(v * K + k)];
        const int32_t m = (int32_t)((w >> 21) & 3u);
        if (sel_m) sel_m[i * K + k] = m;
        if (sel_nbr)
          for (int q = 0; q < 3; ++q) {
            const uint32_t s = (w >> (7 * q)) & 127u;
            sel_nbr[(i * K + k) * 3 + q] =
                (q < m) ? g->perm[(size_t)g->nbr_h[(size_t)(rb + (int32_t)s)]] : -1;
          }
      }
    }
  }
  if (edge_bin && E > 0) {
    std::vector<uint8_t> eb((size_t)E);
    HIP_TRY(ctx, hipMemcpyAsync(eb.data(), h.ebin, E, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int64_t p = 0; p < E; ++p) edge_bin[p] = eb[(size_t)g->orig_to_new_e[(size_t)p]];
  }
  if (dL || tau)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t v = g->inv[(size_t)i];
      if (dL) dL[i] = g->dL_h[(size_t)v];
      if (tau) tau[i] = g->tau_h[(size_t)v];
    }
  return SX_OK;
}

int sx_read_edge_state(sx_ctx *ctx, sx_grid_id id, double *photons_e, uint8_t *layout) {
  Grid *g = nullptr;
  int r = combined_grid(ctx, id, &g);
  if (r) return r;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const GridDev &h = g->hg;
  const int64_t n = h.n, npad = h.npad, E = h.n_edges;
  GridDev cur;
  HIP_TRY(ctx, hipMemcpyAsync(&cur, ctx->table + g->slot, sizeof cur, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  std::vector<uint8_t> lay((size_t)npad);
  HIP_TRY(ctx, hipMemcpyAsync(lay.data(), h.lay[cur.parity], npad, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (layout)
    for (int64_t i = 0; i < n; ++i) layout[i] = lay[(size_t)g->inv[(size_t)i]];
  if (photons_e && E > 0) {
    // O_e = Ipre_e * T of the holder, in the stored precision
    const std::vector<int32_t> to_orig = new_to_orig_edges(g);
    const std::vector<int32_t> &rp = g->row_ptr_h;
    if (h.precision == SX_FP64) {
      std::vector<double> o((size_t)E), t((size_t)h.plane);
      HIP_TRY(ctx, hipMemcpyAsync(o.data(), h.oe[cur.parity], 8 * E, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipMemcpyAsync(t.data(), h.t[cur.parity], 8 * h.plane, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipStreamSynchronize(st));
      for (int64_t v = 0; v < n; ++v)
        for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e)
          photons_e[to_orig[(size_t)e]] =
              lay[(size_t)v] ? (o[(size_t)e] * t[(size_t)v]) * h.unit : 0.0;
    } else {
      std::vector<float> o((size_t)E), t((size_t)h.plane);
      HIP_TRY(ctx, hipMemcpyAsync(o.data(), h.oe[cur.parity], 4 * E, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipMemcpyAsync(t.data(), h.t[cur.parity], 4 * h.plane, hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipStreamSynchronize(st));
      for (int64_t v = 0; v < n; ++v)
        for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) {
          const float ov = o[(size_t)e] * t[(size_t)v];
          photons_e[to_orig[(size_t)e]] = lay[(size_t)v] ? (double)ov * h.unit : 0.0;
        }
    }
  }
  return SX_OK;
}

int sx_grid_restore_edges(sx_ctx *ctx, sx_grid_id id, const double *photons_e,
                          const uint8_t *layout) {
  Grid *g = nullptr;
  int r = combined_grid(ctx, id, &g);
  if (r) return r;
  if (!layout) return fail(ctx, SX_EINVAL, "layout is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  HIP_TRY(ctx, hipStreamSynchronize(st));
  const GridDev &h = g->hg;
  const int64_t n = h.n, npad = h.npad, E = h.n_edges;
  for (int64_t i = 0; i < n; ++i)
    if (layout[i] > 1) return fail(ctx, SX_EINVAL, "layout[%lld] is not 0 or 1", (long long)i);
  if (photons_e)
    for (int64_t p = 0; p < E; ++p)
      if (!(photons_e[p] >= 0.0) || !std::isfinite(photons_e[p]))
        return fail(ctx, SX_EINVAL, "restored photons must be finite and >= 0");
  GridDev cur;
  HIP_TRY(ctx, hipMemcpy(&cur, ctx->table + g->slot, sizeof cur, hipMemcpyDeviceToHost));
  const int par = cur.parity;
  std::vector<uint8_t> lay((size_t)npad, 0);
  for (int64_t i = 0; i < n; ++i) lay[(size_t)g->inv[(size_t)i]] = layout[i];
  const std::vector<int32_t> to_orig = new_to_orig_edges(g);
  const std::vector<int32_t> &rp = g->row_ptr_h;
  // the restored packets are the outgoing share itself: Ipre_e = O_e and
  // T = 1 for the vertices that hold edges (their bins are not read)
  // vertices that hold edges keep zeros in their bins
  const int64_t words = (h.ntiles + 1) * (int64_t)h.kb * sx::kTile * h.bb;
  auto put = [&](auto zero) -> int {
    using T = decltype(zero);
    std::vector<T> o((size_t)E, zero), t((size_t)h.plane), bins((size_t)words);
    HIP_TRY(ctx, hipMemcpy(t.data(), h.t[par], sizeof(T) * h.plane, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(bins.data(), h.o[par], sizeof(T) * words, hipMemcpyDeviceToHost));
    for (int64_t v = 0; v < n; ++v) {
      if (!lay[(size_t)v]) continue;
      t[(size_t)v] = (T)1;
      for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e)
        o[(size_t)e] = photons_e ? (T)(photons_e[to_orig[(size_t)e]] / h.unit) : zero;
      for (int64_t p = 0; p < h.k; ++p)   // every position of the vertex
        bins[(size_t)((((v >> 6) * h.kb + p / h.bb) * sx::kTile + (v & 63)) * h.bb + p % h.bb)] = zero;
    }
    HIP_TRY(ctx, hipMemcpy(h.oe[par], o.data(), sizeof(T) * E, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(h.t[par], t.data(), sizeof(T) * h.plane, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(h.o[par], bins.data(), sizeof(T) * words, hipMemcpyHostToDevice));
    return SX_OK;
  };
  r = h.precision == SX_FP64 ? put(0.0) : put(0.0f);
  if (r) return r;
  HIP_TRY(ctx, hipMemcpy(h.lay[par], lay.data(), npad, hipMemcpyHostToDevice));
  return SX_OK;
}

int sx_read_diffuse(sx_ctx *ctx, sx_grid_id id, double *pending) {
  if (!ctx || !pending) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  const GridDev &h = g->hg;
  const int64_t n = h.n;
  if (!h.diffuse) {
    for (int64_t i = 0; i < n; ++i) pending[i] = 0.0;
    return SX_OK;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  GridDev cur;
  HIP_TRY(ctx, hipMemcpyAsync(&cur, ctx->table + g->slot, sizeof cur, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  const std::vector<int32_t> &rp = g->row_ptr_h;
  auto get = [&](auto zero) -> int {
    using T = decltype(zero);
    std::vector<T> d((size_t)h.plane);
    HIP_TRY(ctx, hipMemcpyAsync(d.data(), h.dsh[cur.parity], sizeof(T) * h.plane,
                                hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) {
      const int64_t v = g->inv[(size_t)i];
      const int deg = rp[(size_t)v + 1] - rp[(size_t)v];
      pending[i] = (double)d[(size_t)v] * (deg > 0 ? (double)deg : 1.0) * h.unit;
    }
    return SX_OK;
  };
  return h.precision == SX_FP64 ? get(0.0) : get(0.0f);
}

int sx_read_ballistic(sx_ctx *ctx, sx_grid_id id, int32_t *bsel, int32_t *bm) {
  Grid *g = nullptr;
  int r = combined_grid(ctx, id, &g);
  if (r) return r;
  const int64_t E = g->hg.n_edges;
  for (int64_t p = 0; p < E; ++p) {
    const int32_t e = g->orig_to_new_e[(size_t)p];
    const int m = g->bm_h[(size_t)e];
    if (bm) bm[p] = m;
    if (bsel)
      for (int q = 0; q < 3; ++q)
        bsel[3 * p + q] = q < m ? g->perm[(size_t)g->nbr_h[(size_t)g->bsel_h[(size_t)(3 * e + q)]]] : -1;
  }
  return SX_OK;
}

int sx_grid_select_removal(sx_ctx *ctx, sx_grid_id id, double tau_remove,
                           double min_spacing, uint8_t *remove, int64_t *n_removed) {
  if (!ctx || !remove) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  if (std::isnan(tau_remove) || std::isnan(min_spacing))
    return fail(ctx, SX_EINVAL, "tau_remove and min_spacing must not be NaN");
  const GridDev &h = g->hg;
  const int64_t n = h.n;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  std::vector<double> y((size_t)h.npad);
  HIP_TRY(ctx, hipMemcpyAsync(y.data(), h.y, 8 * h.npad, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  // candidates: optically thin, finer than the minimum resolution, no source
  struct Cand {
    double od;
    int32_t orig, v;
  };
  std::vector<Cand> c;
  for (int64_t v = 0; v < n; ++v) {
    const double od = y[(size_t)v] * g->tau_h[(size_t)v];
    const bool src = !g->is_src_h.empty() && g->is_src_h[(size_t)v];
    if (od < tau_remove && g->dL_h[(size_t)v] < min_spacing && !src)
      c.push_back({od, g->perm[(size_t)v], (int32_t)v});
  }
  std::sort(c.begin(), c.end(), [](const Cand &a, const Cand &b) {
    return a.od < b.od || (a.od == b.od && a.orig < b.orig);
  });
  // greedy independent set: no two removed vertices are neighbours
  std::vector<uint8_t> blocked((size_t)n, 0), rm((size_t)n, 0);
  int64_t cnt = 0;
  for (const Cand &q : c) {
    if (blocked[(size_t)q.v]) continue;
    rm[(size_t)q.v] = 1;
    ++cnt;
    for (int32_t e = g->row_ptr_h[(size_t)q.v]; e < g->row_ptr_h[(size_t)q.v + 1]; ++e)
      blocked[(size_t)g->nbr_h[(size_t)e]] = 1;
  }
  for (int64_t i = 0; i < n; ++i) remove[i] = rm[(size_t)g->inv[(size_t)i]];
  if (n_removed) *n_removed = cnt;
  return SX_OK;
}

int sx_grid_remap(sx_ctx *ctx, sx_grid_id from, sx_grid_id to, const int32_t *new_of_old) {
  if (!ctx || !new_of_old) return SX_EINVAL;
  if (ctx->poisoned) return fail(ctx, SX_EDEVICE, "context poisoned: %s", ctx->err.c_str());
  Grid *a = find(ctx, from), *b = find(ctx, to);
  if (!a || !b) return fail(ctx, SX_ENOTFOUND, "grid not found");
  if (a->hg.hops > 1 || b->hg.hops > 1)
    return fail(ctx, SX_ENOTSUP, "remap needs grids of one hop per step");
  if (a->hg.transport != b->hg.transport || a->hg.diffuse != b->hg.diffuse)
    return fail(ctx, SX_EINVAL, "remap needs the same transport and the same recombination "
                                "radiation on both grids");
  const int64_t na = a->hg.n, nb = b->hg.n, K = a->hg.k;
  if (b->hg.k != K || a->bins0 != b->bins0 || a->rotated || b->rotated)
    return fail(ctx, SX_EINVAL, "remap needs the same unrotated bins on both grids");
  std::vector<uint8_t> hit((size_t)nb, 0);
  for (int64_t i = 0; i < na; ++i) {
    const int32_t j = new_of_old[i];
    if (j < -1 || j >= nb) return fail(ctx, SX_EINVAL, "new_of_old[%lld] out of range", (long long)i);
    if (j >= 0) {
      if (hit[(size_t)j]) return fail(ctx, SX_EINVAL, "vertex %d of the new grid mapped twice", j);
      hit[(size_t)j] = 1;
    }
  }
  for (int64_t j = 0; j < nb; ++j)
    if (!hit[(size_t)j]) return fail(ctx, SX_EINVAL, "vertex %lld of the new grid has no old vertex", (long long)j);
  const bool comb = a->hg.transport != SX_TRANSPORT_DCT;
  std::vector<double> ya((size_t)na), oa((size_t)(na * K));
  std::vector<int32_t> ma((size_t)(na * K)), mb((size_t)(nb * K));
  sx_tally t{};
  sx_state_out so{nullptr, ya.data(), oa.data(), nullptr, &t};
  int r = sx_read_state(ctx, from, &so);
  if (!r) r = sx_read_tables(ctx, from, nullptr, ma.data(), nullptr, nullptr, nullptr);
  if (!r) r = sx_read_tables(ctx, to, nullptr, mb.data(), nullptr, nullptr, nullptr);
  if (r) return r;
  // combined transport: a vertex that holds edges holds bm O_e for the packet
  // that came along i -> j, filed here in the bin of that edge (the bin a
  // direction-conserving vertex files it in, Sect. 2.2.4); the thinned grid
  // starts with every vertex holding bins
  std::vector<double> extra;
  if (comb) {
    const int64_t E = a->hg.n_edges;
    std::vector<double> pe((size_t)E);
    std::vector<uint8_t> lay((size_t)na);
    std::vector<int32_t> eb((size_t)E), bm((size_t)E);
    r = sx_read_edge_state(ctx, from, pe.data(), lay.data());
    if (!r) r = sx_read_ballistic(ctx, from, nullptr, bm.data());
    if (!r) r = sx_read_tables(ctx, from, nullptr, nullptr, eb.data(), nullptr, nullptr);
    if (r) return r;
    const std::vector<int32_t> n2o = new_to_orig_edges(a);
    const std::vector<int32_t> &rp = a->row_ptr_h, &nbr = a->nbr_h;
    extra.assign((size_t)(na * K), 0.0);
    for (int64_t i = 0; i < na; ++i) {
      if (!lay[(size_t)i]) continue;
      const int32_t v = (int32_t)a->inv[(size_t)i];
      for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) {
        const int32_t u = nbr[(size_t)e];
        int32_t back = -1;   // the edge u -> v in u's row
        for (int32_t f = rp[(size_t)u]; f < rp[(size_t)u + 1]; ++f)
          if (nbr[(size_t)f] == v) { back = f; break; }
        if (back < 0) return fail(ctx, SX_EDEVICE, "neighbour rows are not symmetric");
        const int32_t p = n2o[(size_t)e];
        extra[(size_t)(i * K + eb[(size_t)n2o[(size_t)back]])] += pe[(size_t)p] * (double)bm[(size_t)p];
      }
    }
  }
  // where each old vertex's holdings go: the vertex it maps to, or for a
  // removed one its nearest kept former neighbour (ties: lower id); -1 none
  std::vector<int32_t> dest((size_t)na);
  for (int64_t i = 0; i < na; ++i) {
    int32_t j = new_of_old[i];
    if (j < 0) {
      const int64_t v = a->inv[(size_t)i];
      double best = 0.0;
      int32_t bo = -1;
      for (int32_t e = a->row_ptr_h[(size_t)v]; e < a->row_ptr_h[(size_t)v + 1]; ++e) {
        const int32_t o = a->perm[(size_t)a->nbr_h[(size_t)e]];
        if (new_of_old[o] < 0) continue;
        const double len = a->elen_h[(size_t)e];
        if (bo < 0 || len < best || (len == best && o < bo)) { best = len; bo = o; }
      }
      j = bo >= 0 ? new_of_old[bo] : -1;
    }
    dest[(size_t)i] = j;
  }
  // m O per bin moves to dest in the same bin, added in ascending old id
  std::vector<double> held((size_t)(nb * K), 0.0), yb((size_t)nb, 1.0);
  double lost = 0.0;
  for (int64_t i = 0; i < na; ++i) {
    const int32_t j = dest[(size_t)i];
    if (new_of_old[i] >= 0) yb[(size_t)j] = ya[(size_t)i];
    for (int64_t k = 0; k < K; ++k) {
      double hk = oa[(size_t)(i * K + k)] * (double)ma[(size_t)(i * K + k)];
      if (comb) hk = hk + extra[(size_t)(i * K + k)];
      if (j >= 0) held[(size_t)(j * K + k)] += hk;
      else lost += hk;
    }
  }
  std::vector<double> ob((size_t)(nb * K), 0.0);
  double fly = 0.0;
  for (int64_t q = 0; q < nb * K; ++q) {
    const int32_t m = mb[(size_t)q];
    if (m > 0) {
      ob[(size_t)q] = held[(size_t)q] / (double)m;
      fly += held[(size_t)q];
    } else {
      lost += held[(size_t)q];
    }
  }
  // diffuse recombination photons still to be sent move the same way
  std::vector<double> pb;
  if (a->hg.diffuse) {
    std::vector<double> pa((size_t)na);
    r = sx_read_diffuse(ctx, from, pa.data());
    if (r) return r;
    pb.assign((size_t)nb, 0.0);
    for (int64_t i = 0; i < na; ++i) {
      const int32_t j = dest[(size_t)i];
      if (j >= 0) pb[(size_t)j] += pa[(size_t)i];
      else lost += pa[(size_t)i];
    }
    for (int64_t j = 0; j < nb; ++j) fly += pb[(size_t)j];
  }
  sx_tally tb = t;
  tb.escaped = t.escaped + lost;
  tb.in_flight = fly;
  sx_state_in si{yb.data(), ob.data(), &tb};
  r = sx_grid_restore(ctx, to, &si);
  if (r || pb.empty()) return r;
  // the pending photons go in as each vertex's share per neighbour
  const GridDev &h = b->hg;
  GridDev cur;
  HIP_TRY(ctx, hipMemcpy(&cur, ctx->table + b->slot, sizeof cur, hipMemcpyDeviceToHost));
  auto put = [&](auto zero) -> int {
    using T = decltype(zero);
    std::vector<T> d((size_t)h.plane, zero);
    for (int64_t j = 0; j < nb; ++j) {
      const int64_t v = b->inv[(size_t)j];
      const int deg = b->row_ptr_h[(size_t)v + 1] - b->row_ptr_h[(size_t)v];
      d[(size_t)v] = (T)(pb[(size_t)j] / (deg > 0 ? (double)deg : 1.0) / h.unit);
    }
    HIP_TRY(ctx, hipMemcpy(h.dsh[cur.parity], d.data(), sizeof(T) * h.plane, hipMemcpyHostToDevice));
    return SX_OK;
  };
  return h.precision == SX_FP64 ? put(0.0) : put(0.0f);
}

int sx_grid_info(sx_ctx *ctx, sx_grid_id id, int64_t *n, int32_t *k, int64_t *n_edges,
                 int32_t *precision, double *photon_unit, uint64_t *bytes) {
  if (!ctx) return SX_EINVAL;
  Grid *g = find(ctx, id);
  if (!g) return fail(ctx, SX_ENOTFOUND, "grid %lld not found", (long long)id);
  if (n) *n = g->hg.n;
  if (k) *k = g->hg.k;
  if (n_edges) *n_edges = g->hg.n_edges;
  if (precision) *precision = g->hg.precision;
  if (photon_unit) *photon_unit = g->hg.unit;
  if (bytes) *bytes = g->bytes;
  return SX_OK;
}

}  // extern "C"
