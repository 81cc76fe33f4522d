// sx_internal.h -- device-side grid description shared by the host code and
// the HIP kernels of libsx.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sx.h"

namespace sx {

constexpr int kTile = 64;           // vertices per tile = one wavefront
constexpr int kEmptySlot = 127;     // unused slot marker in packed tables

constexpr int kStageQ = 5;         // halo staging loads per lane and block
constexpr int kHaloMax = 64 * kStageQ;   // halo vertices a staged tile may have;
                                         // LDS entry kHaloMax reads 0

// Halo of a tile: the sorted list of every vertex that neighbours one of
// the tile's 64 vertices.  A block of bins of the halo is staged in LDS once
// per wave; the gathers find a sender there through its 9-bit halo index.  A
// tile whose halo exceeds kHaloMax vertices is "direct": its gathers go to
// global memory through the receiver's neighbour row.
//
// Bins are stored in an order of the library's own: the grid's bins are
// grouped into blocks of BB bins that point in nearby directions (bperm /
// bpos below), so the neighbours that send a block's bins to one vertex are
// few and mostly the same for all of them.  Every kernel that stores or
// reads photons per bin goes through that order; the caller's bin numbers
// are kept everywhere else (selection, edge bins, source shares).
//
// In-word of a (vertex j, block of BB bins) (uint64): which neighbours send
// which of the block's bins to j.  Entry e (bits EB e .. EB e + EB - 1,
// EB = 5 + BB) holds in its low 5 bits the slot of the sender in j's row
// and in the next BB bits the bins of the block it sends; entries are in
// ascending slot (= ascending original sender id), unused entries are 0 (no
// bins).  A word holds 63 / EB entries (7 with 4 bins, 9 with 2).  Bit 63
// is set when the pair also has records (below).  Only slots below
// kSlotRows go into entries; a staged tile finds the halo index of a slot in
// a per-wave LDS table.
// Records (uint32, grouped by (tile, bin position), sorted by position then
// lane) carry what does not fit: senders beyond the in-word's entries (or at
// a slot >= kSlotRows), one record per bin sent, then the vertex's shares of
// source emission for the bin.  Record = lane << 26 | (position mod BB) <<
// 24 | kind << 23 | index; kind 0 = sender (halo index, or row slot in a
// direct tile), kind 1 = emission amount index.
//
// Photon field layout: 16-byte blocks of BB = 16 / sizeof(photon) bins per
// vertex (4 fp32 or 2 fp64), element (v, bin at position p) at block
// ((v / 64) * KB + p / BB) * 64 + v % 64, component p % BB, KB =
// ceil(K/BB).  One extra tile past the last holds zeros.  In-words: one
// per (vertex, block), in the same block order.
constexpr int kSlotRows = 30;      // row slots an in-word entry can name
__host__ __device__ constexpr int inw_entry_bits(int bb) { return 5 + bb; }
__host__ __device__ constexpr int inw_entries(int bb) { return 63 / (5 + bb); }
constexpr int kBlockBytes = 16;
// Record counts and offsets per (tile, bin, group of kRecGroupLanes lanes).
constexpr int kRecGroups = 8;
// The last-level cache (Infinity Cache) of the GPU.  When the photon planes
// of all grids in one sweep launch fit in it, the sweep loads its in-words
// non-temporal, so that the planes stay cached from one sweep to the next;
// on larger launches the hint costs time and is not used.
constexpr int64_t kLlcBytes = 256ll << 20;
constexpr int kRecGroupLanes = kTile / kRecGroups;
constexpr int kRecIdxBits = 23;
// Forward word of a (vertex, bin) pair (selection result):
//   bits 0..20 : three 7-bit slots, best first (127 = none)
//   bits 21..22: m, the number selected

// Everything a kernel needs to know about one grid.  Lives in device memory
// (an array of these for a batch); kernels read it through scalar loads.
struct GridDev {
  int32_t n;          // vertices
  int32_t npad;       // vertices rounded up to kTile
  int32_t ntiles;     // npad / kTile
  int32_t k;          // bins
  int32_t kw;         // ceil(k / 16): words of packed m per lane and tile
  int32_t bb;         // bins per 16-byte block (4 fp32, 2 fp64)
  int32_t kb;         // blocks per vertex, ceil(k / bb)
  int32_t n_sub;      // chemistry substeps
  int32_t mpb;        // max neighbours per bin
  int32_t max_deg;    // largest degree of the grid (sizes the selection's LDS)
  int32_t precision;  // 0 fp64, 1 fp32 transport
  int32_t inw_cap;    // in-word entries the gather-list build fills (<= inw_entries(bb);
                      // fewer only to exercise the record path)
  uint8_t bperm[128]; // bin stored at position p (caller's numbering)
  uint8_t bpos[128];  // position of bin k
  // mutable per-sweep control, advanced by the last workgroup of each sweep launch
  int32_t parity;     // O buffer holding the current field
  int32_t remaining;  // steps still to run in the current request
  int64_t sweeps;     // steps done
  double unit;        // photons per stored unit (power of two)
  double dt;
  double cos_min;
  int64_t plane;      // entries of the per-vertex arrays t[] (npad + a zero tile)
  int64_t n_edges;
  // graph (reordered)
  const int32_t *row_ptr;   // [npad+1]
  const int32_t *nbr;       // [E] new ids, each row sorted by original id
  const uint8_t *rev;       // [E] slot of the row's vertex in the neighbour's row
  const double *edir;       // [3E] unit edge vectors
  const double *bins;       // [3K]
  // selection products
  uint32_t *fwd;            // [npad*K]
  uint8_t *ebin;            // [E]
  uint64_t *inw;            // [ntiles][kb][64]
  uint32_t *mbits;          // [ntiles][kw][64]
  uint32_t *mbits2;         // [ntiles][kw][64] scratch: the new m words of a re-binning
  int32_t *rec_cnt;         // [ntiles*K*kRecGroups+1] scratch: records per (tile, bin, group)
  uint8_t *rec_lane;        // [ntiles*K*64] scratch: records per (tile, bin, receiver lane),
                            // 255 standing for 255 or more
  int32_t *rec_ptr;         // [ntiles*K*kRecGroups+1] first record of each
  int64_t *scan_part;       // [ntiles*K*kRecGroups/1024 + 2] scratch of the record scan
  int32_t *erev;            // [E+1] the edge of nbr[e]'s row that points back at e's row
  uint32_t *smask;          // [4*(E+1)] written by the selection: bit p % 32 of word
                            // (p / 32) (E + 1) + e is set iff the bin at storage
                            // position p of sender nbr[e] selects j (four planes)
  uint32_t *rec;            // [n_rec]
  int64_t rec_cap;
  const int32_t *halo_ptr;  // [ntiles+1]
  const int32_t *halo_vid;  // [halo total] ascending new vertex ids
  const uint16_t *edge_hidx;// [E] halo index of each edge's target (or slot)
  const uint8_t *tile_direct; // [ntiles]
  // sources (per receiving vertex, by bin, then source order)
  const int32_t *em_ptr;    // [npad+1]
  int32_t *em_k;            // [n_em] bin of each share (from its edge)
  const int32_t *em_edge;   // [n_em] the source's edge the share travels along
  const double *em_amt;     // [n_em] photons / unit
  const int32_t *em_beam;   // [n_em] source of a beam share (filed in the bin
                            // closest to the beam), -1 isotropic; null: no beams
  const double *beam_dir;   // [3 n_src] source directions (null: no beams)
  // chemistry coefficients
  const double *tau;        // [npad] n_H sigma dL
  const double *dtnhv;      // [npad] dt * n_H * V
  const double *bcoef;      // [npad] alpha_B * n_H
  double *y;                // [npad] neutral fraction
  double *nin;              // [npad] photons in, last step
  void *o[2];               // [(ntiles+1)*kb*64] blocks: photons per selected
                            // neighbour before attenuation, I/m, double buffered
  void *t[2];               // [plane] transmitted fraction T of each vertex
                            // in the step that wrote o[] (fp32 or fp64)
  double *tally;            // [ntiles*3] absorbed (cum), escaped (cum), in flight
  // combined transport (transport == 1; null otherwise).  Lists are indexed
  // by the incoming edge e = (row of j, slot s), the sender i = nbr[e]:
  int32_t transport;        // 0 direction-conserving, 1 combined
  int32_t dct_ref;          // bin selection w.r.t. 0: the bin, 1: its closest edge
  double tau_switch;        // ballistic where y tau >= tau_switch
  int32_t *kl_ptr;          // [E+1]
  uint8_t *kl;              // bins of i whose selection holds j, as storage
                            // positions, ascending
  int64_t kl_cap;           // entries kl holds
  int32_t *kl_cnt;          // [E+1] scratch: entries per in-edge
  int64_t *kl_part;         // [E/1024 + 2] scratch of their scan
  const int32_t *bl_ptr;    // [E+1]
  const int32_t *bl;        // edges of i (global ids, ascending) whose ballistic
                            // packets go to j
  const int4 *bl4;          // [E] the first four entries of each bl list, -1 padding
  const uint8_t *elane;     // [E] lane (vertex mod 64) of each edge's row
  uint8_t *ebin_in;         // [E] bin of the edge i -> j, for the in-edge (j, slot of i)
  int32_t diffuse;          // recombination photons re-emitted (alpha_A > 0)
  int32_t pad1;
  double dfrac;             // (alpha_A - alpha_B) / alpha_A
  const double *nhv;        // [npad] n_H V
  void *dsh[2];             // [plane] photons / unit each neighbour gets next
                            // step from the vertex's recombinations (the whole
                            // amount for a vertex with no neighbour)
  double *dtally;           // [ntiles] recombination photons made (cum), / unit
  // multi-hop steps (hops > 1; null otherwise): each sweep is one hop, y is
  // updated after the step's last hop (sweeps % hops == hops - 1)
  int32_t hops;
  int32_t pad2;
  double *habs;             // [npad] photons absorbed so far in the step
  double *hnin;             // [npad] photons that arrived so far in the step
  void *xin;                // bin field (layout of o[]): photons from ballistic
                            // senders waiting for their receiver's bin code; zero
                            // between steps
  const uint8_t *bm;        // [E] neighbours chosen for the packet entering j along e
  void *oe[2];              // [E] ballistic photons I/bm per incoming edge (fp32 or fp64)
  uint8_t *lay[2];          // [npad] 1: the vertex held edges in the step that wrote it
};

// Kernel launchers (sx_kernels.hip).  All enqueue on `stream`, return the
// HIP error of the launch.
hipError_t launch_erev(const GridDev *dg, const GridDev &hg, hipStream_t s);
// Selection: forward words, selection masks, and the m words into mout
// (mbits, or mbits2 ahead of a re-binning).
hipError_t launch_select(const GridDev *dg, const GridDev &hg, uint32_t *mout, hipStream_t s);
hipError_t launch_edge_bins(const GridDev *dg, const GridDev &hg, hipStream_t s);
hipError_t launch_inlist_count(const GridDev *dg, const GridDev &hg, hipStream_t s);
hipError_t launch_scan(int32_t *cnt, int32_t *ptr, int64_t *part, int32_t n, hipStream_t s);
hipError_t launch_inlist_fill(const GridDev *dg, const GridDev &hg, hipStream_t s);
// After a rotation of the bins: for every new bin (by storage position), the
// old bins whose photons it takes (the old bins closest in direction to
// it), as storage positions in ascending old bin.
struct RebinMap {
  uint8_t ptr[132];   // by new storage position p: list[ptr[p] .. ptr[p+1])
  uint8_t list[128];  // the old storage positions, in ascending old bin
  uint8_t bin[128];   // the bin at each new position
};
static_assert(SX_MAX_BINS_FP32 < 128 && SX_MAX_BINS_FP64 < 128, "rebin map holds 127 bins");
// The photons each vertex holds move to their new bins (map) and are split
// over the new selection (from fwd; the old m is still in mbits, and is
// replaced); those with no forward neighbour left move to the escape tally.
hipError_t launch_rebin(GridDev *dg, const GridDev &hg, const RebinMap &map, hipStream_t s);
// Bin of each source share from its edge's bin.
hipError_t launch_em_bins(GridDev *dg, const GridDev &hg, int64_t n_em, hipStream_t s);
// Combined transport, from the selection and the edge bins: the bin of each
// in-edge, and per in-edge the sender's bins that hold the receiver (count,
// then fill after a scan of the counts into kl_ptr).
hipError_t launch_ebin_in(const GridDev *dg, const GridDev &hg, hipStream_t s);
hipError_t launch_kl_count(const GridDev *dg, const GridDev &hg, hipStream_t s);
hipError_t launch_kl_fill(const GridDev *dg, const GridDev &hg, hipStream_t s);
hipError_t launch_clear_inw(const GridDev &hg, hipStream_t s);
hipError_t launch_reset_state(GridDev *dg, const GridDev &hg, const double *y0,
                              hipStream_t s);
// One sweep launch: a tile list over grids[] (tile_map null: one grid, tile
// t = t), tpb (1, 2 or 4) waves per workgroup, XCD-contiguous workgroup
// numbering or not, and the grids to advance when the launch completes (adv
// null: grids[0 .. n_adv)).  done: a zeroed device counter that no other
// launch uses concurrently.
struct SweepLaunch {
  GridDev *grids;
  const int2 *map;
  int32_t n_tiles;
  const int32_t *adv;
  int32_t n_adv;
  uint32_t *done;
  int32_t xcd_remap;
  int32_t tpb, precision;   // tpb: waves per workgroup
  int32_t split;            // waves per tile (1, 2, 4; tpb a multiple)
  int32_t transport;
  int32_t nt;   // in-words loaded non-temporal (the photon planes fit kLlcBytes)
};
hipError_t launch_sweep(const SweepLaunch &l, hipStream_t s);
hipError_t add_sweep_node(hipGraph_t graph, const SweepLaunch &l, hipGraphNode_t *prev);
// sx_step_noalloc's device scratch (one file-scope array per device): the
// completion counter at offset 0, per launch class c (< 4) the grids to
// advance at kNoAllocAdvOffset + 4 SX_NOALLOC_MAX_GRIDS c, the tile maps
// from kNoAllocMapOffset (SX_NOALLOC_MAX_TILES int2 shared by the classes).
constexpr int kNoAllocDevices = 64;
constexpr int64_t kNoAllocAdvOffset = 256;
constexpr int64_t kNoAllocMapOffset = 8192;
static_assert(kNoAllocAdvOffset + 4 * 4 * SX_NOALLOC_MAX_GRIDS <= kNoAllocMapOffset,
              "advance lists fit below the tile maps");
// The address of the scratch array on `device` (the current device),
// looked up on the first call for that device and kept.
hipError_t noalloc_scratch_init(int device, void **out);
// Tables of one launch class, by value: grids slot[0..n) (caller order),
// their tiles from first[g] (first[n] = the class's tiles), written at tile
// map entry map_first; clear_done zeroes the completion counter.
struct NoAllocList {
  int32_t n, cls, map_first, clear_done;
  int32_t slot[SX_NOALLOC_MAX_GRIDS];
  int32_t first[SX_NOALLOC_MAX_GRIDS + 1];
};
hipError_t launch_noalloc_tables(uint8_t *base, const NoAllocList &L, hipStream_t s);
hipError_t launch_set_remaining(GridDev *table, const int32_t *slots,
                                const int32_t *values, int32_t n, int32_t add,
                                hipStream_t s);

// For the request loop (sx_serve.cpp), which owns its context:
// sx_solve without the final wait (the sweeps are enqueued on the context
// stream); the wait for them; and the switch that puts the upload, read-back
// and release calls on the context's second stream, so that they overlap
// sweeps of other grids.
int solve_launch(sx_ctx *ctx, const sx_grid_id *ids, int32_t n, const int32_t *n_sweeps);
int wait_sweeps(sx_ctx *ctx);
void set_io_stream(sx_ctx *ctx, bool on);


}  // namespace sx
