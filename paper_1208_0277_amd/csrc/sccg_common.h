// Internal declarations shared by the device library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sccg.h"

namespace sccg {

constexpr int kWave = 64;
constexpr int32_t kMaxSide = 32767;        // largest accepted pair-box side (pixels)
constexpr int32_t kMaxCoord = 1 << 30;     // largest accepted |coordinate|
constexpr int kTile = 64;                  // leaf tile side of the batched path (pixels)
constexpr int kMaxGrid = 8;                // batched split grid is at most 8 x 8 cells

// Device error word bits (latched, reported by sccg_sync).
enum : uint32_t {
  kErrIndex = 1u,     // pair index outside its polygon set
  kErrSide = 2u,      // pair-box side above kMaxSide
  kErrCoord = 4u,     // |coordinate| above kMaxCoord
  kErrWatchdog = 8u,  // a bounded wait in the persistent kernel ran out
};

// Pair classes of the batched path: done in a prepass, swept in index order
// (rings short enough to be held in registers), medium (rings held in
// registers by the second sweep), or heavy (listed for the persistent
// kernel); listed pairs are then marked by their box (small: one leaf tile;
// large: split).
enum : uint8_t { kClsDone = 0, kClsSweep = 1, kClsHeavy = 2, kClsSmall = 3, kClsLarge = 4, kClsMedium = 5 };

struct Polys {
  int64_t n;
  const int64_t* off;
  const int2* xy;
};

// Vertex extent of a polygon: pixels [x0,x1) x [y0,y1).  x0 > x1 marks an
// empty or rejected polygon.
struct Meta {
  int32_t x0, y0, x1, y1;
};

// Number of statistics counters (see sccg_get_stats).
constexpr int kNumStats = 16;

// ------------------------------------------------------------------ launches
// Each returns a hipError_t from the launch.

// Per polygon: vertex extent, |shoelace|/2, coordinate range check.
hipError_t launch_poly_meta(const Polys& P, Meta* meta, int64_t* area, int32_t* big_list, int32_t* big_count,
                            uint32_t* err, hipStream_t s);

struct PlainArgs {
  Polys A, B;
  const Meta* metaA;
  const Meta* metaB;
  const int64_t* areaA;
  const int64_t* areaB;
  int64_t n_pairs;
  const int32_t* pa;
  const int32_t* pb;
  int64_t* inter;
  int64_t* uni;
  uint32_t* err;
  unsigned long long* stats;  // nullable
  int32_t box_threshold;
  int32_t gx, gy;
  int32_t lds_vertex_cap;
};
hipError_t launch_plain(const PlainArgs& a, int wg_size, int grid, hipStream_t s);
int plain_lds_bytes(int wg_size, int lds_vertex_cap);
int plain_occupancy(int wg_size, int lds_vertex_cap);

// A device counter on a cache line of its own, so that claims on different
// counters never contend for one line.
struct alignas(128) Counter {
  unsigned long long v;
  unsigned long long pad[15];
};

// Work is claimed from kStreams interleaved streams (one per XCD): stream s
// owns entries s, s + kStreams, s + 2 kStreams, ... of a list.
constexpr int kStreams = 8;

// Device-side state of the batched path (one block of device memory), reset
// at the start of every call after the slots the previous call touched
// (below max(head, tail) of each queue) are cleared.
// Listed pairs are kept in kLptBuckets lists by vertex count (the cost the
// setup pass can see): at least 4, 2 or 1 times heavy_verts, and the rest;
// the persistent kernel claims the largest bucket first.
constexpr int kLptBuckets = 4;

struct BatchState {
  Counter l_count[kLptBuckets];            // pairs listed per bucket
  Counter l_next[kLptBuckets][kStreams];   // per-stream claim counters over each bucket
  Counter s_next[kStreams];   // per-stream claim counters over pair chunks (the sweep)
  Counter m_count;            // medium pairs listed (by the setup pass and the sweep)
  Counter m_next[kStreams];   // per-stream claim counters over chunks of the medium list
  Counter p_count[kLptBuckets];  // pairs the setup pass listed per bucket (the prepass's share)
  Counter p_next[kStreams];      // per-stream claim counters over the prepass's entries
  Counter q_head[kMaxGrid];   // per-queue ticket counters
  Counter q_tail[kMaxGrid];   // per-queue reservation counters
  unsigned long long stats[kNumStats];
};

// Per-pair record written by the batched setup pass: ring offsets and
// vertex counts of both polygons and the pair's class, so that the sweep
// reads one 32-byte record per pair (through the scalar cache).
struct PairRec {
  int64_t op, oq;
  int32_t np, nq;
  int32_t cls, pad;
};

struct BatchArgs {
  Polys A, B;
  int64_t n_pairs;
  const int32_t* pa;
  const int32_t* pb;
  int64_t* inter;
  int64_t* uni;
  uint32_t* err;
  uint8_t* cls;                  // [n_pairs]
  PairRec* rec;                  // [n_pairs]
  int32_t* l_list;               // [kLptBuckets][n_pairs] listed pairs, bucket b from b * n_pairs
  int32_t* m_list;               // [n_pairs] medium pairs, in the order they were listed
  Meta* hbox;                    // [n_pairs] pair box of a listed pair (by pair index)
  BatchState* st;
  unsigned long long* queue;     // [n_queues * queue_cap] task words, 0 = empty
  int32_t queue_cap;             // slots per queue
  int32_t n_queues;
  int32_t chunk;                 // small pairs per claim
  int32_t heavy_verts;           // pairs with at least this many vertices are claimed first
  int32_t min_cells_to_queue;    // a split pushes its boxes to the queue only from this many boxes
  int32_t min_classify_cells;    // a leaf-level split classifies its tiles only from this many cells
  uint32_t flags;                // SCCG_F_*
  int32_t stats_on;
  // nullable: per wave, (start, end) stamps of the device's constant-rate
  // counter, wave_cap waves per kernel: the sweep, the medium sweep, then
  // the persistent kernel
  unsigned long long* wave_t;
  int32_t wave_cap;
};
// kernels whose waves are stamped (see BatchArgs::wave_t)
constexpr int kStampedKernels = 3;
hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_setup(const BatchArgs& a, hipStream_t s);
// The union sweep (sweep_grid workgroups) then the medium sweep with the
// prepass of the pairs the setup pass listed (medium_grid);
// pair_box: the union sweep also counts the pairs whose pair box fits a leaf
// tile (else the medium sweep does).
hipError_t launch_batch_sweeps(const BatchArgs& a, int sweep_grid, int medium_grid, bool pair_box, hipStream_t s);
// The persistent kernel (grid workgroups).
hipError_t launch_batch_persistent(const BatchArgs& a, int grid, int waves_per_wg, hipStream_t s);
int batch_lds_bytes_per_wave();
int batch_occupancy(int waves_per_wg);
// Workgroups per CU of the union sweep (the instance that counts pair boxes
// or the one that does not) and of the medium sweep.
int batch_sweep_occupancy(bool pair_box);
int batch_medium_occupancy();
int batch_sweep_waves_per_wg();

// Set-level Jaccard: per-set accumulators (a cache line each), a chunk
// counter and `grid` workgroups that claim chunks of the pair range.
struct alignas(128) JacAcc {
  unsigned long long si, su, nn;
  unsigned long long limb[6];  // Fix192 ratio sum as 32-bit limbs, carry-save
};
hipError_t launch_jaccard(int64_t n_sets, const int64_t* set_off, const int64_t* inter, const int64_t* uni,
                          uint32_t flags, int64_t* sum_i, int64_t* sum_u, int64_t* n_contrib, double* j,
                          double* jprime, JacAcc* acc, unsigned long long* next, int grid, hipStream_t s);

// Ring validation.
hipError_t launch_validate(const Polys& P, int64_t* first_bad, hipStream_t s);

// Filter stage (candidate pairs by MBR intersection).
int64_t scan_scratch(int64_t n);
hipError_t launch_join_grid(const Polys& A, const Meta* metaA, const int64_t* a_off, int64_t n_sets, int cell,
                            int4* bbox, int4* grid, int64_t* cells, int64_t* cell_base, int64_t* sums,
                            uint32_t* err, hipStream_t s);
hipError_t launch_join_cells(const Polys& A, const Meta* metaA, const int64_t* a_off, int64_t n_sets,
                             const int4* grid, const int64_t* cell_base, int cell, int mode, int32_t* count,
                             const int64_t* start, int32_t* list, hipStream_t s);
hipError_t launch_join_scan_counts(const int32_t* count, int64_t n, int64_t* start, int64_t* sums, hipStream_t s);
hipError_t launch_join_pairs(const Polys& B, const Meta* metaA, const Meta* metaB, const int64_t* b_off,
                             int64_t n_sets, const int4* grid, const int64_t* cell_base, const int64_t* start,
                             const int32_t* list, int cell, int mode, int32_t* b_count, const int64_t* b_start,
                             int64_t cap, int32_t* out_pa, int32_t* out_pb, hipStream_t s);
hipError_t launch_join_set_off(int64_t n_sets, int64_t n_b, const int64_t* b_off, const int64_t* b_start,
                               int64_t* out_set_off, hipStream_t s);

// Section 3.4's operators from counts and edges.
hipError_t launch_relate(const Polys& A, const Polys& B, const Meta* metaA, const Meta* metaB, const int64_t* areaA,
                         const int64_t* areaB, int64_t n_pairs, const int32_t* pa, const int32_t* pb,
                         const int64_t* inter, uint32_t* out, uint32_t* err, hipStream_t s);

// Diagnostics: 32 integer VALU operations per lane and loop trip, `iters`
// trips, grid workgroups of 256 lanes.
hipError_t launch_valu_peak(int grid, int iters, unsigned long long* sink, hipStream_t s);

// The device error word of a context (read and cleared by the server, which
// owns its context and runs on the context's stream).
uint32_t* ctx_error_word(sccg_ctx* c);

}  // namespace sccg
