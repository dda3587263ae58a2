// Task 1 of the MD step on gfx950: skin test and Verlet-list rebuild.  Included by
// md_kernels.hip.
//
//   k_decide        one block, a wavefront per replica: skin test (Section 2.6) -> rebuild flags
//   k_bin           wrap periodic coordinates, cell of every atom / carbon, cell counts (with a
//                   single replica each block takes the skin decision itself, no k_decide)
//   k_scan          exclusive scan of all cell counts (one pass, decoupled look-back)
//   k_scatter       atom slots / carbon indices into their cells at the ranks k_bin took
//                   (arbitrary order within a cell), with the (cell, id) sort keys; marks
//                   the 27-cell stencil of every occupied carbon cell
//   k_sort_gather   one lane per slot: rank within its cell by (cell, id), gather the atom
//                   state into sorted order (so the final order is canonical); atoms in a
//                   marked carbon cell join the near list
//   k_list_tiles    one block per run of cells of a cell row: the neighbouring rows are
//                   staged in LDS, each atom scans its window of them; copies the sorted
//                   state back.  Its leading blocks build the Cr-C lists (xlist_pass: one
//                   wavefront per near atom).  k_list_rows (one lane per atom from global
//                   memory, for periodic axes with fewer than 3 cells) is followed by
//                   k_xlist, the same Cr-C pass as a launch of its own.
//
// Every build kernel after the decision returns at once when no replica needs a rebuild, so
// a step without a rebuild costs a few empty launches.
#pragma once

#include "md_device.hpp"

namespace md {

struct BuildArgs {
  const RepDesc* R;
  RepState* S;
  const int* tile_rep;   // [ntiles]
  const int* row_rep;    // [nrows] replica of each cell row at capacity
  int2* items;           // [list-build blocks] work items of k_list_tiles: (row, run | runs << 16)
  int* nitems;           // work items of this build
  int* next_item;        // the next work item a k_list_tiles block takes (reset with nitems)
  const int* c_rep;      // [ctot] replica of each carbon
  int* any;              // 1 if some replica rebuilds in this step
  int* abort;            // sticky: a bounded wait of a build gave up; no build runs until
                         // md_clear_flags (which also zeroes the cell counts it left behind)
  double4* q;
  double* v;
  double* f;
  uint8_t* fixed;
  int* id;
  const double* xc;
  double* xref;
  int* cellid;           // [ntot] cell of each atom slot
  int* crank;            // [ntot] rank of the slot among the atoms binned into its cell
  int* perm;             // [ntot] slots by cell (cells in order, arbitrary order within one)
  long long* skey;       // [ntot] (cell, id) sort key of perm's entries
  double4* tq;
  float4* tqf;           // [ntot] sorted positions relative to the replica's grid origin, FP32
  int4* qs;              // [ntot] fixed-point cell-local shadow of q (x, y, z, F' bits)
  long long* bcell;      // [ntot] build cell of each atom slot (pack_cell)
  double* tv;
  double* tf;
  uint8_t* tfixed;
  int* tid;
  int* count;            // [ncell_all]
  int* start;            // [ncell_all + 1]
  int* hcell;            // [ctot]
  int* hrank;            // [ctot] rank of the carbon among those binned into its cell
  int* hlist;            // [ctot] carbons by cell (arbitrary order within a cell)
  double4* hsorted;      // [ctot] carbons by cell, ascending index within a cell: position at
                         // zero indenter displacement, the carbon's index (as bits) in .w
  long long* scan_state; // [scan_blocks] published chunk sums of k_scan
  int* scan_ticket;      // chunk ticket of k_scan
  int* hnear;            // [ncell_all]: carbon cell c has a carbon in its 27-cell stencil
  int* idx;
  int* cnt;
  int* xidx;
  int* xcnt;
  int* near;             // [ntot]: replica r's near atoms at near[a0_r ...]
  double* fme;           // [ntot][4]: last Morse force and energy per atom (0 if none)
  int ncell_all, ncell_cr, ntiles, ctot;
  int nbin;              // tile blocks' worth of work of k_bin, k_scatter, k_sort_gather: the Cr
                         // tiles, then 256-carbon groups (the grids stride over them)
  int near_blocks;       // grid of k_xlist
  int xblocks;           // leading blocks of k_list_tiles that build the Cr-C lists (0: none)
  int persistent;        // k_list_tiles: blocks take work items from a counter (else one block
                         // per item of the table's capacity, the blocks past the items idle)
  int commit_ref;        // k_scan records the indenter position of this build (k_bin decided)
  int copy_f;            // the forces are permuted with the atoms (0 inside md_run: no kick reads
                         // them before the next force pass that stores them)
  int scan_chunk, scan_blocks;
  int spin_limit;        // polls of k_scan's look-back before it gives up (< 0: at once)
  int nrows, nlblk;      // cell rows at capacity; capacity of the work-item table
  int list_tgt;          // atoms a work item aims at (<= LIST_BLOCK)
};

#ifndef MD_LIST_BATCH
#define MD_LIST_BATCH 4
#endif
constexpr int LIST_BATCH = MD_LIST_BATCH;   // candidate loads issued together in k_list_rows
constexpr int MAXC = 512;           // candidates staged per window in k_xlist
#ifndef MD_SG_KEYS
#define MD_SG_KEYS 8
#endif
constexpr int SG_KEYS = MD_SG_KEYS;   // keys of a cell k_sort_gather loads at a time
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;
constexpr int LIST_SEG = 42;      // most cells of one work item of k_list_tiles
#ifndef MD_LIST_STAGE
#define MD_LIST_STAGE 1024
#endif
constexpr int LIST_STAGE = MD_LIST_STAGE;   // candidates k_list_tiles stages in LDS at a time
#ifndef MD_LIST_WAVES
#define MD_LIST_WAVES 7
#endif
#ifndef MD_LIST_WAVES_RESIDENT
#define MD_LIST_WAVES_RESIDENT 6
#endif
#ifndef MD_LIST_BLOCK
#define MD_LIST_BLOCK 256
#endif
#ifndef MD_LIST_TGT
#define MD_LIST_TGT 224
#endif
constexpr int LIST_BLOCK = MD_LIST_BLOCK;           // threads of k_list_tiles
constexpr int LIST_TGT = MD_LIST_TGT;               // atoms per work item aimed at (default)
constexpr int LIST_PT = LIST_STAGE / LIST_BLOCK;    // candidates each thread stages per piece
static_assert(LIST_STAGE % LIST_BLOCK == 0, "a piece is a whole number of candidates per thread");
static_assert(LIST_TGT <= LIST_BLOCK, "a work item's atoms aimed at fit one pass of the threads");
#ifndef MD_LIST_GROUP
#define MD_LIST_GROUP 4
#endif
constexpr int LIST_GROUP = MD_LIST_GROUP;   // candidates screened together per atom in k_list_tiles
static_assert(LIST_GROUP >= 1 && LIST_GROUP <= 32, "a group's passing bits fit the 32-bit mask k_list_tiles appends from");


__device__ __forceinline__ bool rebuild_off(const BuildArgs& A) { return *A.any == 0; }

// One block of DECIDE_THREADS decides every replica (skin test, then the cell grid of the
// build) and ORs the outcomes into the launch-wide flag: the whole block per replica when
// there are few, else a group of lanes per replica (up to a wavefront; see below).
constexpr int DECIDE_THREADS = 1024;
constexpr int DECIDE_BLOCKWIDE = 4;   // replicas up to which the whole block takes each one

// Per-replica part of k_decide.  Reduce(v, op) reduces over the threads that share the
// replica (a wavefront or the block); `lead` marks the thread that writes.
// Skin test (Section 2.6) and cell grid of replica r, the same in every thread that calls it
// (every thread of the block calls it together: maxr is a block or wavefront reduction).
struct BuildGrid {
  int need;
  double glo[3], ginv[3], gedge[3], qscale;
  int gd[3];
};
// The replica's parts are entries first .. first + count - 1 of dmax_tile / tile_box.
template <class MaxReduce>
__device__ __forceinline__ BuildGrid decide_grid(const Consts& K, const BuildArgs& A, int r,
                                                 const double* dmax_tile, const double* tile_box, int force,
                                                 int first, int count, int t0, int tstep, MaxReduce maxr) {
  const RepDesc& d = A.R[r];
  const RepState& s = A.S[r];
  BuildGrid g;
  double m = 0.0;
#pragma unroll 8
  for (int t = t0; t < count; t += tstep) m = fmax(m, dmax_tile[first + t]);   // loads together
  m = maxr(m);
  g.need = !*A.abort && (force || (m > K.half_skin_sq) || (fabs(s.ind_z - s.ind_z_ref) > K.half_skin));
  if (!g.need) return g;   // uniform over the threads of the replica
  // cell grid of this build: the box along periodic axes, the atoms' extent along open ones
  for (int a = 0; a < 3; ++a) {
    if (d.per[a]) {
      g.glo[a] = d.lo[a];
      g.ginv[a] = d.ginv[a];
      g.gedge[a] = d.len[a] / d.gcap[a];
      g.gd[a] = d.gcap[a];
      continue;
    }
    double mn = INFINITY, mx = -INFINITY;
#pragma unroll 4
    for (int t = t0; t < count; t += tstep) {
      mn = fmin(mn, tile_box[6 * (int64_t)(first + t) + a]);
      mx = fmax(mx, tile_box[6 * (int64_t)(first + t) + 3 + a]);
    }
    mn = -maxr(-mn);
    mx = maxr(mx);
    if (!(mn <= mx)) {   // no atoms (or non-finite positions): fall back to the box
      mn = d.lo[a];
      mx = d.lo[a] + d.len[a];
    }
    const double edge = K.rlist * (1.0 + 1e-9);
    const double ext = fmax(mx - mn, edge);
    const int gc = (int)fmin(fmax(floor(ext / edge), 1.0), (double)d.gcap[a]);
    g.glo[a] = mn;
    g.ginv[a] = gc / ext;
    g.gedge[a] = ext / gc;
    g.gd[a] = gc;
  }
  // shadow scale: the longest cell edge spans at most 2^29 units
  const double emax = fmax(g.gedge[0], fmax(g.gedge[1], g.gedge[2]));
  g.qscale = ldexp(1.0, 29 - (int)ceil(log2(emax)));
  return g;
}

// Records the outcome in the replica's state (one thread).
__device__ __forceinline__ void record_grid(RepState& s, const BuildGrid& g) {
  s.rebuild = g.need;
  if (!g.need) return;
  s.nnear_old = s.nnear;
  s.nnear = 0;
  for (int a = 0; a < 3; ++a) {
    s.glo[a] = g.glo[a];
    s.ginv[a] = g.ginv[a];
    s.gedge[a] = g.gedge[a];
    s.gd[a] = g.gd[a];
  }
  s.qscale = g.qscale;
}

template <class MaxReduce>
__device__ __forceinline__ bool decide_replica(const Consts& K, BuildArgs& A, int r, const double* dmax_tile,
                                               const double* tile_box, int force, int ppt, int t0, int tstep,
                                               bool lead, MaxReduce maxr) {
  const BuildGrid g = decide_grid(K, A, r, dmax_tile, tile_box, force, A.R[r].t0 * ppt, A.R[r].nt * ppt, t0,
                                  tstep, maxr);
  if (lead) record_grid(A.S[r], g);
  return g.need;
}

__global__ __launch_bounds__(DECIDE_THREADS) void k_decide(Consts K, BuildArgs A,
                                                           const double* __restrict__ dmax_tile,
                                                           const double* __restrict__ tile_box, int force,
                                                           int ppt) {
  __shared__ int any_sh;
  if (threadIdx.x == 0) any_sh = 0;
  __syncthreads();
  if (K.nrep <= DECIDE_BLOCKWIDE) {
    for (int r = 0; r < K.nrep; ++r) {
      const bool need = decide_replica(K, A, r, dmax_tile, tile_box, force, ppt, threadIdx.x, DECIDE_THREADS,
                                       threadIdx.x == 0, [](double v) { return block_max<DECIDE_THREADS>(v); });
      if (need && threadIdx.x == 0) any_sh = 1;
    }
  } else {
    // groups of G lanes (a power of two, G <= 64), as many as there are replicas up to
    // 1024 / G: group g takes replicas g, g + 1024 / G, ... (so the replicas' loads go out
    // together rather than a wavefront's replicas one after another)
    int G = WAVE;
    while (G > 1 && (DECIDE_THREADS / G) < K.nrep) G >>= 1;
    const int sub = threadIdx.x % G, grp = threadIdx.x / G, ng = DECIDE_THREADS / G;
    for (int r0 = 0; r0 < K.nrep; r0 += ng) {   // (uniform: every group steps together)
      const int r = r0 + grp;
      const bool mine = r < K.nrep;
      // groups past the last replica repeat replica 0's decision without recording it
      const bool need = decide_replica(K, A, mine ? r : 0, dmax_tile, tile_box, force, ppt, sub, G,
                                       mine && sub == 0, [G](double v) {
                                         for (int o = G / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
                                         return v;
                                       });
      if (need && mine && sub == 0) atomicOr(&any_sh, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *A.any = any_sh;
    *A.nitems = 0;   // k_scatter lists the list-build work items of a rebuild
    *A.next_item = 0;
  }
  for (int r = threadIdx.x; r < K.nrep; r += DECIDE_THREADS) {   // builds are counted here
    RepState& s = A.S[r];
    if (s.rebuild) {
      s.nbuilds += 1;
      s.ind_z_ref = s.ind_z;
    }
  }
}

__device__ __forceinline__ int cr_cell_of(const RepDesc& d, const RepState& s, double x, double y, double z) {
  int cx = cell_coord(x, s.glo[0], s.ginv[0], s.gd[0]);
  int cy = cell_coord(y, s.glo[1], s.ginv[1], s.gd[1]);
  int cz = cell_coord(z, s.glo[2], s.ginv[2], s.gd[2]);
  return d.g0 + (cz * s.gd[1] + cy) * s.gd[0] + cx;
}

// Coordinate folded into [lo, lo + len) on a periodic axis (binning of carbons only).
__device__ __forceinline__ double fold(double x, double lo, double len, int per) {
  if (!per) return x;
  return x - len * floor((x - lo) / len);
}

__device__ __forceinline__ void c_cell_coords(const RepDesc& d, double x, double y, double z, int& hx,
                                              int& hy, int& hz) {
  hx = cell_coord(fold(x, d.lo[0], d.len[0], d.per[0]), d.lo[0], d.hinv[0], d.hd[0]);
  hy = cell_coord(fold(y, d.lo[1], d.len[1], d.per[1]), d.lo[1], d.hinv[1], d.hd[1]);
  hz = cell_coord(fold(z, d.lo[2], d.len[2], d.per[2]), d.lo[2], d.hinv[2], d.hd[2]);
}

// Rank of this lane's atom among the atoms binned into cell `cid`: consecutive lanes with
// the same cell (the common case, atoms arrive in the previous build's cell order) form a
// run that takes its ranks with one atomic add.  Every lane of the wave calls it together.
__device__ __forceinline__ int bin_rank(int* count, int cid, bool live) {
  const int lane = threadIdx.x % WAVE;
  const int key = live ? cid : -1;
  const int prev = __shfl_up(key, 1, WAVE);
  const bool head = live && (lane == 0 || prev != key);
  const unsigned long long heads = __ballot(head);
  const unsigned long long stops = __ballot(head || !live);   // first lane of the next run
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const unsigned long long below = heads & upto;                // heads at lanes <= lane
  const int start = below ? 63 - __builtin_clzll(below) : 0;
  int base = 0;
  if (head) {
    const unsigned long long after = stops & ~upto;
    const int end = after ? __builtin_ctzll(after) : WAVE;
    base = atomicAdd(&count[cid], end - lane);
  }
  base = __shfl(base, start, WAVE);
  return base + (lane - start);
}

// The nparts per-part displacement maxima and boxes of a single replica reduced to
// gridDim.x partial ones in the same layout (block b takes a contiguous chunk): the
// maximum, the minima and the maxima of each axis (the neutral values where a chunk is
// empty).  The skin decision then reads those few instead of every part.
__global__ __launch_bounds__(BLOCK) void k_parts_reduce(const double* __restrict__ dmax_tile,
                                                        const double* __restrict__ tile_box, int nparts,
                                                        double* __restrict__ dmax_out,
                                                        double* __restrict__ box_out) {
  const int chunk = (nparts + gridDim.x - 1) / gridDim.x;
  const int p0 = blockIdx.x * chunk, p1 = min(p0 + chunk, nparts);
  // the maximum, then per axis the negated minimum and the maximum
  double v[7] = {0.0, -INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int p = p0 + threadIdx.x; p < p1; p += BLOCK) {
    v[0] = fmax(v[0], dmax_tile[p]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v[1 + a] = fmax(v[1 + a], -tile_box[6 * (int64_t)p + a]);
      v[4 + a] = fmax(v[4 + a], tile_box[6 * (int64_t)p + 3 + a]);
    }
  }
  block_max_to0<BLOCK, 7>(v);
  if (threadIdx.x == 0) {
    dmax_out[blockIdx.x] = v[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      box_out[6 * blockIdx.x + a] = -v[1 + a];
      box_out[6 * blockIdx.x + 3 + a] = v[4 + a];
    }
  }
}

// Blocks [0, ntiles): one tile of Cr atoms each.  Blocks [ntiles, ...): 256 carbons each.
// DECIDE (single replica, no forced build): every block takes the skin decision and the
// cell grid itself from the nparts per-part maxima and boxes (or their partial reductions by
// k_parts_reduce; so no separate decision launch), all blocks alike; block 0 records them.
// The indenter reference position, which every block reads for the decision, is recorded by
// k_scan.
template <bool DECIDE>
__global__ __launch_bounds__(BLOCK) void k_bin(Consts K, BuildArgs A, const double* __restrict__ dmax_tile,
                                               const double* __restrict__ tile_box, int nparts) {
  BuildGrid g1;
  if (DECIDE) {
    g1 = decide_grid(K, A, 0, dmax_tile, tile_box, 0, 0, nparts, threadIdx.x, BLOCK,
                     [](double v) { return block_max<BLOCK>(v); });
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      RepState& s0 = A.S[0];
      record_grid(s0, g1);
      if (g1.need) s0.nbuilds += 1;
      *A.any = g1.need;
      *A.nitems = 0;   // k_scatter lists the list-build work items of a rebuild
      *A.next_item = 0;
    }
    if (!g1.need) return;
  } else if (rebuild_off(A)) {
    return;
  }
  if (blockIdx.x == 0) {   // fresh state for this build's k_scan
    for (int t = threadIdx.x; t < A.scan_blocks; t += BLOCK) A.scan_state[t] = 0;
    if (threadIdx.x == 0) *A.scan_ticket = 0;
  }
  for (int b = blockIdx.x; b < A.nbin; b += gridDim.x) {   // (b uniform over the block)
  if (b < A.ntiles) {
    const int r = A.tile_rep[b];
    if (!DECIDE && !A.S[r].rebuild) continue;
    const RepDesc& d = A.R[r];
    const int64_t i = (int64_t)b * TILE + threadIdx.x;
    const bool live = i < (int64_t)d.a0 + d.n;
    int cid = -1;
    if (live) {
      double4 p = A.q[i];
      double xyz[3] = {p.x, p.y, p.z};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (!d.per[a]) continue;
        const double hi = d.lo[a] + d.len[a];
        if (xyz[a] >= hi)
          xyz[a] -= d.len[a];
        else if (xyz[a] < d.lo[a])
          xyz[a] += d.len[a];
      }
      p.x = xyz[0];
      p.y = xyz[1];
      p.z = xyz[2];
      if (DECIDE) {   // the grid just decided (block 0 may be recording it meanwhile)
        const int cx = cell_coord(p.x, g1.glo[0], g1.ginv[0], g1.gd[0]);
        const int cy = cell_coord(p.y, g1.glo[1], g1.ginv[1], g1.gd[1]);
        const int cz = cell_coord(p.z, g1.glo[2], g1.ginv[2], g1.gd[2]);
        cid = d.g0 + (cz * g1.gd[1] + cy) * g1.gd[0] + cx;
      } else {
        cid = cr_cell_of(d, A.S[r], p.x, p.y, p.z);   // before the stores (which could alias S)
      }
      A.q[i] = p;
      A.cellid[i] = cid;
    }
    const int rank = bin_rank(A.count, cid, live);
    if (live) A.crank[i] = rank;
  } else {
    const int64_t k = (int64_t)(b - A.ntiles) * BLOCK + threadIdx.x;
    int r = -1;
    if (k < A.ctot) {
      r = A.c_rep[k];
      if (!DECIDE && !A.S[r].rebuild) r = -1;
    }
    if (r >= 0) {
      const RepDesc& d = A.R[r];
      const double z = A.xc[3 * k + 2] + A.S[r].ind_z;
      int hx, hy, hz;
      c_cell_coords(d, A.xc[3 * k + 0], A.xc[3 * k + 1], z, hx, hy, hz);
      const int hid = d.h0 + (hz * d.hd[1] + hy) * d.hd[0] + hx;
      A.hcell[k] = hid;
      A.hrank[k] = atomicAdd(&A.count[hid], 1);
    }
  }
  }
}

// Exclusive scan of all cell counts in one launch: each block scans SCAN_CHUNK cells and
// finds the sum of the chunks before it by looking back over the published chunk states
// (single-pass scan with decoupled look-back, Merrill and Garland 2016).  Chunks are
// taken in ticket order, so a block only waits for blocks that are already running; the
// wait is bounded and a timeout is reported in the status words.
constexpr int SCAN_PER_THREAD = 8;
constexpr long long SCAN_AGG = 1ll << 32, SCAN_INCL = 2ll << 32;

__global__ __launch_bounds__(BLOCK) void k_scan(BuildArgs A) {
  if (rebuild_off(A)) return;
  __shared__ int chunk_sh, excl_sh;
  if (threadIdx.x == 0) chunk_sh = atomicAdd(A.scan_ticket, 1);
  __syncthreads();
  const int b = chunk_sh;
  if (A.commit_ref && b == 0 && threadIdx.x == 0) {   // k_bin decided: this build's indenter position
    RepState& s0 = A.S[0];
    s0.ind_z_ref = s0.ind_z;
  }
  const int c0 = b * A.scan_chunk + threadIdx.x * SCAN_PER_THREAD;
  int v[SCAN_PER_THREAD];
  int sum = 0;
#pragma unroll
  for (int u = 0; u < SCAN_PER_THREAD; ++u) {
    v[u] = (c0 + u < A.ncell_all) ? A.count[c0 + u] : 0;
    sum += v[u];
  }
  int tot;
  const int pre = block_exclusive_scan(sum, &tot);
  // wave 0 publishes this chunk and looks back 64 chunks at a time.  A published word holds
  // both the flag and the sum, and nothing else a chunk writes is read before the next
  // launch, so the atomics are relaxed (agent scope): a release or acquire here would write
  // back or invalidate the per-XCD L2 at every publication and poll.
  if (threadIdx.x < WAVE) {
    const int lane = threadIdx.x;
    long long* st = A.scan_state;
    int excl = 0;
    if (b == 0) {
      if (lane == 0)
        __hip_atomic_store(&st[0], SCAN_INCL | (unsigned)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(&st[b], SCAN_AGG | (unsigned)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int top = b - 1, spins = 0;
      while (true) {
        const int j = top - lane;   // lane 0 is the nearest predecessor; j < 0 reads as prefix 0
        const long long w =
            j >= 0 ? __hip_atomic_load(&st[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : SCAN_INCL;
        const long long flag = w & ~0xffffffffll;
        const unsigned long long incl = __ballot(flag == SCAN_INCL);
        const unsigned long long ready = __ballot(flag != 0);
        const int first = incl ? __builtin_ctzll(incl) : WAVE;   // nearest inclusive prefix
        const unsigned long long need = first < WAVE ? ((2ull << first) - 1ull) : ~0ull;
        if ((ready & need) != need || A.spin_limit < 0) {   // some chunk in between has not published yet
          if (++spins > A.spin_limit) {
            // give up: this build is invalid.  The later build kernels of this step see no
            // rebuild (so nothing is scattered with a wrong prefix), and no build runs until
            // md_clear_flags.
            if (lane == 0) {
              A.S[0].sync_timeout = 1;
              *A.abort = 1;
              *A.any = 0;
            }
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += wave_sum(lane <= first ? (int)(unsigned)(w & 0xffffffffll) : 0);
        if (first < WAVE) break;
        top -= WAVE;
      }
      if (lane == 0)
        __hip_atomic_store(&st[b], SCAN_INCL | (unsigned)(excl + tot), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      excl_sh = excl;
      if (b == A.scan_blocks - 1) A.start[A.ncell_all] = excl + tot;
    }
  }
  __syncthreads();
  int run = excl_sh + pre;
#pragma unroll
  for (int u = 0; u < SCAN_PER_THREAD; ++u) {
    if (c0 + u < A.ncell_all) {
      A.start[c0 + u] = run;
      A.hnear[c0 + u] = 0;
    }
    run += v[u];
  }
}

// Work items of k_list_tiles for cell row g (capacity numbering) of a rebuilding replica:
// the row is cut into as many runs of cells as keep a run's atoms near list_tgt (and no run
// longer than LIST_SEG cells); empty rows get none.  Returns the number of runs.
__device__ __forceinline__ int row_runs(const BuildArgs& A, int64_t g) {
  if (g >= A.nrows) return 0;
  const int r = A.row_rep[g];
  const RepState& S = A.S[r];
  if (!S.rebuild) return 0;
  const RepDesc& d = A.R[r];
  const int gx = S.gd[0], gy = S.gd[1], gz = S.gd[2];
  const int l = (int)(g - d.rb0), cy = l % gy, cz = l / gy;
  if (cz >= gz) return 0;
  const int crow = d.g0 + (cz * gy + cy) * gx;
  const int n = A.start[crow + gx] - A.start[crow];
  if (n == 0) return 0;
  return min(min(d.nseg, gx), max((gx + LIST_SEG - 1) / LIST_SEG, (n + A.list_tgt - 1) / A.list_tgt));
}

__global__ __launch_bounds__(BLOCK) void k_scatter(Consts K, BuildArgs A) {
  if (rebuild_off(A)) return;
  // list-build work items, one cell row per thread, appended with one atomic per wavefront
  // (their order is immaterial: each item writes only its own atoms' lists)
  const int lane = threadIdx.x % WAVE;
  for (int64_t g0 = (int64_t)blockIdx.x * BLOCK; g0 < A.nrows; g0 += (int64_t)gridDim.x * BLOCK) {
    const int64_t g = g0 + threadIdx.x;
    const int nr = row_runs(A, g);
    int incl = nr;   // inclusive prefix over the wavefront
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int t = __shfl_up(incl, o, WAVE);
      if (lane >= o) incl += t;
    }
    int base = 0;
    if (lane == WAVE - 1 && incl > 0) base = atomicAdd(A.nitems, incl);
    base = __shfl(base, WAVE - 1, WAVE);
    for (int k = 0, at = base + incl - nr; k < nr; ++k, ++at)
      if (at < A.nlblk) A.items[at] = make_int2((int)g, k | (nr << 16));
  }
  for (int b = blockIdx.x; b < A.nbin; b += gridDim.x) {   // (b uniform over the block)
  if (b < A.ntiles) {
    const int r = A.tile_rep[b];
    if (!A.S[r].rebuild) continue;
    const RepDesc& d = A.R[r];
    const int64_t i = (int64_t)b * TILE + threadIdx.x;
    if (i >= (int64_t)d.a0 + d.n) continue;
    const int cid = A.cellid[i];
    const int pos = d.a0 + (A.start[cid] - A.start[d.g0]) + A.crank[i];
    A.perm[pos] = (int)i;
    A.skey[pos] = ((long long)cid << 32) | (unsigned)A.id[i];
    // the Cr-C records (force, energy) are nonzero only at near-list slots: zeroing those of
    // the previous build's near list (lane k takes entry k) leaves every record zero, and the
    // Cr-C pass rewrites the new near atoms' records
    const int64_t k = i - d.a0;
    if (k < A.S[r].nnear_old) {
      const int64_t pn = A.near[d.a0 + k];
      A.fme[4 * pn + 0] = 0.0;
      A.fme[4 * pn + 1] = 0.0;
      A.fme[4 * pn + 2] = 0.0;
      A.fme[4 * pn + 3] = 0.0;
    }
  } else {
    const int64_t k = (int64_t)(b - A.ntiles) * BLOCK + threadIdx.x;
    if (k >= A.ctot) continue;
    const int r = A.c_rep[k];
    if (!A.S[r].rebuild) continue;
    const RepDesc& d = A.R[r];
    const int hid = A.hcell[k];
    const int rank = A.hrank[k];
    A.hlist[d.c0 + (A.start[hid] - A.start[d.h0]) + rank] = (int)k;
    if (rank == 0) {
      // one carbon per occupied carbon cell: every cell of its stencil can hold Cr atoms
      // within reach of a carbon (k_scan cleared the marks).  The descriptor is read into
      // registers first: a store could alias it and would make every read after it wait.
      const int h0 = d.h0, hd0 = d.hd[0], hd1 = d.hd[1], hd2 = d.hd[2];
      const int p0 = d.per[0], p1 = d.per[1], p2 = d.per[2];
      int* __restrict__ hn = A.hnear + h0;
      const int lc = hid - h0;
      const int hx = lc % hd0, hy = (lc / hd0) % hd1, hz = lc / (hd0 * hd1);
      const int msx = stencil_n(hd0, p0), msy = stencil_n(hd1, p1), msz = stencil_n(hd2, p2);
      for (int tz = 0; tz < msz; ++tz) {
        const int z = stencil_cell(hz, tz, hd2, p2);
        for (int ty = 0; ty < msy; ++ty) {
          const int y = stencil_cell(hy, ty, hd1, p1);
          for (int tx = 0; tx < msx; ++tx) {
            const int x = stencil_cell(hx, tx, hd0, p0);
            if (x >= 0 && y >= 0 && z >= 0) hn[(z * hd1 + y) * hd0 + x] = 1;
          }
        }
      }
    }
  }
  }
}

// One lane per slot in cell order.  Blocks [0, ntiles): Cr slots, one tile each; blocks
// [ntiles, ...): 256 carbon slots each.  A slot's final position is the start of its cell
// plus the number of atoms of that cell with a smaller (cell, id) key (cells hold a few
// atoms), so the final order is canonical; the atom's state is gathered there.
__global__ __launch_bounds__(BLOCK) void k_sort_gather(Consts K, BuildArgs A) {
  if (rebuild_off(A)) return;
  for (int b = blockIdx.x; b < A.nbin; b += gridDim.x) {   // (b uniform over the block)
  if (b < A.ntiles) {
    const int r = A.tile_rep[b];
    RepState& S = A.S[r];
    if (!S.rebuild) continue;
    const RepDesc& d = A.R[r];
    const int u = b * TILE + threadIdx.x;
    bool near = false;
    int p = 0;
    if (u < d.a0 + d.n) {
      const long long key = A.skey[u];
      const int c = (int)(key >> 32);
      const int sbase = d.a0 - A.start[d.g0];
      const int s0 = sbase + A.start[c], s1 = sbase + A.start[c + 1];
      const int e = A.perm[u];
      int rank = 0;
      // SG_KEYS independent key loads at a time: the index is clamped into the cell (which
      // holds this atom) rather than the load made conditional, so that no load waits on
      // the one before it
      for (int t = s0; t < s1; t += SG_KEYS) {
        long long kk[SG_KEYS];
#pragma unroll
        for (int u = 0; u < SG_KEYS; ++u) kk[u] = A.skey[min(t + u, s1 - 1)];
#pragma unroll
        for (int u = 0; u < SG_KEYS; ++u) rank += (t + u < s1 && kk[u] < key) ? 1 : 0;
      }
      if (u == s0) A.count[c] = 0;   // zero again for the next rebuild
      p = s0 + rank;
      // the atom's state, each value stored as it arrives (measured faster here than all
      // loads first)
      const double4 qe = A.q[e];
      A.tq[p] = qe;
      A.tqf[p] = make_float4((float)(qe.x - S.glo[0]), (float)(qe.y - S.glo[1]), (float)(qe.z - S.glo[2]), 0.0f);
      A.tv[3 * p + 0] = A.v[3 * e + 0];
      A.tv[3 * p + 1] = A.v[3 * e + 1];
      A.tv[3 * p + 2] = A.v[3 * e + 2];
      if (A.copy_f) {
        A.tf[3 * p + 0] = A.f[3 * e + 0];
        A.tf[3 * p + 1] = A.f[3 * e + 1];
        A.tf[3 * p + 2] = A.f[3 * e + 2];
      }
      A.tfixed[p] = A.fixed[e];
      A.tid[p] = A.id[e];
      // no Cr-C list until the Cr-C list build of this rebuild says otherwise (k_scatter
      // zeroed the Cr-C records)
      A.xcnt[p] = 0;
      if (d.nc > 0) {   // in the stencil of an occupied carbon cell: the atom gets a Cr-C list
        int hx, hy, hz;
        c_cell_coords(d, qe.x, qe.y, qe.z, hx, hy, hz);
        near = A.hnear[d.h0 + (hz * d.hd[1] + hy) * d.hd[0] + hx] != 0;
      }
    }
    const int lane = threadIdx.x % WAVE;
    const unsigned long long nm = __ballot(near);
    if (nm) {   // append this wave's near atoms (order within the near list is irrelevant)
      const int lead = __builtin_ctzll(nm);
      int first = 0;
      if (lane == lead) first = atomicAdd(&S.nnear, __popcll(nm));
      first = __shfl(first, lead, WAVE);
      if (near) A.near[d.a0 + first + __popcll(nm & ((1ull << lane) - 1ull))] = p;
    }
  } else {
    const int64_t u = (int64_t)(b - A.ntiles) * BLOCK + threadIdx.x;
    if (u >= A.ctot) continue;
    const int r = A.c_rep[u];   // carbon slots of a replica are its carbon index range
    if (!A.S[r].rebuild) continue;
    const RepDesc& d = A.R[r];
    const int e = A.hlist[u];
    const int c = A.hcell[e];
    const int hb = d.c0 - A.start[d.h0];
    const int s0 = hb + A.start[c], s1 = hb + A.start[c + 1];
    int rank = 0;
    for (int t = s0; t < s1; t += SG_KEYS) {   // SG_KEYS independent loads at a time (as above)
      int hh[SG_KEYS];
#pragma unroll
      for (int u = 0; u < SG_KEYS; ++u) hh[u] = A.hlist[min(t + u, s1 - 1)];
#pragma unroll
      for (int u = 0; u < SG_KEYS; ++u) rank += (t + u < s1 && hh[u] < e) ? 1 : 0;
    }
    A.hsorted[s0 + rank] = make_double4(A.xc[3 * e + 0], A.xc[3 * e + 1], A.xc[3 * e + 2],
                                        __longlong_as_double((long long)e));
    if (u == s0) A.count[c] = 0;   // zero again for the next rebuild
  }
  }
}

// Cr-Cr lists, one lane per sorted Cr atom.  The candidates of the atom are those of the
// cells around its own: nine cell rows (y, z), each holding x-cells cx-1 .. cx+1, which are
// one contiguous range of the sorted order (two where the row wraps around a periodic x
// axis).  Entries are written rows in order (z-major), along x, then by slot, at the
// interleaved positions the tpa lanes of the force passes read.  Along a periodic axis with
// >= 3 cells the periodic image of a candidate is fixed by the cell it comes from
// (separation + 0 or -+ length: the same rounding as the minimum image for every pair
// inside the list radius); along a periodic axis with fewer cells each cell is visited once
// and the minimum image is taken pair by pair.
template <bool SCREEN>
__global__ __launch_bounds__(BLOCK) void k_list_rows(Consts K, BuildArgs A) {
  if (rebuild_off(A)) return;
  const int T = K.lt;
  const int tile = blockIdx.x;
  const int r = A.tile_rep[tile];
  RepState& S = A.S[r];
  if (!S.rebuild) return;
  const RepDesc& d = A.R[r];
  const int p = tile * TILE + threadIdx.x;
  const bool live = p < d.a0 + d.n;
  const int cap = K.cap;
  if (live) {
    const double4 pi = A.tq[p];
    const int gx = S.gd[0], gy = S.gd[1], gz = S.gd[2];
    const int cx = cell_coord(pi.x, S.glo[0], S.ginv[0], gx);
    const int cy = cell_coord(pi.y, S.glo[1], S.ginv[1], gy);
    const int cz = cell_coord(pi.z, S.glo[2], S.ginv[2], gz);
    const int sbase = d.a0 - A.start[d.g0];   // sorted slot = sbase + start[cell]
    const double rl2 = K.rlist_sq;
    const double4* __restrict__ tq = A.tq;
    const float4* __restrict__ tqf = A.tqf;
    // entry k at idx[(k / T) * row + k % T]: wp walks the slots in entry order
    const int64_t row = K.ntot * T;
    int* __restrict__ wp = A.idx + (int64_t)p * T;
    // pairwise minimum image on periodic axes with fewer than 3 cells (no FP32 screen then)
    const bool mx = !SCREEN && d.per[0] && gx < 3, my = !SCREEN && d.per[1] && gy < 3,
               mz = !SCREEN && d.per[2] && gz < 3;
    // FP32 screen: r2f, the squared separation from FP32 coordinates relative to the grid
    // origin, decides the pair when it lies outside [rl2 - delta, rl2 + delta); pairs inside
    // that band get the exact FP64 test.  With u = 2^-24, coordinates within E of the origin
    // and a periodic length L, each separation component carries an error of at most
    // eta = u (2E + 2L + 3R) for |component| <= R = r_list + 1, so |r2f - r2| <= sum over axes
    // of (2 R eta + eta^2) + 4 u (rl2 + R^2); delta is twice that.  Pairs farther than R
    // apart are far outside the band.
    float lo_f = 0.0f, hi_f = 0.0f;
    if (SCREEN) {
      const double u = 0x1p-24, R = K.rlist + 1.0;
      const int g[3] = {gx, gy, gz};
      double err = 4.0 * u * (rl2 + R * R);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double E = g[a] / S.ginv[a] + 2.0 * R;
        const double eta = u * (2.0 * E + (d.per[a] ? 2.0 * d.len[a] : 0.0) + 3.0 * R);
        err += 2.0 * R * eta + eta * eta;
      }
      const double delta = 2.0 * err + 1e-6;
      lo_f = (float)(rl2 - delta);
      hi_f = (float)(rl2 + delta);
    }
    const float4 pf = SCREEN ? tqf[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    // x segments (first cell, last cell, shift), the same for every row
    int xa0 = cx - 1, xb0 = cx + 1, xa1 = 0, xb1 = -1;
    double sh0 = 0.0, sh1 = 0.0;
    if (mx) {
      xa0 = 0;
      xb0 = gx - 1;
    } else if (d.per[0]) {
      if (cx == 0) {
        xa0 = gx - 1; xb0 = gx - 1; sh0 = -d.len[0];
        xa1 = 0; xb1 = 1;
      } else if (cx == gx - 1) {
        xa0 = gx - 2; xb0 = gx - 1;
        xa1 = 0; xb1 = 0; sh1 = d.len[0];
      }
    } else {
      xa0 = max(xa0, 0);
      xb0 = min(xb0, gx - 1);
    }
    const int nsy = stencil_n(gy, d.per[1]), nsz = stencil_n(gz, d.per[2]);
    int count = 0;
    auto append = [&](int j) {
      if (count < cap) *wp = j;
      ++count;
      wp += (count & (T - 1)) ? 1 : row - (T - 1);
    };
    for (int rr = 0; rr < 9; ++rr) {
      const int tz = rr / 3, ty = rr % 3;
      if (tz >= nsz || ty >= nsy) continue;
      const int z = stencil_cell(cz, tz, gz, d.per[2]);
      const int y = stencil_cell(cy, ty, gy, d.per[1]);
      if (z < 0 || y < 0) continue;
      const int uz = cz + tz - 1, uy = cy + ty - 1;   // unwrapped row (image shift)
      const double shz = (d.per[2] && !mz) ? (uz < 0 ? -d.len[2] : (uz >= gz ? d.len[2] : 0.0)) : 0.0;
      const double shy = (d.per[1] && !my) ? (uy < 0 ? -d.len[1] : (uy >= gy ? d.len[1] : 0.0)) : 0.0;
      const int crow = d.g0 + (z * gy + y) * gx;
      for (int sg = 0; sg < 2; ++sg) {
        const int xa = sg ? xa1 : xa0, xb = sg ? xb1 : xb0;
        if (xb < xa) continue;
        const double shx = sg ? sh1 : sh0;
        const int j0 = sbase + A.start[crow + xa], j1 = sbase + A.start[crow + xb + 1];
        auto exact = [&](int j) {
          const double4 pj = tq[j];
          double ex = pj.x - pi.x, ey = pj.y - pi.y, ez = pj.z - pi.z;
          ex = mx ? min_image(ex, d.len[0], d.half[0], 1) : ex + shx;
          ey = my ? min_image(ey, d.len[1], d.half[1], 1) : ey + shy;
          ez = mz ? min_image(ez, d.len[2], d.half[2], 1) : ez + shz;
          return dist_sq_exact(ex, ey, ez) < rl2;
        };
        if (SCREEN) {
          const float fx = (float)shx, fy = (float)shy, fz = (float)shz;
          auto test = [&](const float4& cf, int j) {
            const float ex = (cf.x - pf.x) + fx, ey = (cf.y - pf.y) + fy, ez = (cf.z - pf.z) + fz;
            const float r2f = ex * ex + ey * ey + ez * ez;
            bool in = r2f < lo_f;
            if (__builtin_expect(!in && !(r2f >= hi_f), 0)) in = exact(j);   // band (or NaN)
            if (in && j != p) append(j);
          };
          int j = j0;
          for (; j + LIST_BATCH <= j1; j += LIST_BATCH) {   // LIST_BATCH loads in flight
            float4 cf[LIST_BATCH];
#pragma unroll
            for (int u = 0; u < LIST_BATCH; ++u) cf[u] = tqf[j + u];
#pragma unroll
            for (int u = 0; u < LIST_BATCH; ++u) test(cf[u], j + u);
          }
          for (; j < j1; ++j) test(tqf[j], j);
        } else {
          for (int j = j0; j < j1; ++j)
            if (j != p && exact(j)) append(j);
        }
      }
    }
    A.cnt[p] = min(count, cap);
    if (count > cap) atomicMax(&S.overflow, count);
    {
      // copy-back of the sorted state, all loads before the first store
      const double v0 = A.tv[3 * p + 0], v1 = A.tv[3 * p + 1], v2 = A.tv[3 * p + 2];
      const bool cf = A.copy_f;
      const double f0 = cf ? A.tf[3 * p + 0] : 0.0, f1 = cf ? A.tf[3 * p + 1] : 0.0, f2 = cf ? A.tf[3 * p + 2] : 0.0;
      const uint8_t fx = A.tfixed[p];
      const int ide = A.tid[p];
      A.q[p] = pi;
      if (K.shadow) {
        const long long bc = pack_cell(cx, cy, cz);
        A.bcell[p] = bc;
        A.qs[p] = cell_local(S, bc, pi.x, pi.y, pi.z, (float)pi.w);
      }
      A.xref[3 * p + 0] = pi.x;
      A.xref[3 * p + 1] = pi.y;
      A.xref[3 * p + 2] = pi.z;
      A.v[3 * p + 0] = v0;
      A.v[3 * p + 1] = v1;
      A.v[3 * p + 2] = v2;
      if (cf) {
        A.f[3 * p + 0] = f0;
        A.f[3 * p + 1] = f1;
        A.f[3 * p + 2] = f2;
      }
      A.fixed[p] = fx;
      A.id[p] = ide;
    }
  }
}

// Cr-C list {k : |xc_k + ind_z - q_p|^2 < (rc + skin)^2}, atom-major: xidx[p * xcap + n],
// for the atoms of the near list of each rebuilding replica.  One wavefront per near atom
// (stride over those of all rebuilding replicas), its lanes sharing the 27 carbon cells
// around the atom; the passing carbons are compacted in candidate order with a ballot.  Runs
// in blocks bid of nb blocks of BLOCK threads; cand and pre are the block's LDS scratch
// (WAVES_PER_BLOCK x MAXC slots, XL_FLAT_MAXREP + 1 prefixes).  Reads the sorted positions
// (tq) and the near list written by k_sort_gather, so it may run beside the Cr-Cr list build.
constexpr int XL_FLAT_MAXREP = FLAT_MAXREP - 1;   // replicas of the flattened index space
__device__ __forceinline__ void xlist_pass(const Consts& K, const BuildArgs& A, int (*cand_sh)[MAXC], int* pre,
                                           int bid, int nb) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int gw = bid * WAVES_PER_BLOCK + w, nw = nb * WAVES_PER_BLOCK;
  auto one = [&](int r, int item) {   // near atom `item` of replica r, on this wavefront
    RepState& S = A.S[r];
    const RepDesc& d = A.R[r];
    const double iz = S.ind_z;
    const int hbase = A.start[d.h0];
    const int msx = stencil_n(d.hd[0], d.per[0]), msy = stencil_n(d.hd[1], d.per[1]),
              msz = stencil_n(d.hd[2], d.per[2]);
    const int ms = msx * msy * msz;
    const int64_t pa = A.near[d.a0 + item];
    const double4 pi = A.tq[pa];
    int hx, hy, hz;
    c_cell_coords(d, pi.x, pi.y, pi.z, hx, hy, hz);
    int ks = 0, kn = 0;
    if (lane < ms) {
      const int tx = lane % msx, ty = (lane / msx) % msy, tz = lane / (msx * msy);
      const int x = stencil_cell(hx, tx, d.hd[0], d.per[0]);
      const int y = stencil_cell(hy, ty, d.hd[1], d.per[1]);
      const int z = stencil_cell(hz, tz, d.hd[2], d.per[2]);
      if (x >= 0 && y >= 0 && z >= 0) {
        const int hid = d.h0 + (z * d.hd[1] + y) * d.hd[0] + x;
        ks = d.c0 + (A.start[hid] - hbase);
        kn = A.start[hid + 1] - A.start[hid];
      }
    }
    int pref = kn;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int y = __shfl_up(pref, o, WAVE);
      if (lane >= o) pref += y;
    }
    const int total = __shfl(pref, WAVE - 1, WAVE);
    pref -= kn;
    int n = 0;
    for (int w0 = 0; w0 < total; w0 += MAXC) {
      const int lo = max(0, w0 - pref), hi = min(kn, w0 + MAXC - pref);
      for (int e = lo; e < hi; ++e) cand_sh[w][pref + e - w0] = ks + e;   // sorted carbon slots
      wave_sync();
      const int wn = min(MAXC, total - w0);
      for (int k0 = 0; k0 < wn; k0 += WAVE) {
        bool pred = false;
        int k = 0;
        if (k0 + lane < wn) {
          const double4 c4 = A.hsorted[cand_sh[w][k0 + lane]];
          k = (int)__double_as_longlong(c4.w);
          const double ex = min_image(c4.x - pi.x, d.len[0], d.half[0], d.per[0]);
          const double ey = min_image(c4.y - pi.y, d.len[1], d.half[1], d.per[1]);
          const double ez = min_image((c4.z + iz) - pi.z, d.len[2], d.half[2], d.per[2]);
          pred = dist_sq_exact(ex, ey, ez) < K.rxlist_sq;
        }
        const unsigned long long m2 = __ballot(pred);
        const int below = __popcll(m2 & ((1ull << lane) - 1ull));
        if (pred && n + below < K.xcap) A.xidx[pa * K.xcap + n + below] = k;
        n += __popcll(m2);
      }
      wave_sync();
    }
    if (lane == 0) {
      A.xcnt[pa] = min(n, K.xcap);
      if (n > K.xcap) atomicMax(&S.xoverflow, n);
    }
  };
  if (K.nrep <= XL_FLAT_MAXREP) {   // near atoms of all rebuilding replicas as one index space
    const int total = flat_prefix(K.nrep, pre, [&](int r) { return A.S[r].rebuild ? A.S[r].nnear : 0; });
    for (int g = gw; g < total; g += nw) {
      const int r = flat_replica(pre, K.nrep, g);
      one(r, g - pre[r]);
    }
  } else {
    for (int r = 0; r < K.nrep; ++r) {
      if (!A.S[r].rebuild) continue;
      for (int item = gw; item < A.S[r].nnear; item += nw) one(r, item);
    }
  }
}

// Cr-Cr lists with LDS-staged candidates (replicas whose periodic axes all have >= 3 list
// cells).  A work item is a run of cells of one cell row (listed by k_scatter, see
// row_runs), sized so that one pass of a block's threads covers a run's atoms, one center
// per thread; a grid that fills the chip once, each block taking items from a counter.  For each of the nine neighbouring cell rows (z-major, then y) the block
// stages that row's atoms of x-cells x0-1 .. x1+1 -- with the cell seen across a periodic
// x face placed at the end it is seen from -- into LDS as FP32 coordinates relative to the
// grid origin plus the row's image shift, with the slot in the fourth word.  The nine
// staged rows are laid end to end; a center's candidates in one row, x-cells cx-1 .. cx+1,
// are a contiguous window of it, so the candidate order (rows, along x, by slot) is the
// same as in k_list_rows and the lists are identical.  All nine rows are staged with one
// round of loads when they fit LIST_STAGE candidates (else in pieces of that size), so a
// block waits on few dependent memory round trips.  The FP32 screen and its exact FP64
// band are those of k_list_rows.

// Image shift (FP64) of neighbouring row rr (z-major, then y) of the row (cy, cz).
__device__ __forceinline__ void row_shift(int rr, int cy, int cz, int gy, int gz, int per1, int per2,
                                          double len1, double len2, double& shy, double& shz) {
  const int uz = cz + rr / 3 - 1, uy = cy + rr % 3 - 1;
  shz = per2 ? (uz < 0 ? -len2 : (uz >= gz ? len2 : 0.0)) : 0.0;
  shy = per1 ? (uy < 0 ? -len1 : (uy >= gy ? len1 : 0.0)) : 0.0;
}

// Occupancy floor: this kernel hides the latency of its LDS and global reads with waves, so
// its registers are held to what WAVES wavefronts per SIMD can share: MD_LIST_WAVES with one
// block per work item, MD_LIST_WAVES_RESIDENT for resident blocks that take items from a
// counter (measured best on the 8M-atom film: 1.42 against 1.46 ms per rebuild at 7, while
// the 216k-atom film's one block per item does best at 7, 62 against 69 us at 6).
template <int WAVES>
__global__ __launch_bounds__(LIST_BLOCK, WAVES) void k_list_tiles(Consts K, BuildArgs A) {
  if (rebuild_off(A)) return;
  __shared__ float4 sq[LIST_STAGE];        // staged candidates: x, y, z, slot bits
  __shared__ int toff[9][LIST_SEG + 4];    // per row: row-local staged offset of cells x0-1 .. x1+2
  __shared__ int rinfo[9][2];   // per row: row-local end of the main piece; staged total
  __shared__ int4 rslot[9];     // per row: slot of row-local candidate g is g + .x (g < .w),
                                // g + .y (g < end of the main piece), else g + .z
  __shared__ float2 rsh[9];     // per row: FP32 image shift along y and z
  static_assert(LIST_BLOCK == BLOCK && sizeof(sq) >= sizeof(int) * (WAVES_PER_BLOCK * MAXC + XL_FLAT_MAXREP + 1),
                "the Cr-C list blocks run with BLOCK threads in the staging buffer");
  if ((int)blockIdx.x < A.xblocks) {   // leading blocks: the Cr-C lists
    int* scratch = reinterpret_cast<int*>(sq);
    xlist_pass(K, A, reinterpret_cast<int(*)[MAXC]>(scratch), scratch + WAVES_PER_BLOCK * MAXC, blockIdx.x,
               A.xblocks);
    return;
  }
  // the other blocks either stay resident and take work items one at a time from a counter
  // until none is left (zero items in a step without a rebuild), or take one item each
  __shared__ int item_sh;
  const int nitems = uniform(*A.nitems);
  for (int pass = 0;; ++pass) {
  if (!A.persistent && pass > 0) break;
  if (A.persistent) {
    __syncthreads();   // the previous item's LDS tables and stage are no longer read
    if (threadIdx.x == 0) item_sh = atomicAdd(A.next_item, 1);
    __syncthreads();
  }
  const int b = A.persistent ? uniform(item_sh) : (int)blockIdx.x - A.xblocks;
  if (b >= nitems) break;
  const int2 it = A.items[b];
  const int grow = uniform(it.x), sx = uniform(it.y & 0xFFFF), nseg = uniform(it.y >> 16);
  const int r = uniform(A.row_rep[grow]);
  RepState& S = A.S[r];
  const RepDesc& d = A.R[r];
  const int gx = uniform(S.gd[0]), gy = uniform(S.gd[1]), gz = uniform(S.gd[2]);
  // descriptor values used in the loops, held in scalar registers
  const int per0 = uniform(d.per[0]), per1 = uniform(d.per[1]), per2 = uniform(d.per[2]);
  const double len0 = uniform(d.len[0]), len1 = uniform(d.len[1]), len2 = uniform(d.len[2]);
  const int l = grow - uniform(d.rb0);
  const int cy = l % gy, cz = l / gy;
  const int g0 = uniform(d.g0);
  const int crow = g0 + (cz * gy + cy) * gx;
  const int x0 = sx * gx / nseg, x1 = (sx + 1) * gx / nseg - 1;   // this item's cells
  const int sbase = uniform(d.a0 - A.start[g0]);   // sorted slot = sbase + start[cell]
  const int cbeg = sbase + uniform(A.start[crow + x0]);
  const int m = uniform(A.start[crow + x1 + 1]) - (cbeg - sbase);
  if (m == 0) continue;
  const double rl2 = K.rlist_sq;
  const int cap = K.cap, T = K.lt;
  const int64_t row = K.ntot * T;   // entry k of atom p at idx[(k / T) * row + p * T + k % T]
  const double4* __restrict__ tq = A.tq;
  const float4* __restrict__ tqf = A.tqf;
  const bool shadow = K.shadow;   // entries carry relative cells only for the FP32 shadow
  // FP32 screen bounds (see k_list_rows); the staged coordinate already includes the image
  // shift, which the error bound covers
  float lo_f, hi_f;
  {
    const double u = 0x1p-24, R = K.rlist + 1.0;
    const int gg[3] = {gx, gy, gz};
    double err = 4.0 * u * (rl2 + R * R);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double E = gg[a] / S.ginv[a] + 2.0 * R;
      const double eta = u * (3.0 * E + (d.per[a] ? 2.0 * d.len[a] : 0.0) + 3.0 * R);
      err += 2.0 * R * eta + eta * eta;
    }
    const double delta = 2.0 * err + 1e-6;
    lo_f = uniform((float)(rl2 - delta));
    hi_f = uniform((float)(rl2 + delta));
  }
  const unsigned band_bits = __float_as_uint(hi_f - lo_f);   // hi - lo, exact
  const int xa = max(x0 - 1, 0), xb = min(x1 + 1, gx - 1);   // main piece of a staged row
  const bool wl = per0 && x0 == 0, wr = per0 && x1 == gx - 1;   // wrapped end cells
  const int nt = x1 - x0 + 4;
  const bool tiny = gx < 3 || gy < 3 || gz < 3;   // a center may meet its own images
  const float fxl = (float)(-len0), fxr = (float)len0;
  // the first pass's centers: their loads go out before the tables' round of loads
  const int cfirst = min((int)threadIdx.x, m - 1);
  const float4 pf_first = tqf[cbeg + cfirst];
  const double px_first = tq[cbeg + cfirst].x;
  {   // the nine rows' tables: all loads first (one round), then the LDS writes
    constexpr int NIT = (9 * (LIST_SEG + 4) + LIST_BLOCK - 1) / LIST_BLOCK;
    int tv[NIT], ts[NIT], tl[NIT], tm[NIT], tr[NIT], tL[NIT], tR[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      // every load is unconditional and inside row rw (a row of this replica whether or not
      // entry t names one), so that none waits on a branch
      const int t = threadIdx.x + it * LIST_BLOCK;
      const int rr = min(t / nt, 8), k = t % nt;
      const bool in = t < 9 * nt;
      const int z = stencil_cell(cz, rr / 3, gz, per2), y = stencil_cell(cy, rr % 3, gy, per1);
      const bool row_ok = in && z >= 0 && y >= 0;
      const int rw = row_ok ? g0 + (z * gy + y) * gx : g0;
      const int u = min(max(x0 - 1 + k, xa), xb + 1);   // unwrapped cell, clamped
      const int s_a = A.start[rw + xa], s_m = A.start[rw + xb + 1], s_u = A.start[rw + u];
      const int s_0 = A.start[rw], s_1 = A.start[rw + 1];
      const int s_l = A.start[rw + gx - 1], s_r = A.start[rw + gx];
      ts[it] = s_a;
      tl[it] = wl ? s_r - s_l : 0;
      tm[it] = s_m;
      tr[it] = wr ? s_1 - s_0 : 0;
      tv[it] = row_ok ? s_u : (in ? -2 : -1);
      tL[it] = s_l;
      tR[it] = s_0;
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int t = threadIdx.x + it * LIST_BLOCK;
      if (tv[it] == -1) continue;
      const int rr = t / nt, k = t % nt;
      int v = 0;
      if (tv[it] != -2) {
        const int sa = ts[it], nl = tl[it], nm = tm[it] - sa, nr = tr[it];
        const int u = x0 - 1 + k;   // unwrapped cell
        v = u < xa ? 0 : (u <= xb + 1 ? nl + (tv[it] - sa) : nl + nm + nr);
        if (k == 0) {
          rinfo[rr][0] = nl + nm;
          rinfo[rr][1] = nl + nm + nr;
          rslot[rr] = make_int4(sbase + tL[it], sbase + sa - nl, sbase + tR[it] - (nl + nm), nl);
          double shy, shz;
          row_shift(rr, cy, cz, gy, gz, per1, per2, len1, len2, shy, shz);
          rsh[rr] = make_float2((float)shy, (float)shz);
        }
      } else if (k == 0) {
        rinfo[rr][1] = 0;
      }
      toff[rr][k] = v;
    }
  }
  __syncthreads();
  // start of each row in the staged sequence (scalar registers)
  int roff[10];
  roff[0] = 0;
#pragma unroll
  for (int rr = 0; rr < 9; ++rr) roff[rr + 1] = roff[rr] + uniform(rinfo[rr][1]);
  const int tot = roff[9];
  for (int c0 = 0; c0 < m; c0 += LIST_BLOCK) {
    const int c = c0 + threadIdx.x;
    const bool live = c < m;
    const int p = cbeg + (live ? c : 0);
    const float4 pf = c0 == 0 ? pf_first : tqf[p];
    const int cx = cell_coord(c0 == 0 ? px_first : tq[p].x, uniform(S.glo[0]), uniform(S.ginv[0]), gx);
    int count = 0;
    int* __restrict__ wp = A.idx + (int64_t)p * T;
    auto append = [&](int j) {
      if (count < cap) *wp = j;
      ++count;
      wp += (count & (T - 1)) ? 1 : row - (T - 1);
    };
    for (int G0 = 0; G0 < tot; G0 += LIST_STAGE) {   // uniform over the block
      const int nch = min(LIST_STAGE, tot - G0);
      if (c0 > 0 || G0 > 0) __syncthreads();   // the previous piece is no longer read
      {
        // slot and image shift of each staged position into LDS at once, the coordinate
        // loads in flight meanwhile; then the coordinates are added in
        float3 pc[LIST_PT];
#pragma unroll
        for (int u = 0; u < LIST_PT; ++u) {
          const int s = threadIdx.x + u * LIST_BLOCK;
          if (s < nch) {
            const int G = G0 + s;
            int rr = 0, g = G;   // the row of staged position G and its row-local index
#pragma unroll
            for (int k = 1; k < 9; ++k)
              if (G >= roff[k]) {
                rr = k;
                g = G - roff[k];
              }
            const int4 rs = rslot[rr];
            const int nlm = rinfo[rr][0];
            const int j = g + (g < rs.w ? rs.x : (g < nlm ? rs.y : rs.z));
            const float4* c4 = tqf + j;
            pc[u] = make_float3(c4->x, c4->y, c4->z);
            const float2 yz = rsh[rr];
            sq[s] = make_float4(g < rs.w ? fxl : (g < nlm ? 0.0f : fxr), yz.x, yz.y, __int_as_float(j));
          }
        }
#pragma unroll
        for (int u = 0; u < LIST_PT; ++u) {
          const int s = threadIdx.x + u * LIST_BLOCK;
          if (s < nch) {
            float4 e = sq[s];
            e.x += pc[u].x;
            e.y += pc[u].y;
            e.z += pc[u].z;
            sq[s] = e;
          }
        }
      }
      __syncthreads();
      if (live) {
        // the center's staged position (middle row, main piece), relative to this piece
        const int s_self = roff[4] + (p - rslot[4].y) - G0;
#pragma unroll 1
        for (int rr = 0; rr < 9; ++rr) {   // this center's window in each row
          const int* to = toff[rr] + (cx - x0);
          const int w0 = roff[rr] + to[0], w1 = roff[rr] + to[3];
          const int e0 = max(w0, G0) - G0, e1 = min(w1, G0 + nch) - G0;
          if (e0 >= e1) continue;
          const int b1 = roff[rr] + to[1], b2 = roff[rr] + to[2];
          const int rcode = 9 * (rr / 3) + 3 * (rr % 3);
          // exact FP64 test of staged candidate s (in the band, or NaN in the single-candidate
          // loop)
          auto exact = [&](int s) {
            double shy, shz;
            row_shift(rr, cy, cz, gy, gz, per1, per2, len1, len2, shy, shz);
            const int g = G0 + s - roff[rr];
            const double shx = g < rslot[rr].w ? -len0 : (g < rinfo[rr][0] ? 0.0 : len0);
            const double4 pi = tq[p], pj4 = tq[__float_as_int(sq[s].w)];
            return dist_sq_exact((pj4.x - pi.x) + shx, (pj4.y - pi.y) + shy, (pj4.z - pi.z) + shz) < rl2;
          };
          // The passing candidates of up to 32 consecutive staged positions from sb on are
          // gathered as bits of one mask and appended in order together: the appending
          // loop then runs as often as the most passing candidates of a lane in those 32,
          // not once per group for the lane with the most in each group.
          // With three or more cells along every axis the center occurs once among the
          // staged positions, in the middle row: its bit is cleared from the mask, and
          // while all of a mask's entries fit under the capacity they are stored with no
          // further test.  Smaller grids, and a lane about to overflow, test every entry.
          auto flush = [&](unsigned acc, int sb) {
            if (!tiny && rr == 4) {
              const unsigned d = (unsigned)(s_self - sb);
              if (d < 32u) acc &= ~(1u << d);
            }
            if (!tiny && count + __builtin_popcount(acc) <= cap) {
              for (; acc; acc &= acc - 1) {
                const int su = sb + __builtin_ctz(acc);
                const int j = __float_as_int(sq[su].w);
                *wp = shadow ? j | ((rcode + (su + G0 >= b1) + (su + G0 >= b2)) << LIST_IDX_BITS) : j;
                ++count;
                wp += (count & (T - 1)) ? 1 : row - (T - 1);
              }
            } else {
              for (; acc; acc &= acc - 1) {
                const int su = sb + __builtin_ctz(acc);
                const int j = __float_as_int(sq[su].w);
                if (j != p) append(shadow ? j | ((rcode + (su + G0 >= b1) + (su + G0 >= b2)) << LIST_IDX_BITS) : j);
              }
            }
          };
          unsigned acc = 0;
          int sb = e0;
          // LIST_GROUP candidates at a time: the FP32 screen gives their in bits, and the
          // rare candidates in the band get the exact test
          int s = e0;
          for (; s + LIST_GROUP <= e1; s += LIST_GROUP) {
            if (s - sb > 32 - LIST_GROUP) {   // the same step for every lane of the loop
              flush(acc, sb);
              acc = 0;
              sb = s;
            }
            // d = |r2| - lo: in when negative (its sign bit); in the band when
            // 0 <= d < hi - lo, which compares as unsigned bit patterns (both differences
            // are exact there, by Sterbenz's lemma, and d >= lo beyond 2 lo).  The absolute
            // value clears the sign of a NaN, which then falls in neither: out, as the
            // exact test would decide.
            unsigned in = 0, dmin = ~0u;
            float d[LIST_GROUP];
#pragma unroll
            for (int u = 0; u < LIST_GROUP; ++u) {
              const float4 cf = sq[s + u];
              const float ex = cf.x - pf.x, ey = cf.y - pf.y, ez = cf.z - pf.z;
              d[u] = fabsf(ex * ex + ey * ey + ez * ez) - lo_f;
              in |= (__float_as_uint(d[u]) >> 31) << u;
              dmin = min(dmin, __float_as_uint(d[u]));   // one test for the whole group
            }
            if (__builtin_expect(dmin < band_bits, 0)) {
#pragma unroll
              for (int u = 0; u < LIST_GROUP; ++u)
                if (__float_as_uint(d[u]) < band_bits && exact(s + u)) in |= 1u << u;
            }
            acc |= in << (s - sb);
          }
          for (; s < e1; ++s) {
            if (s - sb > 31) {
              flush(acc, sb);
              acc = 0;
              sb = s;
            }
            const float4 cf = sq[s];
            const float ex = cf.x - pf.x, ey = cf.y - pf.y, ez = cf.z - pf.z;
            const float r2f = ex * ex + ey * ey + ez * ez;
            bool ok = r2f < lo_f;
            if (__builtin_expect(!ok && !(r2f >= hi_f), 0)) ok = exact(s);
            acc |= (ok ? 1u : 0u) << (s - sb);
          }
          flush(acc, sb);
        }
      }
    }
    if (live) {
      // all loads before the first store (a store could alias a later load, which would
      // then wait for it)
      const double4 pi = tq[p];
      const double v0 = A.tv[3 * p + 0], v1 = A.tv[3 * p + 1], v2 = A.tv[3 * p + 2];
      const bool cf = A.copy_f;
      const double f0 = cf ? A.tf[3 * p + 0] : 0.0, f1 = cf ? A.tf[3 * p + 1] : 0.0, f2 = cf ? A.tf[3 * p + 2] : 0.0;
      const uint8_t fx = A.tfixed[p];
      const int ide = A.tid[p];
      A.cnt[p] = min(count, cap);
      if (count > cap) atomicMax(&S.overflow, count);
      A.q[p] = pi;
      if (K.shadow) {
        const long long bc = pack_cell(cx, cy, cz);
        A.bcell[p] = bc;
        A.qs[p] = cell_local(S, bc, pi.x, pi.y, pi.z, (float)pi.w);
      }
      A.xref[3 * p + 0] = pi.x;
      A.xref[3 * p + 1] = pi.y;
      A.xref[3 * p + 2] = pi.z;
      A.v[3 * p + 0] = v0;
      A.v[3 * p + 1] = v1;
      A.v[3 * p + 2] = v2;
      if (cf) {
        A.f[3 * p + 0] = f0;
        A.f[3 * p + 1] = f1;
        A.f[3 * p + 2] = f2;
      }
      A.fixed[p] = fx;
      A.id[p] = ide;
    }
  }
  }
}

__global__ __launch_bounds__(BLOCK) void k_xlist(Consts K, BuildArgs A) {
  if (rebuild_off(A)) return;
  __shared__ int cand_sh[WAVES_PER_BLOCK][MAXC];
  __shared__ int pre[XL_FLAT_MAXREP + 1];
  xlist_pass(K, A, cand_sh, pre, blockIdx.x, gridDim.x);
}

// Section 2.6's inner list, refilled every step from the outer (Verlet) list: atom i's outer
// entries whose pair is closer than the largest Cr-Cr cutoff at the current positions
// (minimum image, the list build's exact FP64 predicate), in their outer-list order and in
// the outer list's layout and entry format.  INNER_G lanes share an atom and test INNER_G
// consecutive outer entries at a time (the next ones' indices loaded while the current
// positions are gathered); a ballot over the group gives each kept entry its place, so the
// order is the outer list's.  One block per 256 / INNER_G atoms.
#ifndef MD_INNER_G
#define MD_INNER_G 16   // 4: 978 us on the 216k-atom film (paper's form); 8: 823; 16: 790
#endif
constexpr int INNER_G = MD_INNER_G;

// FP32 positions relative to the replica's grid origin at the current positions, for the
// inner-list screen (one lane per atom slot; the list build's scratch copy, free between
// builds).
__global__ __launch_bounds__(BLOCK) void k_inner_pos(const RepDesc* __restrict__ R, const RepState* __restrict__ S,
                                                     const int* __restrict__ tile_rep, const double4* __restrict__ q,
                                                     float4* __restrict__ qf) {
  static_assert(TILE == BLOCK, "one block per tile");
  const int r = tile_rep[blockIdx.x];
  const int64_t i = (int64_t)blockIdx.x * TILE + threadIdx.x;
  if (i >= (int64_t)R[r].a0 + R[r].n) return;
  const double4 p = q[i];
  const RepState& s = S[r];
  qf[i] = make_float4((float)(p.x - s.glo[0]), (float)(p.y - s.glo[1]), (float)(p.z - s.glo[2]), 0.0f);
}

__device__ __forceinline__ float min_image_f(float d, float len, float half, int per) {
  float s = (per && d > half) ? -len : 0.0f;
  s = (per && d < -half) ? len : s;
  return d + s;
}

// The screen: the FP32 squared separation from those positions decides outside a band
// around r*^2 that covers its error (the list build's bound, with R = r* + 1 and positions
// within R of the grid); the band gets the exact FP64 test.  On a replica with a periodic
// length under 2 R + 1 the FP32 minimum image could pick the other image of a pair inside
// r*, and every entry gets the exact test.
__global__ __launch_bounds__(BLOCK) void k_inner_list(Consts K, const RepDesc* __restrict__ R,
                                                      RepState* __restrict__ S, const int* __restrict__ tile_rep,
                                                      const double4* __restrict__ q, const float4* __restrict__ qf,
                                                      const int* __restrict__ idx, const int* __restrict__ cnt,
                                                      int* __restrict__ iidx, int* __restrict__ icnt) {
  static_assert(WAVE % INNER_G == 0 && INNER_G < 32, "a lane group lies in one wavefront, its mask in 32 bits");
  constexpr int APB = BLOCK / INNER_G;   // atoms per block
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int tile = lb / INNER_G;
  const int r = tile_rep[tile];
  const RepDesc& d = R[r];
  const int sub = threadIdx.x % INNER_G;
  const int64_t i = (int64_t)tile * TILE + (lb % INNER_G) * APB + threadIdx.x / INNER_G;
  const bool live = i < (int64_t)d.a0 + d.n;
  const double4 pi = live ? q[i] : make_double4(0.0, 0.0, 0.0, 0.0);
  const float4 pif = live ? qf[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const bool img = wave_near_face(d, live, pi.x, pi.y, pi.z, K.rlist + 2.0 * K.half_skin);
  // every lane takes part in the ballots (atoms past the replica with an empty list)
  const int n = live ? cnt[i] : 0;
  int nw = n;   // the wavefront's longest list
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) nw = max(nw, __shfl_xor(nw, o, WAVE));
  const int T = K.lt, sh = K.lt_shift;
  const unsigned stride = (unsigned)K.ntot * T, base = (unsigned)(live ? i : 0) * T;
  // word offset of entry k of atom i (32-bit: the lists hold fewer than 2^31 words)
  auto at_k = [&](int k) { return ((unsigned)k >> sh) * stride + base + (unsigned)(k & (T - 1)); };
  const int icap = K.icap;
  const double rc2 = K.icut_sq;
  float lo_f = -1.0f, hi_f = INFINITY;   // (everything in the band)
  {
    const RepState& s = S[r];
    const double u = 0x1p-24, Rr = sqrt(rc2) + 1.0;
    double err = 4.0 * u * (rc2 + Rr * Rr);
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double E = s.gd[a] / s.ginv[a] + 2.0 * Rr;
      const double eta = u * (3.0 * E + (d.per[a] ? 2.0 * d.len[a] : 0.0) + 3.0 * Rr);
      err += 2.0 * Rr * eta + eta * eta;
      ok = ok && !(d.per[a] && d.len[a] <= 2.0 * Rr + 1.0);
    }
    if (ok) {
      const double delta = 2.0 * err + 1e-6;
      lo_f = (float)(rc2 - delta);
      hi_f = (float)(rc2 + delta);
    }
  }
  const float len0 = (float)d.len[0], len1 = (float)d.len[1], len2 = (float)d.len[2];
  const float hf0 = (float)d.half[0], hf1 = (float)d.half[1], hf2 = (float)d.half[2];
  const int gshift = (int)(threadIdx.x % WAVE) - sub;   // the group's first lane
  const unsigned below = (1u << sub) - 1u;
  int c = 0;        // entries kept so far
  int e = sub < n ? idx[at_k(sub)] : 0;   // (slot 0 stands in for an entry past the list)
  for (int m0 = 0; m0 < nw; m0 += INNER_G) {
    const int k = m0 + sub;
    const float4 pjf = qf[list_slot(e)];
    const int en = k + INNER_G < n ? idx[at_k(k + INNER_G)] : 0;
    float fx = pjf.x - pif.x, fy = pjf.y - pif.y, fz = pjf.z - pif.z;
    if (img) {
      fx = min_image_f(fx, len0, hf0, d.per[0]);
      fy = min_image_f(fy, len1, hf1, d.per[1]);
      fz = min_image_f(fz, len2, hf2, d.per[2]);
    }
    const float r2f = fx * fx + fy * fy + fz * fz;
    bool keep = r2f < lo_f;
    if (k < n && !keep && !(r2f >= hi_f)) {   // the band (or NaN): the exact test
      const double4 pj = q[list_slot(e)];
      double ex = pj.x - pi.x, ey = pj.y - pi.y, ez = pj.z - pi.z;
      if (img) {
        ex = min_image(ex, d.len[0], d.half[0], d.per[0]);
        ey = min_image(ey, d.len[1], d.half[1], d.per[1]);
        ez = min_image(ez, d.len[2], d.half[2], d.per[2]);
      }
      keep = dist_sq_exact(ex, ey, ez) < rc2;
    }
    keep = keep && k < n;
    const unsigned gm = (unsigned)(__ballot(keep) >> gshift) & ((1u << INNER_G) - 1u);
    if (keep) {
      const int j = c + __popc(gm & below);
      if (j < icap) iidx[at_k(j)] = e;
    }
    c += __popc(gm);
    e = en;
  }
  if (live && sub == 0) {
    icnt[i] = min(c, icap);
    if (c > icap) atomicMax(&S[r].ioverflow, c);
  }
}

}  // namespace md
