// HIP kernels of the MD step for CDNA4 (gfx950).  Included by md_api.hip.
//
//   k_kick_drift   Tasks 2 + 3 (Eqs. A11-A12) and the per-tile displacement maxima
//   k_decide       skin test of Section 2.6 -> per-replica rebuild flag
//   k_rebuild      Task 1: wrap, bin, sort by (cell, id), permute, build lists (persistent)
//   k_density      Task 4a: rho_i, F'(rho_i)
//   k_force        Task 4b: Eq. (1) [+ Task 4c Morse] [+ Task 5 kick]
//   k_morse        Task 4c on its own
//   k_kick         Task 5 on its own
//   k_kinetic / k_reduce   Task 4d: energies, virial, load (fixed-order FP64 reductions)
//
// Every force-path kernel is owner-computes: one lane per atom gathers over that atom's
// full neighbour list and writes only that atom, so no atomics touch forces or densities.
#pragma once

#include "md_device.hpp"

namespace md {

// Per-tile blocks: block b of an atom-parallel launch covers tile t = xcd_block(b) (256 atoms).
struct TileCtx {
  int tile, r;
  int64_t i;        // atom slot of this thread
  bool live;        // slot holds an atom (not padding)
};

__device__ __forceinline__ TileCtx tile_ctx(const int* tile_rep, const RepDesc* R) {
  TileCtx c;
  c.tile = xcd_block(blockIdx.x, gridDim.x);
  c.r = tile_rep[c.tile];
  c.i = (int64_t)c.tile * TILE + threadIdx.x;
  const RepDesc& d = R[c.r];
  c.live = c.i < (int64_t)d.a0 + d.n;
  return c;
}

// ------------------------------------------------------------------------------------
// Tasks 2 + 3
// ------------------------------------------------------------------------------------
// v(t + dt/2) = v + a dt / 2 and r(t + dt) = r + v(t + dt/2) dt (algebraically Eq. A11) for
// mobile atoms; the indenter moves by v_ind dt.  Writes max |r - r_ref|^2 of each tile.
__global__ __launch_bounds__(BLOCK) void k_kick_drift(Consts K, const RepDesc* __restrict__ R,
                                                      RepState* __restrict__ S,
                                                      const int* __restrict__ tile_rep,
                                                      double4* __restrict__ q, double* __restrict__ v,
                                                      const double* __restrict__ f,
                                                      const uint8_t* __restrict__ fixed,
                                                      const double* __restrict__ xref,
                                                      double* __restrict__ dmax_tile) {
  TileCtx c = tile_ctx(tile_rep, R);
  double d2 = 0.0;
  if (c.live) {
    const int64_t i = c.i;
    double4 p = q[i];
    if (!fixed[i]) {
      const double h = 0.5 * K.dt * K.acc;
      double vx = v[3 * i + 0] + h * f[3 * i + 0];
      double vy = v[3 * i + 1] + h * f[3 * i + 1];
      double vz = v[3 * i + 2] + h * f[3 * i + 2];
      p.x += vx * K.dt;
      p.y += vy * K.dt;
      p.z += vz * K.dt;
      v[3 * i + 0] = vx;
      v[3 * i + 1] = vy;
      v[3 * i + 2] = vz;
      q[i] = p;
    }
    double ex = p.x - xref[3 * i + 0];
    double ey = p.y - xref[3 * i + 1];
    double ez = p.z - xref[3 * i + 2];
    d2 = (ex * ex + ey * ey) + ez * ez;
    if (!(d2 == d2)) d2 = INFINITY;   // NaN positions force a rebuild (and get flagged there)
  }
  d2 = block_max<BLOCK>(d2);
  if (threadIdx.x == 0) {
    dmax_tile[c.tile] = d2;
    if (c.tile == R[c.r].t0) S[c.r].ind_z += K.v_ind * K.dt;   // Task 2, once per replica
  }
}

// ------------------------------------------------------------------------------------
// Task 1a: skin test.  One block per replica.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_decide(Consts K, const RepDesc* __restrict__ R,
                                                  RepState* __restrict__ S,
                                                  const double* __restrict__ dmax_tile, int force,
                                                  int* __restrict__ any) {
  const int r = blockIdx.x;
  const RepDesc& d = R[r];
  double m = 0.0;
  for (int t = threadIdx.x; t < d.nt; t += BLOCK) m = fmax(m, dmax_tile[d.t0 + t]);
  m = block_max<BLOCK>(m);
  if (threadIdx.x == 0) {
    RepState& s = S[r];
    int need = force || (m > K.half_skin_sq) || (fabs(s.ind_z - s.ind_z_ref) > K.half_skin);
    s.rebuild = need;
    if (need) {
      s.czmin = ordered_bits(INFINITY);
      s.czmax = ordered_bits(-INFINITY);
      atomicOr(any, 1);
    }
  }
}

// ------------------------------------------------------------------------------------
// Task 1b-1c: the rebuild, one persistent launch with grid-wide waits between phases.
// ------------------------------------------------------------------------------------
struct RebuildArgs {
  const RepDesc* R;
  RepState* S;
  const int* tile_rep;
  int* any;               // set by k_decide, cleared at the end of a rebuild
  double4* q;
  double* v;
  double* f;
  uint8_t* fixed;
  int* id;
  const double* xc;
  double* xref;
  double* dmax_tile;
  // scratch
  int* cellid;            // [ntot] cell of each atom (global index)
  int* perm;              // [ntot]
  double4* tq;
  double* tv;
  double* tf;
  uint8_t* tfixed;
  int* tid;
  int* count;             // [ncell_all]: Cr cells then carbon cells
  int* start;             // [ncell_all + 1]
  int* hcell;             // [c_total] carbon cell (global index)
  int* hlist;             // [c_total] carbon indices sorted by cell
  int* bsum;              // [grid]
  unsigned* bar;          // [2] grid barrier: count, generation
  // lists
  int* idx;
  int* cnt;
  int* xidx;
  int* xcnt;
  int ncell_all;          // Cr cells + carbon cells of all replicas
  int ncell_cr;           // Cr cells of all replicas
  int ntiles;
  int c_total;
};

constexpr int MAXREP = 1024;

// Grid-wide wait.  All blocks of the launch are resident (the grid is sized from the
// occupancy of this kernel), so every block reaches every wait; the spin is bounded all
// the same and a timeout is flagged instead of hanging.
__device__ void grid_sync(unsigned* bar, int* timeout_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    unsigned arrived = atomicAdd(&bar[0], 1u);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(4);
        if (++spins > (1l << 22)) {
          *timeout_flag = 1;
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
}

__device__ __forceinline__ int cr_cell_of(const RepDesc& d, double x, double y, double z) {
  int cx = cell_coord(x, d.lo[0], d.ginv[0], d.gd[0]);
  int cy = cell_coord(y, d.lo[1], d.ginv[1], d.gd[1]);
  int cz = cell_coord(z, d.lo[2], d.ginv[2], d.gd[2]);
  return d.g0 + (cz * d.gd[1] + cy) * d.gd[0] + cx;
}

// Coordinate folded into [lo, lo + len) on a periodic axis (for binning carbon atoms).
__device__ __forceinline__ double fold(double x, double lo, double len, int per) {
  if (!per) return x;
  return x - len * floor((x - lo) / len);
}

__device__ __forceinline__ int c_cell_of(const RepDesc& d, double x, double y, double z) {
  x = fold(x, d.lo[0], d.len[0], d.per[0]);
  y = fold(y, d.lo[1], d.len[1], d.per[1]);
  z = fold(z, d.lo[2], d.len[2], d.per[2]);
  int cx = cell_coord(x, d.lo[0], d.hinv[0], d.hd[0]);
  int cy = cell_coord(y, d.lo[1], d.hinv[1], d.hd[1]);
  int cz = cell_coord(z, d.lo[2], d.hinv[2], d.hd[2]);
  return d.h0 + (cz * d.hd[1] + cy) * d.hd[0] + cx;
}

// Block-wide exclusive scan of one int per thread; returns the prefix, *total = block sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
  __shared__ int sh[BLOCK / WAVE];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  int x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) sh[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BLOCK / WAVE; ++i) {
    if (i < w) off += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ __launch_bounds__(BLOCK) void k_rebuild(Consts K, RebuildArgs A) {
  __shared__ int reb[MAXREP];
  if (*(volatile int*)A.any == 0) return;   // the skin test passed everywhere: nothing to do
  const int nrep = K.nrep;
  for (int r = threadIdx.x; r < nrep; r += BLOCK) reb[r] = A.S[r].rebuild;
  __syncthreads();
  const int G = gridDim.x;
  const int gtid = blockIdx.x * BLOCK + threadIdx.x;
  const int gthreads = G * BLOCK;
  int* tflag = &A.S[0].sync_timeout;

  // ---- phase 1: wrap positions into the box, bin atoms and carbons, carbon z extent
  for (int t = blockIdx.x; t < A.ntiles; t += G) {
    const int r = A.tile_rep[t];
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const int64_t i = (int64_t)t * TILE + threadIdx.x;
    if (i >= (int64_t)d.a0 + d.n) continue;
    double4 p = A.q[i];
    double xyz[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!d.per[a]) continue;
      double hi = d.lo[a] + d.len[a];
      if (xyz[a] >= hi)
        xyz[a] -= d.len[a];
      else if (xyz[a] < d.lo[a])
        xyz[a] += d.len[a];
    }
    p.x = xyz[0];
    p.y = xyz[1];
    p.z = xyz[2];
    A.q[i] = p;
    int cid = cr_cell_of(d, p.x, p.y, p.z);
    A.cellid[i] = cid;
    atomicAdd(&A.count[cid], 1);
  }
  for (int r = 0; r < nrep; ++r) {
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const double iz = A.S[r].ind_z;
    double zmin = INFINITY, zmax = -INFINITY;
    for (int k = gtid; k < d.nc; k += gthreads) {
      const int kk = d.c0 + k;
      double z = A.xc[3 * kk + 2] + iz;
      int hid = c_cell_of(d, A.xc[3 * kk + 0], A.xc[3 * kk + 1], z);
      A.hcell[kk] = hid;
      atomicAdd(&A.count[hid], 1);
      zmin = fmin(zmin, z);
      zmax = fmax(zmax, z);
    }
    zmin = -block_max<BLOCK>(-zmin);
    zmax = block_max<BLOCK>(zmax);
    if (threadIdx.x == 0 && d.nc > 0 && zmin <= zmax) {
      atomicMin(&A.S[r].czmin, ordered_bits(zmin));
      atomicMax(&A.S[r].czmax, ordered_bits(zmax));
    }
  }
  grid_sync(A.bar, tflag);

  // ---- phase 2: exclusive scan of all cell counts (three sub-phases)
  const int M = A.ncell_all;
  const int chunk = (M + G - 1) / G;
  const int cbeg = min(blockIdx.x * chunk, M), cend = min(cbeg + chunk, M);
  {
    int s = 0;
    for (int c = cbeg + threadIdx.x; c < cend; c += BLOCK) s += A.count[c];
    int tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) A.bsum[blockIdx.x] = tot;
  }
  grid_sync(A.bar, tflag);
  if (blockIdx.x == 0) {
    int carry = 0;
    for (int b0 = 0; b0 < G; b0 += BLOCK) {
      int b = b0 + threadIdx.x;
      int v = b < G ? A.bsum[b] : 0;
      int tot;
      int ex = block_exclusive_scan(v, &tot);
      if (b < G) A.bsum[b] = carry + ex;
      carry += tot;
    }
    if (threadIdx.x == 0) A.start[M] = carry;
  }
  grid_sync(A.bar, tflag);
  {
    int carry = A.bsum[blockIdx.x];
    for (int c0 = cbeg; c0 < cend; c0 += BLOCK) {
      int c = c0 + threadIdx.x;
      int v = c < cend ? A.count[c] : 0;
      int tot;
      int ex = block_exclusive_scan(v, &tot);
      if (c < cend) {
        A.start[c] = carry + ex;
        A.count[c] = 0;   // reused as the fill cursor of phase 3
      }
      carry += tot;
    }
  }
  grid_sync(A.bar, tflag);

  // ---- phase 3: scatter atom slots and carbon indices into their cells
  for (int t = blockIdx.x; t < A.ntiles; t += G) {
    const int r = A.tile_rep[t];
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const int64_t i = (int64_t)t * TILE + threadIdx.x;
    if (i >= (int64_t)d.a0 + d.n) continue;
    const int cid = A.cellid[i];
    const int slot = atomicAdd(&A.count[cid], 1);
    A.perm[d.a0 + (A.start[cid] - A.start[d.g0]) + slot] = (int)i;
  }
  for (int r = 0; r < nrep; ++r) {
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    for (int k = gtid; k < d.nc; k += gthreads) {
      const int kk = d.c0 + k;
      const int hid = A.hcell[kk];
      const int slot = atomicAdd(&A.count[hid], 1);
      A.hlist[d.c0 + (A.start[hid] - A.start[d.h0]) + slot] = kk;
    }
  }
  grid_sync(A.bar, tflag);

  // ---- phase 4: order each cell by atom id (carbons by index): the order is canonical
  for (int r = 0; r < nrep; ++r) {
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const int ncr = d.gd[0] * d.gd[1] * d.gd[2];
    const int nch = d.hd[0] * d.hd[1] * d.hd[2];
    for (int c = gtid; c < ncr + nch; c += gthreads) {
      const bool crc = c < ncr;
      const int cid = crc ? d.g0 + c : d.h0 + (c - ncr);
      const int base = crc ? d.a0 + (A.start[cid] - A.start[d.g0]) : d.c0 + (A.start[cid] - A.start[d.h0]);
      const int m = A.start[cid + 1] - A.start[cid];
      int* seg = crc ? A.perm + base : A.hlist + base;
      for (int a = 1; a < m; ++a) {
        int e = seg[a];
        int key = crc ? A.id[e] : e;
        int b = a - 1;
        while (b >= 0 && (crc ? A.id[seg[b]] : seg[b]) > key) {
          seg[b + 1] = seg[b];
          --b;
        }
        seg[b + 1] = e;
      }
    }
  }
  grid_sync(A.bar, tflag);

  // ---- phase 5: gather the atom state into sorted order
  for (int t = blockIdx.x; t < A.ntiles; t += G) {
    const int r = A.tile_rep[t];
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const int64_t p = (int64_t)t * TILE + threadIdx.x;
    if (p >= (int64_t)d.a0 + d.n) continue;
    const int i = A.perm[p];
    A.tq[p] = A.q[i];
    A.tv[3 * p + 0] = A.v[3 * i + 0];
    A.tv[3 * p + 1] = A.v[3 * i + 1];
    A.tv[3 * p + 2] = A.v[3 * i + 2];
    A.tf[3 * p + 0] = A.f[3 * i + 0];
    A.tf[3 * p + 1] = A.f[3 * i + 1];
    A.tf[3 * p + 2] = A.f[3 * i + 2];
    A.tfixed[p] = A.fixed[i];
    A.tid[p] = A.id[i];
  }
  grid_sync(A.bar, tflag);

  // ---- phase 6: copy back; reference positions for the skin test
  for (int t = blockIdx.x; t < A.ntiles; t += G) {
    const int r = A.tile_rep[t];
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const int64_t p = (int64_t)t * TILE + threadIdx.x;
    if (threadIdx.x == 0) A.dmax_tile[t] = 0.0;
    if (p >= (int64_t)d.a0 + d.n) continue;
    const double4 x = A.tq[p];
    A.q[p] = x;
    A.xref[3 * p + 0] = x.x;
    A.xref[3 * p + 1] = x.y;
    A.xref[3 * p + 2] = x.z;
    A.v[3 * p + 0] = A.tv[3 * p + 0];
    A.v[3 * p + 1] = A.tv[3 * p + 1];
    A.v[3 * p + 2] = A.tv[3 * p + 2];
    A.f[3 * p + 0] = A.tf[3 * p + 0];
    A.f[3 * p + 1] = A.tf[3 * p + 1];
    A.f[3 * p + 2] = A.tf[3 * p + 2];
    A.fixed[p] = A.tfixed[p];
    A.id[p] = A.tid[p];
  }
  grid_sync(A.bar, tflag);

  // ---- phase 7: Verlet lists (full Cr-Cr list; Cr-C list) from the 27 surrounding cells
  const int64_t ntot = K.ntot;
  for (int t = blockIdx.x; t < A.ntiles; t += G) {
    const int r = A.tile_rep[t];
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const int64_t i = (int64_t)t * TILE + threadIdx.x;
    if (i >= (int64_t)d.a0 + d.n) continue;
    const double4 pi = A.q[i];
    const int cx = cell_coord(pi.x, d.lo[0], d.ginv[0], d.gd[0]);
    const int cy = cell_coord(pi.y, d.lo[1], d.ginv[1], d.gd[1]);
    const int cz = cell_coord(pi.z, d.lo[2], d.ginv[2], d.gd[2]);
    const int sbase = A.start[d.g0];
    int n = 0;
    const int nsz = stencil_n(d.gd[2], d.per[2]), nsy = stencil_n(d.gd[1], d.per[1]),
              nsx = stencil_n(d.gd[0], d.per[0]);
    for (int tz = 0; tz < nsz; ++tz) {
      const int z = stencil_cell(cz, tz, d.gd[2], d.per[2]);
      if (z < 0) continue;
      for (int ty = 0; ty < nsy; ++ty) {
        const int y = stencil_cell(cy, ty, d.gd[1], d.per[1]);
        if (y < 0) continue;
        for (int tx = 0; tx < nsx; ++tx) {
          const int x = stencil_cell(cx, tx, d.gd[0], d.per[0]);
          if (x < 0) continue;
          const int cid = d.g0 + (z * d.gd[1] + y) * d.gd[0] + x;
          const int jb = d.a0 + (A.start[cid] - sbase);
          const int je = d.a0 + (A.start[cid + 1] - sbase);
          for (int j = jb; j < je; ++j) {
            if (j == i) continue;
            const double4 pj = A.q[j];
            double ex = min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]);
            double ey = min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]);
            double ez = min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]);
            if (dist_sq_exact(ex, ey, ez) < K.rlist_sq) {
              if (n < K.cap) A.idx[(int64_t)n * ntot + i] = j;
              ++n;
            }
          }
        }
      }
    }
    if (n > K.cap) atomicMax(&A.S[r].overflow, n);
    A.cnt[i] = min(n, K.cap);

    // Cr-C list
    int nx = 0;
    if (d.nc > 0) {
      const double iz = A.S[r].ind_z;
      const double zlo = from_ordered_bits(A.S[r].czmin), zhi = from_ordered_bits(A.S[r].czmax);
      const double rx = sqrt(K.rxlist_sq);
      const bool near = d.per[2] || (pi.z >= zlo - rx && pi.z <= zhi + rx);
      if (near) {
        const int hbase = A.start[d.h0];
        double fx = fold(pi.x, d.lo[0], d.len[0], d.per[0]);
        double fy = fold(pi.y, d.lo[1], d.len[1], d.per[1]);
        double fz = fold(pi.z, d.lo[2], d.len[2], d.per[2]);
        const int hx = cell_coord(fx, d.lo[0], d.hinv[0], d.hd[0]);
        const int hy = cell_coord(fy, d.lo[1], d.hinv[1], d.hd[1]);
        const int hz = cell_coord(fz, d.lo[2], d.hinv[2], d.hd[2]);
        const int msz = stencil_n(d.hd[2], d.per[2]), msy = stencil_n(d.hd[1], d.per[1]),
                  msx = stencil_n(d.hd[0], d.per[0]);
        for (int tz = 0; tz < msz; ++tz) {
          const int z = stencil_cell(hz, tz, d.hd[2], d.per[2]);
          if (z < 0) continue;
          for (int ty = 0; ty < msy; ++ty) {
            const int y = stencil_cell(hy, ty, d.hd[1], d.per[1]);
            if (y < 0) continue;
            for (int tx = 0; tx < msx; ++tx) {
              const int x = stencil_cell(hx, tx, d.hd[0], d.per[0]);
              if (x < 0) continue;
              const int hid = d.h0 + (z * d.hd[1] + y) * d.hd[0] + x;
              const int kb = d.c0 + (A.start[hid] - hbase);
              const int ke = d.c0 + (A.start[hid + 1] - hbase);
              for (int s = kb; s < ke; ++s) {
                const int k = A.hlist[s];
                double ex = min_image(A.xc[3 * k + 0] - pi.x, d.len[0], d.half[0], d.per[0]);
                double ey = min_image(A.xc[3 * k + 1] - pi.y, d.len[1], d.half[1], d.per[1]);
                double ez = min_image((A.xc[3 * k + 2] + iz) - pi.z, d.len[2], d.half[2], d.per[2]);
                if (dist_sq_exact(ex, ey, ez) < K.rxlist_sq) {
                  if (nx < K.xcap) A.xidx[(int64_t)nx * ntot + i] = k;
                  ++nx;
                }
              }
            }
          }
        }
      }
    }
    if (nx > K.xcap) atomicMax(&A.S[r].xoverflow, nx);
    A.xcnt[i] = min(nx, K.xcap);
  }
  // counts are zero again for the next rebuild
  for (int r = 0; r < nrep; ++r) {
    if (!reb[r]) continue;
    const RepDesc& d = A.R[r];
    const int ncr = d.gd[0] * d.gd[1] * d.gd[2];
    const int nch = d.hd[0] * d.hd[1] * d.hd[2];
    for (int c = gtid; c < ncr; c += gthreads) A.count[d.g0 + c] = 0;
    for (int c = gtid; c < nch; c += gthreads) A.count[d.h0 + c] = 0;
  }
  grid_sync(A.bar, tflag);
  if (blockIdx.x == 0) {
    for (int r = threadIdx.x; r < nrep; r += BLOCK) {
      if (!reb[r]) continue;
      RepState& s = A.S[r];
      s.rebuild = 0;
      s.nbuilds += 1;
      s.ind_z_ref = s.ind_z;
    }
    if (threadIdx.x == 0) *A.any = 0;
  }
}

// ------------------------------------------------------------------------------------
// Task 4a: electron density and embedding derivative (Section 3.3.1.2)
// ------------------------------------------------------------------------------------
template <bool MIXED, bool ENERGY>
__global__ __launch_bounds__(BLOCK) void k_density(Consts K, const RepDesc* __restrict__ R,
                                                   RepState* __restrict__ S,
                                                   const int* __restrict__ tile_rep,
                                                   double4* __restrict__ q,
                                                   const int* __restrict__ idx,
                                                   const int* __restrict__ cnt,
                                                   double* __restrict__ rho_out,
                                                   double* __restrict__ part) {
  TileCtx c = tile_ctx(tile_rep, R);
  const RepDesc& d = R[c.r];
  double e_embed = 0.0;
  if (c.live) {
    const int64_t i = c.i;
    const double4 pi = q[i];
    const int n = cnt[i];
    double rho;
    if (MIXED) {
      float acc = 0.0f;
      const float dd = (float)K.d, dd2 = (float)K.d_sq;
      for (int k = 0; k < n; ++k) {
        const int j = idx[(int64_t)k * K.ntot + i];
        const double4 pj = q[j];
        float ex = (float)min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]);
        float ey = (float)min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]);
        float ez = (float)min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]);
        float r2 = ex * ex + ey * ey + ez * ez;
        if (r2 < dd2) {
          float u = __fsqrt_rn(r2) - dd;
          acc += u * u;
        }
      }
      rho = (double)acc;
    } else {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) {
        const int j = idx[(int64_t)k * K.ntot + i];
        const double4 pj = q[j];
        double ex = min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]);
        double ey = min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]);
        double ez = min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]);
        double r2 = ex * ex + ey * ey + ez * ez;
        if (r2 < K.d_sq) {
          double u = sqrt(r2) - K.d;
          acc += u * u;
        }
      }
      rho = acc;
    }
    double sr = sqrt(rho);
    double dF = rho > 0.0 ? -K.A / (2.0 * sr) : 0.0;
    q[i].w = dF;
    if (rho_out) rho_out[i] = rho;
    if (ENERGY) e_embed = -K.A * sr;
    if (!(rho == rho)) S[c.r].nonfinite = 1;
  }
  if (ENERGY) {
    double vals[1] = {e_embed};
    block_sum_store<1, BLOCK>(vals, part + c.tile);
  }
}

// ------------------------------------------------------------------------------------
// Task 4b (+4c, +5): forces
// ------------------------------------------------------------------------------------
// Partial-sum slots written per tile by the force kernels.
enum { P_PAIR = 0, P_MORSE, P_WXX, P_WYY, P_WZZ, P_WXY, P_WXZ, P_WYZ, P_FX, P_FY, P_FZ, NP_FORCE };

template <bool MIXED, bool ENERGY>
__device__ __forceinline__ void morse_gather(const Consts& K, const RepDesc& d, double iz, double4 pi,
                                             const double* __restrict__ xc, const int* __restrict__ xidx,
                                             int nx, int64_t i, double fm[3], double& em) {
  for (int k = 0; k < nx; ++k) {
    const int kk = xidx[(int64_t)k * K.ntot + i];
    double ex = min_image(xc[3 * kk + 0] - pi.x, d.len[0], d.half[0], d.per[0]);
    double ey = min_image(xc[3 * kk + 1] - pi.y, d.len[1], d.half[1], d.per[1]);
    double ez = min_image((xc[3 * kk + 2] + iz) - pi.z, d.len[2], d.half[2], d.per[2]);
    if (MIXED) {
      float fx = (float)ex, fy = (float)ey, fz = (float)ez;
      float r2 = fx * fx + fy * fy + fz * fz;
      if (r2 < (float)K.mrc_sq) {
        float rinv = __frsqrt_rn(r2);
        float r = r2 * rinv;
        float e = __expf(-(float)K.alpha * (r - (float)K.r0));
        float g = 2.0f * (float)(K.alpha * K.D) * (e - e * e);   // phiM'(r)
        float s = g * rinv;                                       // F_i = phiM'(r) (q_k - q_i)/r
        fm[0] += s * fx;
        fm[1] += s * fy;
        fm[2] += s * fz;
        if (ENERGY) em += (double)((float)K.D * (e * e - 2.0f * e)) - K.mshift;
      }
    } else {
      double r2 = ex * ex + ey * ey + ez * ez;
      if (r2 < K.mrc_sq) {
        double r = sqrt(r2);
        double e = exp(-K.alpha * (r - K.r0));
        double g = 2.0 * K.alpha * K.D * (e - e * e);
        double s = g / r;
        fm[0] += s * ex;
        fm[1] += s * ey;
        fm[2] += s * ez;
        if (ENERGY) em += K.D * (e * e - 2.0 * e) - K.mshift;
      }
    }
  }
}

template <bool MIXED, bool MORSE, bool KICK, bool ENERGY>
__global__ __launch_bounds__(BLOCK) void k_force(Consts K, const RepDesc* __restrict__ R,
                                                 RepState* __restrict__ S,
                                                 const int* __restrict__ tile_rep,
                                                 const double4* __restrict__ q,
                                                 double* __restrict__ v, double* __restrict__ f,
                                                 const uint8_t* __restrict__ fixed,
                                                 const int* __restrict__ idx,
                                                 const int* __restrict__ cnt,
                                                 const double* __restrict__ xc,
                                                 const int* __restrict__ xidx,
                                                 const int* __restrict__ xcnt,
                                                 double* __restrict__ part) {
  TileCtx c = tile_ctx(tile_rep, R);
  const RepDesc& d = R[c.r];
  double acc[NP_FORCE];
#pragma unroll
  for (int k = 0; k < NP_FORCE; ++k) acc[k] = 0.0;
  if (c.live) {
    const int64_t i = c.i;
    const double4 pi = q[i];
    const int n = cnt[i];
    double fx, fy, fz;
    if (MIXED) {
      const float cc = (float)K.c, dd = (float)K.d, c2 = (float)K.c2, rv = (float)K.rv,
                  pmin = (float)K.pmin, csq = (float)K.c_sq, dsq = (float)K.d_sq;
      const float Fi = (float)pi.w;
      float ax = 0.f, ay = 0.f, az = 0.f;
      float ep = 0.f, w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f, w4 = 0.f, w5 = 0.f;
      for (int k = 0; k < n; ++k) {
        const int j = idx[(int64_t)k * K.ntot + i];
        const double4 pj = q[j];
        float ex = (float)min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]);
        float ey = (float)min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]);
        float ez = (float)min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]);
        float r2 = ex * ex + ey * ey + ez * ez;
        if (r2 < csq) {
          float rinv = __frsqrt_rn(r2);
          float r = r2 * rinv;
          float u = r - cc, t = r - rv;
          float p = pmin + c2 * t * t;                 // c0 + c1 r + c2 r^2 in vertex form
          float g = u * (2.0f * p + u * (2.0f * c2 * t));   // phi'(r)
          if (r2 < dsq) g += (Fi + (float)pj.w) * (2.0f * (r - dd));
          float s = g * rinv;                           // F_i += g (q_j - q_i) / r
          ax += s * ex;
          ay += s * ey;
          az += s * ez;
          if (ENERGY) {
            ep += 0.5f * u * u * p;
            w0 -= 0.5f * s * ex * ex;
            w1 -= 0.5f * s * ey * ey;
            w2 -= 0.5f * s * ez * ez;
            w3 -= 0.5f * s * ex * ey;
            w4 -= 0.5f * s * ex * ez;
            w5 -= 0.5f * s * ey * ez;
          }
        }
      }
      fx = ax;
      fy = ay;
      fz = az;
      if (ENERGY) {
        acc[P_PAIR] = ep;
        acc[P_WXX] = w0;
        acc[P_WYY] = w1;
        acc[P_WZZ] = w2;
        acc[P_WXY] = w3;
        acc[P_WXZ] = w4;
        acc[P_WYZ] = w5;
      }
    } else {
      const double Fi = pi.w;
      double ax = 0.0, ay = 0.0, az = 0.0;
      for (int k = 0; k < n; ++k) {
        const int j = idx[(int64_t)k * K.ntot + i];
        const double4 pj = q[j];
        double ex = min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]);
        double ey = min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]);
        double ez = min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]);
        double r2 = ex * ex + ey * ey + ez * ez;
        if (r2 < K.c_sq) {
          double rinv = rsqrt(r2);
          double r = r2 * rinv;
          double u = r - K.c;
          double p = K.c0 + r * (K.c1 + r * K.c2);
          double g = u * (2.0 * p + u * (K.c1 + 2.0 * K.c2 * r));   // phi'(r)
          if (r2 < K.d_sq) g += (Fi + pj.w) * (2.0 * (r - K.d));
          double s = g * rinv;
          ax += s * ex;
          ay += s * ey;
          az += s * ez;
          if (ENERGY) {
            acc[P_PAIR] += 0.5 * u * u * p;
            acc[P_WXX] -= 0.5 * s * ex * ex;
            acc[P_WYY] -= 0.5 * s * ey * ey;
            acc[P_WZZ] -= 0.5 * s * ez * ez;
            acc[P_WXY] -= 0.5 * s * ex * ey;
            acc[P_WXZ] -= 0.5 * s * ex * ez;
            acc[P_WYZ] -= 0.5 * s * ey * ez;
          }
        }
      }
      fx = ax;
      fy = ay;
      fz = az;
    }
    if (MORSE) {
      const int nx = xcnt[i];
      if (nx > 0) {
        double fm[3] = {0.0, 0.0, 0.0}, em = 0.0;
        morse_gather<MIXED, ENERGY>(K, d, S[c.r].ind_z, pi, xc, xidx, nx, i, fm, em);
        fx += fm[0];
        fy += fm[1];
        fz += fm[2];
        if (ENERGY) {
          acc[P_MORSE] = em;
          acc[P_FX] = -fm[0];
          acc[P_FY] = -fm[1];
          acc[P_FZ] = -fm[2];
        }
      }
    }
    f[3 * i + 0] = fx;
    f[3 * i + 1] = fy;
    f[3 * i + 2] = fz;
    if (!(fx == fx && fy == fy && fz == fz && fabs(fx) + fabs(fy) + fabs(fz) < INFINITY))
      S[c.r].nonfinite = 1;
    if (KICK && !fixed[i]) {
      const double h = 0.5 * K.dt * K.acc;
      v[3 * i + 0] += h * fx;
      v[3 * i + 1] += h * fy;
      v[3 * i + 2] += h * fz;
    }
  }
  if (ENERGY) block_sum_store<NP_FORCE, BLOCK>(acc, part + (int64_t)c.tile * NP_FORCE);
}

// Task 4c alone: adds the Morse forces (and optionally their half kick) to f.
template <bool MIXED, bool KICK, bool ENERGY>
__global__ __launch_bounds__(BLOCK) void k_morse(Consts K, const RepDesc* __restrict__ R,
                                                 RepState* __restrict__ S,
                                                 const int* __restrict__ tile_rep,
                                                 const double4* __restrict__ q,
                                                 double* __restrict__ v, double* __restrict__ f,
                                                 const uint8_t* __restrict__ fixed,
                                                 const double* __restrict__ xc,
                                                 const int* __restrict__ xidx,
                                                 const int* __restrict__ xcnt,
                                                 double* __restrict__ part) {
  TileCtx c = tile_ctx(tile_rep, R);
  const RepDesc& d = R[c.r];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};   // E_morse, load x, y, z
  if (c.live) {
    const int64_t i = c.i;
    const int nx = xcnt[i];
    if (nx > 0) {
      double fm[3] = {0.0, 0.0, 0.0}, em = 0.0;
      morse_gather<MIXED, ENERGY>(K, d, S[c.r].ind_z, q[i], xc, xidx, nx, i, fm, em);
      f[3 * i + 0] += fm[0];
      f[3 * i + 1] += fm[1];
      f[3 * i + 2] += fm[2];
      if (KICK && !fixed[i]) {
        const double h = 0.5 * K.dt * K.acc;
        v[3 * i + 0] += h * fm[0];
        v[3 * i + 1] += h * fm[1];
        v[3 * i + 2] += h * fm[2];
      }
      acc[0] = em;
      acc[1] = -fm[0];
      acc[2] = -fm[1];
      acc[3] = -fm[2];
    }
  }
  if (ENERGY) block_sum_store<4, BLOCK>(acc, part + (int64_t)c.tile * 4);
}

// Task 5 alone.
__global__ __launch_bounds__(BLOCK) void k_kick(Consts K, const RepDesc* __restrict__ R,
                                                const int* __restrict__ tile_rep,
                                                double* __restrict__ v, const double* __restrict__ f,
                                                const uint8_t* __restrict__ fixed) {
  TileCtx c = tile_ctx(tile_rep, R);
  if (!c.live || fixed[c.i]) return;
  const int64_t i = c.i;
  const double h = 0.5 * K.dt * K.acc;
  v[3 * i + 0] += h * f[3 * i + 0];
  v[3 * i + 1] += h * f[3 * i + 1];
  v[3 * i + 2] += h * f[3 * i + 2];
}

// ------------------------------------------------------------------------------------
// Task 4d: energies
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_kinetic(Consts K, const RepDesc* __restrict__ R,
                                                   const int* __restrict__ tile_rep,
                                                   const double* __restrict__ v,
                                                   const uint8_t* __restrict__ fixed,
                                                   double* __restrict__ part) {
  TileCtx c = tile_ctx(tile_rep, R);
  double ke[1] = {0.0};
  if (c.live && !fixed[c.i]) {
    const int64_t i = c.i;
    double v2 = (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1]) + v[3 * i + 2] * v[3 * i + 2];
    ke[0] = K.ke_fac * v2;
  }
  block_sum_store<1, BLOCK>(ke, part + c.tile);
}

// One block per replica: sums the tile partials of that replica in tile order.
// out[r][MD_NOBS].  Partial arrays that were not produced are passed as NULL.
__global__ __launch_bounds__(BLOCK) void k_reduce(const RepDesc* __restrict__ R,
                                                  const RepState* __restrict__ S,
                                                  const double* __restrict__ p_embed,
                                                  const double* __restrict__ p_force,
                                                  const double* __restrict__ p_morse,
                                                  const double* __restrict__ p_kin,
                                                  double* __restrict__ out) {
  const int r = blockIdx.x;
  const RepDesc& d = R[r];
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int t = d.t0 + threadIdx.x; t < d.t0 + d.nt; t += BLOCK) {
    if (p_embed) acc[MD_E_EMBED] += p_embed[t];
    if (p_kin) acc[MD_E_KIN] += p_kin[t];
    if (p_force) {
      const double* pf = p_force + (int64_t)t * NP_FORCE;
      acc[MD_E_PAIR] += pf[P_PAIR];
      acc[MD_E_MORSE] += pf[P_MORSE];
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[MD_W_XX + k] += pf[P_WXX + k];
      acc[MD_F_IND_X] += pf[P_FX];
      acc[MD_F_IND_X + 1] += pf[P_FY];
      acc[MD_F_IND_X + 2] += pf[P_FZ];
    }
    if (p_morse) {
      const double* pm = p_morse + (int64_t)t * 4;
      acc[MD_E_MORSE] += pm[0];
      acc[MD_F_IND_X] += pm[1];
      acc[MD_F_IND_X + 1] += pm[2];
      acc[MD_F_IND_X + 2] += pm[3];
    }
  }
  block_sum_store<16, BLOCK>(acc, out + (int64_t)r * MD_NOBS);
  if (threadIdx.x == 0) {
    out[(int64_t)r * MD_NOBS + MD_IND_Z] = S[r].ind_z;
    out[(int64_t)r * MD_NOBS + MD_NBUILDS] = (double)S[r].nbuilds;
    out[(int64_t)r * MD_NOBS + 15] = 0.0;
  }
}

// Status flags, folded over replicas.
__global__ void k_status(const RepState* __restrict__ S, int nrep, int* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int o = 0, xo = 0, nf = 0, nb = 0, to = 0;
  for (int r = 0; r < nrep; ++r) {
    o = max(o, S[r].overflow);
    xo = max(xo, S[r].xoverflow);
    nf |= S[r].nonfinite;
    nb += S[r].nbuilds;
    to |= S[r].sync_timeout;
  }
  out[0] = o;
  out[1] = xo;
  out[2] = nf;
  out[3] = nb;
  out[4] = to;
}

__global__ void k_clear_flags(RepState* __restrict__ S, int nrep) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrep) return;
  S[r].overflow = 0;
  S[r].xoverflow = 0;
  S[r].nonfinite = 0;
  S[r].sync_timeout = 0;
}

}  // namespace md
