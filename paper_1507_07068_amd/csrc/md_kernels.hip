// HIP kernels of the MD step for CDNA4 (gfx950).  Included by md_api.hip.
//
//   k_kick_drift   Tasks 2 + 3 (Eqs. A11-A12) and the per-tile displacement maxima
//   k_decide ... k_list   Task 1: skin test and list rebuild (md_rebuild.hip)
//   k_density, k_force, k_morse, k_kick   Task 4a-4c and Task 5 (md_forces.hip)
//   k_kinetic / k_reduce   Task 4d: energies, virial, load (fixed-order FP64 reductions)
//
// Every force-path kernel is owner-computes: one lane per atom gathers over that atom's
// full neighbour list and writes only that atom, so no atomics touch forces or densities.
#pragma once

#include "md_device.hpp"
#include "md_rebuild.hip"
#include "md_forces.hip"

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
// Bounding box of the tile's atoms along the open axes of its replica:
// box[6 t + a] = min, box[6 t + 3 + a] = max (used to size the cell grid).
__device__ __forceinline__ void tile_box_store(const RepDesc& d, bool live, double4 p, double* box) {
  const double x[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d.per[a]) continue;   // uniform over the block
    const double mn = -block_max<BLOCK>(live ? -x[a] : -INFINITY);
    const double mx = block_max<BLOCK>(live ? x[a] : -INFINITY);
    if (threadIdx.x == 0) {
      box[a] = mn;
      box[3 + a] = mx;
    }
  }
}

// v(t + dt/2) = v + a dt / 2 and r(t + dt) = r + v(t + dt/2) dt (algebraically Eq. A11) for
// mobile atoms, and their cell-local shadow; the indenter moves by v_ind dt.  Writes
// max |r - r_ref|^2 of each tile and the tile's bounding box along open axes.  Without
// KICK the velocity is already v(t + dt/2) (the previous force pass gave a full kick) and
// only the drift is done.
template <bool KICK>
__global__ __launch_bounds__(BLOCK) void k_kick_drift(Consts K, const RepDesc* __restrict__ R,
                                                      RepState* __restrict__ S,
                                                      const int* __restrict__ tile_rep,
                                                      double4* __restrict__ q, double* __restrict__ v,
                                                      const double* __restrict__ f,
                                                      const uint8_t* __restrict__ fixed,
                                                      const double* __restrict__ xref,
                                                      double* __restrict__ dmax_tile,
                                                      double* __restrict__ tile_box,
                                                      int4* __restrict__ qs,
                                                      const long long* __restrict__ bcell) {
  TileCtx c = tile_ctx(tile_rep, R);
  double d2 = 0.0;
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
  if (c.live) {
    const int64_t i = c.i;
    p = q[i];
    if (!fixed[i]) {
      double vx = v[3 * i + 0], vy = v[3 * i + 1], vz = v[3 * i + 2];
      if (KICK) {
        const double h = 0.5 * K.dt * K.acc;
        vx += h * f[3 * i + 0];
        vy += h * f[3 * i + 1];
        vz += h * f[3 * i + 2];
        v[3 * i + 0] = vx;
        v[3 * i + 1] = vy;
        v[3 * i + 2] = vz;
      }
      p.x += vx * K.dt;
      p.y += vy * K.dt;
      p.z += vz * K.dt;
      q[i] = p;
      if (K.shadow) qs[i] = cell_local(S[c.r], bcell[i], p.x, p.y, p.z, (float)p.w);   // shadow
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
  tile_box_store(R[c.r], c.live, p, tile_box + 6 * (int64_t)c.tile);
}

// Positions (and their shadow) from the second buffer back into the caller's arrays.
__global__ __launch_bounds__(BLOCK) void k_copy_positions(int64_t n, const double4* __restrict__ q2,
                                                          double4* __restrict__ q, const int4* __restrict__ qs2,
                                                          int4* __restrict__ qs, int shadow) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  q[i] = q2[i];
  if (shadow) qs[i] = qs2[i];
}

// Tile bounding boxes of the current positions (before a forced build).
__global__ __launch_bounds__(BLOCK) void k_tile_box(const RepDesc* __restrict__ R,
                                                    const int* __restrict__ tile_rep,
                                                    const double4* __restrict__ q,
                                                    double* __restrict__ tile_box) {
  TileCtx c = tile_ctx(tile_rep, R);
  const double4 p = c.live ? q[c.i] : make_double4(0.0, 0.0, 0.0, 0.0);
  tile_box_store(R[c.r], c.live, p, tile_box + 6 * (int64_t)c.tile);
}

// ------------------------------------------------------------------------------------
// Task 4d: energies
// ------------------------------------------------------------------------------------
// Per tile: kinetic energy of mobile atoms and the Morse energy / indenter load from the
// per-atom Morse results (atom order).
__global__ __launch_bounds__(BLOCK) void k_kinetic(Consts K, const RepDesc* __restrict__ R,
                                                   const int* __restrict__ tile_rep,
                                                   const double* __restrict__ v,
                                                   const uint8_t* __restrict__ fixed,
                                                   const double* __restrict__ fme,
                                                   double* __restrict__ p_kin,
                                                   double* __restrict__ p_morse) {
  TileCtx c = tile_ctx(tile_rep, R);
  double ke[1] = {0.0};
  double mo[4] = {0.0, 0.0, 0.0, 0.0};
  if (c.live) {
    const int64_t i = c.i;
    if (!fixed[i]) {
      const double v2 = (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1]) + v[3 * i + 2] * v[3 * i + 2];
      ke[0] = K.ke_fac * v2;
    }
    mo[0] = fme[4 * i + 3];
    mo[1] = -fme[4 * i + 0];
    mo[2] = -fme[4 * i + 1];
    mo[3] = -fme[4 * i + 2];
  }
  block_sum_store<1, BLOCK>(ke, p_kin + c.tile);
  block_sum_store<4, BLOCK>(mo, p_morse + (int64_t)c.tile * 4);
}

// Task 4d sums in two fixed-order stages, so that a large replica's partials are read by
// many blocks: each replica's tiles are cut into chunks of REDUCE_CHUNK tiles (the cut
// depends only on the replica's own tile count, so a replica's sums do not depend on the
// batch), one block sums a chunk's partials, then one block per replica sums its chunks in
// order.  Partial arrays that were not produced are passed as NULL; tpe / tpf are the
// blocks per tile of the density / force launches that wrote p_embed / p_force, tpk of the
// launch that wrote p_kin and p_morse (k_kinetic: 1, a force pass that took them: T).
constexpr int REDUCE_CHUNK = 512;

__global__ __launch_bounds__(BLOCK) void k_reduce_chunks(const int2* __restrict__ chunks,
                                                         const double* __restrict__ p_embed, int tpe,
                                                         const double* __restrict__ p_force, int tpf,
                                                         const double* __restrict__ p_morse,
                                                         const double* __restrict__ p_kin, int tpk,
                                                         double* __restrict__ chunk_out) {
  const int2 ch = chunks[blockIdx.x];   // first tile, tile count
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  if (p_embed)
    for (int b = ch.x * tpe + threadIdx.x; b < (ch.x + ch.y) * tpe; b += BLOCK) acc[MD_E_EMBED] += p_embed[b];
  if (p_force)
    for (int b = ch.x * tpf + threadIdx.x; b < (ch.x + ch.y) * tpf; b += BLOCK) {
      const double* pf = p_force + (int64_t)b * NP_FORCE;
      acc[MD_E_PAIR] += pf[P_PAIR];
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[MD_W_XX + k] += pf[P_WXX + k];
    }
  for (int t = ch.x * tpk + threadIdx.x; t < (ch.x + ch.y) * tpk; t += BLOCK) {
    if (p_kin) acc[MD_E_KIN] += p_kin[t];
    if (p_morse) {
      const double* pm = p_morse + (int64_t)t * 4;
      acc[MD_E_MORSE] += pm[0];
      acc[MD_F_IND_X] += pm[1];
      acc[MD_F_IND_X + 1] += pm[2];
      acc[MD_F_IND_X + 2] += pm[3];
    }
  }
  block_sum_store<16, BLOCK>(acc, chunk_out + (int64_t)blockIdx.x * 16);
}

// One block per replica: its chunks' sums in chunk order -> out[r][MD_NOBS].
__global__ __launch_bounds__(BLOCK) void k_reduce(const RepDesc* __restrict__ R,
                                                  const RepState* __restrict__ S,
                                                  const double* __restrict__ chunk_out,
                                                  double* __restrict__ out, int ind_obs) {
  const int r = blockIdx.x;
  const RepDesc& d = R[r];
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int c = d.ch0 + threadIdx.x; c < d.ch0 + d.nch; c += BLOCK)
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] += chunk_out[(int64_t)c * 16 + k];
  block_sum_store<16, BLOCK>(acc, out + (int64_t)r * MD_NOBS);
  if (threadIdx.x == 0) {
    // (ind_obs: a force pass that took the energies has moved the indenter on already)
    out[(int64_t)r * MD_NOBS + MD_IND_Z] = ind_obs ? S[r].ind_z_obs : S[r].ind_z;
    out[(int64_t)r * MD_NOBS + MD_NBUILDS] = (double)S[r].nbuilds;
    out[(int64_t)r * MD_NOBS + 15] = 0.0;
  }
}

// Each replica's list-build count (md_run's trace).
__global__ __launch_bounds__(BLOCK) void k_record_builds(const RepState* __restrict__ S, int nrep,
                                                         int* __restrict__ out) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r < nrep) out[r] = S[r].nbuilds;
}

// Status flags, folded over replicas.
__global__ void k_status(const RepState* __restrict__ S, int nrep, int* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int o = 0, xo = 0, nf = 0, nb = 0, to = 0, nn = 0, io = 0;
  for (int r = 0; r < nrep; ++r) {
    o = max(o, S[r].overflow);
    io = max(io, S[r].ioverflow);
    xo = max(xo, S[r].xoverflow);
    nf |= S[r].nonfinite;
    nb += S[r].nbuilds;
    to |= S[r].sync_timeout;
    nn += S[r].nnear;
  }
  out[0] = o;
  out[1] = xo;
  out[2] = nf;
  out[3] = nb;
  out[4] = to;
  out[5] = nn;
  out[6] = io;
}

// Cell counts back to zero and the abort word of a build that gave up lifted.
__global__ __launch_bounds__(BLOCK) void k_clear_build(int* __restrict__ count, int ncell, int* __restrict__ abort) {
  for (int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * BLOCK) count[c] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *abort = 0;
}

__global__ void k_clear_flags(RepState* __restrict__ S, int nrep) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrep) return;
  S[r].overflow = 0;
  S[r].xoverflow = 0;
  S[r].ioverflow = 0;
  S[r].nonfinite = 0;
  S[r].sync_timeout = 0;
}

}  // namespace md
