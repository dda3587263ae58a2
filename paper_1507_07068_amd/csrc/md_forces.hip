// Task 4 (and the fused Task 5 kick) of the MD step on gfx950.  Included by md_kernels.hip.
//
//   k_density<T>   rho_i = sum_j f(r_ij), F'(rho_i) -> q[i].w   (Section 3.3.1.2)
//                  (FP32-mixed: separations from the fixed-point cell-local shadow of q)
//   k_force<T>     Eq. (1): F_i = -sum_j [(F'_i + F'_j) f'(r) + phi'(r)] (q_i - q_j) / r
//   k_morse        Cr-C Morse forces: one wavefront per Cr atom that has carbons in range
//   k_kick         Task 5 on its own
//
// T lanes cooperate on one atom (entries k = sub, sub + T, ... of its list; the list is
// interleaved by T so those lanes read adjacent words) and combine their partial sums with
// a fixed butterfly, so results do not depend on scheduling.  Each atom's sums are written
// by one lane only: no atomics.
#pragma once

#include <type_traits>

#include "md_device.hpp"

namespace md {

// Sum over the T lanes of one atom (T a power of two <= 64).
template <int T, class V>
__device__ __forceinline__ V group_sum(V v) {
#pragma unroll
  for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Visit the entries k = sub, sub + T, ... (< n) of atom i's list in order, calling
// body(fetch(e), e) for each entry e (the neighbour's slot and relative cell, see
// list_slot / list_code).  Entries go U at a time: the U gathers of one group are in
// flight together with the U index loads of the next.
#ifndef MD_UNROLL
#define MD_UNROLL 2
#endif
constexpr int UNROLL = MD_UNROLL;

template <int T, int U, class Fetch, class Body>
__device__ __forceinline__ void for_entries(const int* __restrict__ idx, int i, int n, int sub, int ntot,
                                            int shift, Fetch fetch, Body body) {
  // this lane's entries k = sub + m T (m = 0 .. nl - 1) sit one stride apart, at
  // idx[(m ntot + i) T + sub]; 32-bit word offsets (the list holds fewer than 2^31 words),
  // running by the stride, and the index loads ahead clamped to the last entry so that they
  // need no branch
  const int nl = n > sub ? ((n - 1 - sub) >> shift) + 1 : 0;
  if (nl == 0) return;
  const unsigned stride = (unsigned)ntot * T;
  const unsigned first = (unsigned)i * T + sub;
  const unsigned last = first + (unsigned)(nl - 1) * stride;
  unsigned base = first;   // offset of entry m
  int e[U];
#pragma unroll
  for (int u = 0; u < U; ++u) e[u] = idx[min(base + u * stride, last)];
  int m = 0;
  for (; m + U <= nl; m += U) {
    decltype(fetch(0)) p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) p[u] = fetch(e[u]);
    base += U * stride;
    int en[U];
#pragma unroll
    for (int u = 0; u < U; ++u) en[u] = idx[min(base + u * stride, last)];
#pragma unroll
    for (int u = 0; u < U; ++u) body(p[u], e[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) e[u] = en[u];
  }
  // fewer than U entries remain (m + U > nl); their indices are already in e[]
#pragma unroll
  for (int u = 0; u < U - 1; ++u)
    if (m + u < nl) body(fetch(e[u]), e[u]);
}

// Offsets of the 27 relative cells of a list entry in the block's replica, in shadow units:
// the separation of two atoms is (shadow_j - shadow_i + offset[code]) / qscale.
__device__ __forceinline__ void fill_cell_offsets(int4* tab, const RepState& s) {
  const int t = threadIdx.x;
  if (t < 27) {
    const double q = s.qscale;
    tab[t] = make_int4((t % 3 - 1) * (int)rint(s.gedge[0] * q), (t / 3 % 3 - 1) * (int)rint(s.gedge[1] * q),
                       (t / 9 - 1) * (int)rint(s.gedge[2] * q), 0);
  }
  __syncthreads();
}

// Atom of this thread in a launch with T lanes per atom and one block per 256/T atoms.
struct AtomCtx {
  int blk;       // logical block (XCD-aware)
  int r;         // replica
  int sub;       // lane within the atom's group
  int64_t i;     // atom slot
  bool live;
};

template <int T>
__device__ __forceinline__ AtomCtx atom_ctx(const int* tile_rep, const RepDesc* R, int bid, int nb) {
  constexpr int APB = BLOCK / T;
  AtomCtx c;
  c.blk = xcd_block(bid, nb);
  const int tile = c.blk / T;
  c.r = tile_rep[tile];
  c.sub = threadIdx.x % T;
  c.i = (int64_t)tile * TILE + (c.blk % T) * APB + threadIdx.x / T;
  const RepDesc& d = R[c.r];
  c.live = c.i < (int64_t)d.a0 + d.n;
  return c;
}

// Task 4c: Cr-C Morse forces, F_i += -phiM'(r) (q_i - q_k)/r over atom i's Cr-C list.
// One wavefront per atom of the replicas' near lists (grid-stride over all of them); the
// 64 lanes share that atom's carbons and combine their sums with a fixed butterfly.
// fme[i] receives (F_i, E_i) of the atom, which the energy pass sums in atom order; with
// ADD_F the force is also added into f (and, with KICK, its half kick into v).  Without
// ADD_F the pass runs in extra blocks of the density launch and the force pass adds fme.
template <bool MIXED, bool KICK, bool ADD_F>
__device__ __forceinline__ void morse_pass(const Consts& K, const RepDesc* __restrict__ R,
                                           const RepState* __restrict__ S,
                                           const double4* __restrict__ q,
                                           double* __restrict__ v, double* __restrict__ f,
                                           const uint8_t* __restrict__ fixed,
                                           const double* __restrict__ xc,
                                           const int* __restrict__ xidx,
                                           const int* __restrict__ xcnt,
                                           const int* __restrict__ near,
                                           double* __restrict__ fme, int bid, int nb) {
  const int lane = threadIdx.x % WAVE;
  const int gw = bid * (BLOCK / WAVE) + threadIdx.x / WAVE, nw = nb * (BLOCK / WAVE);
  auto one = [&](int r, int item) {   // near atom `item` of replica r, on this wavefront
    const RepDesc& d = R[r];
    const double iz = S[r].ind_z;
    {
      const int64_t pa = near[d.a0 + item];
      const int na = xcnt[pa];
      const double4 pi = q[pa];
      double fm0 = 0.0, fm1 = 0.0, fm2 = 0.0, em = 0.0;
      for (int k = lane; k < na; k += WAVE) {
        const int kk = xidx[pa * K.xcap + k];
        const double ex = min_image(xc[3 * kk + 0] - pi.x, d.len[0], d.half[0], d.per[0]);
        const double ey = min_image(xc[3 * kk + 1] - pi.y, d.len[1], d.half[1], d.per[1]);
        const double ez = min_image((xc[3 * kk + 2] + iz) - pi.z, d.len[2], d.half[2], d.per[2]);
        if (MIXED) {
          const float fx = (float)ex, fy = (float)ey, fz = (float)ez;
          const float r2 = fx * fx + fy * fy + fz * fz;
          if (r2 < (float)K.mrc_sq) {
            const float rinv = __frsqrt_rn(r2);
            const float rr = r2 * rinv;
            const float e = __expf(-(float)K.alpha * (rr - (float)K.r0));
            const float g = 2.0f * (float)(K.alpha * K.D) * (e - e * e);   // phiM'(r)
            const float s = g * rinv;                                     // F_i += g (q_k - q_i)/r
            fm0 += s * fx;
            fm1 += s * fy;
            fm2 += s * fz;
            em += (double)((float)K.D * (e * e - 2.0f * e)) - K.mshift;
          }
        } else {
          // the cutoff test on r = sqrt((ex ex + ey ey) + ez ez), rounded exactly as the plain
          // definition does it: the unshifted force jumps at the cutoff, so a pair within an
          // ulp of it must fall on the same side
          const double rr = sqrt(dist_sq_exact(ex, ey, ez));
          if (rr < K.mrc) {
            const double e = exp(-K.alpha * (rr - K.r0));
            const double g = 2.0 * K.alpha * K.D * (e - e * e);
            const double s = g / rr;
            fm0 += s * ex;
            fm1 += s * ey;
            fm2 += s * ez;
            em += K.D * (e * e - 2.0 * e) - K.mshift;
          }
        }
      }
      fm0 = wave_sum(fm0);
      fm1 = wave_sum(fm1);
      fm2 = wave_sum(fm2);
      em = wave_sum(em);
      if (lane == 0) {
        if (ADD_F) {
          f[3 * pa + 0] += fm0;
          f[3 * pa + 1] += fm1;
          f[3 * pa + 2] += fm2;
        }
        if (KICK && !fixed[pa]) {
          const double h = 0.5 * K.dt * K.acc;
          v[3 * pa + 0] += h * fm0;
          v[3 * pa + 1] += h * fm1;
          v[3 * pa + 2] += h * fm2;
        }
        fme[4 * pa + 0] = fm0;
        fme[4 * pa + 1] = fm1;
        fme[4 * pa + 2] = fm2;
        fme[4 * pa + 3] = em;
      }
    }
  };
  __shared__ int pre[FLAT_MAXREP + 1];
  if (K.nrep <= FLAT_MAXREP) {
    const int total = flat_prefix(K.nrep, pre, [&](int r) { return S[r].nnear; });
    for (int g = gw; g < total; g += nw) {
      const int r = flat_replica(pre, K.nrep, g);
      one(r, g - pre[r]);
    }
  } else {
    for (int r = 0; r < K.nrep; ++r)
      for (int item = gw; item < S[r].nnear; item += nw) one(r, item);
  }
}

template <bool MIXED, bool KICK, bool ADD_F>
__global__ __launch_bounds__(BLOCK) void k_morse(Consts K, const RepDesc* __restrict__ R,
                                                 const RepState* __restrict__ S,
                                                 const double4* __restrict__ q,
                                                 double* __restrict__ v, double* __restrict__ f,
                                                 const uint8_t* __restrict__ fixed,
                                                 const double* __restrict__ xc,
                                                 const int* __restrict__ xidx,
                                                 const int* __restrict__ xcnt,
                                                 const int* __restrict__ near,
                                                 double* __restrict__ fme) {
  morse_pass<MIXED, KICK, ADD_F>(K, R, S, q, v, f, fixed, xc, xidx, xcnt, near, fme, blockIdx.x, gridDim.x);
}

// The Cr-C pass that the leading M.nblocks blocks of a density launch run (Task 4c does
// not depend on the density, so it overlaps with it).
struct MorseIn {
  const double* xc;
  const int* xidx;
  const int* xcnt;
  const int* near;
  double* fme;
  int nblocks;
};

// SHADOW (with MIXED): separations from the fixed-point cell-local shadow qs and the entries'
// relative cells; otherwise FP64 positions (rounded to FP32 for the MIXED arithmetic).
// PAPER: the paper's form -- rho_i = sum f, P_i = sum f^2, F'(rho_i) into q.w and M'(P_i)
// into dm[i] (the second derivative of the paper's per-atom array).
template <int T, bool MIXED, bool SHADOW, bool ENERGY, bool PAPER = false>
__global__ __launch_bounds__(BLOCK) void k_density(Consts K, const RepDesc* __restrict__ R,
                                                   RepState* __restrict__ S,
                                                   const int* __restrict__ tile_rep,
                                                   double4* __restrict__ q,
                                                   int4* __restrict__ qs,
                                                   const int* __restrict__ idx,
                                                   const int* __restrict__ cnt,
                                                   double* __restrict__ rho_out,
                                                   double* __restrict__ part, MorseIn M,
                                                   double* __restrict__ dm) {
  if ((int)blockIdx.x < M.nblocks) {   // uniform over the block
    morse_pass<MIXED, false, false>(K, R, S, q, nullptr, nullptr, nullptr, M.xc, M.xidx, M.xcnt, M.near, M.fme,
                                    blockIdx.x, M.nblocks);
    return;
  }
  const AtomCtx c = atom_ctx<T>(tile_rep, R, (int)blockIdx.x - M.nblocks, (int)gridDim.x - M.nblocks);
  const RepDesc& d = R[c.r];
  __shared__ int4 ctab[27];
  if (SHADOW) fill_cell_offsets(ctab, S[c.r]);
  // FP64 separations: the minimum image only in wavefronts with an atom near a periodic face
  const double4 pi = (!SHADOW && c.live) ? q[c.i] : make_double4(0.0, 0.0, 0.0, 0.0);
  const bool img = !SHADOW && wave_near_face(d, c.live, pi.x, pi.y, pi.z, K.rlist + 2.0 * K.half_skin);
  double rho = 0.0, pp = 0.0;   // pp: P_i (paper's form)
  if (c.live) {
    const int64_t i = c.i;
    const int n = cnt[i];
    if constexpr (PAPER) {
      if (MIXED) {
        float ar = 0.0f, ap = 0.0f;
        const float rcs = (float)K.P.rc_sq;
        auto add = [&](float ex, float ey, float ez) {
          const float r2 = ex * ex + ey * ey + ez * ez;
          const bool in = r2 < rcs;
          const float f = paper_f32(K.P, __frsqrt_rn(in ? r2 : 1.0f));
          ar += in ? f : 0.0f;
          ap += in ? f * f : 0.0f;
        };
        if (SHADOW) {
          const int4 ps = qs[i];
          const float qi = (float)(1.0 / S[c.r].qscale);
          for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                                 [&](int e) { return qs[list_slot(e)]; },
                                 [&](const int4& pj, int e) {
            const int4 o = ctab[list_code(e)];
            add((float)(pj.x - ps.x + o.x) * qi, (float)(pj.y - ps.y + o.y) * qi, (float)(pj.z - ps.z + o.z) * qi);
          });
        } else {
          auto pass = [&](auto img_c) {
            constexpr bool IMG = decltype(img_c)::value;
            for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                                   [&](int e) { return q[list_slot(e)]; },
                                   [&](const double4& pj, int) {
              add((float)(IMG ? min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.x - pi.x),
                  (float)(IMG ? min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.y - pi.y),
                  (float)(IMG ? min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.z - pi.z));
            });
          };
          if (img) pass(std::true_type{}); else pass(std::false_type{});
        }
        rho = (double)ar;
        pp = (double)ap;
      } else {
        auto pass = [&](auto img_c) {
          constexpr bool IMG = decltype(img_c)::value;
          for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                                 [&](int e) { return q[list_slot(e)]; },
                                 [&](const double4& pj, int) {
            const double ex = IMG ? min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.x - pi.x;
            const double ey = IMG ? min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.y - pi.y;
            const double ez = IMG ? min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.z - pi.z;
            const double r2 = ex * ex + ey * ey + ez * ez;
            const bool in = r2 < K.P.rc_sq;
            const double f = paper_f(K.P, rsq_nr(in ? r2 : 1.0));
            rho += in ? f : 0.0;
            pp += in ? f * f : 0.0;
          });
        };
        if (img) pass(std::true_type{}); else pass(std::false_type{});
      }
    } else if (MIXED && SHADOW) {
      const int4 ps = qs[i];
      const float qi = (float)(1.0 / S[c.r].qscale);
      float acc = 0.0f;
      const float dd = (float)K.d, dd2 = (float)K.d_sq;
      for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                             [&](int e) { return qs[list_slot(e)]; },
                             [&](const int4& pj, int e) {
        const int4 o = ctab[list_code(e)];
        const float ex = (float)(pj.x - ps.x + o.x) * qi, ey = (float)(pj.y - ps.y + o.y) * qi,
                    ez = (float)(pj.z - ps.z + o.z) * qi;
        const float r2 = ex * ex + ey * ey + ez * ez;
        const float u = __fsqrt_rn(r2) - dd;
        acc += (r2 < dd2) ? u * u : 0.0f;
      });
      rho = (double)acc;
    } else if (MIXED) {
      float acc = 0.0f;
      const float dd = (float)K.d, dd2 = (float)K.d_sq;
      auto pass = [&](auto img_c) {
        constexpr bool IMG = decltype(img_c)::value;
        for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                               [&](int e) { return q[list_slot(e)]; },
                               [&](const double4& pj, int) {
          const float ex = (float)(IMG ? min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.x - pi.x);
          const float ey = (float)(IMG ? min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.y - pi.y);
          const float ez = (float)(IMG ? min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.z - pi.z);
          const float r2 = ex * ex + ey * ey + ez * ez;
          const float u = __fsqrt_rn(r2) - dd;
          acc += (r2 < dd2) ? u * u : 0.0f;
        });
      };
      if (img) pass(std::true_type{}); else pass(std::false_type{});
      rho = (double)acc;
    } else {
      auto pass = [&](auto img_c) {
        constexpr bool IMG = decltype(img_c)::value;
        for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                               [&](int e) { return q[list_slot(e)]; },
                               [&](const double4& pj, int) {
          const double ex = IMG ? min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.x - pi.x;
          const double ey = IMG ? min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.y - pi.y;
          const double ez = IMG ? min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.z - pi.z;
          const double r2 = ex * ex + ey * ey + ez * ez;
          const bool in = r2 < K.d_sq;
          const double u = r2 * rsq_nr(in ? r2 : 1.0) - K.d;   // r - d (r = r2 / sqrt(r2))
          rho += in ? u * u : 0.0;
        });
      };
      if (img) pass(std::true_type{}); else pass(std::false_type{});
    }
  }
  rho = group_sum<T>(rho);
  if (PAPER) pp = group_sum<T>(pp);
  double e_embed = 0.0;
  if (c.live && c.sub == 0) {
    double dF, en;
    if constexpr (PAPER) {
      const PaperEmbed pe = paper_embed(K.P, rho, pp);
      dF = pe.dF;
      en = pe.F + pe.M;
      dm[c.i] = pe.dM;
      if (!(pp == pp)) S[c.r].nonfinite = 1;
    } else {
      const double sr = sqrt(rho);
      dF = rho > 0.0 ? -K.A / (2.0 * sr) : 0.0;
      en = -K.A * sr;
    }
    q[c.i].w = dF;
    if (SHADOW) qs[c.i].w = __float_as_int((float)dF);
    if (rho_out) rho_out[c.i] = rho;
    if (ENERGY) e_embed = en;
    if (!(rho == rho)) S[c.r].nonfinite = 1;
  }
  if (ENERGY) {
    double vals[1] = {e_embed};
    block_sum_store<1, BLOCK>(vals, part + c.blk);
  }
}

// Partial sums written per block by k_force.
enum { P_PAIR = 0, P_WXX, P_WYY, P_WZZ, P_WXY, P_WXZ, P_WYZ, NP_FORCE };

// With DRIFT (and a full kick) the pass also does the next step's Task 2 + 3: the new
// positions (and their fixed-point shadow) go to the other position buffer, with the
// displacement maxima and open-axis boxes of each block's atoms (T parts per tile) for the
// next rebuild decision, and the indenter moves.
struct DriftOut {
  double4* q;             // next step's positions (the other buffer)
  int4* qs;               // and their shadow
  const double* xref;
  const long long* bcell;
  double* dmax;           // [tile * T + part]
  double* tbox;           // [6 (tile * T + part) + ...]
};

// An energy step of md_run whose end velocities are observed but which is not the last (the
// pass with ENERGY and DRIFT): it kicks to the whole step, takes the kinetic energy and the
// Cr-C sums there (the k_kinetic terms, as partials per block), then gives the next step's
// first half kick too and drifts.  Each velocity sees the same two kicks, in the same order,
// as with the separate passes.
struct KinOut {
  double* kin;            // [tile * T + part] kinetic energy
  double* morse;          // [4 (tile * T + part) + ...] Cr-C energy and indenter load
};

// Occupancy floor of the force pass (wavefronts per SIMD its registers must allow); the
// pass that takes energies and drifts (KinOut) is held to MD_FORCE_KIN_WAVES, but for the
// paper's form (whose registers would spill there).
#ifndef MD_FORCE_WAVES
#define MD_FORCE_WAVES 1
#endif
#ifndef MD_FORCE_KIN_WAVES
#define MD_FORCE_KIN_WAVES 5
#endif

// A neighbour's record with its M'(P_j) (paper's form).
struct QM {
  double4 q;
  double m;
};
struct SM {
  int4 q;
  double m;
};

// PAPER: the paper's form, dm[j] = M'(P_j) from the density pass.
template <int T, bool MIXED, bool SHADOW, bool KICK, bool ENERGY, bool DRIFT = false, bool PAPER = false>
__global__ __launch_bounds__(BLOCK, (ENERGY && DRIFT && !PAPER) ? MD_FORCE_KIN_WAVES : MD_FORCE_WAVES) void k_force(Consts K, const RepDesc* __restrict__ R,
                                                 RepState* __restrict__ S,
                                                 const int* __restrict__ tile_rep,
                                                 const double4* __restrict__ q,
                                                 const int4* __restrict__ qs,
                                                 double* __restrict__ v, double* __restrict__ f,
                                                 const uint8_t* __restrict__ fixed,
                                                 const int* __restrict__ idx,
                                                 const int* __restrict__ cnt,
                                                 double* __restrict__ part,
                                                 const int* __restrict__ xcnt,
                                                 const double* __restrict__ fme, double kick_h,
                                                 DriftOut D, const double* __restrict__ dm, int store_f,
                                                 KinOut KO) {
  const AtomCtx c = atom_ctx<T>(tile_rep, R, blockIdx.x, gridDim.x);
  const RepDesc& d = R[c.r];
  __shared__ int4 ctab[27];
  if (SHADOW) fill_cell_offsets(ctab, S[c.r]);
  // FP64 separations: the minimum image only in wavefronts with an atom near a periodic face
  const double4 pi = (!SHADOW && c.live) ? q[c.i] : make_double4(0.0, 0.0, 0.0, 0.0);
  const bool img = !SHADOW && wave_near_face(d, c.live, pi.x, pi.y, pi.z, K.rlist + 2.0 * K.half_skin);
  double acc[NP_FORCE];
#pragma unroll
  for (int k = 0; k < NP_FORCE; ++k) acc[k] = 0.0;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (c.live) {
    const int64_t i = c.i;
    const int n = cnt[i];
    if constexpr (PAPER) {
      // dE/dr = Phi'(r) [x < d] + f'(r) [r < rc] ((F'_i + F'_j) + (M'_i + M'_j) 2 f(r)), Phi' by
      // Horner in x = r / re; all lanes evaluate and the cutoffs select, with F'_j and M'_j
      // used on every path (so the neighbour's record is loaded ahead of the arithmetic)
      const PaperConsts& P = K.P;
      if (MIXED) {
        const float rcs = (float)P.rc_sq, phs = (float)P.phi_sq, ire = (float)P.inv_re, dd = (float)P.d,
                    b0 = (float)P.b0, b1 = (float)P.b1, b2 = (float)P.b2, b3 = (float)P.b3, beta = (float)P.beta;
        float ax = 0.f, ay = 0.f, az = 0.f;
        double ep = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0, w4 = 0.0, w5 = 0.0;
        auto pair = [&](float ex, float ey, float ez, float Fij, float Mij) {
          const float r2 = ex * ex + ey * ey + ez * ez;
          const bool in_f = r2 < rcs, in_p = r2 < phs, inc = in_f || in_p;
          const float rinv = __frsqrt_rn(inc ? r2 : 1.0f);
          const float r = r2 * rinv, x = r * ire, u = x - dd, t = x - 1.0f;
          const float poly = ((b3 * t + b2) * t + b1) * t + b0, dpoly = (3.0f * b3 * t + 2.0f * b2) * t + b1;
          const float fr = paper_f32(P, rinv);
          const float dfr = in_f ? -beta * fr * rinv : 0.0f;
          const float g = (in_p ? (2.0f * u * poly + u * u * dpoly) * ire : 0.0f) + dfr * (Fij + Mij * (2.0f * fr));
          const float sc = inc ? g * rinv : 0.0f;
          ax += sc * ex;
          ay += sc * ey;
          az += sc * ez;
          if (ENERGY) {
            ep += (double)(in_p ? 0.5f * u * u * poly : 0.0f);
            const float hs = 0.5f * sc;
            w0 -= (double)(hs * ex * ex);
            w1 -= (double)(hs * ey * ey);
            w2 -= (double)(hs * ez * ez);
            w3 -= (double)(hs * ex * ey);
            w4 -= (double)(hs * ex * ez);
            w5 -= (double)(hs * ey * ez);
          }
        };
        const float Mi = (float)dm[i];
        if (SHADOW) {
          const int4 ps = qs[i];
          const float qi = (float)(1.0 / S[c.r].qscale);
          const float Fi = __int_as_float(ps.w);
          for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                                 [&](int e) { const int j = list_slot(e); return SM{qs[j], dm[j]}; },
                                 [&](const SM& pj, int e) {
            const int4 o = ctab[list_code(e)];
            pair((float)(pj.q.x - ps.x + o.x) * qi, (float)(pj.q.y - ps.y + o.y) * qi,
                 (float)(pj.q.z - ps.z + o.z) * qi, Fi + __int_as_float(pj.q.w), Mi + (float)pj.m);
          });
        } else {
          const float Fi = (float)pi.w;
          auto pass = [&](auto img_c) {
            constexpr bool IMG = decltype(img_c)::value;
            for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                                   [&](int e) { const int j = list_slot(e); return QM{q[j], dm[j]}; },
                                   [&](const QM& pj, int) {
              pair((float)(IMG ? min_image(pj.q.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.q.x - pi.x),
                   (float)(IMG ? min_image(pj.q.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.q.y - pi.y),
                   (float)(IMG ? min_image(pj.q.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.q.z - pi.z),
                   Fi + (float)pj.q.w, Mi + (float)pj.m);
            });
          };
          if (img) pass(std::true_type{}); else pass(std::false_type{});
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
        const double Fi = pi.w, Mi = dm[i];
        auto pass = [&](auto img_c) {
          constexpr bool IMG = decltype(img_c)::value;
          for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                                 [&](int e) { const int j = list_slot(e); return QM{q[j], dm[j]}; },
                                 [&](const QM& pj, int) {
            const double ex = IMG ? min_image(pj.q.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.q.x - pi.x;
            const double ey = IMG ? min_image(pj.q.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.q.y - pi.y;
            const double ez = IMG ? min_image(pj.q.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.q.z - pi.z;
            const double r2 = ex * ex + ey * ey + ez * ez;
            const bool in_f = r2 < P.rc_sq, in_p = r2 < P.phi_sq, inc = in_f || in_p;
            const double rinv = rsq_nr(inc ? r2 : 1.0);
            const double r = r2 * rinv, x = r * P.inv_re, u = x - P.d;
            const double poly = ((P.a3 * x + P.a2) * x + P.a1) * x + P.a0;
            const double dpoly = (3.0 * P.a3 * x + 2.0 * P.a2) * x + P.a1;
            const double fr = paper_f(P, rinv);
            const double dfr = in_f ? -P.beta * fr * rinv : 0.0;
            const double g = (in_p ? (2.0 * u * poly + u * u * dpoly) * P.inv_re : 0.0) +
                             dfr * ((Fi + pj.q.w) + (Mi + pj.m) * (2.0 * fr));
            const double sc = inc ? g * rinv : 0.0;
            fx += sc * ex;
            fy += sc * ey;
            fz += sc * ez;
            if (ENERGY) {
              acc[P_PAIR] += in_p ? 0.5 * u * u * poly : 0.0;
              acc[P_WXX] -= 0.5 * sc * ex * ex;
              acc[P_WYY] -= 0.5 * sc * ey * ey;
              acc[P_WZZ] -= 0.5 * sc * ez * ez;
              acc[P_WXY] -= 0.5 * sc * ex * ey;
              acc[P_WXZ] -= 0.5 * sc * ex * ez;
              acc[P_WYZ] -= 0.5 * sc * ey * ez;
            }
          });
        };
        if (img) pass(std::true_type{}); else pass(std::false_type{});
      }
    } else if (MIXED) {
      const float cc = (float)K.c, dd = (float)K.d, c2 = (float)K.c2, rv = (float)K.rv,
                  pmin = (float)K.pmin, csq = (float)K.c_sq, dsq = (float)K.d_sq;
      float ax = 0.f, ay = 0.f, az = 0.f;
      // energy and virial terms are FP32 products, summed in FP64
      double ep = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0, w4 = 0.0, w5 = 0.0;
      // pair term for separation (ex, ey, ez) and neighbour F' fj
      auto pair = [&](float ex, float ey, float ez, float Fi, float fj) {
        const float r2 = ex * ex + ey * ey + ez * ez;
        // all lanes evaluate; the cutoffs select (no branch)
        const bool inc = r2 < csq;
        const float rinv = __frsqrt_rn(inc ? r2 : 1.0f);
        const float r = r2 * rinv;
        const float u = r - cc, t = r - rv;
        const float p = pmin + c2 * t * t;                      // c0 + c1 r + c2 r^2, vertex form
        float g = u * (2.0f * p + u * (2.0f * c2 * t));          // phi'(r)
        g += (r2 < dsq) ? (Fi + fj) * (2.0f * (r - dd)) : 0.0f;
        const float s = inc ? g * rinv : 0.0f;                   // F_i += g (q_j - q_i) / r
        ax += s * ex;
        ay += s * ey;
        az += s * ez;
        if (ENERGY) {
          ep += (double)(inc ? 0.5f * u * u * p : 0.0f);
          const float hs = 0.5f * s;
          w0 -= (double)(hs * ex * ex);
          w1 -= (double)(hs * ey * ey);
          w2 -= (double)(hs * ez * ez);
          w3 -= (double)(hs * ex * ey);
          w4 -= (double)(hs * ex * ez);
          w5 -= (double)(hs * ey * ez);
        }
      };
      if (SHADOW) {
        const int4 ps = qs[i];
        const float qi = (float)(1.0 / S[c.r].qscale);
        const float Fi = __int_as_float(ps.w);
        for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                               [&](int e) { return qs[list_slot(e)]; },
                               [&](const int4& pj, int e) {
          const int4 o = ctab[list_code(e)];
          pair((float)(pj.x - ps.x + o.x) * qi, (float)(pj.y - ps.y + o.y) * qi,
               (float)(pj.z - ps.z + o.z) * qi, Fi, __int_as_float(pj.w));
        });
      } else {
        const float Fi = (float)pi.w;
        auto pass = [&](auto img_c) {
          constexpr bool IMG = decltype(img_c)::value;
          for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                                 [&](int e) { return q[list_slot(e)]; },
                                 [&](const double4& pj, int) {
            pair((float)(IMG ? min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.x - pi.x),
                 (float)(IMG ? min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.y - pi.y),
                 (float)(IMG ? min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.z - pi.z), Fi,
                 (float)pj.w);
          });
        };
        if (img) pass(std::true_type{}); else pass(std::false_type{});
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
      auto pass = [&](auto img_c) {
      constexpr bool IMG = decltype(img_c)::value;
      for_entries<T, UNROLL>(idx, (int)i, n, c.sub, (int)K.ntot, K.lt_shift,
                             [&](int e) { return q[list_slot(e)]; },
                             [&](const double4& pj, int) {
        const double ex = IMG ? min_image(pj.x - pi.x, d.len[0], d.half[0], d.per[0]) : pj.x - pi.x;
        const double ey = IMG ? min_image(pj.y - pi.y, d.len[1], d.half[1], d.per[1]) : pj.y - pi.y;
        const double ez = IMG ? min_image(pj.z - pi.z, d.len[2], d.half[2], d.per[2]) : pj.z - pi.z;
        const double r2 = ex * ex + ey * ey + ez * ez;
        // all lanes evaluate; the cutoffs select (no branch: the whole 32-byte gather is
        // consumed up front)
        const bool inc = r2 < K.c_sq;
        const double rinv = rsq_nr(inc ? r2 : 1.0);
        const double r = r2 * rinv;
        const double u = r - K.c;
        const double p = K.c0 + r * (K.c1 + r * K.c2);
        double g = u * (2.0 * p + u * (K.c1 + 2.0 * K.c2 * r));     // phi'(r)
        // F'_j used on every path (times zero beyond d), so that the whole record is loaded
        // ahead of the arithmetic rather than its last word behind a branch
        g += (Fi + pj.w) * ((r2 < K.d_sq) ? 2.0 * (r - K.d) : 0.0);
        const double s = inc ? g * rinv : 0.0;
        fx += s * ex;
        fy += s * ey;
        fz += s * ez;
        if (ENERGY) {
          acc[P_PAIR] += inc ? 0.5 * u * u * p : 0.0;
          acc[P_WXX] -= 0.5 * s * ex * ex;
          acc[P_WYY] -= 0.5 * s * ey * ey;
          acc[P_WZZ] -= 0.5 * s * ez * ez;
          acc[P_WXY] -= 0.5 * s * ex * ey;
          acc[P_WXZ] -= 0.5 * s * ex * ez;
          acc[P_WYZ] -= 0.5 * s * ey * ez;
        }
      });
      };
      if (img) pass(std::true_type{}); else pass(std::false_type{});
    }
  }
  fx = group_sum<T>(fx);
  fy = group_sum<T>(fy);
  fz = group_sum<T>(fz);
  const bool own = c.live && c.sub == 0;
  constexpr bool KIN = ENERGY && DRIFT;   // the k_kinetic terms into KO (see KinOut)
  double ke[1] = {0.0}, mo[4] = {0.0, 0.0, 0.0, 0.0};
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0);   // with DRIFT: the atom's next position
  double d2 = 0.0;                                 // and its squared displacement since the build
  if (own) {
    const int64_t i = c.i;
    // every value read here is loaded before the first store (a store could alias a later
    // load, which would then wait for it) and used on every path (selects, not branches: a
    // load used only past a branch is made there), so the loads go out together
    const int xn = fme ? xcnt[i] : 0;
    const bool move = KICK && !fixed[i];
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (KICK) {
      v0 = v[3 * i + 0];
      v1 = v[3 * i + 1];
      v2 = v[3 * i + 2];
    }
    double4 qi = make_double4(0.0, 0.0, 0.0, 0.0);
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
    if (DRIFT) {
      qi = SHADOW ? q[i] : pi;   // (loaded above on the FP64-separation paths)
      r0 = D.xref[3 * i + 0];
      r1 = D.xref[3 * i + 1];
      r2 = D.xref[3 * i + 2];
    }
    if (xn > 0) {   // the Cr-C force of this step (atoms with carbons in range)
      fx += fme[4 * i + 0];
      fy += fme[4 * i + 1];
      fz += fme[4 * i + 2];
      if (KIN) {   // (records of atoms without carbons in range are zero)
        mo[0] = fme[4 * i + 3];
        mo[1] = -fme[4 * i + 0];
        mo[2] = -fme[4 * i + 1];
        mo[3] = -fme[4 * i + 2];
      }
    }
    if (!DRIFT && store_f) {   // (a pass that also gives the next step's first half kick
                               // leaves f alone: no kick reads it before the next pass that
                               // stores it; drifting passes are such passes)
      f[3 * i + 0] = fx;
      f[3 * i + 1] = fy;
      f[3 * i + 2] = fz;
    }
    if (!(fabs(fx) + fabs(fy) + fabs(fz) < INFINITY)) S[c.r].nonfinite = 1;
    if (KICK) {   // kick_h = dt a / 2 (Task 5), or dt a (with the next Task 3's); fixed atoms
                  // keep their velocity (written back unchanged)
      double vx = move ? v0 + kick_h * fx : v0, vy = move ? v1 + kick_h * fy : v1,
             vz = move ? v2 + kick_h * fz : v2;
      if (KIN) {   // kinetic energy at the whole step, then the next half kick
        if (move) {
          ke[0] = K.ke_fac * ((vx * vx + vy * vy) + vz * vz);
          vx += kick_h * fx;
          vy += kick_h * fy;
          vz += kick_h * fz;
        }
      }
      v[3 * i + 0] = vx;
      v[3 * i + 1] = vy;
      v[3 * i + 2] = vz;
      if (DRIFT) {   // x(t + dt) = x + v(t + dt/2) dt into the other buffer (fixed: copied)
        p = qi;
        if (move) {
          p.x += vx * K.dt;
          p.y += vy * K.dt;
          p.z += vz * K.dt;
        }
      }
    } else if (DRIFT) {
      p = qi;
    }
    if (DRIFT) {
      D.q[i] = p;
      if (K.shadow) D.qs[i] = cell_local(S[c.r], D.bcell[i], p.x, p.y, p.z, (float)p.w);
      const double ex = p.x - r0, ey = p.y - r1, ez = p.z - r2;
      d2 = (ex * ex + ey * ey) + ez * ez;
      if (!(d2 == d2)) d2 = INFINITY;   // NaN positions force a rebuild (and get flagged there)
    }
  }
  if (DRIFT) {
    // the part's displacement maximum and box (minima as maxima of the negated coordinates)
    double m[7] = {d2, own ? -p.x : -INFINITY, own ? -p.y : -INFINITY, own ? -p.z : -INFINITY,
                   own ? p.x : -INFINITY, own ? p.y : -INFINITY, own ? p.z : -INFINITY};
    block_max_to0<BLOCK, 7>(m);
    if (threadIdx.x == 0) {
      D.dmax[c.blk] = m[0];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        D.tbox[6 * (int64_t)c.blk + a] = -m[1 + a];
        D.tbox[6 * (int64_t)c.blk + 3 + a] = m[4 + a];
      }
      if (c.blk == d.t0 * T) {   // Task 2, once per replica (the observed step's position kept)
        if (KIN) S[c.r].ind_z_obs = S[c.r].ind_z;
        S[c.r].ind_z += K.v_ind * K.dt;
      }
    }
  }
  if (ENERGY) block_sum_store<NP_FORCE, BLOCK>(acc, part + (int64_t)c.blk * NP_FORCE);
  if (KIN) {
    block_sum_store<1, BLOCK>(ke, KO.kin + c.blk);
    block_sum_store<4, BLOCK>(mo, KO.morse + (int64_t)c.blk * 4);
  }
}

// Task 5 alone.
__global__ __launch_bounds__(BLOCK) void k_kick(Consts K, const RepDesc* __restrict__ R,
                                                const int* __restrict__ tile_rep,
                                                double* __restrict__ v, const double* __restrict__ f,
                                                const uint8_t* __restrict__ fixed) {
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const RepDesc& d = R[tile_rep[tile]];
  const int64_t i = (int64_t)tile * TILE + threadIdx.x;
  if (i >= (int64_t)d.a0 + d.n || fixed[i]) return;
  const double h = 0.5 * K.dt * K.acc;
  v[3 * i + 0] += h * f[3 * i + 0];
  v[3 * i + 1] += h * f[3 * i + 1];
  v[3 * i + 2] += h * f[3 * i + 2];
}

}  // namespace md
