// Device-side data structures and helpers shared by the MD kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md.h"

namespace md {

constexpr int TILE = MD_TILE;   // atoms per tile (replica ranges are tile aligned)
constexpr int BLOCK = 256;      // threads of the atom-parallel kernels (one tile per block)
constexpr int WAVE = 64;

// (eV / (Angstrom u)) -> Angstrom / fs^2, from e = 1.602176634e-19 C and u = 1.66053906660e-27 kg.
constexpr double ACC_CONV = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;

// One replica as the kernels see it (read only).
struct RepDesc {
  double lo[3];
  double len[3];
  double half[3];
  int per[3];
  int a0, n, npad;      // first atom slot, atom count, padded slot count
  int c0, nc;           // first carbon, carbon count
  int t0, nt;           // first tile, tile count
  int g0, gcap[3];      // Cr-Cr cell grid: first cell (global), allocated dims (the dims in
                        // use along open axes follow the atoms, see RepState)
  int h0, hd[3];        // Cr-C cell grid: first cell (global, after all Cr grids), dims
  int rb0, nseg;        // list build: first cell row at capacity (global numbering), most runs per row
  int ch0, nch;         // energy sums: first chunk of tiles, chunk count
  double ginv[3];       // cells per Angstrom of the Cr grid along periodic axes
  double hinv[3];       // cells per Angstrom of the carbon grid
};

// Mutable per-replica flags and counters.
struct alignas(64) RepState {
  double ind_z;           // indenter displacement along z
  double ind_z_ref;       // ind_z at the last list build
  double ind_z_obs;       // ind_z of the step whose energies a force pass took (KinOut)
  int rebuild;            // 1: the next k_rebuild rebuilds this replica
  int nbuilds;
  int overflow;           // needed Cr-Cr capacity (0 = fits)
  int xoverflow;          // needed Cr-C capacity
  int nonfinite;
  int sync_timeout;
  int nnear;              // Cr atoms within reach of the carbons (entries of the near list)
  int nnear_old;          // entries of the previous build's near list (during a rebuild)
  int ioverflow;          // needed inner-list capacity (two-tier lists; 0 = fits)
  // Cr cell grid of the current build: origin, cells per Angstrom, dims (<= gcap).  Along
  // periodic axes it is the box; along open axes it spans the atoms' current extent.
  double glo[3], ginv[3];
  double gedge[3];        // cell edge of that grid (1 / ginv)
  double qscale;          // fixed-point scale of the shadow positions (a power of two)
  int gd[3];
};

// A Cr-Cr list entry holds the neighbour's slot in its low LIST_IDX_BITS bits and, above
// them, the neighbour's cell relative to the atom's cell at the build: code = 9 (dz + 1) +
// 3 (dy + 1) + (dx + 1) with dx, dy, dz in {-1, 0, 1}, counted across periodic faces.
constexpr int LIST_IDX_BITS = 27;
constexpr int LIST_IDX_MASK = (1 << LIST_IDX_BITS) - 1;
__device__ __forceinline__ int list_slot(int e) { return e & LIST_IDX_MASK; }
__device__ __forceinline__ int list_code(int e) { return (int)((unsigned)e >> LIST_IDX_BITS); }

// Build cell of an atom, packed 21 bits per axis.
__device__ __forceinline__ long long pack_cell(int cx, int cy, int cz) {
  return (long long)cx | ((long long)cy << 21) | ((long long)cz << 42);
}
// Shadow position of an atom for the FP32-mixed passes: its offset from the centre of its
// build cell in fixed point (units of 1 / qscale, with qscale chosen so a cell edge is at
// most 2^29 units), and F' as FP32 bits in w.  The separation of two atoms is then an exact
// integer sum -- shadow_j - shadow_i + (relative cell) x edge -- rounded once to FP32, the
// same rounding as an FP64 separation converted to FP32.
__device__ __forceinline__ int4 cell_local(const RepState& s, long long bc, double x, double y, double z, float w) {
  const int cx = (int)(bc & 0x1FFFFF), cy = (int)((bc >> 21) & 0x1FFFFF), cz = (int)((bc >> 42) & 0x1FFFFF);
  return make_int4((int)rint((x - (s.glo[0] + (cx + 0.5) * s.gedge[0])) * s.qscale),
                   (int)rint((y - (s.glo[1] + (cy + 0.5) * s.gedge[1])) * s.qscale),
                   (int)rint((z - (s.glo[2] + (cz + 0.5) * s.gedge[2])) * s.qscale), __float_as_int(w));
}

// The paper's EAM form (Appendix, Eqs. A1-A4), in the terms the kernels use.
struct PaperConsts {
  double Fo, n, rho_e, alpha, P_e, fe, re, beta;
  double a0, a1, a2, a3, d;
  double rc_sq;       // f (and f^2) for r < rc
  double phi_sq;      // Phi for r < d re
  double inv_re, re2;
  double b0, b1, b2, b3;   // the same cubic in t = x - 1 (b_k = poly^(k)(1) / k!, in FP64): its
                           // terms stay small near the neighbour shells, so FP32 evaluation does
                           // not lose digits to the cancelling large a_k
  int bh;             // beta / 2 when it is a whole number 1..8 (then f needs r^2 only), else 0
};

// f(r) = fe (re / r)^beta from r^2 and 1/r: (re^2 / r^2)^(beta/2) by repeated squaring when
// beta / 2 is a whole number, else through pow.
__device__ __forceinline__ double paper_f(const PaperConsts& P, double rinv) {
  if (P.bh > 0) {
    const double t = P.re2 * (rinv * rinv);
    double f = 1.0, b = t;
    for (int e = P.bh; e; e >>= 1) {   // uniform over the wavefront
      if (e & 1) f *= b;
      b *= b;
    }
    return P.fe * f;
  }
  return P.fe * pow(P.re * rinv, P.beta);
}
__device__ __forceinline__ float paper_f32(const PaperConsts& P, float rinv) {
  if (P.bh > 0) {
    const float t = (float)P.re2 * (rinv * rinv);
    float f = 1.0f, b = t;
    for (int e = P.bh; e; e >>= 1) {
      if (e & 1) f *= b;
      b *= b;
    }
    return (float)P.fe * f;
  }
  return (float)P.fe * __powf((float)P.re * rinv, (float)P.beta);
}

// Per atom: F(rho), F'(rho) (0 without neighbours), M(P), M'(P) of Eq. A3, in FP64.
//   F' = Fo n^2 (rho/rho_e)^n ln(rho/rho_e) / rho;  M' = (2 alpha / P_e) u (1 - u^2) exp(-u^2),
//   u = P / P_e - 1.
struct PaperEmbed {
  double F, dF, M, dM;
};
__device__ __forceinline__ PaperEmbed paper_embed(const PaperConsts& P, double rho, double p) {
  PaperEmbed e;
  if (rho > 0.0) {
    const double lt = log(rho / P.rho_e), tn = exp(P.n * lt);
    e.F = -P.Fo * (1.0 - P.n * lt) * tn;
    e.dF = P.Fo * P.n * P.n * tn * lt / rho;
  } else {
    e.F = 0.0;
    e.dF = 0.0;
  }
  const double u = p / P.P_e - 1.0, w = exp(-u * u);
  e.M = P.alpha * u * u * w;
  e.dM = 2.0 * P.alpha / P.P_e * u * (1.0 - u * u) * w;
  return e;
}

// Constants of the potential and the integrator (passed by value).
struct Consts {
  // EAM
  double A, c, d, c0, c1, c2;
  double c_sq, d_sq;      // cutoffs squared
  double rv, pmin;        // vertex form of c0 + c1 r + c2 r^2 = pmin + c2 (r - rv)^2
  // Morse
  double D, alpha, r0, mrc, mrc_sq, mshift;
  // integration / lists
  double acc;             // ACC_CONV / mass: acceleration per unit force
  double ke_fac;          // mass / (2 ACC_CONV): kinetic energy per v^2
  double dt, v_ind;
  double half_skin, half_skin_sq;
  double rlist_sq, rxlist_sq;
  double rlist;           // cutoff + skin
  double icut_sq;         // two-tier lists: the inner list's radius (the largest Cr-Cr cutoff), squared
  int cap, xcap;
  int icap;               // two-tier lists: inner-list capacity (0: one list)
  int nrep;
  int lt;                 // list interleave: entries k..k+lt-1 of an atom are adjacent
  int lt_shift;           // log2(lt)
  int shadow;             // 1: keep the FP32 cell-local shadow of the positions
  int pot;                // MD_POT_FS or MD_POT_PAPER
  int64_t ntot;           // atom slots (all replicas)
  PaperConsts P;          // the paper's form (pot == MD_POT_PAPER)
};

// Order-preserving map of a double to an unsigned 64-bit integer (for atomic min/max).
__device__ __forceinline__ unsigned long long ordered_bits(double v) {
  unsigned long long b = __double_as_longlong(v);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered_bits(unsigned long long b) {
  b = (b & 0x8000000000000000ull) ? (b & 0x7fffffffffffffffull) : ~b;
  return __longlong_as_double(b);
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run of
// logical blocks so that neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nb) {
  int per = nb >> 3;
  if (bid < (per << 3)) return (bid & 7) * per + (bid >> 3);
  return bid;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Sum K values over a block of NT threads (NT multiple of 64) in a fixed order; thread
// t < K of the block receives sum k = t in out[t].  Contains __syncthreads.
template <int K, int NT>
__device__ __forceinline__ void block_sum_store(double (&v)[K], double* out) {
  constexpr int NW = NT / WAVE;
  __shared__ double sh[K][NW];
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += sh[threadIdx.x][i];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Maxima over the block of N values per thread, delivered to thread 0 only (one barrier;
// call once per block).
template <int NT, int N>
__device__ __forceinline__ void block_max_to0(double (&v)[N]) {
  constexpr int NW = NT / WAVE;
  __shared__ double sh[NW][N];
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_max(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) sh[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k)
      for (int i = 1; i < NW; ++i) v[k] = fmax(v[k], sh[i][k]);
}

template <int NT>
__device__ __forceinline__ double block_max(double v) {
  constexpr int NW = NT / WAVE;
  __shared__ double sh[NW];
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  v = wave_max(v);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double m = sh[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) m = fmax(m, sh[i]);
  __syncthreads();
  return m;
}

// Minimum-image component of a separation along one axis: d - len if d > len/2, d + len if
// d < -len/2 (periodic axes only).  Written as selects so that it compiles without branches.
__device__ __forceinline__ double min_image(double d, double len, double half, int per) {
  // d + (-len) rounds exactly like d - len; the shift is chosen with selects on constants
  double s = (per && d > half) ? -len : 0.0;
  s = (per && d < -half) ? len : s;
  return d + s;
}

// 1/sqrt(x) for a positive normal x: the hardware estimate refined by one cubic Newton step
// (y (1 + e/2 + 3 e^2 / 8) with e = 1 - x y^2), accurate to about an ulp.  The same
// steps as the math library's rsqrt without its fix-up of zero, infinite and denormal
// arguments, which the callers never pass.
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// True if some live atom of the wavefront lies within `margin` of a periodic face of its
// replica's box (every lane calls it).  A listed pair can cross a face only if one of its
// atoms was within r_list of that face at the build and has moved less than skin / 2 since,
// so with margin = r_list + skin every listed pair of a wavefront for which this is false
// has its minimum image equal to the plain difference of the positions.
__device__ __forceinline__ bool wave_near_face(const RepDesc& d, bool live, double x, double y, double z,
                                               double margin) {
  const double p[3] = {x, y, z};
  bool near = false;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    near |= d.per[a] && !(p[a] - d.lo[a] >= margin && d.lo[a] + d.len[a] - p[a] >= margin);
  return __ballot(live && near) != 0;
}

// Squared length (dx dx + dy dy) + dz dz with every product and sum rounded on its own:
// the exact list predicate, evaluated identically wherever a list is built.
__device__ __forceinline__ double dist_sq_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double xx = dx * dx;
  double yy = dy * dy;
  double zz = dz * dz;
  double s = xx + yy;
  return s + zz;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Cell coordinate along one axis, clamped into the grid (also for far-away or NaN x).
__device__ __forceinline__ int cell_coord(double x, double lo, double inv, int dim) {
  double t = floor((x - lo) * inv);
  t = fmin(fmax(t, 0.0), (double)(dim - 1));
  return (int)t;
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

// Value of `v` in lane `l` (l uniform across the wavefront), as a scalar.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffull), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Orders the LDS accesses of one wavefront (lanes exchanging data through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work items spread over replicas (e.g. each replica's near atoms), flattened into one index
// space so that every wavefront of a launch gets the same share whatever the replica sizes:
// pre[r] = items of replicas before r (a block-wide scan into shared memory, called by the
// whole block), and item g belongs to the replica r with pre[r] <= g < pre[r + 1].
constexpr int FLAT_MAXREP = 2048;

template <class Count>
__device__ int flat_prefix(int nrep, int* pre, Count count) {
  int carry = 0;
  for (int r0 = 0; r0 < nrep; r0 += BLOCK) {
    const int r = r0 + threadIdx.x;
    const int c = r < nrep ? count(r) : 0;
    int tot;
    const int ex = block_exclusive_scan(c, &tot);
    if (r < nrep) pre[r] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) pre[nrep] = carry;
  __syncthreads();
  return carry;
}

__device__ __forceinline__ int flat_replica(const int* pre, int nrep, int g) {
  int lo = 0, hi = nrep - 1;   // the largest r with pre[r] <= g (empty replicas are skipped)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Slot of entry k of atom i in the Cr-Cr list (interleave T: entries k..k+T-1 of one atom
// are adjacent, so T lanes of one atom read consecutive words).
__device__ __forceinline__ int list_pos(int k, int i, int ntot, int T, int Tshift) {
  return ((k >> Tshift) * ntot + i) * T + (k & (T - 1));
}

// Values the same on every lane of a wavefront, moved to scalar registers (the compiler
// keeps loads through pointers it cannot prove read-only in vector registers).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The 27-cell stencil, one axis at a time: offsets t = 0..stencil_n-1 map to cells
// c-1, c, c+1 (periodic wrap, or -1 = outside an open axis).  A periodic axis with fewer
// than 3 cells visits each of its cells once instead, so no cell is met twice.
__device__ __forceinline__ int stencil_n(int gd, int per) { return (per && gd < 3) ? gd : 3; }
__device__ __forceinline__ int stencil_cell(int c, int t, int gd, int per) {
  if (per && gd < 3) return t;
  int x = c + t - 1;
  if (per) return x < 0 ? x + gd : (x >= gd ? x - gd : x);
  return (x < 0 || x >= gd) ? -1 : x;
}

}  // namespace md
