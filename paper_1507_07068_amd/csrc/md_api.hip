// Host side of the C ABI declared in include/md.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "md.h"
#include "md_kernels.hip"

using namespace md;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Byte offsets of the workspace regions.
struct Layout {
  size_t desc, state, tile_rep, row_rep, items, c_rep, misc, chunks, chunk_out, xref, dmax, tbox, cellid, crank, perm, skey, tq, tqf, qs, q2, qs2, bcell, tv,
      tf, tfixed, tid, count, start, hcell, hrank, hlist, hsorted, scan_state, hnear, near, fme, p_embed, p_force,
      p_morse, p_kin, dm, dmax_p, tbox_p, total;
};

constexpr int MISC_INTS = 16;    // rebuild flag, status words
// The list build takes one block per work item while the item table's capacity is at most
// this many waves of resident blocks (six per compute unit): measured faster on the
// 216k-atom film (3 waves: 63 against 76 us per rebuild), slower on the 1M-atom film (15
// waves: 203 against 196 us, and 6.7 against 4.4 us for a step without a rebuild) and on the
// 8M-atom film (~110 waves of idle blocks per step), even on the 64-replica ensemble (~32).
constexpr int LIST_ONE_PER_ITEM_WAVES = 8;
constexpr int SCAN_CHUNK = 2048; // cells per block of the cell-count scan
constexpr int64_t DECIDE_IN_BIN_MAX_LOADS = (int64_t)1 << 22;   // part loads over all k_bin blocks
constexpr int PARTS_REDUCED = 64;   // partial reductions of a large single replica's parts
constexpr int MAXREP = 16384;    // replicas per system

}  // namespace

struct md_system {
  md_params p;
  int nrep;
  std::vector<RepDesc> desc;
  std::vector<int> tile_rep;
  std::vector<int> row_rep;    // replica of each cell row at capacity
  std::vector<int> c_rep;
  std::vector<int2> chunks;    // energy sums: (first tile, tile count) of each chunk
  int64_t ntot, ctot;
  int ntiles;
  int nlblk;     // blocks of the list build (most work items)
  int nrows;     // cell rows at capacity, all replicas
  int ncell_cr, ncell_all;
  Consts K;
  Layout L;
  char* ws;
  int scan_blocks;
  bool list_mix;   // some periodic axis has fewer than 3 list cells
  bool have_embed, have_force;
  // md_run's energy steps other than the last take the kinetic energy inside the force pass
  // (KinOut); MD_FUSE_ENERGY=0 in the environment at creation: by a pass of its own
  bool fuse_energy = true;
  // Inside md_run the positions alternate between the caller's q (with the workspace
  // shadow qs) and the workspace pair q2, qs2: cur says which holds the current ones
  // (outside md_run always the caller's).  ppt: parts per tile of the last displacement
  // maxima and boxes (1 from the kick-drift pass, T from a force pass with the drift).
  int cur = 0, ppt = 1;
  // grids of the build kernels that stride over their work (set at bind from the device):
  // tile kernels (256 threads) and the persistent list build
  int tile_grid = 2048, list_grid = 2048;
  int list_tgt = LIST_TGT;   // atoms a list-build work item aims at
  int static_dev = -1;   // device whose static scratch is the workspace (md_workspace_bind_static)
};

// The workspace of md_workspace_bind_static: a file-scope device array, one copy per GPU
// (each at its own address), held until the process ends.  Host code never names it except
// to look up that address: g_scratch_ptr[dev] holds it, taken once per device with the
// device current.
static __device__ __align__(256) unsigned char scratch[MD_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];                            // device address of `scratch`
std::atomic<const md_system*> g_scratch_owner[MAX_DEVICES];  // the system bound to it

// A workspace is bound, and if it is a device's static scratch no other system has taken
// that scratch over since.
bool bound(const md_system* s) {
  return s->ws && (s->static_dev < 0 || g_scratch_owner[s->static_dev].load() == s);
}
}  // namespace

namespace {

int cells_along(double len, double edge) {
  double n = std::floor(len / (edge * (1.0 + 1e-9)));
  return n < 1.0 ? 1 : (int)n;
}

Layout make_layout(const md_system& s) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t n = (size_t)s.ntot, nt = (size_t)s.ntiles;
  L.desc = take(sizeof(RepDesc) * s.nrep);
  L.state = take(sizeof(RepState) * s.nrep);
  L.tile_rep = take(sizeof(int) * nt);
  L.row_rep = take(sizeof(int) * (size_t)s.nrows);
  L.items = take(sizeof(int2) * (size_t)s.nlblk);
  L.c_rep = take(sizeof(int) * (size_t)s.ctot);
  L.misc = take(sizeof(int) * MISC_INTS);
  L.chunks = take(sizeof(int2) * s.chunks.size());
  L.chunk_out = take(sizeof(double) * 16 * s.chunks.size());
  L.xref = take(sizeof(double) * 3 * n);
  L.dmax = take(sizeof(double) * nt * 8);       // per tile, or per part of a tile (up to 8)
  L.tbox = take(sizeof(double) * 6 * nt * 8);
  L.cellid = take(sizeof(int) * n);
  L.crank = take(sizeof(int) * n);
  L.perm = take(sizeof(int) * n);
  L.skey = take(sizeof(long long) * n);
  L.tq = take(sizeof(double) * 4 * n);
  L.tqf = take(sizeof(float) * 4 * n);
  L.qs = take(sizeof(int) * 4 * n);
  L.q2 = take(sizeof(double) * 4 * n);   // md_run's second position buffer
  L.qs2 = take(sizeof(int) * 4 * n);
  L.bcell = take(sizeof(long long) * n);
  L.tv = take(sizeof(double) * 3 * n);
  L.tf = take(sizeof(double) * 3 * n);
  L.tfixed = take(n);
  L.tid = take(sizeof(int) * n);
  L.count = take(sizeof(int) * (size_t)s.ncell_all);
  L.start = take(sizeof(int) * ((size_t)s.ncell_all + 1));
  L.hcell = take(sizeof(int) * (size_t)s.ctot);
  L.hrank = take(sizeof(int) * (size_t)s.ctot);
  L.hlist = take(sizeof(int) * (size_t)s.ctot);
  L.hsorted = take(sizeof(double4) * (size_t)s.ctot);
  L.scan_state = take(sizeof(long long) * (size_t)s.scan_blocks);
  L.hnear = take(sizeof(int) * (size_t)s.ncell_all);
  L.near = take(sizeof(int) * n);
  L.fme = take(sizeof(double) * 4 * n);
  L.dm = take(sizeof(double) * n);       // M'(P_i) of the paper's form
  L.dmax_p = take(sizeof(double) * PARTS_REDUCED);   // k_parts_reduce's partial maxima and boxes
  L.tbox_p = take(sizeof(double) * 6 * PARTS_REDUCED);
  L.p_embed = take(sizeof(double) * nt * s.K.lt);
  L.p_force = take(sizeof(double) * nt * s.K.lt * NP_FORCE);
  // k_kinetic's partials per tile, or those of a force pass that takes them (per block)
  L.p_morse = take(sizeof(double) * nt * s.K.lt * 4);
  L.p_kin = take(sizeof(double) * nt * s.K.lt);
  L.total = o;
  return L;
}

template <class T>
T* at(const md_system* s, size_t off) {
  return reinterpret_cast<T*>(s->ws + off);
}

int hip_status(hipError_t e) {
  if (e == hipSuccess) return MD_OK;
  std::fprintf(stderr, "md: HIP error %d: %s\n", (int)e, hipGetErrorString(e));
  return MD_ERR_HIP;
}

int check_launch() { return hip_status(hipGetLastError()); }

bool atoms_ok(const md_atoms* a) {
  return a && a->q && a->v && a->f && a->fixed && a->id;
}

bool lists_ok(const md_system* s, const md_lists* l) {
  return l && l->idx && l->cnt && l->xidx && l->xcnt && (s->p.icap == 0 || (l->iidx && l->icnt));
}

// The Cr-Cr list the density and force passes read: the inner list with two-tier lists.
const int* pass_idx(const md_system* s, const md_lists* l) { return s->p.icap ? l->iidx : l->idx; }
const int* pass_cnt(const md_system* s, const md_lists* l) { return s->p.icap ? l->icnt : l->cnt; }

int grid_tiles(const md_system* s) { return s->ntiles; }

// Current and next position buffers (see md_system::cur).
double4* qcur(md_system* s, const md_atoms* a) {
  return s->cur ? at<double4>(s, s->L.q2) : reinterpret_cast<double4*>(a->q);
}
double4* qnext(md_system* s, const md_atoms* a) {
  return s->cur ? reinterpret_cast<double4*>(a->q) : at<double4>(s, s->L.q2);
}
int4* qscur(md_system* s) { return at<int4>(s, s->cur ? s->L.qs2 : s->L.qs); }
int4* qsnext(md_system* s) { return at<int4>(s, s->cur ? s->L.qs : s->L.qs2); }

// Polls of the cell-count scan's bounded wait before a build gives up: 2^22, or the value of
// MD_SCAN_SPIN_LIMIT in the environment at the time of the build (a negative value gives up
// at once: tests force the give-up path with it).
int scan_spin_limit() {
  const char* e = std::getenv("MD_SCAN_SPIN_LIMIT");
  return e ? std::atoi(e) : (1 << 22);
}

// The list build's work distribution (see build_chain).
bool list_persistent(const md_system* s) {
  const char* e = std::getenv("MD_LIST_PERSISTENT");
  if (e && *e) return std::atoi(e) != 0;
  return s->nlblk > LIST_ONE_PER_ITEM_WAVES * s->list_grid;
}

// Grid of the kernels that walk the near-indenter atoms (one wavefront per atom, grid-stride).
int near_blocks(const md_system* s) { return std::max(1, std::min(2048, s->ntiles)); }
// Blocks of the Cr-C pass inside a density launch: about one wavefront per three carbons'
// worth of near atoms (their count is known only on the device), 64 .. 2048.
int morse_fused_blocks(const md_system* s) {
  return (int)std::min<int64_t>(2048, std::max<int64_t>(64, (s->ctot + 11) / 12));
}

}  // namespace

namespace {

template <int T>
// morse: the leading blocks of the launch also run the Cr-C pass into fme (for a force
// pass that adds it)
void launch_density(md_system* s, const md_atoms* a, const md_lists* l, bool mixed, bool energy,
                    double* rho_out, bool morse, hipStream_t st) {
  const RepDesc* R = at<RepDesc>(s, s->L.desc);
  RepState* S = at<RepState>(s, s->L.state);
  const int* tr = at<int>(s, s->L.tile_rep);
  double4* q = qcur(s, a);
  double* pe = at<double>(s, s->L.p_embed);
  const MorseIn M{a->xc, l->xidx, l->xcnt, at<int>(s, s->L.near), at<double>(s, s->L.fme),
                  morse ? morse_fused_blocks(s) : 0};
  const int nb = s->ntiles * T + M.nblocks;
  int4* qs = qscur(s);
  double* dm = at<double>(s, s->L.dm);
  const int *li = pass_idx(s, l), *lc = pass_cnt(s, l);
#define DENS(M_, SH, E, PA) \
  k_density<T, M_, SH, E, PA><<<nb, BLOCK, 0, st>>>(s->K, R, S, tr, q, qs, li, lc, rho_out, pe, M, dm)
#define DENS_P(M_, SH, E) \
  if (s->K.pot == MD_POT_PAPER) DENS(M_, SH, E, true); else DENS(M_, SH, E, false)
  if (mixed && s->K.shadow && !s->list_mix) { if (energy) { DENS_P(true, true, true); } else { DENS_P(true, true, false); } }
  else if (mixed) { if (energy) { DENS_P(true, false, true); } else { DENS_P(true, false, false); } }
  else { if (energy) { DENS_P(false, false, true); } else { DENS_P(false, false, false); } }
#undef DENS_P
#undef DENS
}

template <int T>
// add_fme: the force includes the Cr-C force of this step from fme; full_kick: the kick is
// dt a (the two half kicks of Task 5 and the next step's Task 3 at once), else dt a / 2;
// drift (with full_kick or fuse_ke): the pass also drifts the atoms into the next position
// buffer; fuse_ke (with kick and energy): the two half kicks around an observed whole step,
// with its kinetic energy and Cr-C sums (KinOut).
void launch_force(md_system* s, const md_atoms* a, const md_lists* l, bool mixed, bool kick, bool energy,
                  bool add_fme, hipStream_t st, bool full_kick, bool drift, bool fuse_ke) {
  const double kick_h = (full_kick ? 1.0 : 0.5) * s->K.dt * s->K.acc;
  const int store_f = (full_kick || fuse_ke) ? 0 : 1;
  // (an energy pass with the drift takes the kinetic terms: fuse_ke implies drift, and only
  // such a pass drifts with energies)
  const KinOut KO{at<double>(s, s->L.p_kin), at<double>(s, s->L.p_morse)};
  const DriftOut D{qnext(s, a), qsnext(s), at<double>(s, s->L.xref), at<long long>(s, s->L.bcell),
                   at<double>(s, s->L.dmax), at<double>(s, s->L.tbox)};
  const RepDesc* R = at<RepDesc>(s, s->L.desc);
  RepState* S = at<RepState>(s, s->L.state);
  const int* tr = at<int>(s, s->L.tile_rep);
  const double4* q = qcur(s, a);
  double* pf = at<double>(s, s->L.p_force);
  const int nb = s->ntiles * T;
  const int4* qs = qscur(s);
  const double* dm = at<double>(s, s->L.dm);
  const bool paper = s->K.pot == MD_POT_PAPER;
  const int *li = pass_idx(s, l), *lc = pass_cnt(s, l);
#define FORCE1(M, SH, KI, E, PA)                                                                                \
  k_force<T, M, SH, KI, E, false, PA><<<nb, BLOCK, 0, st>>>(s->K, R, S, tr, q, qs, a->v, a->f, a->fixed, li,     \
                                                             lc, pf, l->xcnt,                                    \
                                                             add_fme ? at<double>(s, s->L.fme) : nullptr, kick_h, D, dm, store_f, KO)
#define FORCE(M, SH, KI, E) \
  if (paper) FORCE1(M, SH, KI, E, true); else FORCE1(M, SH, KI, E, false)
#define FORCE_DRIFT1(M, SH, E, PA)                                                                               \
  k_force<T, M, SH, true, E, true, PA><<<nb, BLOCK, 0, st>>>(                                                    \
      s->K, R, S, tr, q, qs, a->v, a->f, a->fixed, li, lc, pf, l->xcnt,                                          \
      add_fme ? at<double>(s, s->L.fme) : nullptr, kick_h, D, dm, store_f, KO)
#define FORCE_DRIFT2(M, SH, E) \
  if (paper) FORCE_DRIFT1(M, SH, E, true); else FORCE_DRIFT1(M, SH, E, false)
#define FORCE_DRIFT(M, SH) \
  if (energy) { FORCE_DRIFT2(M, SH, true); } else { FORCE_DRIFT2(M, SH, false); }
#define FORCE_E(M, SH, KI) \
  if (energy) { FORCE(M, SH, KI, true); } else { FORCE(M, SH, KI, false); }
#define FORCE_K(M, SH) \
  if (kick) { FORCE_E(M, SH, true); } else { FORCE_E(M, SH, false); }
  if (drift) {
    if (mixed && s->K.shadow && !s->list_mix) { FORCE_DRIFT(true, true); }
    else if (mixed) { FORCE_DRIFT(true, false); }
    else { FORCE_DRIFT(false, false); }
  } else if (mixed && s->K.shadow && !s->list_mix) { FORCE_K(true, true); }
  else if (mixed) { FORCE_K(true, false); }
  else { FORCE_K(false, false); }
#undef FORCE_DRIFT
#undef FORCE_DRIFT2
#undef FORCE_DRIFT1
#undef FORCE_K
#undef FORCE_E
#undef FORCE
#undef FORCE1
}

// add_f: the Cr-C forces are added into f (else only recorded in fme)
void launch_morse(md_system* s, const md_atoms* a, const md_lists* l, bool mixed, bool kick, bool add_f,
                  hipStream_t st) {
  const RepDesc* R = at<RepDesc>(s, s->L.desc);
  const RepState* S = at<RepState>(s, s->L.state);
  const double4* q = qcur(s, a);
  const int* nr = at<int>(s, s->L.near);
  double* fme = at<double>(s, s->L.fme);
  const int nb = near_blocks(s);
#define MORSE(M, KI, AF) \
  k_morse<M, KI, AF><<<nb, BLOCK, 0, st>>>(s->K, R, S, q, a->v, a->f, a->fixed, a->xc, l->xidx, l->xcnt, nr, fme)
  if (!add_f) { if (mixed) MORSE(true, false, false); else MORSE(false, false, false); }
  else if (mixed) { if (kick) MORSE(true, true, true); else MORSE(true, false, true); }
  else { if (kick) MORSE(false, true, true); else MORSE(false, false, true); }
#undef MORSE
}

}  // namespace

extern "C" {

MD_API const char* md_strerror(int code) {
  switch (code) {
    case MD_OK: return "ok";
    case MD_ERR_ARG: return "invalid argument";
    case MD_ERR_HIP: return "HIP runtime error";
    case MD_ERR_STATE: return "no workspace bound";
    default: return "unknown error";
  }
}

MD_API int md_system_create(const md_replica_desc* reps, int32_t nrep, const md_params* p,
                            md_system** out) {
  if (!out) return MD_ERR_ARG;
  *out = nullptr;
  if (!reps || !p || nrep < 1 || nrep > MAXREP) return MD_ERR_ARG;
  if (!(p->mass > 0) || !(p->dt > 0) || !(p->skin >= 0) || p->cap < 1 || p->xcap < 1) return MD_ERR_ARG;
  if (p->tpa != 1 && p->tpa != 2 && p->tpa != 4 && p->tpa != 8) return MD_ERR_ARG;
  if (p->cap % p->tpa != 0) return MD_ERR_ARG;
  if (p->icap < 0 || p->icap % p->tpa != 0) return MD_ERR_ARG;
  if (p->list_tgt != 0 && (p->list_tgt < 32 || p->list_tgt > LIST_BLOCK)) return MD_ERR_ARG;
  if (p->potential != MD_POT_FS && p->potential != MD_POT_PAPER) return MD_ERR_ARG;
  if (p->potential == MD_POT_FS && (!(p->eam.c > 0) || !(p->eam.d > 0) || !(p->eam.d <= p->eam.c)))
    return MD_ERR_ARG;
  if (p->potential == MD_POT_PAPER) {
    const md_eam_paper_params& q = p->paper;
    if (!(q.rc > 0) || !(q.re > 0) || !(q.d > 0) || !(q.rho_e > 0) || !(q.P_e > 0) || !(q.fe >= 0) ||
        !std::isfinite(q.beta) || !std::isfinite(q.n) || !std::isfinite(q.Fo) || !std::isfinite(q.alpha))
      return MD_ERR_ARG;
  }
  if (!(p->morse.rc > 0) || !(p->morse.alpha > 0)) return MD_ERR_ARG;
  md_system* s = new (std::nothrow) md_system();
  if (!s) return MD_ERR_ARG;
  s->p = *p;
  s->nrep = nrep;
  s->ws = nullptr;
  s->have_embed = s->have_force = false;
  s->list_mix = false;
  s->list_tgt = p->list_tgt ? p->list_tgt : LIST_TGT;
  // the list holds pairs within the potential's largest Cr-Cr cutoff + skin
  const double cut = p->potential == MD_POT_PAPER ? std::max(p->paper.rc, p->paper.d * p->paper.re) : p->eam.c;
  const double rlist = cut + p->skin;
  const double rxlist = p->morse.rc + p->skin;
  int64_t a0 = 0, c0 = 0, nlblk = 0;
  int t0 = 0, g0 = 0;
  std::vector<int> hcells(nrep);
  for (int r = 0; r < nrep; ++r) {
    const md_replica_desc& rd = reps[r];
    if (rd.n < 0 || rd.n_c < 0) { delete s; return MD_ERR_ARG; }
    RepDesc d{};
    for (int a = 0; a < 3; ++a) {
      if (!(rd.len[a] > 0) || !std::isfinite(rd.lo[a])) { delete s; return MD_ERR_ARG; }
      d.lo[a] = rd.lo[a];
      d.len[a] = rd.len[a];
      d.half[a] = 0.5 * rd.len[a];
      d.per[a] = rd.periodic[a] ? 1 : 0;
      // allocated cells along the axis: the box along periodic axes; room for the atoms to
      // spread to about twice the given extent along open axes (beyond that cells stretch)
      const int nb = cells_along(rd.len[a], rlist);
      d.gcap[a] = d.per[a] ? nb : std::max(2 * nb, nb + 8);
      if (d.per[a] && nb < 3) s->list_mix = true;
      d.hd[a] = rd.n_c > 0 ? cells_along(rd.len[a], rxlist) : 1;
      // the minimum image must be the only image within the list radius
      if (d.per[a] && !(rd.len[a] > 2.0 * rlist)) { delete s; return MD_ERR_ARG; }
      if (d.per[a] && rd.n_c > 0 && !(rd.len[a] > 2.0 * rxlist)) { delete s; return MD_ERR_ARG; }
      d.ginv[a] = nb / rd.len[a];
      d.hinv[a] = d.hd[a] / rd.len[a];
    }
    d.a0 = (int)a0;
    d.n = rd.n;
    int ntile = std::max(1, (rd.n + TILE - 1) / TILE);
    d.npad = ntile * TILE;
    d.t0 = t0;
    d.nt = ntile;
    d.c0 = (int)c0;
    d.nc = rd.n_c;
    int64_t ncr = (int64_t)d.gcap[0] * d.gcap[1] * d.gcap[2];
    int64_t nch = (int64_t)d.hd[0] * d.hd[1] * d.hd[2];
    if (ncr > (1 << 28) || nch > (1 << 28)) { delete s; return MD_ERR_ARG; }
    d.g0 = g0;
    g0 += (int)ncr;
    hcells[r] = (int)nch;
    a0 += d.npad;
    c0 += rd.n_c;
    t0 += ntile;
    if (a0 > (int64_t)INT32_MAX / 2 || c0 > (int64_t)INT32_MAX / 2) { delete s; return MD_ERR_ARG; }
    s->desc.push_back(d);
    for (int t = 0; t < ntile; ++t) s->tile_rep.push_back(r);
    // list build: rows at capacity, each cut into at most nseg runs of cells (twice the
    // runs of LIST_SEG cells, so that dense rows can be cut finer); one block per run
    s->desc.back().rb0 = (int)s->row_rep.size();
    s->desc.back().nseg = 2 * ((d.gcap[0] + LIST_SEG - 1) / LIST_SEG) * ((224 + s->list_tgt - 1) / s->list_tgt);
    const int64_t nrw = (int64_t)d.gcap[1] * d.gcap[2];
    nlblk += (int64_t)s->desc.back().nseg * nrw;
    if ((int64_t)s->row_rep.size() + nrw > (int64_t)INT32_MAX / 2 || nlblk > (int64_t)INT32_MAX / 2) {
      delete s;
      return MD_ERR_ARG;
    }
    s->row_rep.insert(s->row_rep.end(), (size_t)nrw, r);
    s->desc.back().ch0 = (int)s->chunks.size();
    for (int t = 0; t < ntile; t += REDUCE_CHUNK)
      s->chunks.push_back(make_int2(t0 - ntile + t, std::min(REDUCE_CHUNK, ntile - t)));
    s->desc.back().nch = (int)s->chunks.size() - s->desc.back().ch0;
    for (int k = 0; k < rd.n_c; ++k) s->c_rep.push_back(r);
  }
  s->ncell_cr = g0;
  int h = g0;
  for (int r = 0; r < nrep; ++r) {
    s->desc[r].h0 = h;
    h += hcells[r];
  }
  s->ncell_all = h;
  // list entries keep the slot in 27 bits; list offsets are 32-bit
  if (a0 >= ((int64_t)1 << 27)) { delete s; return MD_ERR_ARG; }
  if ((int64_t)p->cap * a0 >= (int64_t)INT32_MAX || (int64_t)p->xcap * a0 >= (int64_t)INT32_MAX ||
      (int64_t)p->icap * a0 >= (int64_t)INT32_MAX) {
    delete s;
    return MD_ERR_ARG;
  }
  s->scan_blocks = (h + SCAN_CHUNK - 1) / SCAN_CHUNK;
  s->ntot = a0;
  s->ctot = c0;
  s->ntiles = t0;
  s->nlblk = (int)nlblk;
  s->nrows = (int)s->row_rep.size();

  Consts& K = s->K;
  std::memset(&K, 0, sizeof K);
  K.A = p->eam.A;
  K.c = p->eam.c;
  K.d = p->eam.d;
  K.c0 = p->eam.c0;
  K.c1 = p->eam.c1;
  K.c2 = p->eam.c2;
  K.c_sq = p->eam.c * p->eam.c;
  K.d_sq = p->eam.d * p->eam.d;
  if (p->eam.c2 != 0.0) {
    K.rv = -p->eam.c1 / (2.0 * p->eam.c2);
    K.pmin = p->eam.c0 - p->eam.c1 * p->eam.c1 / (4.0 * p->eam.c2);
  }
  K.D = p->morse.D;
  K.alpha = p->morse.alpha;
  K.r0 = p->morse.r0;
  K.mrc = p->morse.rc;
  K.mrc_sq = p->morse.rc * p->morse.rc;
  {
    double e = std::exp(-p->morse.alpha * (p->morse.rc - p->morse.r0));
    K.mshift = p->morse.D * (e * e - 2.0 * e);
  }
  K.acc = ACC_CONV / p->mass;
  K.ke_fac = p->mass / (2.0 * ACC_CONV);
  K.dt = p->dt;
  K.v_ind = p->v_ind;
  K.half_skin = 0.5 * p->skin;
  K.half_skin_sq = K.half_skin * K.half_skin;
  K.rlist_sq = rlist * rlist;
  K.rlist = rlist;
  K.icut_sq = cut * cut;
  K.rxlist_sq = rxlist * rxlist;
  K.cap = p->cap;
  K.xcap = p->xcap;
  K.icap = p->icap;
  K.nrep = nrep;
  K.lt = p->tpa;
  K.lt_shift = p->tpa == 1 ? 0 : (p->tpa == 2 ? 1 : (p->tpa == 4 ? 2 : 3));
  K.shadow = p->shadow ? 1 : 0;
  K.ntot = s->ntot;
  K.pot = p->potential;
  if (p->potential == MD_POT_PAPER) {
    const md_eam_paper_params& q = p->paper;
    PaperConsts& P = K.P;
    P.Fo = q.Fo; P.n = q.n; P.rho_e = q.rho_e; P.alpha = q.alpha; P.P_e = q.P_e;
    P.fe = q.fe; P.re = q.re; P.beta = q.beta;
    P.a0 = q.a0; P.a1 = q.a1; P.a2 = q.a2; P.a3 = q.a3; P.d = q.d;
    P.rc_sq = q.rc * q.rc;
    P.phi_sq = (q.d * q.re) * (q.d * q.re);
    P.inv_re = 1.0 / q.re;
    P.re2 = q.re * q.re;
    P.b0 = q.a3 + q.a2 + q.a1 + q.a0;
    P.b1 = 3.0 * q.a3 + 2.0 * q.a2 + q.a1;
    P.b2 = 3.0 * q.a3 + q.a2;
    P.b3 = q.a3;
    const double bh = 0.5 * q.beta;
    P.bh = (bh == std::floor(bh) && bh >= 1.0 && bh <= 8.0) ? (int)bh : 0;
  }
  {
    const char* fe = std::getenv("MD_FUSE_ENERGY");
    s->fuse_energy = !(fe && std::atoi(fe) == 0);
  }
  s->L = make_layout(*s);
  *out = s;
  return MD_OK;
}

MD_API void md_system_destroy(md_system* s) {
  if (s && s->static_dev >= 0) {
    const md_system* me = s;
    g_scratch_owner[s->static_dev].compare_exchange_strong(me, nullptr);
  }
  delete s;
}

MD_API int64_t md_system_atoms(const md_system* s) { return s ? s->ntot : -1; }
MD_API int64_t md_system_carbons(const md_system* s) { return s ? s->ctot : -1; }
MD_API int64_t md_replica_offset(const md_system* s, int32_t r) {
  if (!s || r < 0 || r >= s->nrep) return -1;
  return s->desc[r].a0;
}

MD_API size_t md_workspace_bytes(const md_system* s) { return s ? s->L.total : 0; }

namespace {

// Takes ws as the workspace of s: cleared, descriptors written, stream synchronised.
int bind_workspace(md_system* s, void* ws, hipStream_t st) {
  s->ws = (char*)ws;
  int e;
  if ((e = hip_status(hipMemsetAsync(ws, 0, s->L.total, st)))) return e;
  if ((e = hip_status(hipMemcpyAsync(at<RepDesc>(s, s->L.desc), s->desc.data(),
                                     sizeof(RepDesc) * s->nrep, hipMemcpyHostToDevice, st))))
    return e;
  if ((e = hip_status(hipMemcpyAsync(at<int>(s, s->L.row_rep), s->row_rep.data(),
                                     sizeof(int) * s->nrows, hipMemcpyHostToDevice, st))))
    return e;
  if ((e = hip_status(hipMemcpyAsync(at<int>(s, s->L.tile_rep), s->tile_rep.data(),
                                     sizeof(int) * s->ntiles, hipMemcpyHostToDevice, st))))
    return e;
  if (s->ctot > 0 &&
      (e = hip_status(hipMemcpyAsync(at<int>(s, s->L.c_rep), s->c_rep.data(), sizeof(int) * s->ctot,
                                     hipMemcpyHostToDevice, st))))
    return e;
  if ((e = hip_status(hipMemcpyAsync(at<int2>(s, s->L.chunks), s->chunks.data(), sizeof(int2) * s->chunks.size(),
                                     hipMemcpyHostToDevice, st))))
    return e;
  s->have_embed = s->have_force = false;
  s->cur = 0;
  s->ppt = 1;
  // the build kernels that stride over their work fill the chip once: as many blocks as its
  // compute units hold at once
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hip_status(hipGetDevice(&dev)))) return e;
  if ((e = hip_status(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)))) return e;
  if ((e = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_list_tiles<MD_LIST_WAVES_RESIDENT>, LIST_BLOCK, 0)))) return e;
  s->list_grid = std::max(1, cus * std::max(1, per_cu));
  s->tile_grid = std::max(1, cus * (2048 / BLOCK));
  return hip_status(hipStreamSynchronize(st));
}

}  // namespace

MD_API int md_workspace_bind(md_system* s, void* ws, size_t bytes, void* stream) {
  if (!s || !ws || bytes < s->L.total) return MD_ERR_ARG;
  if (((uintptr_t)ws) % ALIGN) return MD_ERR_ARG;
  if (s->static_dev >= 0) {   // give up a static scratch this system held
    const md_system* me = s;
    g_scratch_owner[s->static_dev].compare_exchange_strong(me, nullptr);
    s->static_dev = -1;
  }
  return bind_workspace(s, ws, (hipStream_t)stream);
}

MD_API int md_workspace_bind_static(md_system* s, void* stream) {
  if (!s) return MD_ERR_ARG;
  if (s->L.total > (size_t)MD_SCRATCH_BYTES) {
    std::fprintf(stderr,
                 "md_workspace_bind_static: this system needs %zu bytes of workspace, more than the "
                 "%d bytes of the static scratch; bind a caller-owned workspace with md_workspace_bind\n",
                 s->L.total, (int)MD_SCRATCH_BYTES);
    return MD_ERR_ARG;
  }
  int dev = 0, e;
  if ((e = hip_status(hipGetDevice(&dev)))) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return MD_ERR_ARG;
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {   // once per device, with that device current
      void* p = nullptr;
      if ((e = hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))))) return e;
      if (!p) return MD_ERR_HIP;
      g_scratch_ptr[dev] = p;
    }
    ptr = g_scratch_ptr[dev];
    g_scratch_owner[dev].store(s);   // earlier systems bound to it are now refused
  }
  s->static_dev = dev;
  return bind_workspace(s, ptr, (hipStream_t)stream);
}

namespace {

// The list build; ev0 / ev1 (or null) are recorded just before and after the Cr-Cr list
// kernel.
// copy_f: the forces are permuted with the atoms (md_run passes false: its kicks read a->f
// only after a force pass has stored it since the last build).
int build_chain(md_system* s, const md_atoms* a, const md_lists* l, uint32_t flags, hipStream_t st,
                hipEvent_t ev0, hipEvent_t ev1, bool copy_f = true) {
  int* misc = at<int>(s, s->L.misc);
  BuildArgs A;
  A.R = at<RepDesc>(s, s->L.desc);
  A.S = at<RepState>(s, s->L.state);
  A.tile_rep = at<int>(s, s->L.tile_rep);
  A.row_rep = at<int>(s, s->L.row_rep);
  A.items = at<int2>(s, s->L.items);
  A.nitems = misc + 2;
  A.next_item = misc + 4;
  A.nrows = s->nrows;
  A.nlblk = s->nlblk;
  A.list_tgt = s->list_tgt;
  A.c_rep = at<int>(s, s->L.c_rep);
  A.any = misc + 0;
  A.abort = misc + 3;
  A.spin_limit = scan_spin_limit();
  A.q = qcur(s, a);
  A.v = a->v;
  A.f = a->f;
  A.copy_f = copy_f ? 1 : 0;
  A.fixed = a->fixed;
  A.id = a->id;
  A.xc = a->xc;
  A.xref = at<double>(s, s->L.xref);
  A.cellid = at<int>(s, s->L.cellid);
  A.crank = at<int>(s, s->L.crank);
  A.perm = at<int>(s, s->L.perm);
  A.skey = at<long long>(s, s->L.skey);
  A.tq = at<double4>(s, s->L.tq);
  A.tqf = at<float4>(s, s->L.tqf);
  A.qs = qscur(s);
  A.bcell = at<long long>(s, s->L.bcell);
  A.tv = at<double>(s, s->L.tv);
  A.tf = at<double>(s, s->L.tf);
  A.tfixed = at<uint8_t>(s, s->L.tfixed);
  A.tid = at<int>(s, s->L.tid);
  A.count = at<int>(s, s->L.count);
  A.start = at<int>(s, s->L.start);
  A.hcell = at<int>(s, s->L.hcell);
  A.hrank = at<int>(s, s->L.hrank);
  A.hlist = at<int>(s, s->L.hlist);
  A.hsorted = at<double4>(s, s->L.hsorted);
  A.scan_state = at<long long>(s, s->L.scan_state);
  A.scan_ticket = misc + 1;
  A.idx = l->idx;
  A.cnt = l->cnt;
  A.xidx = l->xidx;
  A.xcnt = l->xcnt;
  A.near = at<int>(s, s->L.near);
  A.hnear = at<int>(s, s->L.hnear);
  A.fme = at<double>(s, s->L.fme);
  A.near_blocks = near_blocks(s);
  A.ncell_all = s->ncell_all;
  A.ncell_cr = s->ncell_cr;
  A.ntiles = s->ntiles;
  A.ctot = (int)s->ctot;
  static_assert(SCAN_CHUNK == BLOCK * SCAN_PER_THREAD, "k_scan covers SCAN_CHUNK cells per block");
  A.scan_chunk = SCAN_CHUNK;
  A.scan_blocks = s->scan_blocks;
  const int cblocks = (int)((s->ctot + BLOCK - 1) / BLOCK);
  A.nbin = s->ntiles + cblocks;
  const int tgrid = std::min(A.nbin, s->tile_grid);   // k_bin, k_scatter, k_sort_gather
  // a single replica without a forced build: the skin decision is taken inside k_bin, every
  // block reducing the per-part maxima, while those redundant loads stay few (they grow as
  // blocks x parts: 1.4 M on the 216k-atom film); else (2e9 on an 8M-atom one) from
  // PARTS_REDUCED partial reductions of them by a launch of many blocks
  const int64_t bin_blocks = tgrid, nparts = (int64_t)s->ntiles * s->ppt;
  const bool decide_in_bin = !(flags & MD_B_FORCE) && s->K.nrep == 1;
  A.commit_ref = decide_in_bin ? 1 : 0;
  if (decide_in_bin && bin_blocks * nparts <= DECIDE_IN_BIN_MAX_LOADS) {
    k_bin<true><<<tgrid, BLOCK, 0, st>>>(s->K, A, at<double>(s, s->L.dmax), at<double>(s, s->L.tbox),
                                         (int)nparts);
  } else if (decide_in_bin) {
    k_parts_reduce<<<PARTS_REDUCED, BLOCK, 0, st>>>(at<double>(s, s->L.dmax), at<double>(s, s->L.tbox),
                                                    (int)nparts, at<double>(s, s->L.dmax_p),
                                                    at<double>(s, s->L.tbox_p));
    k_bin<true><<<tgrid, BLOCK, 0, st>>>(s->K, A, at<double>(s, s->L.dmax_p), at<double>(s, s->L.tbox_p),
                                         PARTS_REDUCED);
  } else {
    if (flags & MD_B_FORCE)
      k_tile_box<<<s->ntiles, BLOCK, 0, st>>>(A.R, A.tile_rep, A.q, at<double>(s, s->L.tbox));
    k_decide<<<1, DECIDE_THREADS, 0, st>>>(s->K, A, at<double>(s, s->L.dmax), at<double>(s, s->L.tbox),
                                  (flags & MD_B_FORCE) ? 1 : 0, (flags & MD_B_FORCE) ? 1 : s->ppt);
    k_bin<false><<<tgrid, BLOCK, 0, st>>>(s->K, A, nullptr, nullptr, 0);
  }
  k_scan<<<s->scan_blocks, BLOCK, 0, st>>>(A);
  k_scatter<<<tgrid, BLOCK, 0, st>>>(s->K, A);
  k_sort_gather<<<tgrid, BLOCK, 0, st>>>(s->K, A);
  int e;
  if (ev0 && (e = hip_status(hipEventRecord(ev0, st)))) return e;
  // the Cr-C lists: leading blocks of the staged Cr-Cr list launch, else a launch of their own
  A.xblocks = (s->list_mix || s->ctot == 0) ? 0 : morse_fused_blocks(s);
  // the Cr-Cr list: one block per work item while the item table's capacity is a few waves
  // of resident blocks (the idle blocks then cost less than taking items from a counter),
  // else resident blocks that take items from a counter (MD_LIST_PERSISTENT=0/1 in the
  // environment overrides the choice)
  A.persistent = list_persistent(s);
  if (s->list_mix)
    k_list_rows<false><<<s->ntiles, BLOCK, 0, st>>>(s->K, A);
  else if (A.persistent)
    k_list_tiles<MD_LIST_WAVES_RESIDENT><<<A.xblocks + std::min(s->nlblk, s->list_grid), LIST_BLOCK, 0, st>>>(s->K, A);
  else
    k_list_tiles<MD_LIST_WAVES><<<A.xblocks + s->nlblk, LIST_BLOCK, 0, st>>>(s->K, A);
  if (ev1 && (e = hip_status(hipEventRecord(ev1, st)))) return e;
  if (s->list_mix && s->ctot > 0) k_xlist<<<A.near_blocks, BLOCK, 0, st>>>(s->K, A);
  return check_launch();
}

}  // namespace

MD_API int md_build_neighbors(md_system* s, const md_atoms* a, const md_lists* l, uint32_t flags,
                              void* stream) {
  if (!s || !atoms_ok(a) || !lists_ok(s, l) || (s->ctot > 0 && !a->xc)) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  return build_chain(s, a, l, flags, (hipStream_t)stream, nullptr, nullptr);
}

namespace {

// Two-tier lists: the inner list refilled from the outer one at the current positions.
int inner_list(md_system* s, const md_atoms* a, const md_lists* l, hipStream_t st) {
  if (!s->p.icap) return MD_OK;
  k_inner_pos<<<grid_tiles(s), BLOCK, 0, st>>>(at<RepDesc>(s, s->L.desc), at<RepState>(s, s->L.state),
                                               at<int>(s, s->L.tile_rep), qcur(s, a), at<float4>(s, s->L.tqf));
  k_inner_list<<<grid_tiles(s) * INNER_G, BLOCK, 0, st>>>(s->K, at<RepDesc>(s, s->L.desc), at<RepState>(s, s->L.state),
                                                at<int>(s, s->L.tile_rep), qcur(s, a), at<float4>(s, s->L.tqf),
                                                l->idx, l->cnt, l->iidx, l->icnt);
  return check_launch();
}

// The density pass (morse: with the Cr-C pass in the same launch; inner: the inner list is
// refilled first).
int eam_density(md_system* s, const md_atoms* a, const md_lists* l, uint32_t flags, double* rho_out, bool morse,
                hipStream_t st, bool inner = true) {
  const bool mixed = flags & MD_F_MIXED, energy = flags & MD_F_ENERGY;
  if (inner) {
    const int e = inner_list(s, a, l, st);
    if (e) return e;
  }
  switch (s->K.lt) {
    case 1: launch_density<1>(s, a, l, mixed, energy, rho_out, morse, st); break;
    case 2: launch_density<2>(s, a, l, mixed, energy, rho_out, morse, st); break;
    case 4: launch_density<4>(s, a, l, mixed, energy, rho_out, morse, st); break;
    default: launch_density<8>(s, a, l, mixed, energy, rho_out, morse, st); break;
  }
  s->have_embed = energy;
  return check_launch();
}

// The force pass (add_fme: the Cr-C forces recorded in fme this step are included;
// full_kick: see launch_force).
int eam_force(md_system* s, const md_atoms* a, const md_lists* l, uint32_t flags, bool add_fme, hipStream_t st,
              bool full_kick = false, bool drift = false, bool fuse_ke = false) {
  const bool mixed = flags & MD_F_MIXED, energy = flags & MD_F_ENERGY, kick = flags & MD_F_KICK;
  switch (s->K.lt) {
    case 1: launch_force<1>(s, a, l, mixed, kick, energy, add_fme, st, full_kick, drift, fuse_ke); break;
    case 2: launch_force<2>(s, a, l, mixed, kick, energy, add_fme, st, full_kick, drift, fuse_ke); break;
    case 4: launch_force<4>(s, a, l, mixed, kick, energy, add_fme, st, full_kick, drift, fuse_ke); break;
    default: launch_force<8>(s, a, l, mixed, kick, energy, add_fme, st, full_kick, drift, fuse_ke); break;
  }
  s->have_force = energy;
  return check_launch();
}

}  // namespace

MD_API int md_eam_forces(md_system* s, const md_atoms* a, const md_lists* l, uint32_t flags,
                         double* rho_out, void* stream) {
  if (!s || !atoms_ok(a) || !lists_ok(s, l)) return MD_ERR_ARG;
  if ((flags & MD_F_MORSE) && s->ctot > 0 && !a->xc) return MD_ERR_ARG;
  if ((flags & MD_F_MIXED) && s->K.pot == MD_POT_FS && s->p.eam.c2 == 0.0) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  // With a force pass, the Cr-C forces go in with the Eq. 1 forces: computed into fme by
  // extra blocks of the density launch when there is one, else by their own launch first.
  const bool morse = (flags & MD_F_MORSE) && (flags & MD_F_FORCE) && s->ctot > 0;
  const bool fused = morse && (flags & MD_F_DENSITY);
  int e;
  if ((flags & MD_F_DENSITY) && (e = eam_density(s, a, l, flags, rho_out, fused, st))) return e;
  if (flags & MD_F_FORCE) {
    if (morse && !fused) launch_morse(s, a, l, flags & MD_F_MIXED, false, false, st);
    if ((e = eam_force(s, a, l, flags, morse, st))) return e;
  }
  return MD_OK;
}

MD_API int md_morse_forces(md_system* s, const md_atoms* a, const md_lists* l, uint32_t flags,
                           void* stream) {
  if (!s || !atoms_ok(a) || !lists_ok(s, l)) return MD_ERR_ARG;
  if (s->ctot > 0 && !a->xc) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  if (s->ctot > 0) launch_morse(s, a, l, flags & MD_F_MIXED, flags & MD_F_KICK, true, (hipStream_t)stream);
  return check_launch();
}

namespace {

// Tasks 2 + 3 (kick: the half kick first; else the velocities are at the half step already).
void launch_kick_drift(md_system* s, const md_atoms* a, hipStream_t st, bool kick) {
#define KD(KI)                                                                                                  \
  k_kick_drift<KI><<<grid_tiles(s), BLOCK, 0, st>>>(                                                           \
      s->K, at<RepDesc>(s, s->L.desc), at<RepState>(s, s->L.state), at<int>(s, s->L.tile_rep),                 \
      qcur(s, a), a->v, a->f, a->fixed, at<double>(s, s->L.xref), at<double>(s, s->L.dmax),                    \
      at<double>(s, s->L.tbox), qscur(s), at<long long>(s, s->L.bcell))
  if (kick) KD(true); else KD(false);
#undef KD
  s->ppt = 1;
}

}  // namespace

MD_API int md_verlet_step(md_system* s, int32_t phase, const md_atoms* a, void* stream) {
  if (!s || !atoms_ok(a)) return MD_ERR_ARG;
  if (phase != MD_PHASE_KICK_DRIFT && phase != MD_PHASE_KICK) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  const RepDesc* R = at<RepDesc>(s, s->L.desc);
  const int* tr = at<int>(s, s->L.tile_rep);
  const int nb = grid_tiles(s);
  if (phase == MD_PHASE_KICK_DRIFT)
    launch_kick_drift(s, a, st, true);
  else
    k_kick<<<nb, BLOCK, 0, st>>>(s->K, R, tr, a->v, a->f, a->fixed);
  return check_launch();
}

namespace {

// Task 4d: the per-replica sums of the last passes' partials into out (tpk: blocks per tile
// of the pass that wrote the kinetic and Cr-C partials; ind_obs: that pass, taking them
// (KinOut) with the drift, has moved the indenter on and kept the observed step's position).
int energy_sums(md_system* s, double* out, int tpk, bool ind_obs, hipStream_t st) {
  k_reduce_chunks<<<(int)s->chunks.size(), BLOCK, 0, st>>>(
      at<int2>(s, s->L.chunks), s->have_embed ? at<double>(s, s->L.p_embed) : nullptr, s->K.lt,
      s->have_force ? at<double>(s, s->L.p_force) : nullptr, s->K.lt, at<double>(s, s->L.p_morse),
      at<double>(s, s->L.p_kin), tpk, at<double>(s, s->L.chunk_out));
  k_reduce<<<s->nrep, BLOCK, 0, st>>>(at<RepDesc>(s, s->L.desc), at<RepState>(s, s->L.state),
                                      at<double>(s, s->L.chunk_out), out, ind_obs ? 1 : 0);
  return check_launch();
}

}  // namespace

MD_API int md_energy(md_system* s, const md_atoms* a, double* out, void* stream) {
  if (!s || !atoms_ok(a) || !out) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  const RepDesc* R = at<RepDesc>(s, s->L.desc);
  const int* tr = at<int>(s, s->L.tile_rep);
  double* pk = at<double>(s, s->L.p_kin);
  double* pm = at<double>(s, s->L.p_morse);
  k_kinetic<<<grid_tiles(s), BLOCK, 0, st>>>(s->K, R, tr, a->v, a->fixed, at<double>(s, s->L.fme), pk, pm);
  return energy_sums(s, out, 1, false, st);
}

MD_API int md_run(md_system* s, const md_atoms* a, const md_lists* l, int32_t nsteps, uint32_t flags,
                  int32_t energy_every, double* obs, const md_trace* trace, void* stream) {
  if (!s || !atoms_ok(a) || !lists_ok(s, l) || nsteps < 0) return MD_ERR_ARG;
  if (energy_every > 0 && !obs) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t mixed = flags & MD_F_MIXED;
  int e;
  // Velocity Verlet (Eqs. A11-A13, Task 5).  Where the velocities at the end of a step are
  // not observed (no energies, not the last step), its final half kick and the next step's
  // first one are given together by the force pass (a full kick of the same force), and
  // the next Task 3 only drifts.
  // The force pass of such a step also does the next step's drift (into the other position
  // buffer and shadow; the positions come back to the caller's q at the end).
  bool drifted = false;   // this step's Task 2 + 3 was done by the previous force pass
  bool whole = true;      // the velocities are at a whole step
  for (int k = 1; k <= nsteps; ++k) {
    const bool en = energy_every > 0 && k % energy_every == 0;
    const bool full = k < nsteps && !en;
    // an observed step other than the last: its energies taken inside the force pass, which
    // then also gives the next step's first half kick (KinOut)
    const bool fuse = en && k < nsteps && s->fuse_energy;
    const bool drift = full || fuse;
    if (!drifted) launch_kick_drift(s, a, st, whole);
    hipEvent_t ev[MD_TRACE_EVENTS] = {};
    if (trace && trace->events)
      for (int u = 0; u < MD_TRACE_EVENTS; ++u) ev[u] = (hipEvent_t)trace->events[MD_TRACE_EVENTS * (k - 1) + u];
    if ((e = build_chain(s, a, l, 0, st, ev[2], ev[3], false))) return e;
    // Task 4c runs in the density launch; the force pass includes it and gives the kick
    const bool morse = s->ctot > 0;
    const uint32_t ef = mixed | (en ? MD_F_ENERGY : 0);
    if (ev[6] && (e = hip_status(hipEventRecord(ev[6], st)))) return e;
    if ((e = inner_list(s, a, l, st))) return e;
    if (ev[7] && (e = hip_status(hipEventRecord(ev[7], st)))) return e;
    if (ev[4] && (e = hip_status(hipEventRecord(ev[4], st)))) return e;
    if ((e = eam_density(s, a, l, MD_F_DENSITY | ef, nullptr, morse, st, false))) return e;
    if (ev[5] && (e = hip_status(hipEventRecord(ev[5], st)))) return e;
    if (ev[0] && (e = hip_status(hipEventRecord(ev[0], st)))) return e;
    if ((e = eam_force(s, a, l, MD_F_FORCE | MD_F_KICK | ef, morse, st, full, drift, fuse))) return e;
    if (ev[1] && (e = hip_status(hipEventRecord(ev[1], st)))) return e;
    if (trace && trace->builds) {
      k_record_builds<<<(s->nrep + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(
          at<RepState>(s, s->L.state), s->nrep, trace->builds + (int64_t)(k - 1) * s->nrep);
      if ((e = check_launch())) return e;
    }
    if (drift) {
      s->cur ^= 1;
      s->ppt = s->K.lt;
    }
    drifted = drift;
    whole = !(full || fuse);
    if (en) {
      double* out = obs + (int64_t)(k / energy_every - 1) * s->nrep * MD_NOBS;
      if ((e = fuse ? energy_sums(s, out, s->K.lt, drift, st) : md_energy(s, a, out, stream))) return e;
    }
  }
  if (s->cur) {   // the positions back into the caller's q
    k_copy_positions<<<(int)((s->ntot + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(
        s->ntot, at<double4>(s, s->L.q2), reinterpret_cast<double4*>(a->q), at<int4>(s, s->L.qs2),
        at<int4>(s, s->L.qs), s->K.shadow);
    s->cur = 0;
    if ((e = check_launch())) return e;
  }
  return MD_OK;
}

MD_API int md_graph_create(md_system* s, const md_atoms* a, const md_lists* l, int32_t nsteps,
                           uint32_t flags, int32_t energy_every, double* obs, void* stream,
                           void** graph_exec) {
  if (!graph_exec) return MD_ERR_ARG;
  *graph_exec = nullptr;
  hipStream_t st = (hipStream_t)stream;
  if (!st) return MD_ERR_ARG;   // the null stream cannot be captured
  int e;
  if ((e = hip_status(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)))) return e;
  int rc = md_run(s, a, l, nsteps, flags, energy_every, obs, nullptr, stream);
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if ((e = hip_status(ce))) return e;
  hipGraphExec_t ex = nullptr;
  e = hip_status(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  (void)hipGraphDestroy(g);
  if (e) return e;
  *graph_exec = (void*)ex;
  return MD_OK;
}

MD_API int md_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return MD_ERR_ARG;
  return hip_status(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
}

MD_API int md_graph_destroy(void* graph_exec) {
  if (!graph_exec) return MD_ERR_ARG;
  return hip_status(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
}

MD_API int md_set_indenter_velocity(md_system* s, double v_ind) {
  if (!s || !std::isfinite(v_ind)) return MD_ERR_ARG;
  s->p.v_ind = v_ind;
  s->K.v_ind = v_ind;
  return MD_OK;
}

MD_API int md_check(md_system* s, md_status* st_out, void* stream) {
  if (!s || !st_out) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  int* misc = at<int>(s, s->L.misc);
  k_status<<<1, 64, 0, st>>>(at<RepState>(s, s->L.state), s->nrep, misc + 8);
  int e = check_launch();
  if (e) return e;
  int host[8] = {0};
  if ((e = hip_status(hipMemcpyAsync(host, misc + 8, sizeof(int) * 7, hipMemcpyDeviceToHost, st)))) return e;
  if ((e = hip_status(hipStreamSynchronize(st)))) return e;
  std::memset(st_out, 0, sizeof *st_out);
  st_out->overflow = host[0];
  st_out->xoverflow = host[1];
  st_out->nonfinite = host[2];
  st_out->nbuilds = host[3];
  st_out->sync_timeout = host[4];
  st_out->nnear = host[5];
  st_out->ioverflow = host[6];
  return MD_OK;
}

MD_API int md_clear_flags(md_system* s, void* stream) {
  if (!s) return MD_ERR_ARG;
  if (!bound(s)) return MD_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  k_clear_flags<<<(s->nrep + 63) / 64, 64, 0, st>>>(at<RepState>(s, s->L.state), s->nrep);
  // a build that gave up left its cell counts behind: zero them and lift the abort word
  k_clear_build<<<std::min(4096, (s->ncell_all + BLOCK - 1) / BLOCK + 1), BLOCK, 0, st>>>(
      at<int>(s, s->L.count), s->ncell_all, at<int>(s, s->L.misc) + 3);
  return check_launch();
}

}  // extern "C"
