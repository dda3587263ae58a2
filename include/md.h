/*
 * md.h -- C ABI of the MI355X (gfx950) short-range molecular-dynamics step:
 * cell binning + Verlet neighbour lists, two-pass Embedded Atom Method (EAM) forces for
 * Cr-Cr, Morse forces between Cr and a rigid carbon indenter, velocity-Verlet update.
 *
 * The calls follow the five tasks of one MD time step in the paper (Section 2.1 and
 * Table 1):
 *   Task 1  neighbour-list update             -> md_build_neighbors
 *   Task 2  indenter motion                   -> md_verlet_step (MD_PHASE_KICK_DRIFT)
 *   Task 3  positions + half-step velocities  -> md_verlet_step (MD_PHASE_KICK_DRIFT)
 *   Task 4  density, forces, energies         -> md_eam_forces, md_morse_forces, md_energy
 *   Task 5  final velocity update             -> md_verlet_step (MD_PHASE_KICK), or fused
 *                                                into md_eam_forces with MD_F_KICK
 *
 * Conventions shared by every call
 *   - Units: eV, Angstrom, fs, u.  All state is FP64.
 *   - Every pointer inside md_atoms / md_lists and the workspace is DEVICE memory owned by
 *     the caller; the library never allocates or frees device memory.  The md_system
 *     handle is host memory allocated by md_system_create and freed by md_system_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls only
 *     enqueue work; they return before the GPU is done, except md_check and
 *     md_workspace_bind, which synchronise the stream.
 *   - Return value: MD_OK (0) or an MD_ERR_* code, detected on the host before anything is
 *     enqueued (bad arguments) or reported by the HIP runtime.  Conditions found on the
 *     GPU (list overflow, non-finite forces) are raised as device flags read by md_check.
 *   - Atoms of one system ("replica") occupy a contiguous range of the atom arrays,
 *     padded up to a multiple of MD_TILE atoms; several replicas are laid out one after
 *     the other (batched mode).  Padding slots are never read or written.
 *   - The library is not thread safe for one md_system; distinct systems are independent.
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MD_API __attribute__((visibility("default")))

/* Status codes */
#define MD_OK 0
#define MD_ERR_ARG 1       /* invalid argument (NULL pointer, bad size, box too small, ...) */
#define MD_ERR_HIP 2       /* a HIP runtime call failed */
#define MD_ERR_STATE 3     /* call out of order (e.g. no workspace bound) */

/* Atoms per tile: replica ranges are padded to a multiple of this. */
#define MD_TILE 256

/* Arithmetic of the pair/density loops. */
#define MD_FP64 0          /* everything in FP64 */
#define MD_MIXED 1         /* pair, density and force arithmetic in FP32; state, Verlet update
                              and energy/virial reductions in FP64 */

/* md_verlet_step phases */
#define MD_PHASE_KICK_DRIFT 1  /* Tasks 2 + 3: indenter moves by v_ind*dt; v += a dt/2; x += v dt */
#define MD_PHASE_KICK 2        /* Task 5: v += a dt/2 */

/* md_eam_forces / md_morse_forces flags */
#define MD_F_DENSITY 0x01  /* pass 1: rho_i, F'(rho_i) into q[i][3] */
#define MD_F_FORCE 0x02    /* pass 2: Eq. (1) forces into f (overwrites f) */
#define MD_F_MORSE 0x04    /* pass 2 also adds the Cr-C Morse forces (fused Task 4c) */
#define MD_F_KICK 0x08     /* pass 2 also applies the Task 5 half kick with the total force */
#define MD_F_ENERGY 0x10   /* write per-block energy / virial / load partials for md_energy */
#define MD_F_MIXED 0x20    /* FP32 pair arithmetic (MD_MIXED) */

/* md_build_neighbors flags */
#define MD_B_FORCE 0x01    /* rebuild now, whatever the skin test says */

/* Observables written by md_energy, per replica (MD_NOBS doubles each). */
#define MD_E_EMBED 0       /* sum_i F(rho_i) (+ M(P_i) with the paper's form) (Eq. A1, first and third terms) */
#define MD_E_PAIR 1        /* 1/2 sum_{i != j} phi(r_ij)             (Eq. A1, second term) */
#define MD_E_MORSE 2       /* sum over Cr-C pairs of phiM(r) - phiM(rc) */
#define MD_E_KIN 3         /* 1/2 m v^2 over mobile atoms */
#define MD_W_XX 4          /* EAM virial W_ab = sum_{i<j} (q_i-q_j)_a F_ij,b: xx yy zz xy xz yz */
#define MD_F_IND_X 10      /* load on the indenter = -(sum of Morse forces on Cr), x y z */
#define MD_IND_Z 13        /* indenter displacement along z */
#define MD_NBUILDS 14      /* number of list builds so far */
#define MD_NOBS 16

/* ---------------------------------------------------------------------------------- */
/* Descriptions                                                                         */
/* ---------------------------------------------------------------------------------- */

/* Synthetic Finnis-Sinclair-form EAM (Section 3.1, Eq. 1; energy of Eq. A1 without M):
 *   phi(r) = (r-c)^2 (c0 + c1 r + c2 r^2), r < c;  f(r) = (r-d)^2, r < d;  F(rho) = -A sqrt(rho). */
typedef struct md_eam_params {
    double A, c, d, c0, c1, c2;
} md_eam_params;

/* Cr-C Morse (form of Eq. A5): phiM(r) = D [exp(-2 alpha (r-r0)) - 2 exp(-alpha (r-r0))],
 * r < rc; the energy is shifted by -phiM(rc), the force is not. */
typedef struct md_morse_params {
    double D, alpha, r0, rc;
} md_morse_params;

/* The paper's own EAM form (Appendix, Eqs. A1-A4), selected with potential = MD_POT_PAPER:
 *   F(rho) = -Fo [1 - n ln(rho/rho_e)] (rho/rho_e)^n,  M(P) = alpha (P/P_e - 1)^2 exp(-(P/P_e - 1)^2),
 *   f(r) = fe (re/r)^beta for r < rc,  Phi(r) = (x-d)^2 (a3 x^3 + a2 x^2 + a1 x + a0) for
 *   x = r/re < d,  rho_i = sum_j f(r_ij), P_i = sum_j f(r_ij)^2, E = sum_i [F(rho_i) + M(P_i)]
 *   + 1/2 sum_{i != j} Phi(r_ij).  Forces: Eq. (1) with V = Phi and the M term in the same form,
 *   F_i = -sum_j [(F'_i + F'_j) f' + (M'_i + M'_j) 2 f f' + Phi'] (q_i - q_j) / r.
 *   F'(0) is taken as 0.  beta / 2 a whole number from 1 to 8 takes a faster path. */
typedef struct md_eam_paper_params {
    double Fo, n, rho_e, alpha, P_e, fe, re, beta, a0, a1, a2, a3, d, rc;
} md_eam_paper_params;

#define MD_POT_FS 0        /* md_params.potential: the Finnis-Sinclair-form `eam` */
#define MD_POT_PAPER 1     /* the paper's form `paper` */

typedef struct md_params {
    md_eam_params eam;
    md_morse_params morse;
    double mass;        /* Cr mass, u */
    double dt;          /* time step, fs */
    double v_ind;       /* indenter velocity along z, Angstrom/fs (Task 2) */
    double skin;        /* Verlet skin, Angstrom; lists hold pairs closer than cutoff + skin */
    int32_t cap;        /* Cr-Cr list capacity per atom */
    int32_t xcap;       /* Cr-C list capacity per atom */
    int32_t tpa;        /* lanes per atom in the density / force passes: 1, 2, 4 or 8 (the
                           Cr-Cr list is interleaved by tpa to match; cap must be a multiple
                           of tpa) */
    int32_t shadow;     /* 1: keep an FP32 copy of the positions relative to each atom's cell
                           (updated by the list build and md_verlet_step), from which the
                           MD_F_MIXED passes take their separations; 0: those passes round FP64
                           separations instead */
    int32_t potential;  /* MD_POT_FS (eam) or MD_POT_PAPER (paper); the list radius is the
                           potential's largest Cr-Cr cutoff + skin */
    int32_t icap;       /* two-tier lists (Section 2.6) when > 0: the Cr-Cr list (md_lists.idx,
                           radius cutoff + skin) is the outer list, rebuilt by the half-skin
                           rule, and before every density pass the inner list (md_lists.iidx,
                           capacity icap per atom, a multiple of tpa) is refilled with the
                           outer list's entries whose pair is now closer than the potential's
                           largest Cr-Cr cutoff; the passes then read the inner list.  0: one
                           list, read by the passes */
    md_eam_paper_params paper;
    int32_t list_tgt;   /* atoms a work item of the Cr-Cr list build aims at (a launch-shape
                           choice, 32 .. 256; 0: 224); results do not depend on it */
    int32_t pad;
} md_params;

/* One system (replica). */
typedef struct md_replica_desc {
    double lo[3];       /* box lower corner */
    double len[3];      /* periodic length (periodic axes) or extent of the cell grid (open
                           axes; atoms outside are still handled correctly) */
    int32_t periodic[3];
    int32_t n;          /* Cr atoms */
    int32_t n_c;        /* carbon atoms of the indenter (may be 0) */
    int32_t pad;
} md_replica_desc;

/* Device arrays of all replicas (n_total = md_system_atoms(sys) slots). */
typedef struct md_atoms {
    double *q;          /* [n_total][4]: x, y, z and F'(rho) -- the paper's position +
                           embedding-derivative array (Section 3.1) */
    double *v;          /* [n_total][3] velocities, Angstrom/fs */
    double *f;          /* [n_total][3] forces, eV/Angstrom */
    uint8_t *fixed;     /* [n_total] 1 = atom held fixed (bottom layer) */
    int32_t *id;        /* [n_total] caller's atom id; permuted together with the atoms */
    const double *xc;   /* [c_total][3] carbon positions at zero indenter displacement */
} md_atoms;

/* Device neighbour lists (caller-owned, written by md_build_neighbors). */
typedef struct md_lists {
    int32_t *idx;       /* [cap * n_total]: entry k of atom i at
                           idx[(k / tpa) * n_total * tpa + i * tpa + k % tpa]; its low 27 bits
                           are the neighbour's atom slot, the bits above 9 (dz + 1) + 3 (dy + 1)
                           + (dx + 1) for the neighbour's cell relative to atom i's at the build
                           when shadow is set (else 0, as when a periodic axis has fewer than 3
                           cells); entries are ordered
                           by the cell row (dz, then dy), then along x, then by slot */
    int32_t *cnt;       /* [n_total] */
    int32_t *xidx;      /* [n_total][xcap]: carbon indices (into xc) of atom i's Cr-C list */
    int32_t *xcnt;      /* [n_total] */
    int32_t *iidx;      /* two-tier lists only (else NULL): the inner list, [icap * n_total] in
                           idx's layout and entry format, atom i's entries in the order they
                           have in its outer list */
    int32_t *icnt;      /* [n_total] */
} md_lists;

/* Host copy of the device status flags (md_check). */
typedef struct md_status {
    int32_t overflow;       /* largest Cr-Cr list count that did not fit in cap (0 = none) */
    int32_t xoverflow;      /* same for the Cr-C list and xcap */
    int32_t nonfinite;      /* 1 if a non-finite force or density was produced */
    int32_t nbuilds;        /* list builds so far (summed over replicas) */
    int32_t sync_timeout;   /* a bounded device-side wait of a list build gave up: that build
                               is invalid (its later kernels did nothing; the lists, reference
                               positions and order are those of the build before, the positions
                               may have been wrapped) and no list build runs until
                               md_clear_flags.  The wait is 2^22 polls, or MD_SCAN_SPIN_LIMIT
                               from the environment at the time of the build (negative: give up
                               at once, for tests of this path) */
    int32_t nnear;          /* Cr atoms whose carbon cells are within reach of a carbon at the
                               last build (the candidates of the Cr-C lists), all replicas */
    int32_t ioverflow;      /* largest inner-list count that did not fit in icap (0 = none) */
    int32_t pad;
} md_status;

typedef struct md_system md_system;

/* ---------------------------------------------------------------------------------- */
/* Set-up                                                                               */
/* ---------------------------------------------------------------------------------- */

/* Create a handle for nrep replicas (host allocation only).  Checks that every periodic
 * axis holds at least 3 list cells (length >= 3 (c + skin)).  MD_ERR_ARG on bad input. */
MD_API int md_system_create(const md_replica_desc *reps, int32_t nrep, const md_params *p,
                            md_system **out);
MD_API void md_system_destroy(md_system *sys);

/* Atom slots (n_total), carbon slots (c_total), and the first atom slot of replica r. */
MD_API int64_t md_system_atoms(const md_system *sys);
MD_API int64_t md_system_carbons(const md_system *sys);
MD_API int64_t md_replica_offset(const md_system *sys, int32_t r);

/* Bytes of device workspace the system needs (cell grids, sort buffers, reference
 * positions, flags, reduction partials). */
MD_API size_t md_workspace_bytes(const md_system *sys);

/* Bind a caller-owned device workspace of at least md_workspace_bytes bytes: writes the
 * replica descriptors, clears flags, and synchronises `stream`.  MD_ERR_ARG if too small. */
MD_API int md_workspace_bind(md_system *sys, void *ws, size_t bytes, void *stream);

/* Bytes of the library's static device scratch (one per GPU): see md_workspace_bind_static. */
#define MD_SCRATCH_BYTES (16 << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same as md_workspace_bind, with the
 * library's own static device array of MD_SCRATCH_BYTES bytes as the workspace in place of a
 * caller-owned buffer.  Nothing is allocated here or by any later call on `sys` (the atom and
 * list arrays are still the caller's).  The array lives on every GPU the library runs on
 * (each GPU its own copy, at its own address, looked up at the first such call on that GPU,
 * which must be current) until the process ends.  MD_ERR_ARG, with a message on stderr, when
 * md_workspace_bytes(sys) exceeds MD_SCRATCH_BYTES (about 60,000 atoms).
 * One scratch per GPU: binding a system takes it over, clears it and keeps nothing of the
 * previous system; calls on a system bound to it earlier then return MD_ERR_STATE (bind that
 * system again to use it).  Calls on one GPU whose work overlaps on the device (several
 * streams or host threads) race on the array.  Synchronises `stream`; a set-up call, not
 * for use under stream capture (md_run and md_graph_create are). */
MD_API int md_workspace_bind_static(md_system *sys, void *stream);

/* ---------------------------------------------------------------------------------- */
/* The step                                                                             */
/* ---------------------------------------------------------------------------------- */

/* Task 1 (Section 2.6): if any atom moved more than skin/2 since the last build (or the
 * indenter did, or MD_B_FORCE), wrap periodic coordinates into the box, bin atoms into
 * cells of edge >= cutoff + skin, sort the atoms of each replica by (cell, id) -- the atom
 * arrays q, v, f, fixed, id are permuted in place --, record reference positions and
 * rebuild the full Cr-Cr list {j != i: |q_j - q_i|^2 < (c+skin)^2} and the Cr-C list
 * {k: |xc_k + ind_z - q_i|^2 < (rc+skin)^2}.  The test runs on the device; when it fails
 * the call costs one short kernel.  Overflow is flagged, not fatal: the list keeps cap
 * entries and md_check reports the count needed. */
MD_API int md_build_neighbors(md_system *sys, const md_atoms *a, const md_lists *l,
                              uint32_t flags, void *stream);

/* Task 4a/4b (Section 3.1, Eq. 1; Section 3.3.1.2-3): MD_F_DENSITY computes
 * rho_i = sum_j f(r_ij) and stores F'(rho_i) in q[i][3] (rho_out, if not NULL, receives rho
 * per atom slot; the paper's form also takes P_i = sum_j f^2 and keeps M'(P_i) in the
 * workspace, the second derivative of Section 3.1's array); MD_F_FORCE computes
 *   F_i = - sum_j [(F'(rho_i) + F'(rho_j)) f'(r_ij) + phi'(r_ij)] (q_i - q_j) / r_ij
 * into f over the Cr-Cr list (each atom gathers over its full list: no atomics).  With
 * MD_F_MORSE (and MD_F_FORCE) the Cr-C Morse forces of md_morse_forces are included in f:
 * they are computed by extra blocks of the density launch when MD_F_DENSITY is also set
 * (Task 4c does not depend on the density), else by a launch of their own before the force
 * pass.  With MD_F_KICK the Task 5 half kick v += F/m dt/2 of the whole force follows
 * (mobile atoms).  MD_F_MIXED selects FP32 arithmetic.  Lists must be current
 * (md_build_neighbors in the same step).  With two-tier lists (icap > 0) MD_F_DENSITY first
 * refills the inner list from the outer one at the current positions (Section 2.6, Task 1:
 * the inner list is updated every step), and both passes read it. */
MD_API int md_eam_forces(md_system *sys, const md_atoms *a, const md_lists *l, uint32_t flags,
                         double *rho_out, void *stream);

/* Task 4c: Cr-C Morse forces added into f (F_i += -phiM'(r) (q_i - q_k)/r over the Cr-C
 * list), recorded per atom for the load on the indenter (minus their sum) and the Morse
 * energy reported by md_energy.  Flags: MD_F_KICK applies the half kick of these forces
 * only, MD_F_MIXED FP32 arithmetic. */
MD_API int md_morse_forces(md_system *sys, const md_atoms *a, const md_lists *l, uint32_t flags,
                           void *stream);

/* Tasks 2+3 (MD_PHASE_KICK_DRIFT, Eqs. A11-A12) or Task 5 (MD_PHASE_KICK) for all mobile
 * atoms, a = F/m.  KICK_DRIFT also moves the indenter and measures displacements for the
 * skin test of the next md_build_neighbors.  Positions are not wrapped here. */
MD_API int md_verlet_step(md_system *sys, int32_t phase, const md_atoms *a, void *stream);

/* Task 4d: energies, virial, indenter load and counters (MD_NOBS doubles per replica,
 * device pointer out[nrep][MD_NOBS]), reduced in a fixed order in FP64: embedding and pair
 * energy and virial from the partials of the last md_eam_forces call made with
 * MD_F_ENERGY, Morse energy and load from the last Morse evaluation (zero before any and
 * after a list build), kinetic energy of the current velocities. */
MD_API int md_energy(md_system *sys, const md_atoms *a, double *out, void *stream);

/* ---------------------------------------------------------------------------------- */
/* Whole steps                                                                          */
/* ---------------------------------------------------------------------------------- */

/* Records md_run can make of its steps, for measurement (each member may be NULL). */
#define MD_TRACE_EVENTS 8  /* events per step */
typedef struct md_trace {
    void *const *events;  /* MD_TRACE_EVENTS * nsteps hipEvent_t handles created by the caller
                             (NULL entries are skipped), recorded on the stream around step k's
                             kernels: [8k], [8k+1] the EAM force kernel (Eq. 1); [8k+2], [8k+3]
                             the Cr-Cr list kernel (which returns at once when no rebuild is
                             due); [8k+4], [8k+5] the density kernel (with the Cr-C pass);
                             [8k+6], [8k+7] the inner-list refill (two-tier lists only) */
    int32_t *builds;      /* device int32[nsteps][nrep]: each replica's list-build count after
                             each step (a step rebuilt a replica's lists iff its count grew) */
} md_trace;

/* Enqueue nsteps whole time steps in the order of Table 1 (Tasks 2+3 -> 1 -> 4 -> 5) for
 * every replica: md_verlet_step(KICK_DRIFT), md_build_neighbors, then the Task 4 passes
 * with the Cr-C forces included in the Eq. 1 pass and the final half kick applied by it
 * (as md_eam_forces(DENSITY | FORCE | MORSE | KICK)).  Where a step's end velocities are
 * not observed (no energies after it, not the last step), its final half kick and the next
 * step's first one are given together (a full kick of the same force) and the next Task 3
 * only drifts: the same velocity Verlet steps, rounded once per kick pair instead of twice.
 * That drift is done by the force pass itself, into a second position buffer (and FP32
 * shadow) in the workspace.  The force pass of such a step leaves a->f alone: no
 * kick reads the force before the next pass that stores it (within md_run a->f is stale
 * meanwhile).  After md_run the velocities are at the last whole step, the positions are
 * back in a->q and a->f holds the forces at them.
 * flags: MD_F_MIXED selects FP32 arithmetic.  energy_every > 0: after step k with
 * k % energy_every == 0 the energies are written as by md_energy to
 * obs[(k / energy_every - 1) * nrep * MD_NOBS ...] (device memory, caller-owned).  For such
 * a step other than the last, the force pass takes the kinetic energy and the Cr-C sums at
 * the whole step itself and then gives the next step's first half kick as well (the same
 * sums grouped per block of the pass, equal to md_energy's to rounding).
 * trace: NULL, or timing and rebuild records of the steps (see md_trace).
 * Lists must have been built and forces evaluated once before the first step
 * (md_build_neighbors with MD_B_FORCE, md_eam_forces with DENSITY|FORCE|MORSE). */
MD_API int md_run(md_system *sys, const md_atoms *a, const md_lists *l, int32_t nsteps,
                  uint32_t flags, int32_t energy_every, double *obs, const md_trace *trace,
                  void *stream);

/* Capture md_run(nsteps, flags, energy_every, obs, no events) on `stream` into an
 * instantiated HIP graph (*graph_exec, host handle) that replays the same steps on the
 * same buffers with one launch.  The graph holds no memset nodes. */
MD_API int md_graph_create(md_system *sys, const md_atoms *a, const md_lists *l, int32_t nsteps,
                           uint32_t flags, int32_t energy_every, double *obs, void *stream,
                           void **graph_exec);
MD_API int md_graph_launch(void *graph_exec, void *stream);
MD_API int md_graph_destroy(void *graph_exec);

/* Task 2 of later steps moves the indenter by v_ind * dt along z (Angstrom/fs; the value given
 * at md_system_create until changed here), for the load-unload protocol of Section 2.5: relax
 * with 0, load with a negative, withdraw with a positive velocity.  Host state only: calls
 * enqueued after it use the new value; a HIP graph keeps the value it was captured with. */
MD_API int md_set_indenter_velocity(md_system *sys, double v_ind);

/* Synchronise `stream` and copy the device flags to *st (summed / maxed over replicas). */
MD_API int md_check(md_system *sys, md_status *st, void *stream);

/* Clear overflow / non-finite / sync_timeout flags (e.g. after enlarging the lists), and
 * after a list build that gave up, reset what it left behind (cell counts) so that builds run
 * again; the next build should then be forced (MD_B_FORCE). */
MD_API int md_clear_flags(md_system *sys, void *stream);

MD_API const char *md_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
