/*
 * dmts.h -- C ABI of the MI355X (gfx950) library for the hot path of distilled
 * multi-time-step (DMTS) molecular dynamics with neural network potentials.
 *
 * The method (the paper's Methods section and Algorithm 1): a cheap one-interaction
 * potential with a 3.5 A cutoff is integrated at a short inner step; every n_slow inner
 * steps the outer level applies the slow correction F_large - F_small of an expensive
 * two-interaction potential as a half-kick on both sides of the inner loop.
 *
 * Conventions for every entry point
 *   - Units: Angstrom, femtosecond, atomic mass unit, electron-volt; forces eV/A,
 *     velocities A/fs.
 *   - Array arguments are DEVICE pointers owned by the caller, unless the name says
 *     "host_".  Coordinate-like arrays are structure-of-arrays [3][n_atoms] (all x, then
 *     all y, then all z), contiguous.
 *   - species: int32 codes 0..n_species-1 (H=0, C=1, N=2, O=3, S=4 for the 5-species
 *     models).  box: edge of a periodic cube, or 0.0 for open boundaries.
 *   - sys_offsets (optional, device, int32 [n_sys+1]): CSR ranges of independent
 *     molecules of a batch.  With open boundaries pairs never cross molecules; with a
 *     periodic box sys_offsets must be NULL.
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  Every call only
 *     enqueues work on that stream; none synchronizes the host unless documented.
 *   - Handles are opaque, not thread-safe, and must be used from one stream at a time.
 *     The library owns their internal device memory; it never frees, reallocates or
 *     retains caller arrays beyond the enqueued work.
 *   - Errors: every call returns a dmts_status.  Argument and shape errors are detected
 *     on the host before anything is enqueued and leave all state unchanged; the
 *     message is available from dmts_last_error() (thread-local).  Conditions found on
 *     the device (neighbor capacity overflow, non-finite values) set bits in a device
 *     flag word of the handle, read back by nnp_nlist_flags() and dmts_state_flags(),
 *     and reported by dmts_step() when it returns.  No C++ exception crosses the ABI.
 */
#ifndef DMTS_H
#define DMTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmts_status;
enum {
  DMTS_OK = 0,
  DMTS_E_ARG = 1,        /* bad argument, unsupported shape, NULL pointer          */
  DMTS_E_BOX = 2,        /* cutoff >= box/2 for a periodic box                      */
  DMTS_E_CAPACITY = 3,   /* a neighbor list overflowed its capacity                 */
  DMTS_E_NONFINITE = 4,  /* NaN/Inf met in positions, energies or forces            */
  DMTS_E_HIP = 5,        /* a HIP runtime call failed                               */
  DMTS_E_OOM = 6,        /* device allocation failed                                */
  DMTS_E_STATE = 7       /* handle used inconsistently (sizes changed, ...)         */
};

/* Device flag bits. */
#define DMTS_FLAG_NBR_OVERFLOW 0x1u
#define DMTS_FLAG_NONFINITE 0x2u

/* Model kinds (see nnp_model_create). */
#define NNP_KIND_ONE_INTERACTION 0
#define NNP_KIND_TWO_INTERACTION 1
/* Arithmetic of the dense (MLP) contractions. */
#define NNP_PREC_FP32 0
#define NNP_PREC_BF16 1

typedef struct nnp_model nnp_model;
typedef struct nnp_nlist nnp_nlist;
typedef struct dmts_state dmts_state;

typedef struct {
  int32_t kind;          /* NNP_KIND_*                                               */
  int32_t n_rbf;         /* Gaussian radial functions K (16 or 32)                   */
  int32_t width;         /* hidden width F (64 for kind 0, 128 for kind 1)           */
  int32_t emb_dim;       /* species embedding width (16)                             */
  int32_t n_species;     /* rows of the embedding table (<= 8)                       */
  int32_t precision;     /* NNP_PREC_*                                               */
  double cutoff;         /* r_c in A                                                 */
  double energy_scale;   /* s_E in eV (0.01 for the synthetic models)                */
} nnp_model_desc;

/* ---------------------------------------------------------------- errors, version */
const char* dmts_last_error(void);
const char* dmts_version(void);

/* ---------------------------------------------------------------- models
 * The two potentials that stand in for the paper's fast distilled model (one
 * message-passing interaction, short cutoff) and its reference model (two
 * interactions) (Methods: neural network architectures).
 *
 * kind 0 (fast level):   a_ij = W_pair [b(r_ij); e_zi; e_zj],  m_ij = f_c(r_ij) SiLU(a_ij),
 *                        h_i = sum_j m_ij,  E_i = s_E w_atom2 . SiLU(W_atom1 h_i).
 * kind 1 (reference):    two interactions with messages m^t_ij = f_c SiLU(W_pair_t
 *                        [b; s^t_i; s^t_j]) (s^1 = e_z, s^2 = h^1), l <= 2 Cartesian moments
 *                        of u_ij = d_ij/r_c, invariants q = [M0; |M1|^2; |M2|^2] per
 *                        channel, h^1 = SiLU(U1 q^1), h^2 = h^1 + SiLU(U2 q^2),
 *                        E_i = s_E w_out2 . SiLU(W_out1 h^2).
 * with Gaussian radial functions b_k(r) = exp(-(r - k r_c/(K-1))^2 / (2 (r_c/(K-1))^2)),
 * cosine cutoff f_c(r) = (cos(pi r / r_c) + 1)/2 for r < r_c, and no biases.
 *
 * host_weights: float32 blob of n_weights entries, row-major tensors in this order
 *   kind 0: emb [Z][D], W_pair [F][K+2D], W_atom1 [F][F], w_atom2 [F]
 *   kind 1: emb [Z][D], W_pair1 [F][K+2D], U1 [F][3F], W_pair2 [F][K+2F], U2 [F][3F],
 *           W_out1 [F][F], w_out2 [F]
 * The blob is copied; the caller keeps ownership.  Supported shapes: kind 0 with
 * (K, F) = (16, 64); kind 1 with (K, F) = (32, 128); D = 16; n_species <= 8.
 * Blocking: synchronizes the device once (weight upload).  Returns DMTS_E_ARG for an
 * unsupported shape or a wrong n_weights.
 */
dmts_status nnp_model_create(const nnp_model_desc* desc, const float* host_weights,
                             int64_t n_weights, nnp_model** out);
void nnp_model_destroy(nnp_model* model);

/* Launch shapes (the batching form's tiles, chosen by an autotuner).  Every kernel of a
 * model computes each receiver and each atom row with a fixed arithmetic whatever
 * work-group holds it, so a shape changes speed only, never a result bit.
 *   receivers_per_group  two-interaction pair kernels: receivers per work-group, one
 *                        wave each, sharing the work-group's staged weights: 2, 4 or 8;
 *   atom_tiles           two-interaction per-atom MLP chains: 16-atom row tiles per
 *                        work-group (each weight load feeds them all): 1 or 2;
 *   keep_derivatives     one-interaction model: 1 keeps the radial derivative factors of a
 *                        receiver's first 32 pairs in registers across its readout (three
 *                        waves per SIMD), 0 recomputes them (four waves per SIMD);
 *   work_groups          grid-stride kernels: 0 = one work-group per group of receivers
 *                        (one persistent round when that is between one and two rounds of
 *                        resident work-groups), k > 0 = a persistent grid of at most k.
 * A model holds a default shape (4, 2, 1, 0 at creation) and one shape per size bucket
 * (systems with the same number of bits in their atom count).
 * nnp_model_set_shape: n_atoms <= 0 sets the default and forgets every bucket's shape;
 *   n_atoms > 0 sets the shape of n_atoms' bucket.  DMTS_E_ARG for a value outside the
 *   lists above.  nnp_model_get_shape: the shape a system of n_atoms uses (n_atoms <= 0:
 *   the default).
 * nnp_model_set_grid / nnp_model_get_grid: work_groups of the default shape (set_grid also
 *   sets it in every bucket's shape).
 * nnp_autotune times energy+force evaluations of the given system (list built from pos)
 *   for every candidate shape: the values above that the model's kind uses, times
 *   work_groups in {0, 256, 512, 1024, 2048, 4096} (median of `reps` timings after a
 *   warm-up, each over four back-to-back evaluations between two HIP events on `stream`,
 *   so that the events' own cost does not decide between close shapes), keeps the fastest
 *   as the shape of n_atoms' bucket and returns it in *chosen (host) with its time per
 *   evaluation in *best_ms (host).  Blocking: synchronizes the stream and allocates
 *   scratch. */
typedef struct {
  int32_t receivers_per_group;
  int32_t atom_tiles;
  int32_t keep_derivatives;
  int32_t work_groups;
} nnp_tile_shape;
dmts_status nnp_model_set_shape(nnp_model* model, int32_t n_atoms, const nnp_tile_shape* shape);
dmts_status nnp_model_get_shape(nnp_model* model, int32_t n_atoms, nnp_tile_shape* shape);
dmts_status nnp_model_set_grid(nnp_model* model, int32_t work_groups);
dmts_status nnp_model_get_grid(nnp_model* model, int32_t* work_groups);
dmts_status nnp_autotune(nnp_model* model, nnp_nlist* nl, const double* pos,
                         const int32_t* species, int32_t n_atoms, double box,
                         const int32_t* sys_offsets, int32_t n_sys, int32_t reps, void* stream,
                         nnp_tile_shape* chosen, double* best_ms);

/* ---------------------------------------------------------------- neighbor lists
 * A full (both directions) list of ordered pairs {(i, j): j != i, |d_ij| < cutoff},
 * d_ij = x_j - x_i under the minimum-image convention of the cube (or plain difference
 * for open boundaries, restricted to one molecule when sys_offsets is given).  The
 * paper does not describe its neighbor search; this is the pair set its message
 * passing sums over.
 *
 * Storage is CSR with each row padded to a multiple of row_align (1, 16 or 32) with
 * entries -1; rev[p] is the position of the reverse pair (j, i) for every real entry.
 * Rows are filled in a fixed order, so the list is bitwise reproducible.
 *
 * nnp_nlist_create: capacity for max_atoms atoms and max_pairs padded entries.
 *   Blocking (allocates).
 * nnp_build_neighbors: rebuilds the list for pos ([3][n_atoms] float64).  A periodic box
 *   needs cutoff < box/2 (else DMTS_E_BOX).  A list that would exceed max_pairs sets
 *   DMTS_FLAG_NBR_OVERFLOW on the device and is then incomplete.  Asynchronous.
 * nnp_filter_neighbors: rebuilds child as the list at cutoff (<= the parent's) for pos,
 *   from the rows of parent (built for the same atoms, at a longer cutoff, from positions
 *   none of which has since moved more than half the cutoff difference): each parent row
 *   filtered to |d_ij| < cutoff at pos, which keeps it sorted, so the child equals a list
 *   built at cutoff with nnp_build_neighbors (a fast model of the reference kind reuses
 *   the reference model's list this way).  child and parent must differ; the child's
 *   row_align and capacity apply; DMTS_E_ARG for a cutoff outside (0, parent cutoff] or a
 *   child with room for fewer atoms.  Asynchronous.
 * nnp_nlist_flags: synchronizes the stream, returns the flag word in *host_flags and
 *   clears it.
 * nnp_nlist_download: synchronizes, copies offs [n_atoms+1], nbr and rev [offs[n]] to
 *   host arrays of capacity host_cap entries (DMTS_E_CAPACITY if too small); a test
 *   and debugging aid.  *n_entries receives offs[n_atoms].
 */
dmts_status nnp_nlist_create(int32_t max_atoms, int64_t max_pairs, int32_t row_align,
                             nnp_nlist** out);
void nnp_nlist_destroy(nnp_nlist* nl);
dmts_status nnp_build_neighbors(nnp_nlist* nl, const double* pos, int32_t n_atoms,
                                double box, const int32_t* sys_offsets, int32_t n_sys,
                                double cutoff, void* stream);
dmts_status nnp_filter_neighbors(nnp_nlist* child, const nnp_nlist* parent, const double* pos,
                                 double cutoff, void* stream);
dmts_status nnp_nlist_flags(nnp_nlist* nl, void* stream, uint32_t* host_flags);
dmts_status nnp_nlist_download(nnp_nlist* nl, void* stream, int32_t* host_offs,
                               int32_t* host_nbr, int32_t* host_rev, int64_t host_cap,
                               int64_t* n_entries);

/* ---------------------------------------------------------------- energy and forces
 * Energy per system (float64, device [n_sys]) and forces F = -dE/dx (float32, device
 * [3][n_atoms], or NULL for energy only) of one model on the pairs of nl, which must
 * have been built from the same pos with cutoff >= the model's cutoff.  Pairs beyond
 * the model's cutoff contribute zero.  Per-atom energies (float32, device [n_atoms]) are
 * written to atom_energy when it is not NULL.  n_sys = 1 and sys_offsets = NULL for one
 * system.  Asynchronous; the model's workspace grows (blocking) when a larger system or
 * list than before is seen.
 */
dmts_status nnp_energy_forces(nnp_model* model, nnp_nlist* nl, const double* pos,
                              const int32_t* species, int32_t n_atoms, double box,
                              const int32_t* sys_offsets, int32_t n_sys, double* energy,
                              float* forces, float* atom_energy, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): nnp_energy_forces of a
 * one-interaction (fast) model that allocates nothing.  Same arguments, results (bit for
 * bit) and asynchrony as nnp_energy_forces; the caller still passes inputs, outputs and a
 * built list (nnp_nlist_create allocates, once).  Its workspace is a fixed array of
 * 13 MiB in device memory, one per GPU the library runs on, held until the process ends;
 * it holds systems of at most 8,192 atoms: more returns DMTS_E_CAPACITY, a
 * two-interaction model DMTS_E_ARG, both before anything is enqueued.  Every call on one
 * GPU shares that GPU's array (its contents are those of the last call; nothing in it needs
 * to start at zero), so calls that overlap on one GPU (other streams or threads) race:
 * order them on one stream.  The first call on a device looks up the array's address
 * there (hipGetSymbolAddress); with kernel timing (dmts_prof_enable) on, timing events may
 * be created.
 */
dmts_status nnp_energy_forces_noalloc(nnp_model* model, nnp_nlist* nl, const double* pos,
                                      const int32_t* species, int32_t n_atoms, double box,
                                      const int32_t* sys_offsets, int32_t n_sys,
                                      double* energy, float* forces, float* atom_energy,
                                      void* stream);

/* ---------------------------------------------------------------- the RESPA loop
 * Algorithm 1 (BAOAB-RESPA with force splitting).  One outer step of length dt_outer:
 *   v += dt/2 (F - F_small)/m;
 *   n_inner times: v += h/2 F_small/m; x += h/2 v; v <- O_h(v); x += h/2 v;
 *                  F_small <- small(x); v += h/2 F_small/m   (h = dt_outer / n_inner);
 *   F <- large(x); v += dt/2 (F - F_small)/m.
 * O_h is the thermostat of Algorithm 1's middle step, the exact Ornstein-Uhlenbeck update
 * v <- c v + sqrt((1 - c^2) k_B T KAPPA / m) xi with c = exp(-gamma h), off (the
 * identity: NVE) unless dmts_state_set_thermostat gave gamma > 0.
 * Both forces are evaluated on the first step only and carried between calls
 * afterwards (for the same two models: a call with another model, or with a model created
 * since, evaluates both afresh).  With small == NULL the call runs the single-time-step baseline instead:
 * BAOAB with the large model at dt_outer (velocity Verlet when gamma = 0; n_inner is
 * ignored).
 *
 * dmts_state_create: n_atoms atoms in a periodic cube `box` (open boundaries: 0.0),
 *   species (device [n_atoms], borrowed for the life of the state), masses per species
 *   (host, copied).  max_nbrs_* bound the average number of neighbors per atom within
 *   each model's cutoff (the lists are sized n_atoms * max_nbrs).  Blocking.
 * dmts_step: advances x and v (device float64 [3][n_atoms], updated in place) by
 *   n_outer outer steps.  energies_out (device float64 [4], optional) receives
 *   {E_large, E_small, kinetic, E_large + kinetic} at the final positions.  Checks the
 *   device flags once at the end (one host synchronization) and returns
 *   DMTS_E_CAPACITY or DMTS_E_NONFINITE if set.
 * dmts_state_reset: forget the carried forces (call after changing x outside
 *   dmts_step).
 * dmts_state_fallbacks: number of dmts_step calls that had to be redone because an atom
 *   moved farther than the shared neighbor list allows (see the neighbor-list note).
 *
 * Neighbor-list note: each reference evaluation gets one list at
 * max(r_c,large, r_c,small + 1 A) (at r_c,large for the single-time-step baseline), filtered
 * at the current positions from rows kept at that cutoff plus a skin (dmts_state_set_skin);
 * the rows themselves are rebuilt only when some atom has moved half the skin since their
 * last rebuild, so the list is the one a fresh build would give.  The fast model of the
 * next inner steps reuses the reference evaluation's list, which
 * is exact while every atom stays within half the gap to the fast cutoff of where the
 * list was built.  The device checks that bound at every drift; when it fails, the call
 * restores its starting x, v and carried forces and repeats with fresh lists for every
 * evaluation (same results, slower).  The fast model may be of either kind: a
 * one-interaction model compacts the shared rows to its cutoff inside its own kernels; a
 * two-interaction one (the message-passing fast model) gets the shared list filtered to
 * its cutoff (nnp_filter_neighbors) before each evaluation, so max_nbrs_small must hold
 * its rows padded to 16.
 * dmts_state_forces: device pointers to the carried F_large and F_small (float32
 *   [3][n_atoms]) for inspection.
 */
dmts_status dmts_state_create(int32_t n_atoms, double box, const int32_t* species,
                              const double* host_mass_by_species, int32_t n_species,
                              double dt_outer_fs, int32_t n_inner, int32_t max_nbrs_small,
                              int32_t max_nbrs_large, dmts_state** out);
void dmts_state_destroy(dmts_state* st);
dmts_status dmts_step(dmts_state* st, double* x, double* v, nnp_model* small,
                      nnp_model* large, int32_t n_outer, double* energies_out,
                      void* stream);
dmts_status dmts_state_reset(dmts_state* st);
dmts_status dmts_state_fallbacks(dmts_state* st, int64_t* n_calls);

/* Per-atom masses (amu, host array of n_atoms values, each finite and > 0), used instead of
 * the species table by every kick, O-step and kinetic energy of the state: hydrogen mass
 * repartitioning (heavier hydrogens for longer outer steps: the bulk-water stability
 * tests and their table) needs masses that depend on the bonding, not only on the
 * species.  NULL returns to the species table.  Copies the values to device memory the state owns (blocking; call it
 * between steps, not while a dmts_step of this state is in flight).  DMTS_E_ARG for a
 * count other than the state's or a mass that is not finite and positive.
 */
dmts_status dmts_state_set_atom_masses(dmts_state* st, const double* host_masses,
                                       int32_t n_atoms);

/* Langevin thermostat of Algorithm 1 (the O-step; the paper's production runs use
 * gamma = 1 ps^-1 = 0.001 fs^-1).  gamma_per_fs >= 0 (0 turns it off), temperature_K >= 0,
 * seed: the key of the noise.  Resets the O-step counter to 0; DMTS_E_ARG for a negative
 * or non-finite gamma or temperature.
 * The k-th O-step of the state (k = 0, 1, ...) gives atom i the standard normals
 * xi = (sqrt(-2 ln u0) cos(2 pi u1), sqrt(-2 ln u0) sin(2 pi u1), sqrt(-2 ln u2) cos(2 pi u3)),
 * u_j = (r_j + 1/2) / 2^32, r = Philox4x32-10 (Salmon et al., SC 2011) of counter
 * (i, k mod 2^32, k div 2^32, 0) and key (seed mod 2^32, seed div 2^32), so that any
 * implementation of the generator reproduces the noise.  A call redone with exact lists
 * reuses its O-step numbers.  dmts_state_o_steps returns the number of O-steps taken.
 */
dmts_status dmts_state_set_thermostat(dmts_state* st, double gamma_per_fs,
                                      double temperature_K, uint64_t seed);
dmts_status dmts_state_o_steps(dmts_state* st, uint64_t* n_o_steps);

/* Force-difference monitor (the paper's guard against holes in the fast model: where
 * |F - F_small| of an atom exceeds an unphysical threshold, 150 kcal/mol/A = 6.505 eV/A in
 * the paper, the integrator temporarily reverts to single-time-step integration; Results,
 * protein-ligand complexes).
 * dmts_state_set_fdiff_threshold: eV_per_A > 0 turns the check on (0, the default, off;
 *   DMTS_E_ARG for a negative or non-finite value).  With the check on, dmts_step takes its
 *   n_outer outer steps one at a time: both slow kicks of a step test |F_i - F_small,i| of
 *   every atom, and when any atom exceeds the threshold the step is rolled back to its
 *   starting x, v and carried forces and redone as n_inner single-time-step steps of length
 *   dt_outer / n_inner with the reference model (same O-step numbers); the next step then
 *   evaluates both models afresh.  A breach seen while a step is redone with exact lists
 *   (neighbor-list note) is acted on the same way.  Each step backs up its starting state
 *   and reads the device flags once (one host synchronization per outer step).
 * dmts_state_fdiff: the number of outer steps redone that way since the state was created,
 *   and the largest breaching |F - F_small| (eV/A) seen by the last dmts_step call (0 if
 *   none breached).
 */
dmts_status dmts_state_set_fdiff_threshold(dmts_state* st, double eV_per_A);
dmts_status dmts_state_fdiff(dmts_state* st, int64_t* n_sts_redos, double* last_breach);
dmts_status dmts_state_forces(dmts_state* st, const float** f_large, const float** f_small);
dmts_status dmts_state_flags(dmts_state* st, void* stream, uint32_t* host_flags);

/* Skin of the reference evaluations' lists (neighbor-list note; not a passage of the paper,
 * which leaves the neighbor search open: a Verlet-list skin as in any molecular-dynamics
 * code).
 * dmts_state_set_skin: skin_A >= 0 (finite; DMTS_E_ARG otherwise), 1.5 A by default; 0
 *   builds the list afresh at every reference evaluation.  The skin is also dropped (fresh
 *   builds) for an open box or when cutoff + skin reaches half the box edge.  A change
 *   takes effect at the next reference evaluation (which rebuilds).  Results do not depend
 *   on the skin: the lists, and so every sum, are the same.  Rows at cutoff + skin may hold
 *   up to 512 entries (twice a list row's 256, so that a skin does not lower the density a
 *   state can run at); a longer one raises DMTS_FLAG_NBR_OVERFLOW (DMTS_E_CAPACITY from
 *   dmts_step) as an overlong row of a fresh build does.
 * dmts_state_get_skin: the skin in use (A).
 * dmts_state_list_builds: the number of row rebuilds so far (blocking: synchronizes the
 *   device).
 */
dmts_status dmts_state_set_skin(dmts_state* st, double skin_A);
dmts_status dmts_state_get_skin(dmts_state* st, double* skin_A);
dmts_status dmts_state_list_builds(dmts_state* st, int64_t* n_builds);

/* ---------------------------------------------------------------- kernel timing
 * Optional HIP-event timing of individual kernel classes, for measurement harnesses.
 * dmts_prof_enable takes a bit mask (bit k = class k, 0 = off, the default).  Each launch
 * of an enabled class is bracketed by two hipEventRecord calls on its stream (a few
 * microseconds of overhead per launch); disabled classes cost nothing.  dmts_prof_read synchronizes on the recorded events and returns the summed
 * duration in milliseconds and the number of launches of one class since the last reset.
 * dmts_prof_sample(every): time only the first of every `every` launches of each enabled
 * class (counted from the last reset; 1, the default, times all), so that a harness can
 * time a kernel inside a throughput measurement while adding the events' cost to a
 * fraction of its launches.  DMTS_E_ARG for 0.
 */
enum {
  DMTS_K_SMALL_FORWARD = 0,
  DMTS_K_SMALL_BACKWARD = 1,
  DMTS_K_PAIR1_FORWARD = 2,
  DMTS_K_PAIR2_FORWARD = 3,
  DMTS_K_PAIR2_BACKWARD = 4,
  DMTS_K_PAIR1_BACKWARD = 5,
  DMTS_K_NEIGHBORS = 6,      /* a whole neighbor-list build (all its kernels)          */
  DMTS_K_ATOM_GEMM = 7,      /* each per-atom MFMA GEMM                                */
  DMTS_K_GATHER = 8,         /* sender and force gathers                               */
  DMTS_K_INTEGRATE = 9,      /* fused kick/drift launches                              */
  DMTS_K_COUNT = 10
};
dmts_status dmts_prof_enable(uint32_t class_mask);
dmts_status dmts_prof_sample(uint32_t every);
dmts_status dmts_prof_reset(void);
dmts_status dmts_prof_read(int32_t kernel_class, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* DMTS_H */
