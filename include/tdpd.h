/*
 * tdpd.h -- C ABI of the MI355X tDPD + red-blood-cell time-step library.
 *
 * The library advances the particle system of transport dissipative particle
 * dynamics with RBC membranes (Blumers et al., arXiv:1611.06163):
 *   - pair forces: conservative, dissipative and random, Eqs. (3)-(5), with
 *     the fluctuation-dissipation pairing of Eq. (6), summed as in Eq. (2);
 *   - concentration fluxes: Fickian and random, Eqs. (8)-(9) with the pairing
 *     of Eq. (10), summed as in Eq. (7), for n_species species per particle;
 *   - membrane bonded terms (Section 2.2): WLC and POW springs, Eqs. (13)-(14),
 *     bond viscosity and its random partner, Eqs. (15)-(16), global and local
 *     area and global volume constraints, Eqs. (17)-(18), bending, Eq. (19);
 *   - velocity-Verlet integration of Eqs. (1)-(2) and (7).
 * Every step runs in HIP kernels on the device; the host only enqueues.
 *
 * Conventions shared by all calls:
 *   - Every function returns a tdpd_status: 0 on success, < 0 on error.
 *     Nothing throws across the ABI.  tdpd_last_error() gives a message.
 *   - Host buffers passed in are read during the call and stay owned by the
 *     caller; host buffers passed out are caller-allocated with the stated
 *     size.  Device memory belongs to the library; it is obtained through
 *     the caller's allocator callback when one is given, else hipMalloc.
 *   - Particle arrays are in gid order: gid = index in the array given to
 *     tdpd_set_state.  Vectors are AoS [n][3] float32, concentrations
 *     [n][n_species] float32.
 *   - The HIP stream given at creation is borrowed; every kernel is enqueued
 *     on it.  Calls are not thread-safe for one system.
 */
#ifndef TDPD_H
#define TDPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TDPD_OK = 0,
  TDPD_ERR_INVALID_ARG = -1,   /* bad pointer, size or parameter */
  TDPD_ERR_BOX_TOO_SMALL = -2, /* fewer than 3 cells of size > max(rc, rcc) per side */
  TDPD_ERR_OOM = -3,           /* device allocation failed */
  TDPD_ERR_HIP = -4,           /* a HIP runtime call failed */
  TDPD_ERR_NONFINITE = -5,     /* a force or state value became NaN/Inf */
  TDPD_ERR_BOND_OVEREXTENDED = -6, /* a WLC bond reached its maximum length */
  TDPD_ERR_STATE = -7,         /* call out of order (e.g. step before set_state) */
  TDPD_ERR_UNSUPPORTED = -8,   /* valid request outside what the library handles */
  TDPD_ERR_CAPACITY = -9,      /* an output buffer was too small */
  TDPD_ERR_IO = -10,           /* a checkpoint file could not be read or written, or does not match */
  TDPD_ERR_LIST = -11          /* a neighbour list was invalidated (skin exceeded or list full) */
} tdpd_status;

#define TDPD_MAX_TYPES 4
#define TDPD_MAX_SPECIES 16

/* Terms bitmask (tdpd_params.terms); all set by default. */
#define TDPD_TERM_CONSERVATIVE 1    /* Eq. (3) */
#define TDPD_TERM_DISSIPATIVE 2     /* Eq. (4) */
#define TDPD_TERM_RANDOM 4          /* Eq. (5) */
#define TDPD_TERM_FLUX_FICK 8       /* Eq. (8) */
#define TDPD_TERM_FLUX_RANDOM 16    /* Eq. (9) (needs m_s > 0) */
#define TDPD_TERM_BOND 32           /* Eqs. (13)-(14) */
#define TDPD_TERM_BOND_VISCOUS 64   /* Eq. (15) */
#define TDPD_TERM_BOND_RANDOM 128   /* Eq. (16) */
#define TDPD_TERM_AREA 256          /* Eq. (17) */
#define TDPD_TERM_VOLUME 512        /* Eq. (18) */
#define TDPD_TERM_BENDING 1024      /* Eq. (19) */
#define TDPD_TERM_BODY_FORCE 2048   /* constant external force on mobile particles */
#define TDPD_TERMS_ALL 4095

/* Particle flags word: bits 0-7 type index (< n_types), bit 8 frozen
   (never moved, F = Q = 0, concentrations held fixed; used for walls). */
#define TDPD_FLAG_FROZEN (1u << 8)

typedef struct {
  float box[3];      /* periodic box lengths; positions live in [0, L) */
  float rc;          /* force cutoff r_c, Eqs. (3)-(5) */
  float rcc;         /* flux cutoff r_cc, Eqs. (8)-(9) */
  float dt;          /* time step */
  float kT;          /* k_B T */
  float rho;         /* number density in Eq. (10) */
  float m_s;         /* solute mass ratio in Eq. (10); 0 switches Q^R off */
  float s_exp;       /* w_D = (1 - r/rc)^s_exp, w_R = w_D^(1/2) */
  float sc_exp;      /* w_DC = (1 - r/rcc)^sc_exp, w_RC = w_DC^(1/2) */
  int32_t n_types;   /* 1..TDPD_MAX_TYPES */
  int32_t n_species; /* 1..TDPD_MAX_SPECIES */
  float alpha[TDPD_MAX_TYPES * TDPD_MAX_TYPES]; /* [ti*n_types+tj], symmetric */
  float gamma[TDPD_MAX_TYPES * TDPD_MAX_TYPES];
  float sigma[TDPD_MAX_TYPES * TDPD_MAX_TYPES];
  float kappa[TDPD_MAX_SPECIES * TDPD_MAX_TYPES * TDPD_MAX_TYPES]; /* [(s*T+ti)*T+tj] */
  float body_force[3];
  int32_t wall_axis; /* -1: none; 0-2: mobile particles crossing wall_w or
                        L - wall_w on that axis are reflected; 3: a tube about
                        the x-parallel axis through (L_y/2, L_z/2), see
                        wall_radius */
  float wall_w;
  uint64_t seed;     /* Philox key */
  uint32_t box_id;   /* part of the Philox counter, < 2^24 */
  int32_t terms;     /* TDPD_TERM_* mask */
  float shear_rate;  /* Lees-Edwards shear rate gamma (0: plain periodic box):
                        the periodic image above in y sits
                        delta_k = fl32(fmod(gamma L_y * (k dt), L_x)) further
                        in x at step counter k and moves with
                        u = fl32(gamma L_y) in x (FP64 products of the FP32
                        values); not with walls (TDPD_ERR_UNSUPPORTED) */
  /* Source term Q^S of Eq. (7), the external contribution the paper leaves
     open, read as a zero-order source less a first-order decay of the
     particle's own concentration per species s and particle type t:
     Q^S_i = source[s*n_types + t_i] - decay[s*n_types + t_i] * C_i^s, added
     to the fluxes of mobile particles where they are evaluated (at the
     half-step concentrations).  Zero switches it off; values must be finite. */
  float source[TDPD_MAX_SPECIES * TDPD_MAX_TYPES];
  float decay[TDPD_MAX_SPECIES * TDPD_MAX_TYPES];
  /* Tube radius R for wall_axis = 3 (the Dirichlet cylinder of the paper's
     transport validation, Section 4): a mobile particle that ends a drift
     farther than R from the axis is mirrored along its radius to 2R - r and
     its velocity reversed.  The wall itself is made of frozen particles of
     the input (outside R), which hold their concentration: with kappa to
     the fluid above zero they are a Dirichlet reservoir.  Needs
     0 < R < min(L_y, L_z) / 2. */
  float wall_radius;
} tdpd_params;

typedef struct {
  float p;        /* WLC persistence length, Eq. (13) */
  float x0;       /* rest extension l0 / l_m of every bond */
  float m_pow;    /* POW exponent m, Eq. (14); k_p per bond makes l0 force-free */
  float kb;       /* bending constant, Eq. (19) */
  float theta0;   /* spontaneous angle; NaN = mean dihedral of the rest shape */
  float kg, kl, kv; /* global area, local area, volume constants, Eqs. (17)-(18) */
  float gamma_t, gamma_c; /* bond viscosities, Eqs. (15)-(16); 3 gamma_c >= gamma_t */
} tdpd_mesh_params;

/* One periodic box of a batched ensemble (tdpd_create_batch).  Each box has
   its own geometry and noise key; the random-number counter uses box-local
   gids, so a box gives the same trajectory alone and in a batch. */
typedef struct {
  float box[3];      /* box lengths */
  uint64_t seed;     /* Philox key */
  uint32_t box_id;   /* part of the Philox counter, < 2^24 */
  float shear_rate;  /* Lees-Edwards shear rate, as tdpd_params.shear_rate */
} tdpd_box;

typedef struct tdpd_sys tdpd_sys;
typedef void *(*tdpd_alloc_fn)(size_t bytes, void *user); /* returns device memory or NULL */
typedef void (*tdpd_free_fn)(void *ptr, void *user);

/* Create a system.  p is copied.  hip_stream may be NULL (default stream).
   alloc/free may both be NULL (hipMalloc/hipFree).  Checks: cutoffs > 0,
   n_types/n_species in range, sigma^2 = 2 kT gamma within 1e-4 relative
   (Eq. 6), at least 3 cells of edge > max(rc, rcc) per axis. */
int tdpd_create(const tdpd_params *p, void *hip_stream, tdpd_alloc_fn alloc,
                tdpd_free_fn free_fn, void *user, tdpd_sys **out);

/* Create a batch of n_boxes (1..1024) independent periodic boxes sharing
   every parameter of p except box, seed and box_id, which come from boxes[].
   Every phase of a step is one launch over all boxes (and one captured graph
   per step).  Fills the state with tdpd_set_state_boxes. */
int tdpd_create_batch(const tdpd_params *p, int32_t n_boxes, const tdpd_box *boxes,
                      void *hip_stream, tdpd_alloc_fn alloc, tdpd_free_fn free_fn, void *user,
                      tdpd_sys **out);

/* Set the state of every box: box b owns the next box_count[b] particles of
   the concatenated arrays (gids are global, box-major); positions are in
   that box's coordinates.  Same layout and effects as tdpd_set_state. */
int tdpd_set_state_boxes(tdpd_sys *s, const int64_t *box_count, const float *pos, const float *vel,
                         const float *conc, const uint32_t *flags);

/* Set the whole particle state of a one-box system (Section 2.1: each
   particle carries a position and a velocity, Eqs. (1)-(2), and one
   concentration per species, Eq. (7)): n particles, pos [n][3] (wrapped
   into the box by the library), vel [n][3], conc [n][n_species], flags [n]
   (type, frozen bit).  All host pointers, copied before the call returns.
   Resets the step counter to 0 and drops membranes added before.
   TDPD_ERR_INVALID_ARG for n < 0, a NULL array with n > 0 or a bad flags
   word; TDPD_ERR_NONFINITE for a non-finite value; TDPD_ERR_STATE on a
   batch (which takes tdpd_set_state_boxes). */
int tdpd_set_state(tdpd_sys *s, int64_t n, const float *pos, const float *vel,
                   const float *conc, const uint32_t *flags);

/* Register a membrane mesh: nv vertices of its rest shape ref_xyz [nv][3]
   (FP64, unwrapped), ntri triangles tri [ntri][3] ordered counter-clockwise
   seen from outside, forming a closed connected surface.  Rest quantities
   come from ref_xyz (Section 2.2): per-bond l0, l_m = l0/x0, k_p cancelling
   the WLC force at l0; per-triangle A_{0,j}; A_0 = sum; V_0 = rest volume;
   theta0 as given or the mean rest dihedral. */
int tdpd_add_mesh(tdpd_sys *s, int32_t nv, const double *ref_xyz, int32_t ntri,
                  const int32_t *tri, const tdpd_mesh_params *mp, int32_t *mesh_id);

/* Bind particles [first_gid, first_gid + nv) to one red cell of mesh
   mesh_id (Section 2.2: the membrane vertices are particles of the fluid
   that also carry the membrane forces of Eqs. (13)-(19); Section 3.3)
   (vertex v is particle first_gid + v; all in one box, whose half length
   must exceed 1.25 times the cell's radius plus 1).  Pair forces between
   vertices of the same cell are left to the bonded terms; fluxes act
   between all pairs.  Writes the cell's index to *rbc_id.  Call after
   set_state and before stepping (TDPD_ERR_STATE otherwise).
   TDPD_ERR_INVALID_ARG for an unknown mesh, a gid range outside the state
   or across two boxes, or a particle already bound or frozen;
   TDPD_ERR_UNSUPPORTED for too many cells or a cell too large for its
   box. */
int tdpd_add_rbc(tdpd_sys *s, int32_t mesh_id, int64_t first_gid, int32_t *rbc_id);

/* Evaluate F and Q at the current state with random-number step counter k,
   treating the stored velocities and concentrations as the ones the
   dissipative force and fluxes see.  Asynchronous. */
int tdpd_compute_forces(tdpd_sys *s, uint32_t k);

/* Advance n_steps steps of Eqs. (1), (2) and (7) (positions, velocities,
   concentrations) with velocity Verlet, the forces of Eqs. (3)-(6) and
   (13)-(19) and the fluxes of Eqs. (7)-(10) evaluated once per step; step
   n draws random numbers with counter k = n.  The first call after
   set_state evaluates the forces at k = 0 first.  Asynchronous: errors
   found by kernels surface at the next tdpd_sync or tdpd_get_*.
   TDPD_ERR_INVALID_ARG for n_steps < 0, TDPD_ERR_STATE before set_state,
   TDPD_ERR_UNSUPPORTED once the 32-bit step counter would wrap. */
int tdpd_step(tdpd_sys *s, int32_t n_steps);

/* Wait for the stream, then read and clear the device error word. */
int tdpd_sync(tdpd_sys *s);

/* Copy the state of Eqs. (1), (2) and (7) to host buffers in gid order:
   pos [n][3] (in the box), vel [n][3], conc [n][n_species]; any pointer
   may be NULL.  Waits for the stream; returns a kernel error found since
   the last sync. */
int tdpd_get_state(tdpd_sys *s, float *pos, float *vel, float *conc);
/* Last evaluated forces [n][3] and concentration rates [n][n_species]. */
int tdpd_get_forces(tdpd_sys *s, float *F, float *Q);

/* The neighbour pairs of the pair terms (Section 3.1: particles binned into
   cells of edge >= the cutoff, pairs found over the 27 surrounding cells;
   the distance test is the FP32 rule 0 < d^2 < fl(rcut^2) on the nearest
   periodic or sheared image) at the current positions.
   which = 0 (rcut = rc) or 1 (rcut = rcc): unordered pairs {gid_i < gid_j},
   enumerated by the one-thread-per-particle kernel's cell search (with
   Verlet lists on: from the lists).
   which = 2 (rc) or 3 (rcc): ordered pairs (home gid, partner gid) of every
   mobile home, both orientations, as the default tiled pair kernel's
   candidate path finds them at the current tile shape (stencil filter,
   periodic and sheared lifts included); TDPD_ERR_STATE with Verlet lists.
   Writes up to cap pairs to ij [cap][2] in no particular order and the total
   to *n_out; TDPD_ERR_CAPACITY if n_out > cap. */
int tdpd_get_pairs(tdpd_sys *s, int32_t which, int64_t cap, int32_t *ij, int64_t *n_out);

/* FP64 diagnostics of the conserved and controlled quantities: out[0..2]
   total momentum of mobile particles (conserved by the pair forces,
   Section 2.1), out[3] kT = sum |v - vbar|^2 / (3 (N_mobile - 1)) (the
   temperature of Eq. (6)), out[4..4+S) total concentration per species
   (conserved by the fluxes of Eqs. (8)-(10)), then per cell the total area
   and volume (A^t, V^t) of Eqs. (17)-(18).  cap = doubles available in the
   host buffer out (TDPD_ERR_CAPACITY if short).  Evaluates the forces
   first if the state has none yet; waits for the stream. */
int tdpd_diagnostics(tdpd_sys *s, double *out, int64_t cap);

/* The same diagnostics for callers that cannot allocate: code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc.  It makes no
   allocation of any kind and does not wait: it enqueues on the system's
   stream, writing the same 4 + S + 2 x cells doubles as tdpd_diagnostics
   (the same bits) to out_dev, a device buffer owned by the caller, valid once
   the stream reaches that point.  The workgroup partial sums live in a
   library-wide device scratch of 1.38 MB per GPU (held until the process
   ends), which limits the system to at most 8,388,608 particles
   (TDPD_ERR_CAPACITY beyond).  Needs an evaluated state (tdpd_compute_forces
   or tdpd_step before; else TDPD_ERR_STATE): it never evaluates forces
   itself.  Every call on a GPU shares that GPU's scratch, so calls that
   overlap on one GPU (systems on different streams) race; calls on one
   stream are ordered.  TDPD_ERR_HIP if the scratch could not be located at
   tdpd_create. */
int tdpd_diagnostics_noalloc(tdpd_sys *s, double *out_dev, int64_t cap);

/* Kernel timing with HIP events recorded on the system's stream around each
   phase of a force evaluation.  mask bits: TDPD_PHASE_* (0 disables).
   tdpd_get_timing waits for the stream, returns the summed duration in ms
   and the launch count of one phase since the last call, and resets it. */
#define TDPD_PHASE_PAIR 1      /* pair force + flux kernel */
#define TDPD_PHASE_BIN 2       /* kick/drift/key + radix sort + cell bounds + reorder */
#define TDPD_PHASE_MEMBRANE 4  /* K-Gather + membrane forces */
#define TDPD_PHASE_KICK 8      /* second half kick */
int tdpd_set_timing(tdpd_sys *s, int32_t mask);
int tdpd_get_timing(tdpd_sys *s, int32_t phase, double *total_ms, int64_t *launches);

/* Checkpoint and resume.  The paper's method is an explicit time
   integration (Eqs. 1-2 and 7 advanced by velocity Verlet), so the whole
   state of a run is the particle state in the library's internal (cell)
   order, the last forces and rates, the step counter that keys the random
   numbers, and the per-cell centroids of the volume sums (Eq. 18).
   tdpd_save waits for the stream and writes these to `path` (binary,
   little-endian, with a fingerprint of parameters, boxes, particle count,
   meshes and cells).  tdpd_load reads such a file into a system built the
   same way (same params, boxes, set_state sizes, meshes and cells; the
   particle values given to set_state are replaced).  A run resumed from a
   checkpoint continues bit for bit as the uninterrupted run.
   Errors: TDPD_ERR_IO if the file cannot be opened, is truncated or its
   fingerprint differs; TDPD_ERR_STATE before set_state. */
int tdpd_save(tdpd_sys *s, const char *path);
int tdpd_load(tdpd_sys *s, const char *path);

/* Tile shape of the cell-tiled pair kernel: wavefronts per workgroup (2 or
   4), 64-candidate chunks per wavefront held in registers (1-4), workgroups
   per cell (1-4), and filter (1: candidates of the 27-cell stencil farther
   than max(r_c, r_cc) from the home cell's box are dropped before the pair
   tests, for stencils of up to 768 candidates; 0: the whole stencil is
   tested).  Every shape gives a valid result; summation order, and so the
   last bits, depend on the shape, and results are bit-for-bit reproducible
   for a fixed shape.  tdpd_autotune times every built shape on
   the system's current state (reps launches each, HIP events on the
   system's stream), keeps the fastest and re-evaluates the forces with it.
   With cache_path (may be NULL) it first looks for a line written for the
   same device and workload signature (particle, species, box, cell and RBC
   counts, term mask, in-place or queued flux) and uses it without timing;
   otherwise it appends the result.  *best_ms (may be NULL) gets the chosen
   shape's time, 0 when the tiled kernel is not used (the simple kernel
   selected, or 2^26 particles or more).  One to four species without the
   random flux evaluate the flux in place on every candidate lane; the
   random flux (m_s > 0) and five or more species take the queued-flux
   build, in which the flux pairs are compacted into an LDS queue first;
   both are built in every shape, and both give results within rounding of
   each other.
   tdpd_set_tile returns TDPD_ERR_UNSUPPORTED for a shape that is not built.
   These calls are not part of the paper's method: they choose among
   equivalent evaluation orders of Eqs. (2)-(10). */
int tdpd_autotune(tdpd_sys *s, const char *cache_path, int32_t reps, double *best_ms);
int tdpd_set_tile(tdpd_sys *s, int32_t waves, int32_t chunks, int32_t split, int32_t filter);
int tdpd_get_tile(const tdpd_sys *s, int32_t *waves, int32_t *chunks, int32_t *split,
                  int32_t *filter);

/* ---------------------------------------------------------------------
   Verlet neighbour lists (Section 3.1: the paper's GPU code keeps
   per-particle neighbour lists in a locally transposed layout; Section
   5.2: its benchmarks refresh them every 5 steps).  With every > 0 and skin > 0, each particle
   keeps the list of every other particle closer than max(r_c, r_cc) + skin;
   the lists are rebuilt, together with the cell binning, on every
   every-th force evaluation (the first evaluation after set_state or
   load without stored lists always rebuilds), and the other evaluations
   test only the list entries with the same FP32 pair rule as the cell
   path, so the pair set of every step is the same as the cell path's as
   long as no particle moves more than skin / 2 between rebuilds.  That is
   checked every step: a larger displacement, or a particle with more
   than capacity list entries, makes the next tdpd_sync (and every call
   that syncs) return TDPD_ERR_LIST; the forces of that step are then
   not to be trusted.  A given capacity is rounded up to a multiple of 8 and
   split evenly over the 8 sub-lists a particle's neighbours are dealt
   into (4 sub-lists from 131,072 particles on; the error is raised when
   one of them is full); capacity 0 picks
   three times the mean count at the nominal density rho plus 128, rounded
   up to a multiple of 32 (at most 4096).  Cells are made at least
   max(r_c, r_cc) + skin wide (TDPD_ERR_BOX_TOO_SMALL under 3 per side).
   Call after tdpd_create or tdpd_set_state and before the first step or
   force evaluation of that state (TDPD_ERR_STATE otherwise); skin 0 or
   every 0 switches back to per-step cells.  Not with Lees-Edwards boxes or
   the random flux (TDPD_ERR_UNSUPPORTED).  Device memory: at most 4 * capacity +
   96 bytes per particle.  Results differ from the cell path's only in
   summation order; tdpd_get_pairs then lists pairs from the lists, and
   checkpoints hold the lists, so a resumed run is bit-for-bit the
   uninterrupted one. */
int tdpd_set_verlet(tdpd_sys *s, float skin, int32_t every, int32_t capacity);
int tdpd_get_verlet(const tdpd_sys *s, float *skin, int32_t *every, int32_t *capacity);

/* ---------------------------------------------------------------------
   Membrane surrogate.  Not part of the paper's method: a learned stand-in
   for the bending force (Eq. 19) plus the local-area force (Eq. 17, k_l
   term) of a membrane vertex, with the plain forces as check and fallback.

   Network: 20 inputs -> 128 -> 128 -> 128 (SiLU after each) -> 3, on the
   matrix cores in bfloat16 with FP32 accumulation (weights, inputs and
   hidden activations rounded to bfloat16 where they enter a product).
   Parameters are TDPD_MLP_PARAMS floats, layer by layer [W1 (128 x 20, row
   = output unit), b1, W2 (128 x 128), b2, W3, b3, W4 (3 x 128), b4].

   Inputs of vertex v: the vectors to its 1-ring neighbours (counter-
   clockwise seen from outside, starting at the smallest mesh index) in the
   local frame (e1 = first ring vector projected on the tangent plane,
   e2 = n x e1, n = normalised sum of consecutive ring cross products),
   divided by the mesh's mean rest edge length, six slots (slot 6 zero for a
   degree-5 vertex), then 100 (A - A0)/A0 and 100 (V - V0)/V0 of its cell
   from the previous force evaluation.  Output y in the local frame; force =
   force_scale (y1 e1 + y2 e2 + y3 n).  Vertices of degree other than 5 or 6
   always use the plain forces. */
#define TDPD_MLP_PARAMS 36099
typedef struct tdpd_mlp tdpd_mlp;
/* Network with parameters and Adam moments on the device (caller's allocator
   as for tdpd_create; hip_stream borrowed).  Parameters start undefined. */
int tdpd_mlp_create(void *hip_stream, tdpd_alloc_fn alloc, tdpd_free_fn free_fn, void *user,
                    tdpd_mlp **out);
int64_t tdpd_mlp_num_params(void);
/* Copy TDPD_MLP_PARAMS host floats in (and reset the Adam moments) / out.
   TDPD_ERR_INVALID_ARG for a non-finite value. */
int tdpd_mlp_set_params(tdpd_mlp *m, const float *params);
int tdpd_mlp_get_params(tdpd_mlp *m, float *params);
/* Y [n][3] = network(X [n][20]); host buffers.  One fused kernel: weights
   resident in LDS as bfloat16, activations kept on chip, gfx950's
   16x16x32 bfloat16 matrix cores. */
int tdpd_mlp_forward(tdpd_mlp *m, const float *X, int64_t n, float *Y);
/* Parity/debug: the same forward pass, also returning the three hidden
   layers' FP32 activations before their bfloat16 rounding, H [3][n][128]
   (host buffer, caller-owned). */
int tdpd_mlp_forward_hidden(tdpd_mlp *m, const float *X, int64_t n, float *Y, float *H);
/* Mean over rows and outputs of (y - T/target_scale)^2 and its gradient
   with respect to the parameters (TDPD_MLP_PARAMS floats, may be NULL). */
int tdpd_mlp_loss_grad(tdpd_mlp *m, const float *X, const float *T, int64_t n,
                       float target_scale, double *loss, float *grad);
/* steps Adam updates (lr, beta1 0.9, beta2 0.999, eps 1e-8; moments kept
   across calls) on consecutive full batches of `batch` rows of the data set
   (taken in order, cycling; the caller shuffles), the loss of each batch
   before its update in loss_out [steps] (may be NULL).  The data set is
   copied to the device for the call.  Needs n >= batch. */
int tdpd_mlp_train(tdpd_mlp *m, const float *X, const float *T, int64_t n, float target_scale,
                   int32_t batch, int32_t steps, float lr, double *loss_out);
const char *tdpd_mlp_last_error(const tdpd_mlp *m);
void tdpd_mlp_destroy(tdpd_mlp *m);

/* Training samples of every membrane vertex at the current state: inputs X
   [n_vertices][20], the plain bending + local-area force in the vertex's
   local frame T [n_vertices][3] (not scaled), and whether the vertex may use
   the network ok [n_vertices] (any pointer may be NULL).  Vertices in the
   order of tdpd_add_rbc calls.  TDPD_ERR_STATE without cells. */
int tdpd_surrogate_sample(tdpd_sys *s, float *X, float *T, uint8_t *ok);
/* From now on the bending + local-area force of a vertex comes from a copy
   of the network's current parameters, except where the last check found
   |F_net - F_plain| > tol x (RMS of |F_plain| over the vertex's cell) or the
   vertex's degree is not 5 or 6.  Checks run at steps k with k %
   check_every == 0 (the set-up pass is k = 0).  Forces are re-evaluated at
   the current state.  */
int tdpd_surrogate_enable(tdpd_sys *s, const tdpd_mlp *mlp, float force_scale, float tol,
                          int32_t check_every);
int tdpd_surrogate_disable(tdpd_sys *s);
/* Of the last check: out[0] fraction of vertices on the network, out[1]
   max and out[2] mean relative error over vertices that may use it, out[3]
   fraction of vertices that may use it. */
int tdpd_surrogate_stats(tdpd_sys *s, double *out);

int64_t tdpd_num_particles(const tdpd_sys *s);
int32_t tdpd_num_boxes(const tdpd_sys *s);
int64_t tdpd_step_counter(const tdpd_sys *s);
/* Number of coincident particle pairs (d^2 == 0) met since set_state. */
int64_t tdpd_coincident_pairs(tdpd_sys *s);
const char *tdpd_last_error(const tdpd_sys *s);
void tdpd_destroy(tdpd_sys *s);

#ifdef __cplusplus
}
#endif
#endif /* TDPD_H */
