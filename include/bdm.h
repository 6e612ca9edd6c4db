/*
 * bdm.h -- C ABI of libbdm.so, the MI355X (gfx950) hot path of the BioDynaMo agent-based engine
 * (Breitwieser et al., arXiv 2006.06775): each timestep's mechanical interaction of spherical
 * agents -- a uniform-grid neighbour search followed by the sphere-sphere force and an
 * adherence-gated, clamped displacement -- plus the two workloads the paper runs on the same
 * grid (tumour-spheroid growth/division, SIR epidemiology) and a seeded generator.
 *
 * Conventions that hold for every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller, unless a parameter says
 *     "host".  The library never allocates device memory inside these calls, never frees and
 *     never creates streams.  `stream` is a hipStream_t (NULL = the default stream); every
 *     call is asynchronous on it unless it says "synchronises".
 *   - Arguments are validated synchronously on the host; a violation returns a negative
 *     BDM_E* code and launches nothing.  Conditions only the device can see (capacity or box
 *     overflow, non-finite data, box smaller than the largest agent) set sticky bits in the
 *     workspace that bdm_status() returns; a step that meets one leaves the agent state
 *     untouched.  No C++ exception crosses this boundary.
 *   - Agent state lives in structure-of-arrays form (bdm_soa).  After a grid build the library
 *     keeps agents in box-sorted order, lexicographic in (box key, agent id); every step writes
 *     its results back into the caller's arrays in that order.  id[] says which agent sits in
 *     each slot; bdm_read_agents() restores id order.
 *   - Floating point: binary64 without contraction, correctly rounded sqrt and division, so
 *     results are reproducible bit for bit from run to run.
 */
#ifndef BDM_H
#define BDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------------------------ */
#define BDM_OK 0
#define BDM_EINVAL (-1)   /* an argument is out of its documented range */
#define BDM_ENOWS (-2)    /* workspace missing, too small, or sized for smaller arrays */
#define BDM_EHIP (-3)     /* a HIP runtime call failed; bdm_last_error() has the text */
#define BDM_ENODEV (-4)   /* no usable gfx950 device */

/* ---- sticky device status bits (bdm_status) ---------------------------------------------- */
#define BDM_FLAG_CAPACITY 0x1u   /* a division found no free slot below capacity */
#define BDM_FLAG_BOXES 0x2u      /* the grid needed more than max_boxes boxes */
#define BDM_FLAG_NONFINITE 0x4u  /* a position or diameter was NaN/Inf, or too far out */
#define BDM_FLAG_BOXSMALL 0x8u   /* explicit box edge below the largest diameter */
#define BDM_FLAG_NOGRID 0x10u    /* a step ran without a valid grid of the same agents */
#define BDM_FLAG_SCAN 0x20u      /* a prefix-scan look-back exceeded its spin bound */
#define BDM_FLAG_BADCOUNT 0x40u  /* the live count was outside [0, capacity] */
#define BDM_FLAG_BADID 0x80u     /* an agent id was outside [0, n) where ids must be dense */

/* ---- models for bdm_sim_step ------------------------------------------------------------- */
#define BDM_MODEL_MECH 0      /* grid build + mechanical step (open space) */
#define BDM_MODEL_SPHEROID 1  /* growth + division, then grid build + mechanical step */
#define BDM_MODEL_SIR 2       /* periodic grid build + SIR infection/recovery/movement */
#define BDM_MODEL_ONCOLOGY 3  /* apoptosis, growth + division, Brownian migration, grid + mechanics */

/* ---- batched form ------------------------------------------------------------------------ */
#define BDM_MAX_SLOTS 4096      /* slots of one batch */
#define BDM_SLOT_ALIGN 1024     /* a slot's first agent index is a multiple of this */
#define BDM_BOX_ALIGN 64        /* a slot's first histogram entry is a multiple of this */

/* ---- generator kinds for bdm_generate ---------------------------------------------------- */
#define BDM_GEN_CUBE 0  /* uniform in [0, L)^3, diameter uniform in [dlo, dhi) */
#define BDM_GEN_BALL 1  /* uniform in the ball of radius L about the origin (rejection) */
#define BDM_GEN_SIR 2   /* points uniform in [0, L)^3, ids < n_infected infected */
#define BDM_GEN_SOMA 3  /* as CUBE, with cell type (state) = id mod 2 */

/* Agent state.  Every array has `capacity` elements; `n` points to the device-resident live
 * count (int64).  diam/adh may be NULL for point agents (SIR); fx/fy/fz may be NULL when the
 * forces are not wanted; state may be NULL except for SIR (0 = S, 1 = I, 2 = R), soma
 * clustering (cell type) and cylinders (1 = cylinder).  Where it is kept it travels with its
 * agent: through every sort, to a dividing cell's daughter and with an apoptosis survivor. */
typedef struct bdm_soa {
    int64_t capacity;
    int64_t *n;
    double *x, *y, *z;
    double *diam, *adh;
    double *fx, *fy, *fz;
    uint32_t *id;
    uint8_t *state;
} bdm_soa;

/* Parameters.  Fields a model does not use are ignored. */
typedef struct bdm_params {
    double k, gamma;       /* force F = k*delta - gamma*sqrt(rhat*delta) */
    double dt;             /* displacement = dt * F (> 0) */
    double max_disp;       /* displacement clamp length (> 0) */
    double box;            /* > 0: explicit box edge (>= largest diameter); <= 0: largest diameter */
    int32_t force_bits;    /* 64: binary64 pair force; 32: binary32 pair force, binary64 sums */
    int32_t periodic;      /* 1 only for SIR: periodic cube [0, L)^3 */
    double L;              /* periodic cube edge */
    double r_inf, p_inf, p_rec, walk;  /* SIR radius (inclusive), probabilities, step bound */
    double grow;           /* spheroid: diameter factor per step */
    double div_d;          /* spheroid: division threshold diameter */
    double half_cbrt;      /* spheroid: daughter diameter factor (cube root of 1/2) */
    uint64_t seed, salt;   /* Philox4x64-10 key */
    int32_t skip_static;   /* 1: skip agents in stationary regions (mechanical steps; see below) */
    double p_apo;          /* oncology: probability per step that a cell dies, in [0, 1] */
    double migrate;        /* oncology: bound of the Brownian displacement per axis and step (>= 0) */
    double diff_D;         /* substances: diffusion coefficient (>= 0; D*dt/h^2 <= 1/6) */
    double diff_decay;     /* substances: decay rate (>= 0; decay*dt <= 1) */
    double secrete;        /* soma clustering: quantity a cell adds to its substance per step */
    double chemo_speed;    /* soma clustering: chemotactic displacement per step (>= 0) */
} bdm_params;

/* Stationary regions [paper Sec. 2.3 (iv): detect stationary regions and skip their expensive
 * collision detection].  With skip_static = 1 a plain mechanical step (bdm_grid_build +
 * bdm_mech_step, or bdm_sim_step with BDM_MODEL_MECH) skips the neighbour walk of every agent
 * whose result is known to equal the previous step's: the previous step was also a skip_static
 * step of the same agents on the same workspace, the lattice (box edge, origin, dims) is
 * unchanged, the agent did not move in it, and no agent moved out of or into any box of its
 * neighbourhood that can hold a sphere touching it.  Such an agent keeps its previous force
 * (so it is gated again) and its position, bit for bit: results are identical with and without
 * skipping.  Precondition: between two skip_static steps the agents change only through the
 * library's mechanical steps (after bdm_generate or any other change, take one step with
 * skip_static = 0, or re-initialise the workspace).  The force law (k, gamma, force_bits) must
 * also be unchanged for an agent to be skipped; after a change every agent walks again.  When
 * the last step skipped every agent (so nothing moved), the step has nothing to change: with the
 * same live count, force law and requested box edge, its grid build and neighbour walk return at
 * once and the agents, forces and grid stay as they are (a mechanical step after such a build
 * that asks for another force law sets BDM_FLAG_NOGRID and moves nothing).  The batched and
 * spheroid steps ignore it. */

/* Seeded initial state. */
typedef struct bdm_gen {
    int32_t kind;          /* BDM_GEN_* */
    int64_t n;             /* agents to create (<= capacity) */
    double L;              /* cube edge, or ball radius */
    double dlo, dhi;       /* diameter range */
    double adh;            /* adherence of every agent */
    int64_t n_infected;    /* SIR: agents with id < n_infected start infected */
    uint64_t seed, salt;   /* Philox4x64-10 key */
} bdm_gen;

/* Caller-owned scratch memory sized by bdm_workspace_bytes for at most `capacity` agents and
 * `max_boxes` grid boxes.  It also holds the sorted copies, the grid and the status bits, so
 * one workspace serves one population at a time. */
typedef struct bdm_workspace {
    void *ptr;             /* device, 256-byte aligned */
    size_t bytes;
    int64_t capacity;
    int64_t max_boxes;
} bdm_workspace;

/* Read-back of the device-resident grid description (bdm_grid_info). */
typedef struct bdm_grid_desc {
    double b;              /* box edge */
    int32_t cmin[3];       /* lattice coordinate of box 0 (open space) */
    int32_t dims[3];       /* boxes per axis */
    int64_t nboxes;
    int64_t n;             /* agents binned */
    int32_t valid;         /* 1 when the last build succeeded */
    uint32_t flags;        /* sticky BDM_FLAG_* bits */
    int64_t skipped;       /* agents whose walk the last skip_static mechanical step skipped */
} bdm_grid_desc;

/* A batch: many independent mechanical simulations packed into one population.  Slot s owns
 * the agent indices [agent_off, agent_off + capacity) of the packed arrays (agent_off a
 * multiple of BDM_SLOT_ALIGN) and the histogram entries [box_off, box_off + max_boxes) (box_off a
 * multiple of BDM_BOX_ALIGN: the grid build sorts boxes in buckets of 64); its live
 * count is soa->n[s] (soa->n points to `slots` int64 counts).  Each slot has its own grid, box
 * edge and parameters, so every agent's arithmetic is the same as in a plain call on that slot
 * alone.  The caller keeps slot ranges disjoint. */
typedef struct bdm_batch {
    void *ptr;             /* device workspace, 256-byte aligned */
    size_t bytes;
    int64_t capacity;      /* length of the packed agent arrays */
    int64_t max_boxes;     /* length of the packed histogram */
    int32_t slots;         /* number of slots (1..BDM_MAX_SLOTS) */
    int32_t grid_cap;      /* work split: workgroups the per-tile launches of bdm_batch_step deal
                              the packed tiles to, striding (0 = 8192; else 64..65536), or -1:
                              one workgroup per tile.  Results do not depend on it; keep it fixed
                              while a step is captured. */
} bdm_batch;

/* Size in bytes of the workspace for `capacity` agents and `max_boxes` boxes; 0 when either is
 * negative or the size overflows. */
size_t bdm_workspace_bytes(int64_t capacity, int64_t max_boxes);

/* Prepare a workspace for first use: clears counters, status bits and the box histogram.
 * Must precede every other call that takes `ws`.  Errors: BDM_ENOWS, BDM_EHIP. */
int bdm_workspace_init(const bdm_workspace *ws, void *stream);

/* Seeded generator of the initial state [paper Sec. 3.2 places cells in a ball; Sec. 3.3
 * distributes agents randomly in a cube].  Agent i (0 <= i < gen->n) takes Philox4x64-10 block
 * (counter (1 + attempt*2^8, i, 0, 0), key (seed, salt)); u = (word >> 11) * 2^-53.  CUBE:
 * x, y, z = L*u from words 0..2, diam = dlo + (dhi - dlo)*u(word 3).  BALL: attempt t gives
 * v = 2u - 1 per axis, accepted when |v|^2 <= 1, position L*v.  SIR: CUBE positions, state
 * 1 for id < n_infected else 0.  Writes arrays in id order (id[i] = i) and *soa->n = gen->n.
 * Errors: BDM_EINVAL (n > capacity, missing array). */
int bdm_generate(const bdm_soa *soa, const bdm_gen *gen, void *stream);

/* Uniform grid [paper Sec. 2.1: equal boxes, agents assigned by centre of mass, box edge from
 * the largest agent, neighbourhood = 27 boxes].  Box edge b = params->box or the largest
 * diameter; lattice c = floor(x / b) per axis, box 0 at the minimum c, key = cx + nx*(cy +
 * ny*cz); periodic (SIR): nb = floor(L / box) >= 3 boxes per axis, b = L / nb.  Builds the
 * histogram, its exclusive scan (start offsets) and the sorted copies of the agents in
 * (key, id) order inside the workspace.  Does not modify `soa`.  Errors: BDM_EINVAL, BDM_ENOWS;
 * device: BDM_FLAG_BOXES, BDM_FLAG_NONFINITE, BDM_FLAG_BOXSMALL. */
int bdm_grid_build(const bdm_soa *soa, const bdm_params *params, const bdm_workspace *ws,
                   void *stream);

/* Mechanical step on the grid of the last bdm_grid_build of the same agents [paper Sec. 2.1,
 * "calculate mechanical forces" agent operation; force model of Zubler & Douglas that Sec. 3.4
 * says BioDynaMo shares with Cortex3D].  For each agent i, over candidates j != i in the 27
 * boxes in ascending (key, id) order: delta = (d_i + d_j)/2 - |x_i - x_j|; when delta > 0,
 * F = k*delta - gamma*sqrt(rhat*delta) with rhat = r_i*r_j/(r_i + r_j), and F_i += (F/|.|) *
 * (x_i - x_j).  Then: |F_i| < adh_i -> no move; else disp = dt*F_i, clamped to length
 * max_disp; x_i += disp, synchronously for all agents.  Writes x, y, z, diam, adh, id (and
 * state) in box-sorted order and fx, fy, fz = the summed pre-gate forces.  Errors: BDM_EINVAL,
 * BDM_ENOWS; device: BDM_FLAG_NOGRID. */
int bdm_mech_step(const bdm_soa *soa, const bdm_params *params, const bdm_workspace *ws,
                  void *stream);

/* One full timestep of `model` at step index `step` (used as the Philox counter word 2):
 *   BDM_MODEL_MECH     bdm_grid_build + bdm_mech_step.
 *   BDM_MODEL_SPHEROID [paper Sec. 3.2] every diameter *= grow; each agent with diam >= div_d
 *                      divides: d' = diam*half_cbrt, axis u by rejection from Philox block
 *                      (5 + attempt*2^8, id, step, 0), mother at x - (d'/4)u, daughter at
 *                      x + (d'/4)u with id n + (rank of the mother among dividing mothers by
 *                      id) and the mother's adherence; divisions with no slot below capacity
 *                      are skipped and set BDM_FLAG_CAPACITY; then grid + mechanics.
 *   BDM_MODEL_ONCOLOGY [paper Sec. 3.2: growth, duplication, Brownian migration, apoptosis]
 *                      apoptosis: the cell with id i dies iff draw (6, i, step, 0) has word 0 <
 *                      floor(p_apo*2^64); the survivors are renumbered 0 .. n'-1 in their old id
 *                      order and packed into slots 0 .. n'-1 (slot = id); then growth and
 *                      division as BDM_MODEL_SPHEROID (with the new ids); then every cell moves
 *                      by migrate*(2u - 1) per axis, u from words 0..2 of draw (7, id, step, 0)
 *                      (open space); then grid + mechanics.  BDM_EINVAL for p_apo outside
 *                      [0, 1] or a negative or non-finite migrate.
 *   BDM_MODEL_SIR      [paper Sec. 3.3] on the periodic grid of positions at t: a susceptible
 *                      agent with m infected agents within r_inf (minimum image, inclusive)
 *                      becomes infected iff one of the draws (4 + c*2^8, id, step, 0), c < m,
 *                      has word 0 < floor(p_inf*2^64); an infected agent recovers iff draw
 *                      (3, id, step, 0) has word 0 < floor(p_rec*2^64); every agent moves by
 *                      walk*(2u - 1) per axis (words 0..2 of draw (2, id, step, 0)) and wraps
 *                      into [0, L).  S/I/R totals are kept for bdm_sir_counts.
 * Errors: as the underlying steps. */
int bdm_sim_step(const bdm_soa *soa, int32_t model, const bdm_params *params, int64_t step,
                 const bdm_workspace *ws, void *stream);

/* Copy agents from box-sorted slots into id order: out_*[id[s]] = soa->*[s] for s < n.  Any
 * out pointer may be NULL.  Each out array needs n elements.  Errors: BDM_EINVAL. */
int bdm_read_agents(const bdm_soa *soa, double *out_x, double *out_y, double *out_z,
                    double *out_diam, double *out_fx, double *out_fy, double *out_fz,
                    uint8_t *out_state, void *stream);

/* Spheroid diameter [paper Sec. 3.2: the diameter is derived from the volume of the convex hull
 * that encloses all cells].  These two calls do the O(n) part on the device; the host builds
 * the hull of the few agents they return.  Positions must be finite.
 *
 * bdm_extreme_points: for each direction k < ndir (dirs: device, row k = (ux, uy, uz), binary64),
 * out_slot[k] (device int32) = the smallest slot s < n maximising (ux*x[s] + uy*y[s]) + uz*z[s]
 * (binary64, no contraction).  work: device scratch of ndir uint64, overwritten.
 * 1 <= ndir <= BDM_HULL_MAX_DIRS.  With n = 0 every out_slot is 0x7fffffff.  Errors: BDM_EINVAL.
 *
 * bdm_hull_candidates: every slot s < n whose centre is not strictly inside all nplane
 * half-spaces, i.e. for which some plane k (planes: device, row k = (nx, ny, nz, c)) has
 * (nx*x[s] + ny*y[s]) + nz*z[s] + c >= -tol, is a candidate.  *out_count (device int64) = the
 * number of candidates; the first min(count, max_out) of them are written to out_slot (device
 * int32), in no particular order.  When the planes bound a polytope spanned by agents (faces
 * with outward normals, c the offset) and tol covers the rounding of the plane test, no agent
 * left out is a vertex of the agents' hull.  1 <= nplane <= BDM_HULL_MAX_PLANES, tol >= 0.
 * Errors: BDM_EINVAL. */
#define BDM_HULL_MAX_DIRS 256
#define BDM_HULL_MAX_PLANES 1024
int bdm_extreme_points(const bdm_soa *soa, const double *dirs, int32_t ndir, uint64_t *work,
                       int32_t *out_slot, void *stream);
int bdm_hull_candidates(const bdm_soa *soa, const double *planes, int32_t nplane, double tol,
                        int32_t *out_slot, int64_t max_out, int64_t *out_count, void *stream);

/* Extracellular substances [paper Sec. 2.1: the diffusion of extracellular substances is a
 * standalone operation run once per step; growth-factor secretion and chemotaxis are agent
 * behaviours] on a uniform voxel grid, and the soma-clustering model [the Sec. 3.4 benchmark:
 * two cell types, each secreting its own substance and moving up its gradient, so that cells of
 * one type gather].
 *
 * Voxel (i, j, k) covers [x0 + i*h, x0 + (i+1)*h) x ...; substance s's value at the voxel is
 * element s*V + i + nx*(j + ny*k), V = nx*ny*nz, binary64.  An agent belongs to the voxel
 * floor((x - x0)/h) per axis, clamped into the grid.  All arrays are caller-owned device memory;
 * c and c_next must not overlap. */
typedef struct bdm_field {
    int32_t nx, ny, nz;    /* voxels per axis, in [1, 2^20] (ny <= 1048560), nx*ny*nz <= 2^30 */
    double x0, y0, z0;     /* lower corner */
    double h;              /* voxel edge (> 0) */
    double *c;             /* 2*V values: both substances now */
    double *c_next;        /* 2*V values: receives the next step's values (the caller then swaps) */
    uint32_t *count;       /* 2*V secretion counters: zero between calls */
} bdm_field;

/* c = 0 and count = 0 (both substances).  Errors: BDM_EINVAL. */
int bdm_field_init(const bdm_field *field, void *stream);

/* One diffusion step of both substances, c -> c_next: with lam = (diff_D*dt)/(h*h) and
 * kdec = diff_decay*dt (params->dt is the time step),
 *   c_next = c + (lam*L - kdec*c),  L = ((dx- + dx+) + (dy- + dy+)) + (dz- + dz+),
 * d = neighbour - c; the boundary is closed (a neighbour outside the grid is the voxel itself).
 * BDM_EINVAL unless 0 <= lam <= 1/6 and 0 <= kdec <= 1 (the explicit step's stable range). */
int bdm_diffuse(const bdm_field *field, const bdm_params *params, void *stream);

/* One soma-clustering step.  soa->state holds each cell's type: types 0 and 1 secrete and follow
 * substances 0 and 1, other types are inert.
 *   1. secretion: each voxel's substance s grows by secrete*m, m = its cells of type s (in c);
 *   2. diffusion of both substances, c -> c_next, as bdm_diffuse;
 *   3. chemotaxis: a cell of type s at voxel (i, j, k) takes g = (c(i+1) - c(i-1), c(j+1) -
 *      c(j-1), c(k+1) - c(k-1)) of substance s in c_next (neighbours outside the grid are the
 *      voxel itself) and moves by (chemo_speed/|g|)*g, |g| = sqrt((gx*gx + gy*gy) + gz*gz); no
 *      move where g = 0;
 *   4. grid build + mechanical step, as BDM_MODEL_MECH (positions after chemotaxis).
 * After the call the substances are in field->c_next (and field->c holds the secreted values
 * before diffusion): swap the two pointers before the next step.  Errors: BDM_EINVAL, BDM_ENOWS;
 * device: as bdm_sim_step. */
int bdm_soma_step(const bdm_soa *soa, const bdm_params *params, const bdm_field *field,
                  const bdm_workspace *ws, void *stream);

/* Spheres and cylinders [paper Sec. 2.2: the neuroscience module's neurite elements are
 * cylinders, each a spring with a point mass at its distal end; Sec. 2.1: mechanical forces
 * between agents found in the 27 boxes].  An agent with state 1 is a cylinder whose position
 * (x, y, z) is its distal end q; its proximal end p and diameter dc are in the id-indexed arrays
 * below.  Every other state is a sphere of diameter diam.
 *
 * bdm_geom_step: one mechanical step of such a population.
 *   1. each cylinder's diam is set to its grid diameter 2|q - p| + dc (|v| = sqrt((vx*vx +
 *      vy*vy) + vz*vz)), the diameter of the sphere about q that holds the whole cylinder;
 *   2. grid build on x, y, z and diam, as bdm_grid_build (box = largest diam, or params->box);
 *   3. forces: for each pair in contact, the closest points of the two axes (a sphere's axis is
 *      its centre; segment p -> q parameters from the clamped stationary point of the squared
 *      distance, re-clamped; segments within about 1e-6 rad of parallel start from parameter 0;
 *      a segment of length 0 is its distal end) carry virtual spheres of the bodies' diameters,
 *      and the sphere law of bdm_mech_step acts between them (contact iff delta > 0); a
 *      cylinder's point mass takes the share s in [0, 1] of the force, s the position of its
 *      closest point along p -> q; forces are summed in ascending (key, id) candidate order;
 *   4. gate, clamp and synchronous move as bdm_mech_step; a cylinder moves its distal end (p and
 *      dc do not change).
 * Outputs as bdm_mech_step (box-sorted slots; fx, fy, fz = the summed forces on the point
 * masses); counts (device uint32 per box-sorted slot, may be NULL) = each agent's contacts.
 * params->force_bits must be 64.  Errors: BDM_EINVAL, BDM_ENOWS; device: as bdm_sim_step,
 * BDM_FLAG_BADID for a cylinder id >= capacity. */
typedef struct bdm_cylinders {
    double *px, *py, *pz;  /* device, soa->capacity entries indexed by agent id: proximal ends */
    double *dc;            /* device, indexed by agent id: cylinder diameters */
} bdm_cylinders;

int bdm_geom_step(const bdm_soa *soa, const bdm_cylinders *cyl, const bdm_params *params,
                  const bdm_workspace *ws, uint32_t *counts, void *stream);

/* Sticky status bits of the workspace into *flags (host); clears them when `clear` != 0.
 * Synchronises the stream.  Errors: BDM_ENOWS, BDM_EHIP. */
int bdm_status(const bdm_workspace *ws, uint32_t *flags, int32_t clear, void *stream);

/* S, I, R totals after the last SIR step into counts[3] (host).  Synchronises the stream. */
int bdm_sir_counts(const bdm_workspace *ws, int64_t *counts, void *stream);

/* Grid description of the last build into *desc (host).  Synchronises the stream. */
int bdm_grid_info(const bdm_workspace *ws, bdm_grid_desc *desc, void *stream);

/* Test hook: copies of the last grid build -- key[n] per agent in the input order of that
 * build, order[n] = agent ids in box-sorted order, start[nboxes + 1].  Any pointer may be NULL.
 * Synchronises the stream (it needs n and nboxes). */
int bdm_grid_export(const bdm_workspace *ws, uint32_t *key, uint32_t *order, uint32_t *start,
                    void *stream);

/* Test hook: contact lists of the last grid build, per box-sorted slot s, candidates in the
 * force-sum order.  Mechanical contact (delta > 0 with params->force_bits arithmetic) in open
 * space, or SIR contact (minimum-image squared distance <= r_inf^2, any state) when
 * params->periodic.  Call with ids == NULL to get counts[n]; then with offsets[n] (exclusive
 * prefix of counts, int64) and ids[sum(counts)] to get the agent ids.  Errors: BDM_EINVAL. */
int bdm_contacts(const bdm_workspace *ws, const bdm_params *params, uint32_t *counts,
                 const int64_t *offsets, uint32_t *ids, void *stream);

/* Test hook: bdm_sim_step of model BDM_MODEL_MECH, _SPHEROID or _ONCOLOGY (same arguments, same
 * results) through the traced instantiation of the same kernels, which also records the contact
 * decisions the step's own walk takes [paper Sec. 2.1: the neighbours found in the 27 boxes].
 * For each agent s in the step's output order (box-sorted slots), counts[s] = the number of
 * contacts whose terms the step added to F_s and hashes[s] = h over those contacts in the order
 * they were added, h = h*0x9E3779B1 + p + 1 (mod 2^32, from h = 0) with p the partner's
 * box-sorted position (the index into bdm_grid_export's order[]).  counts and hashes are device
 * arrays of soa->capacity elements; entries of slots >= n are not written.  Errors: as
 * bdm_sim_step; BDM_EINVAL for another model or a NULL counts/hashes. */
int bdm_sim_step_traced(const bdm_soa *soa, int32_t model, const bdm_params *params, int64_t step,
                        const bdm_workspace *ws, uint32_t *counts, uint32_t *hashes, void *stream);

/* For callers that cannot allocate device memory: code under stream or graph capture, tight
 * serving loops, harnesses that forbid allocation.  The same step as bdm_sim_step (any model,
 * same arguments, same results bit for bit) with the library's own static device array of
 * BDM_NOALLOC_SCRATCH_BYTES as the workspace, one copy per device that runs it, held until the
 * process ends; no memory is allocated or freed in the call.  soa->capacity and max_boxes (the
 * grid boxes the workspace must hold, as for bdm_workspace_bytes) must fit the array:
 * bdm_workspace_bytes(capacity, max_boxes) <= BDM_NOALLOC_SCRATCH_BYTES, else BDM_ENOWS
 * (synchronous, nothing launched).  The array is cleared at the start of every call, so nothing
 * carries over between calls (no grid for a later bdm_mech_step, no S/I/R counts to read).
 * flags (device, one uint32, may be NULL) receives the step's sticky status bits (BDM_FLAG_*)
 * when the step completes on the stream.  Calls on one device share its array: calls that
 * overlap in time on one device (other streams, other threads) race and are not allowed.
 * Errors: as bdm_sim_step; BDM_ENOWS as above; BDM_ENODEV, BDM_EHIP from the device lookup. */
#define BDM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int bdm_sim_step_noalloc(const bdm_soa *soa, int32_t model, const bdm_params *params, int64_t step,
                         int64_t max_boxes, uint32_t *flags, void *stream);

/* ---- batched form --------------------------------------------------------------------------
 * Callers: many independent simulations of uneven sizes stepped together (one launch per
 * phase for all of them, capturable in a graph).  The per-slot work is the plain mechanical
 * step (bdm_sim_step with BDM_MODEL_MECH) [paper Sec. 2.1 grid, Sec. 3.4 force model]. */

/* Workspace bytes of a batch; 0 when an argument is out of range. */
size_t bdm_batch_workspace_bytes(int64_t capacity, int64_t max_boxes, int32_t slots);

/* Prepare a batch workspace: every slot idle, histogram and grids cleared.  Errors: BDM_ENOWS,
 * BDM_EINVAL, BDM_EHIP, BDM_ENODEV. */
int bdm_batch_init(const bdm_batch *b, void *stream);

/* Make slot `slot` run `steps` mechanical steps of the agents in [agent_off, agent_off +
 * capacity) with its own histogram range and parameters (k, gamma, dt, max_disp, box,
 * force_bits).  Asynchronous on `stream` (kernel writes, no host copy), so it may sit between
 * graph replays.  The agents themselves are written by the caller (e.g. bdm_generate on a view
 * of the slot's range with n = &soa->n[slot]).  Errors: BDM_EINVAL (range, alignment, params). */
int bdm_batch_set_slot(const bdm_batch *b, int32_t slot, int64_t agent_off, int64_t capacity,
                       int64_t box_off, int64_t max_boxes, int64_t steps, const bdm_params *p,
                       void *stream);

/* Idle slot `slot` and detach its agent range [agent_off, agent_off + capacity) from it. */
int bdm_batch_clear_slot(const bdm_batch *b, int32_t slot, int64_t agent_off, int64_t capacity,
                         void *stream);

/* One mechanical step (grid build + mechanics) of every slot with steps left, then each of
 * those slots' step count drops by one.  Agents of slot s stay in its range, box-sorted.  Fixed
 * launch geometry: the same call sequence is replayable as a graph.  Device conditions set the
 * slot's status bits (bdm_batch_slot_status).  Errors: BDM_EINVAL, BDM_ENOWS. */
int bdm_batch_step(const bdm_soa *packed, const bdm_batch *b, void *stream);

/* Test hook: bdm_batch_step through the traced instantiation of its kernels (see
 * bdm_sim_step_traced); counts/hashes are indexed like the packed arrays (b->capacity
 * elements), positions p are box-sorted positions within the agent's own slot. */
int bdm_batch_step_traced(const bdm_soa *packed, const bdm_batch *b, uint32_t *counts, uint32_t *hashes,
                          void *stream);

/* Status bits and remaining steps of one slot (host).  Synchronises the stream. */
int bdm_batch_slot_status(const bdm_batch *b, int32_t slot, uint32_t *flags, int64_t *steps_left,
                          void *stream);

/* Test hook: element-wise IEEE operations as the kernels compute them, for bitwise checks
 * against the host: out_sqrt[i] = sqrt(a[i]), out_div[i] = a[i] / b[i] in binary64;
 * out_sqrtf[i] = sqrtf((float)a[i]), out_divf[i] = (float)a[i] / (float)b[i] in binary32. */
int bdm_fp_probe(const double *a, const double *b, int64_t n, double *out_sqrt, double *out_div,
                 float *out_sqrtf, float *out_divf, void *stream);

/* Text of a return code; bdm_last_error() gives the detail of the last failure on this
 * thread (empty when none). */
const char *bdm_strerror(int code);
const char *bdm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BDM_H */
