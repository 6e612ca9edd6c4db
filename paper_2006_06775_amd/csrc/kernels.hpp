// kernels.hpp -- argument records and host launchers of the gfx950 kernels (internal).
//
// Every launcher takes a `Slots` record (common.hpp): one slot by value for a plain call, or
// the batch's slot table and tile map.  Launch geometry covers `capacity` array entries in
// tiles of kBlock agents; tiles outside any slot, or beyond a slot's live count, exit at once.
#pragma once

#include "common.hpp"

namespace bdm {

struct SoaIn {
    const double *x, *y, *z, *d, *adh;
    const uint32_t *id;
    const uint8_t *state;
    const double *fx, *fy, *fz;  // the last step's forces (stationary skip only)
};

struct ReadOut {
    double *x, *y, *z, *d, *fx, *fy, *fz;
    uint8_t *state;
};

struct SirArgs {
    double L, half, r2, walk;
    Threshold tinf, trec;
    uint64_t seed, salt, step;
};

struct DivArgs {
    double grow, div_d, half_cbrt;
    uint64_t seed, salt, step;
};

struct ApoArgs {
    Threshold tapo;
    uint64_t seed, salt, step;
};

struct MigArgs {
    double walk;
    uint64_t seed, salt, step;
};

// A substance grid: nx*ny*nz voxels of edge h from (x0, y0, z0), V voxels per substance.
struct FieldDev {
    int32_t nx, ny, nz;
    double x0, y0, z0, h;
    int64_t V;
};

// Cylinder agents: proximal end and diameter by agent id.
struct CylIn {
    const double *px, *py, *pz, *dc;
};

struct GeomArgs {
    double k, gamma, dt, max_disp;
    int64_t capacity;  // entries of the cylinder arrays (ids beyond are rejected)
};

struct GenArgs {
    int32_t kind;
    int64_t n;
    double L, dlo, dhi, adh;
    int64_t n_infected;
    uint64_t seed, salt;
};

// Per-agent contact record of a traced mechanical step (test hook): count and order-sensitive
// hash of the contacts the step adds, indexed like the step's outputs.
struct TraceOut {
    uint32_t *counts, *hashes;
};

struct ContactArgs {
    int32_t mode;       // 0: mechanical FP64, 1: mechanical FP32, 2: periodic radius
    double L, half, r2;
};

// Workgroups of a per-tile launch (one per tile for a plain call, capped for a batch).
unsigned tile_grid(const Slots &sl, int64_t ntiles);
// Grid build (bounds, finalize, key/histogram, scan, scatter, canonical order) of every slot.
// f32_copy: also write the binary32 pre-test copies (read by the crowded mechanics kernel).
// allow_freeze: a plain skipping build may find that nothing changed since the last step and
// skip itself and its step whole (traced steps pass false: they record every contact).
void launch_grid_build(const bdm_soa &s, const Slots &sl, int64_t capacity, bool f32_copy, const Ws &w,
                       hipStream_t st, bool allow_freeze = true);
// Exclusive scan of in[0, len) into out[0, len] (len read on the device).
void launch_scan(uint32_t *in, uint32_t *out, const int64_t *len_ptr, int64_t max_len, const Ws &w,
                 int zero_in, bool prepare, hipStream_t st, bool build = false);
// trace: NULL for the step itself; else the traced instantiation of the same kernels.
void launch_mech(const bdm_soa &s, const Slots &sl, int64_t capacity, int precision, bool crowded, const Ws &w,
                 hipStream_t st, const TraceOut *trace = nullptr);
void launch_sir(const bdm_soa &s, const Slots &sl, int64_t capacity, const SirArgs &a, const Ws &w,
                hipStream_t st);
void launch_grow_divide(const bdm_soa &s, const Slots &sl, int64_t capacity, const DivArgs &a, const Ws &w,
                        hipStream_t st);
// Apoptosis: survivors compacted and renumbered 0 .. n'-1 in id order; n updated on the device.
void launch_apoptosis(const bdm_soa &s, int64_t capacity, const ApoArgs &a, const Ws &w, hipStream_t st);
// Brownian migration of every live agent.
void launch_migrate(const bdm_soa &s, int64_t capacity, const MigArgs &a, hipStream_t st);
// Spheroid-diameter observable: extreme agents per direction; agents outside a set of planes.
void launch_extreme_points(const bdm_soa &s, const double *dirs, int32_t ndir, unsigned long long *work,
                           int32_t *out_slot, hipStream_t st);
void launch_hull_keep(const bdm_soa &s, const double *planes, int32_t nplane, double tol, int32_t *out_slot,
                      int64_t max_out, int64_t *out_count, hipStream_t st);
// Substances: secretion into c (counters left at zero), one diffusion step of both substances
// cin -> cout, chemotaxis along c, zero fill of c and the counters.
void launch_secrete(const bdm_soa &s, int64_t capacity, const FieldDev &f, uint32_t *count, double *c, double q,
                    hipStream_t st);
void launch_diffuse(const FieldDev &f, const double *cin, double *cout, double lam, double kdec, hipStream_t st);
void launch_chemotaxis(const bdm_soa &s, int64_t capacity, const FieldDev &f, const double *c, double speed,
                       hipStream_t st);
void launch_field_fill(double *c, uint32_t *count, int64_t len, hipStream_t st);
// Spheres and cylinders: grid diameters of the cylinders; the mechanical step after a grid build.
void launch_geom_reach(const bdm_soa &s, int64_t capacity, const CylIn &cyl, hipStream_t st);
void launch_geom(const bdm_soa &s, const CylIn &cyl, const GeomArgs &a, const Ws &w, uint32_t *counts,
                 hipStream_t st);
void launch_batch_advance(const Ws &w, hipStream_t st);
void launch_set_slot(const Ws &w, int32_t slot, const SlotDev &rec, int64_t first_tile, int64_t ntile,
                     int32_t value, hipStream_t st);
void launch_contacts(const ContactArgs &a, const Slots &sl, const Ws &w, uint32_t *counts,
                     const int64_t *offsets, uint32_t *ids, hipStream_t st);
void launch_contacts_mech(int f32, const Slots &sl, const Ws &w, uint32_t *counts, const int64_t *offsets,
                          uint32_t *ids, hipStream_t st);
void launch_read_agents(const bdm_soa &s, const ReadOut &o, hipStream_t st);
void launch_generate(const bdm_soa &s, const GenArgs &a, hipStream_t st);
void launch_fp_probe(const double *a, const double *b, int64_t n, double *os, double *od, float *osf,
                     float *odf, hipStream_t st);
void launch_ws_init(const Ws &w, hipStream_t st);
void launch_copy_flags(const Ws &w, uint32_t *out, hipStream_t st);
void launch_mask_starts(uint32_t *p, int64_t n, hipStream_t st);

}  // namespace bdm
