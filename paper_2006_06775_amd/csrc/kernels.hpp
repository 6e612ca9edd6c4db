// kernels.hpp -- argument records and host launchers of the gfx950 kernels (internal).
#pragma once

#include "common.hpp"

namespace bdm {

struct FinalizeArgs {
    double box;         // requested box edge (<= 0: largest diameter; periodic: the request)
    double L;           // periodic cube edge
    int32_t nb;         // periodic boxes per axis
    int32_t periodic;
    int32_t has_d;      // diameters present (spheres) or not (points)
    int64_t max_boxes;
};

struct SoaIn {
    const double *x, *y, *z, *d, *adh;
    const uint32_t *id;
    const uint8_t *state;
};

struct ReadOut {
    double *x, *y, *z, *d, *fx, *fy, *fz;
    uint8_t *state;
};

struct MechArgs {
    double k, gamma, dt, max_disp;
    float kf, gf;       // binary32 copies for the FP32 pair law
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

struct GenArgs {
    int32_t kind;
    int64_t n;
    double L, dlo, dhi, adh;
    int64_t n_infected;
    uint64_t seed, salt;
};

struct ContactArgs {
    int32_t mode;       // 0: mechanical FP64, 1: mechanical FP32, 2: periodic radius
    double L, half, r2;
};

void launch_grid_build(const bdm_soa &s, const FinalizeArgs &fa, const Ws &w, hipStream_t st);
void launch_scan(uint32_t *in, uint32_t *out, const int64_t *len_ptr, const int32_t *gate,
                 int64_t max_len, const Ws &w, int zero_in, bool prepare, hipStream_t st);
void launch_contacts_mech(int f32, const Ws &w, uint32_t *counts, const int64_t *offsets,
                          uint32_t *ids, hipStream_t st);
void launch_read_agents(const bdm_soa &s, const ReadOut &o, hipStream_t st);
void launch_mech(const bdm_soa &s, const MechArgs &a, int force_bits, const Ws &w, hipStream_t st);
void launch_contacts(const ContactArgs &a, const Ws &w, uint32_t *counts, const int64_t *offsets,
                     uint32_t *ids, hipStream_t st);
void launch_sir(const bdm_soa &s, const SirArgs &a, const Ws &w, hipStream_t st);
void launch_grow_divide(const bdm_soa &s, const DivArgs &a, const Ws &w, hipStream_t st);
void launch_generate(const bdm_soa &s, const GenArgs &a, hipStream_t st);
void launch_fp_probe(const double *a, const double *b, int64_t n, double *os, double *od, float *osf,
                     float *odf, hipStream_t st);
void launch_ws_init(const Ws &w, hipStream_t st);

}  // namespace bdm
