// k_mech.hip -- mechanical step on gfx950: 27-box gather, sphere-sphere force, adherence gate,
// clamp and synchronous integration in one kernel (paper Sec. 2.1 "calculate mechanical forces"
// agent operation; Zubler & Douglas force model shared with Cortex3D, Sec. 3.4).
//
// One lane per agent in box-sorted order.  The 27 neighbour boxes are walked as 9 contiguous
// key runs (dz, dy in {-1, 0, 1}; dx = -1..+1 adjacent in key space because x varies fastest),
// so candidates arrive in ascending (key, id) order -- the canonical summation order -- and each
// run costs two start[] reads.  Neighbour records are packed double4 (x, y, z, d), one 32-byte
// load per candidate.  A conservative squared-distance prefilter skips the sqrt of candidates
// that cannot touch; every surviving pair is evaluated exactly as the definition spells it.
#include "kernels.hpp"

namespace bdm {

// Accept when a contact is still possible: a contact needs |x_i - x_j| < r_i + r_j, i.e.
// d2 < (r_i + r_j)^2 in exact arithmetic, and a 1e-4 relative margin covers every rounding of
// both the binary64 and the binary32 evaluation of the test.
__device__ __forceinline__ bool maybe_touch(double d2, double s) { return d2 < s * s * 1.0001; }

template <bool F32>
__device__ __forceinline__ void pair_force(const double4 &p, double ri, float rif, const double4 &q,
                                           const MechArgs &a, double &fx, double &fy, double &fz) {
    const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
    const double rj = 0.5 * q.w;
    const double s = ri + rj;
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    if (!maybe_touch(d2, s)) return;
    if constexpr (!F32) {
        const double dist = __builtin_sqrt(d2);
        const double delta = s - dist;
        if (!(delta > 0.0) || dist == 0.0) return;
        const double rhat = (ri * rj) / s;
        const double F = a.k * delta - a.gamma * __builtin_sqrt(rhat * delta);
        const double sc = F / dist;
        fx = fx + sc * dx;
        fy = fy + sc * dy;
        fz = fz + sc * dz;
    } else {
        const float dxf = float(dx), dyf = float(dy), dzf = float(dz);
        const float dist = __builtin_sqrtf((dxf * dxf + dyf * dyf) + dzf * dzf);
        const float rjf = float(rj);
        const float sf = rif + rjf;
        const float delta = sf - dist;
        if (!(delta > 0.0f) || dist == 0.0f) return;
        const float rhat = (rif * rjf) / sf;
        const float F = a.kf * delta - a.gf * __builtin_sqrtf(rhat * delta);
        const float sc = F / dist;
        fx = fx + double(sc * dxf);
        fy = fy + double(sc * dyf);
        fz = fz + double(sc * dzf);
    }
}

template <bool F32>
__global__ __launch_bounds__(kBlock) void k_mech(const GridDev *__restrict__ g,
                                                 const double4 *__restrict__ pos4,
                                                 const double *__restrict__ adh_s,
                                                 const uint32_t *__restrict__ id_s,
                                                 const uint8_t *__restrict__ state_s,
                                                 const uint32_t *__restrict__ start, MechArgs a,
                                                 bdm_soa out) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!g->valid || s >= g->n || s >= out.capacity) return;
    const double b = g->b;
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    const double4 p = pos4[s];
    const int cx = box_coord(p.x, b, g->cmin[0], nx, false);
    const int cy = box_coord(p.y, b, g->cmin[1], ny, false);
    const int cz = box_coord(p.z, b, g->cmin[2], nz, false);
    const double ri = 0.5 * p.w;
    const float rif = float(ri);
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < nx - 1 ? cx + 1 : nx - 1;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int oz = -1; oz <= 1; ++oz) {
        const int zz = cz + oz;
        if (zz < 0 || zz >= nz) continue;
        for (int oy = -1; oy <= 1; ++oy) {
            const int yy = cy + oy;
            if (yy < 0 || yy >= ny) continue;
            const uint32_t kb = uint32_t(x0) + uint32_t(nx) * (uint32_t(yy) + uint32_t(ny) * uint32_t(zz));
            const uint32_t j0 = start[kb], j1 = start[kb + uint32_t(x1 - x0) + 1u];
            for (uint32_t j = j0; j < j1; ++j) {
                if (j == uint32_t(s)) continue;
                pair_force<F32>(p, ri, rif, pos4[j], a, fx, fy, fz);
            }
        }
    }
    // adherence gate, clamp, integrate (binary64)
    const double adh = adh_s[s];
    double nxp = p.x, nyp = p.y, nzp = p.z;
    const double fn = __builtin_sqrt((fx * fx + fy * fy) + fz * fz);
    if (!(fn < adh)) {
        double ux = a.dt * fx, uy = a.dt * fy, uz = a.dt * fz;
        const double len = __builtin_sqrt((ux * ux + uy * uy) + uz * uz);
        if (len > a.max_disp) {
            const double sc = a.max_disp / len;
            ux = ux * sc;
            uy = uy * sc;
            uz = uz * sc;
        }
        nxp = p.x + ux;
        nyp = p.y + uy;
        nzp = p.z + uz;
    }
    out.x[s] = nxp;
    out.y[s] = nyp;
    out.z[s] = nzp;
    out.diam[s] = p.w;
    out.adh[s] = adh;
    out.id[s] = id_s[s];
    if (out.state) out.state[s] = state_s[s];
    if (out.fx) out.fx[s] = fx;
    if (out.fy) out.fy[s] = fy;
    if (out.fz) out.fz[s] = fz;
}

// Test hook: contact lists per sorted slot in force-sum order (mechanical contact).
__global__ __launch_bounds__(kBlock) void k_contacts_mech(const GridDev *__restrict__ g,
                                                          const double4 *__restrict__ pos4,
                                                          const uint32_t *__restrict__ id_s,
                                                          const uint32_t *__restrict__ start,
                                                          int f32, uint32_t *counts,
                                                          const int64_t *offsets, uint32_t *ids) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!g->valid || s >= g->n) return;
    const double b = g->b;
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    const double4 p = pos4[s];
    const int cx = box_coord(p.x, b, g->cmin[0], nx, false);
    const int cy = box_coord(p.y, b, g->cmin[1], ny, false);
    const int cz = box_coord(p.z, b, g->cmin[2], nz, false);
    const double ri = 0.5 * p.w;
    const float rif = float(ri);
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < nx - 1 ? cx + 1 : nx - 1;
    uint32_t c = 0;
    for (int oz = -1; oz <= 1; ++oz) {
        const int zz = cz + oz;
        if (zz < 0 || zz >= nz) continue;
        for (int oy = -1; oy <= 1; ++oy) {
            const int yy = cy + oy;
            if (yy < 0 || yy >= ny) continue;
            const uint32_t kb = uint32_t(x0) + uint32_t(nx) * (uint32_t(yy) + uint32_t(ny) * uint32_t(zz));
            const uint32_t j0 = start[kb], j1 = start[kb + uint32_t(x1 - x0) + 1u];
            for (uint32_t j = j0; j < j1; ++j) {
                if (j == uint32_t(s)) continue;
                const double4 q = pos4[j];
                const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
                const double rj = 0.5 * q.w;
                bool hit;
                if (!f32) {
                    hit = ((ri + rj) - __builtin_sqrt((dx * dx + dy * dy) + dz * dz)) > 0.0;
                } else {
                    const float dxf = float(dx), dyf = float(dy), dzf = float(dz);
                    hit = ((rif + float(rj)) - __builtin_sqrtf((dxf * dxf + dyf * dyf) + dzf * dzf)) > 0.0f;
                }
                if (hit) {
                    if (ids) ids[offsets[s] + c] = id_s[j];
                    ++c;
                }
            }
        }
    }
    counts[s] = c;
}

void launch_mech(const bdm_soa &s, const MechArgs &a, int force_bits, const Ws &w, hipStream_t st) {
    int64_t nb = (s.capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    if (force_bits == 32)
        hipLaunchKernelGGL(k_mech<true>, dim3(unsigned(nb)), dim3(kBlock), 0, st, w.grid, w.pos4, w.adh,
                           w.ids, w.state, w.start, a, s);
    else
        hipLaunchKernelGGL(k_mech<false>, dim3(unsigned(nb)), dim3(kBlock), 0, st, w.grid, w.pos4, w.adh,
                           w.ids, w.state, w.start, a, s);
}

void launch_contacts_mech(int f32, const Ws &w, uint32_t *counts, const int64_t *offsets, uint32_t *ids,
                          hipStream_t st) {
    int64_t nb = (w.lay.capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_contacts_mech, dim3(unsigned(nb)), dim3(kBlock), 0, st, w.grid, w.pos4, w.ids,
                       w.start, f32, counts, offsets, ids);
}

}  // namespace bdm
