// k_mech.hip -- mechanical step on gfx950: 27-box gather, sphere-sphere force, adherence gate,
// clamp and synchronous integration in one kernel (paper Sec. 2.1 "calculate mechanical forces"
// agent operation; Zubler & Douglas force model shared with Cortex3D, Sec. 3.4).
//
// One lane per agent in box-sorted order.  The 27 neighbour boxes are 9 contiguous key runs
// (dz, dy in {-1, 0, 1}; dx = -1..+1 adjacent in key space because x varies fastest), so
// candidates arrive in ascending (key, id) order -- the canonical summation order.
//
// The work is split in two so that the wavefront does not pay the expensive exact law for
// every candidate of every lane:
//   1. candidate stream: each lane walks its 9 runs as one flattened stream (run table in LDS)
//      and keeps the candidates that pass a cheap conservative squared-distance test in a small
//      per-lane queue in LDS;
//   2. exact pass: the queued candidates, still in canonical order, are re-read and evaluated
//      exactly as the definition spells the law (binary64 or binary32) and summed.
// The packed record holds (x, y, z, r) with r = d/2.
//
// Schedule: a tile is 256 consecutive sorted agents.  A plain call processes its tiles in the
// pencil order built with the grid (rows grouped 16 at a time and swept along z) and gives each
// XCD one contiguous part of that sequence, so the three z-planes a tile reads stay in that
// XCD's L2.  Outputs are written with non-temporal stores: they are not read again in the step.
#include "kernels.hpp"

namespace bdm {

constexpr int kQueue = 8;          // queued candidates per lane before an exact pass
constexpr int kQueueCrowded = 16;  // the same for crowded populations (tens of contacts per agent)

template <bool F32>
__device__ __forceinline__ void exact_pair(const double4 &p, const double4 &q, float rif, const SlotDev &a,
                                           double &fx, double &fy, double &fz) {
    const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
    const double ri = p.w, rj = q.w;
    if constexpr (!F32) {
        const double s = ri + rj;
        const double dist = __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
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

// The 9 key runs of the box (cx, cy, cz) as [lo, hi) ranges of sorted positions, the non-empty
// ones first in canonical order, then the empty ones, in column t; returns the candidate count.
__device__ __forceinline__ uint32_t load_runs(const GridDev *__restrict__ g, const uint32_t *__restrict__ start,
                                              int cx, int cy, int cz, uint2 (*s_run)[kBlock], int t) {
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < nx - 1 ? cx + 1 : nx - 1;
    uint32_t lo[9], hi[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const int zz = cz + r / 3 - 1, yy = cy + r % 3 - 1;
        lo[r] = 0;
        hi[r] = 0;
        if (zz >= 0 && zz < nz && yy >= 0 && yy < ny) {
            const uint32_t kb = uint32_t(x0) + uint32_t(nx) * (uint32_t(yy) + uint32_t(ny) * uint32_t(zz));
            lo[r] = start[kb];
            hi[r] = start[kb + uint32_t(x1 - x0) + 1u];
        }
    }
    uint32_t cnt = 0;
    int k = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r)
        if (hi[r] > lo[r]) {
            s_run[k++][t] = make_uint2(lo[r], hi[r]);
            cnt += hi[r] - lo[r];
        }
    for (int r = k; r < 9; ++r) s_run[r][t] = make_uint2(0u, 0u);  // empty runs after them
    return cnt;
}

// Packed-record loads: a raw buffer resource with 32-bit byte offsets when the sorted arrays
// are below 4 GiB (one shift per address, out-of-range offsets read zero), else global loads.
// operator() reads the binary64 record (x, y, z, r), f() its binary32 pre-test copy.
struct RecBuf {
    void *base, *basef;
    uint32_t bytes;  // of the binary64 records (the binary32 copy is half as long)
    __device__ __forceinline__ double4 operator()(uint32_t j) const {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, 0x00020000);
        const uint32_t off = j * 32u;
        const auto lo = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const auto hi = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
        const double2 a = __builtin_bit_cast(double2, lo), c = __builtin_bit_cast(double2, hi);
        return make_double4(a.x, a.y, c.x, c.y);
    }
    __device__ __forceinline__ float4 f(uint32_t j) const {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(basef, 0, bytes / 2u, 0x00020000);
        return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, j * 16u, 0, 0));
    }
};
struct RecGlobal {
    const double4 *__restrict__ p;
    const float4 *__restrict__ pf;
    __device__ __forceinline__ double4 operator()(uint32_t j) const { return p[j]; }
    __device__ __forceinline__ float4 f(uint32_t j) const { return pf[j]; }
};

// Absolute slack of the binary32 pre-test of a slot.  Stored coordinates are relative to the
// lattice origin o and lie within M = (largest dims + 1) * b of it (plus the rounding of x / b
// at the lattice edges), so each is off by at most 2^-24 M and a difference by at most
// e = 2^-23 (M + b) (with b >= r_i + r_j >= the distance of any contact).  Then the binary32
// squared distance exceeds the true one by at most (1 + 2^-24)^3 (2 sqrt(3) d e + 3 e^2); with
// e doubled, 4 (b + e) e bounds that.  The relative factor 1.001 on (r_i + r_j)^2 covers the
// rounding of the radii, of their sum and square, and the rounding of every exact law's own
// contact test.  So no pair that the exact law counts as a contact can fail the pre-test.
__device__ __forceinline__ float pretest_slack(const GridDev *__restrict__ g) {
    const double b = g->b;
    int dm = g->dims[0];
    if (g->dims[1] > dm) dm = g->dims[1];
    if (g->dims[2] > dm) dm = g->dims[2];
    double omax = 0.0;
    for (int a = 0; a < 3; ++a) omax = fmax(omax, fabs(double(g->cmin[a]) * b));
    const double M = (double(dm) + 1.0) * b + 0x1p-48 * omax;
    const double e = 0x1p-22 * (M + b);
    return float(4.0 * (b + e) * e) * 1.001f;
}

// Conservative contact pre-test in binary32 (every real contact passes; see pretest_slack).
__device__ __forceinline__ bool maybe_touch(const float4 &a, const float4 &c, float slack) {
    const float dx = a.x - c.x, dy = a.y - c.y, dz = a.z - c.z;
    const float d2 = (dx * dx + dy * dy) + dz * dz;
    const float s = a.w + c.w;
    return d2 < (s * s) * 1.001f + slack;
}

// Box coordinates of a key (x fastest) by fast division.
__device__ __forceinline__ void key_coords(const GridDev *__restrict__ g, uint32_t key, int &cx, int &cy, int &cz) {
    const uint32_t row = fastdiv(key, g->div_nx);
    cx = int(key - row * uint32_t(g->dims[0]));
    const uint32_t z = fastdiv(row, g->div_ny);
    cy = int(row - z * uint32_t(g->dims[1]));
    cz = int(z);
}

// Summed force on the agent with record p at sorted position q whose `cnt` candidates are the
// runs in column `col` of s_run (canonical order); the queue uses this lane's column t.
// The candidates are walked as one counted stream, two per iteration with the next record
// loaded one ahead.  Survivors of the pre-test go to the queue (written unconditionally,
// kept when they pass), which the exact law empties in order when full and at the end.
template <bool F32, int kQ, class Rec>
__device__ __forceinline__ void mech_forces(const SlotDev &S, uint32_t q, const double4 &p, const Rec &rec,
                                            float slack, const uint2 (*s_run)[kBlock], int col, uint32_t cnt,
                                            uint32_t (*s_q)[kBlock], int t, double &fx, double &fy, double &fz) {
    const float rif = float(p.w);
    const float4 pf = rec.f(q);
    fx = 0.0;
    fy = 0.0;
    fz = 0.0;
    int qn = 0;
    auto flush = [&]() {
        for (int k = 0; k < qn; ++k) exact_pair<F32>(p, rec(s_q[k][t]), rif, S, fx, fy, fz);
        qn = 0;
    };
    int r = 0;
    uint2 run = s_run[0][col];
    uint32_t j = run.x, left = run.y - run.x;  // current candidate, candidates left in its run
    // position after j (a run switch reads the next packed run)
    auto advance = [&](uint32_t &jj, uint32_t &ll, int &rr) {
        ++jj;
        if (--ll == 0 && rr < 8) {
            const uint2 u = s_run[++rr][col];
            jj = u.x;
            ll = u.y - u.x;
        }
    };
    constexpr bool kSync = kQ == kQueue;
    auto visit = [&](uint32_t jj, const float4 &c) {
        s_q[qn][t] = jj;
        qn += (maybe_touch(pf, c, slack) && jj != q) ? 1 : 0;
        if constexpr (!kSync) {
            if (qn == kQ) flush();
        }
    };
    // with the normal queue the inner loop fills the queue and stops at a full queue or the end
    // of the stream; the exact law then empties it with every lane of the wavefront together (a
    // lane whose queue fills early waits for the others instead of running its own exact pass
    // alone).  In crowded populations nearly every lane fills its longer queue within a few
    // candidates of the others, and each lane empties it where it fills (measured faster there).
    float4 ca = rec.f(cnt ? j : q), cb;
    uint32_t c = 0;
    while (c < cnt) {
        for (;;) {
            uint32_t jn = j, ln = left;
            int rn = r;
            advance(jn, ln, rn);
            cb = rec.f(c + 1 < cnt ? jn : q);
            visit(j, ca);
            j = jn;
            left = ln;
            r = rn;
            if (++c == cnt || (kSync && qn == kQ)) {
                ca = cb;
                break;
            }
            advance(jn, ln, rn);
            ca = rec.f(c + 1 < cnt ? jn : q);
            visit(j, cb);
            j = jn;
            left = ln;
            r = rn;
            if (++c == cnt || (kSync && qn == kQ)) break;
        }
        flush();
    }
}

// One tile: 256 agents of one slot, one lane per agent.  precision: 64 or 32 for a plain call;
// 0 = per slot.
template <int kPrec, int kQ, class Rec>
__device__ __forceinline__ void mech_tile(const Slots &sl, int64_t tile, const Rec &rec,
                                          const double *__restrict__ adh_s, const uint32_t *__restrict__ id_s,
                                          const uint8_t *__restrict__ state_s, const uint32_t *__restrict__ key_s,
                                          const uint32_t *__restrict__ start_all, const bdm_soa &out,
                                          uint2 (*s_run)[kBlock], uint32_t (*s_q)[kBlock]) {
    const int t = threadIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    const GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    const int64_t l = tile * kBlock + t - S.agent_off;  // local (sorted) index in the slot
    if (!g->valid || l >= g->n || l >= S.capacity) return;
    const bool f32 = kPrec == 32 || (kPrec == 0 && S.force_bits == 32);
    const uint32_t q = uint32_t(g->sorted_base + l);
    int cx, cy, cz;
    key_coords(g, key_s[q], cx, cy, cz);
    const uint32_t cnt = load_runs(g, start_all + S.box_off, cx, cy, cz, s_run, t);
    const double4 p = rec(q);
    double fx, fy, fz;
    if (f32)
        mech_forces<true, kQ>(S, q, p, rec, pretest_slack(g), s_run, t, cnt, s_q, t, fx, fy, fz);
    else
        mech_forces<false, kQ>(S, q, p, rec, pretest_slack(g), s_run, t, cnt, s_q, t, fx, fy, fz);

    // adherence gate, clamp, integrate (binary64)
    const double adh = adh_s[q];
    double nxp = p.x, nyp = p.y, nzp = p.z;
    const double fn = __builtin_sqrt((fx * fx + fy * fy) + fz * fz);
    if (!(fn < adh)) {
        double ux = S.dt * fx, uy = S.dt * fy, uz = S.dt * fz;
        const double len = __builtin_sqrt((ux * ux + uy * uy) + uz * uz);
        if (len > S.max_disp) {
            const double sc = S.max_disp / len;
            ux = ux * sc;
            uy = uy * sc;
            uz = uz * sc;
        }
        nxp = p.x + ux;
        nyp = p.y + uy;
        nzp = p.z + uz;
    }
    const int64_t o = S.agent_off + l;
    __builtin_nontemporal_store(nxp, &out.x[o]);
    __builtin_nontemporal_store(nyp, &out.y[o]);
    __builtin_nontemporal_store(nzp, &out.z[o]);
    __builtin_nontemporal_store(2.0 * p.w, &out.diam[o]);
    __builtin_nontemporal_store(adh, &out.adh[o]);
    __builtin_nontemporal_store(id_s[q], &out.id[o]);
    if (out.state) out.state[o] = state_s[q];
    if (out.fx) __builtin_nontemporal_store(fx, &out.fx[o]);
    if (out.fy) __builtin_nontemporal_store(fy, &out.fy[o]);
    if (out.fz) __builtin_nontemporal_store(fz, &out.fz[o]);
}

template <int kPrec, int kQ, class Rec>
__global__ __launch_bounds__(kBlock) void k_mech(Slots sl, int64_t ntiles, const uint32_t *__restrict__ order, Rec rec,
                                                 const double *__restrict__ adh_s,
                                                 const uint32_t *__restrict__ id_s,
                                                 const uint8_t *__restrict__ state_s,
                                                 const uint32_t *__restrict__ key_s,
                                                 const uint32_t *__restrict__ start, bdm_soa out) {
    __shared__ uint2 s_run[9][kBlock];
    __shared__ uint32_t s_q[kQ][kBlock];
    if (order) {  // plain call: pencil order, one contiguous part of it per XCD
        const GridDev *g0 = &sl.grids[0];
        if (!g0->valid) return;
        const uint32_t live_tiles = uint32_t((g0->n + kBlock - 1) / kBlock);
        if (blockIdx.x >= live_tiles) return;
        mech_tile<kPrec, kQ>(sl, order[xcd_tile(blockIdx.x, live_tiles)], rec, adh_s, id_s, state_s, key_s, start, out,
                         s_run, s_q);
        return;
    }
    // batch: the workgroups stride over the tiles (a simulation's tiles spread over all of them),
    // neighbouring tiles of a round going to workgroups of one XCD
    for (int64_t tile = xcd_tile(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x)
        mech_tile<kPrec, kQ>(sl, tile, rec, adh_s, id_s, state_s, key_s, start, out, s_run, s_q);
}

// Test hook: contact lists per sorted slot in force-sum order (mechanical contact, plain calls).
__global__ __launch_bounds__(kBlock) void k_contacts_mech(Slots sl, const double4 *__restrict__ pos4,
                                                          const uint32_t *__restrict__ id_s,
                                                          const uint32_t *__restrict__ start, int f32,
                                                          uint32_t *counts, const int64_t *offsets,
                                                          uint32_t *ids) {
    __shared__ uint2 s_run[9][kBlock];
    const int t = threadIdx.x;
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + t;
    const GridDev *g = &sl.grids[0];
    if (!g->valid || s >= g->n) return;
    const double b = g->b;
    const double4 p = pos4[s];
    const int cx = box_coord(p.x, b, g->cmin[0], g->dims[0], false);
    const int cy = box_coord(p.y, b, g->cmin[1], g->dims[1], false);
    const int cz = box_coord(p.z, b, g->cmin[2], g->dims[2], false);
    load_runs(g, start, cx, cy, cz, s_run, t);
    const double ri = p.w;
    const float rif = float(ri);
    uint32_t c = 0;
    for (int r = 0; r < 9; ++r) {
        const uint2 run = s_run[r][t];
        for (uint32_t j = run.x; j < run.y; ++j) {
            if (j == uint32_t(s)) continue;
            const double4 q = pos4[j];
            const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
            const double rj = q.w;
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
    counts[s] = c;
}

template <class Rec>
static void launch_mech_rec(const bdm_soa &s, const Slots &sl, int64_t ntiles, unsigned nb, int precision,
                            bool crowded, const uint32_t *order, const Rec &rec, const Ws &w, hipStream_t st) {
#define BDM_MECH(P, Q)                                                                                      \
    hipLaunchKernelGGL((k_mech<P, Q, Rec>), dim3(nb), dim3(kBlock), 0, st, sl, ntiles, order, rec, w.adh, w.ids, \
                       w.state, w.rank, w.start, s)
    if (precision == 32) {
        if (crowded)
            BDM_MECH(32, kQueueCrowded);
        else
            BDM_MECH(32, kQueue);
    } else if (precision == 64) {
        if (crowded)
            BDM_MECH(64, kQueueCrowded);
        else
            BDM_MECH(64, kQueue);
    } else {
        BDM_MECH(0, kQueue);
    }
#undef BDM_MECH
}

// crowded: a population packed so densely that agents have tens of contacts (the growing
// spheroid); a longer queue then saves exact-law rounds, at the cost of LDS (occupancy).
void launch_mech(const bdm_soa &s, const Slots &sl, int64_t capacity, int precision, bool crowded, const Ws &w,
                 hipStream_t st) {
    const int64_t ntiles = (capacity + kBlock - 1) / kBlock;
    const unsigned nb = tile_grid(sl, ntiles);
    const uint32_t *order = sl.table ? nullptr : w.flagid;  // plain: order built with the grid
    const uint64_t bytes = uint64_t(w.lay.capacity) * 32u;
    if (bytes <= 0xFFFFFFE0ull) {
        RecBuf rec{static_cast<void *>(w.pos4), static_cast<void *>(w.pos4f), uint32_t(bytes)};
        launch_mech_rec(s, sl, ntiles, nb, precision, crowded, order, rec, w, st);
    } else {
        launch_mech_rec(s, sl, ntiles, nb, precision, crowded, order, RecGlobal{w.pos4, w.pos4f}, w, st);
    }
}

void launch_contacts_mech(int f32, const Slots &sl, const Ws &w, uint32_t *counts, const int64_t *offsets,
                          uint32_t *ids, hipStream_t st) {
    int64_t nb = (w.lay.capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_contacts_mech, dim3(unsigned(nb)), dim3(kBlock), 0, st, sl, w.pos4, w.ids, w.start, f32,
                       counts, offsets, ids);
}

}  // namespace bdm
