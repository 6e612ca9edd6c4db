// k_grid.hip -- uniform-grid build on gfx950 (paper Sec. 2.1: equal boxes, agents binned by
// centre, box edge from the largest agent, 27-box neighbourhood).
//
// Pipeline for every slot at once (one launch each, all device-resident, no host read-back):
//   bounds     min/max of x, y, z and max diameter: one partial record per 1024 agents (batch)
//              or per workgroup (plain call)
//   finalize   one workgroup per slot: reduce its partials, box edge, lattice origin and dims,
//              box count check
//   key_count  box key per agent and its arrival rank in the box (integer atomics)
//   A plain build (other than a spheroid step's) fuses the first and third: it keys
//   the agents on the last build's lattice while it reduces their bounds, and keys them again
//   only when finalize finds that the lattice moved.
//   scan       single-pass decoupled look-back exclusive scan of the packed histogram
//   scatter    ids into their box range in arrival order
//   canon      each agent counts the smaller ids in its box (ascending-id order inside a box)
//              and copies itself into the sorted copy: (x, y, z, r = d/2) packed as double4
//              (halving and doubling a binary64 are exact, so d = 2r is recovered bit for bit),
//              and for mechanics the records that only the conservative
//              contact pre-test reads: an 8-byte fixed-point record (offsets within the box) and,
//              for spheroid steps, a binary32 copy (x - o, y - o, z - o, r) relative to the
//              lattice origin o
//   order      one workgroup: the processing order of the mechanics tiles (pencils of rows
//              swept along z, so that the three z-planes a tile reads stay in one XCD's L2)
#include "kernels.hpp"

namespace bdm {

constexpr int kPencilRows = 16;       // y-rows per pencil of the processing order
constexpr int kBucketLds = 1024;      // agents of a bucket whose ids the sort keeps in LDS
constexpr int kCrowdedGroups = 1024;  // workgroups that rank the boxes of crowded buckets
constexpr int64_t kBoundsGroups = 2048;  // workgroups of a plain call's bounds reduction

// Bounds partial records: min of x, y, z, max of x, y, z, max diameter, non-finite flag.
__device__ __forceinline__ void bounds_identity(double v[8]) {
    for (int a = 0; a < 3; ++a) {
        v[a] = __builtin_inf();
        v[3 + a] = -__builtin_inf();
    }
    v[6] = 0.0;
    v[7] = 0.0;
}

// Adds the agents of bounds tile `btile` (kBoundsTile agents) to this thread's record; false
// when the tile holds no live agent (the same for the whole workgroup).
__device__ __forceinline__ bool bounds_add(const Slots &sl, int64_t btile, const int64_t *n_ptr,
                                           const double *__restrict__ x, const double *__restrict__ y,
                                           const double *__restrict__ z, const double *__restrict__ d,
                                           double v[8]) {
    const int64_t base = btile * kBoundsTile;
    const int slot = slot_of_tile(sl, base / kBlock);
    if (slot < 0) return false;
    const SlotDev S = slot_record(sl, slot);
    const int64_t n = live_count(n_ptr, slot, S.capacity);
    const int64_t l0 = base - S.agent_off;  // local index of the tile's first agent
    if (l0 >= n) return false;
    bool bad = false;
    constexpr int kUnroll = kBoundsTile / kBlock;
    double px[kUnroll], py[kUnroll], pz[kUnroll], pd[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {  // independent loads in flight
        const int64_t l = l0 + u * kBlock + threadIdx.x;
        const int64_t i = (l < n ? l : l0) + S.agent_off;
        px[u] = x[i];
        py[u] = y[i];
        pz[u] = z[i];
        pd[u] = d ? d[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        bad |= !__builtin_isfinite(px[u]) || !__builtin_isfinite(py[u]) || !__builtin_isfinite(pz[u]) ||
               !__builtin_isfinite(pd[u]);
        v[0] = fmin(v[0], px[u]);
        v[3] = fmax(v[3], px[u]);
        v[1] = fmin(v[1], py[u]);
        v[4] = fmax(v[4], py[u]);
        v[2] = fmin(v[2], pz[u]);
        v[5] = fmax(v[5], pz[u]);
        v[6] = fmax(v[6], pd[u]);
    }
    if (bad) v[7] = 1.0;
    return true;
}

// The workgroup's records reduced into one partial record at dst (no atomics).
__device__ __forceinline__ void bounds_store(double v[8], double *dst) {
    __shared__ double s_red[kBlock / 64][8];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = fmin(v[a], __shfl_xor(v[a], s, 64));
            v[3 + a] = fmax(v[3 + a], __shfl_xor(v[3 + a], s, 64));
        }
        v[6] = fmax(v[6], __shfl_xor(v[6], s, 64));
        v[7] = fmax(v[7], __shfl_xor(v[7], s, 64));
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int a = 0; a < 8; ++a) s_red[wave][a] = v[a];
    __syncthreads();
    if (threadIdx.x < 8) {
        const int a = threadIdx.x;
        double r = s_red[0][a];
        for (int w = 1; w < kBlock / 64; ++w) r = (a < 3) ? fmin(r, s_red[w][a]) : fmax(r, s_red[w][a]);
        dst[a] = r;
    }
    __syncthreads();  // s_red is reused by the next tile of this workgroup
}

// A batch: one partial record per bounds tile (each tile belongs to one slot).  A plain call
// (per_group): one record per workgroup over its stride of tiles, so that the reduction in
// k_finalize reads as many records as there are workgroups (2048 at most) instead of one per
// 1024 agents (16 384 at 2^24 agents: 23 us in one workgroup).
__global__ __launch_bounds__(kBlock) void k_bounds(Slots sl, int64_t nbtiles, const int64_t *n_ptr,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ d, double *partials,
                                                   unsigned long long *tiles, int64_t max_tiles, int32_t per_group) {
    if (frozen_plain(&sl.grids[0], sl.table)) return;
    if (blockIdx.x == 0) {  // reset the scan tiles of the coming histogram scan
        for (int64_t t = threadIdx.x; t < max_tiles; t += blockDim.x) tiles[t] = 0ull;
        if (threadIdx.x == 0) {
            sl.grids[0].scan_ticket = 0u;
            sl.grids[0].crowd_n = 0u;
        }
    }
    double v[8];
    if (per_group) {
        bounds_identity(v);
        for (int64_t bt = blockIdx.x; bt < nbtiles; bt += gridDim.x) bounds_add(sl, bt, n_ptr, x, y, z, d, v);
        bounds_store(v, partials + 8 * int64_t(blockIdx.x));
        return;
    }
    for (int64_t bt = blockIdx.x; bt < nbtiles; bt += gridDim.x) {
        bounds_identity(v);
        if (bounds_add(sl, bt, n_ptr, x, y, z, d, v)) bounds_store(v, partials + 8 * bt);
    }
}

// One workgroup per slot: reduce the slot's bounds partials, then box edge, lattice, box count.
// plain_parts: a plain call's number of per-workgroup records (0: a batch, one per bounds tile).
// spec (plain calls): k_key_spec has already keyed and counted the agents on the last build's
// lattice if that build succeeded; this build keeps those keys when its lattice is the same,
// and otherwise asks for the histogram to be cleared (if anything was counted) and for the keys
// to be taken again.
__global__ __launch_bounds__(kBlock) void k_finalize(Slots sl, const int64_t *n_ptr, const double *partials,
                                                     int32_t kind, int64_t plain_parts, int32_t spec) {
    const int slot = int(blockIdx.x);
    if (slot >= sl.nslots) return;
    const SlotDev a = slot_record(sl, slot);
    GridDev *g = &sl.grids[slot];
    if (frozen_plain(g, sl.table)) return;
    const bool counted = spec && g->valid && g->nboxes > 0;  // k_key_spec counted on the last lattice
    g->rekey = 0;
    g->rezero = counted ? 1 : 0;  // a build that fails clears what was counted
    const int64_t n_raw = n_ptr[slot];
    const int64_t n = live_count(n_ptr, slot, a.capacity);
    const bool idle = a.steps_left <= 0 || a.capacity <= 0;
    double v[8];
    for (int i = 0; i < 3; ++i) {
        v[i] = __builtin_inf();
        v[3 + i] = -__builtin_inf();
    }
    v[6] = 0.0;
    v[7] = 0.0;
    if (!idle) {
        const int64_t b0 = plain_parts ? 0 : a.agent_off / kBoundsTile;
        const int64_t nb = plain_parts ? plain_parts : (n + kBoundsTile - 1) / kBoundsTile;
        const double4 *p4 = reinterpret_cast<const double4 *>(partials) + 2 * b0;
#pragma unroll 8
        for (int64_t k = threadIdx.x; k < nb; k += blockDim.x) {  // 64-byte records, loads in flight
            const double4 lo = p4[2 * k], hi = p4[2 * k + 1];
            v[0] = fmin(v[0], lo.x);
            v[1] = fmin(v[1], lo.y);
            v[2] = fmin(v[2], lo.z);
            v[3] = fmax(v[3], lo.w);
            v[4] = fmax(v[4], hi.x);
            v[5] = fmax(v[5], hi.y);
            v[6] = fmax(v[6], hi.z);
            v[7] = fmax(v[7], hi.w);
        }
    }
    __shared__ double s_red[kBlock][8];
    for (int i = 0; i < 8; ++i) s_red[threadIdx.x][i] = v[i];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off)
            for (int i = 0; i < 8; ++i)
                s_red[threadIdx.x][i] = (i < 3) ? fmin(s_red[threadIdx.x][i], s_red[threadIdx.x + off][i])
                                                : fmax(s_red[threadIdx.x][i], s_red[threadIdx.x + off][i]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double lo[3] = {s_red[0][0], s_red[0][1], s_red[0][2]};
    const double hi[3] = {s_red[0][3], s_red[0][4], s_red[0][5]};
    const double dmax = a.has_d ? s_red[0][6] : 0.0;
    const bool bad = s_red[0][7] != 0.0;
    // the last build's lattice and whether the step after it marked its movers (stationary skip)
    const double prev_b = g->b;
    const int32_t prev_cmin[3] = {g->cmin[0], g->cmin[1], g->cmin[2]};
    const int32_t prev_dims[3] = {g->dims[0], g->dims[1], g->dims[2]};
    // (a skipped agent keeps its last force: the force law must be the same too)
    const bool marks = kind == kGridOpenSkip && g->mark_ready && g->valid && g->consumed && g->kind == kGridOpenSkip &&
                       g->law_k == a.k && g->law_gamma == a.gamma && g->law_bits == a.force_bits;
    g->law_k = a.k;
    g->law_gamma = a.gamma;
    g->law_bits = a.force_bits;
    g->law_box = a.box;
    g->mark_ready = 0;
    g->skip_ok = 0;
    g->sir_counts[0] = g->sir_counts[1] = g->sir_counts[2] = 0ull;
    g->valid = 0;
    g->kind = kind;
    g->consumed = 0;
    g->n = 0;
    g->nboxes = 0;
    if (idle) return;  // idle batch slot
    if (n_raw != n) {
        g->flags |= BDM_FLAG_BADCOUNT;
        return;
    }
    g->n = n;
    if (bad) {
        g->flags |= BDM_FLAG_NONFINITE;
        g->n = 0;
        return;
    }
    double b;
    if (a.periodic) {
        if (a.box < dmax) {
            g->flags |= BDM_FLAG_BOXSMALL;
            g->n = 0;
            return;
        }
        b = a.L / double(a.nb);
        for (int i = 0; i < 3; ++i) {
            g->cmin[i] = 0;
            g->dims[i] = a.nb;
        }
    } else {
        if (a.box > 0.0) {
            if (a.box < dmax) {
                g->flags |= BDM_FLAG_BOXSMALL;
                g->n = 0;
                return;
            }
            b = a.box;
        } else {
            b = dmax;
        }
        if (n == 0) {
            g->b = b;
            for (int i = 0; i < 3; ++i) g->cmin[i] = g->dims[i] = 0;
            g->valid = 1;
            return;
        }
        if (!(b > 0.0)) {
            g->flags |= BDM_FLAG_BOXSMALL;
            g->n = 0;
            return;
        }
        // The span of each axis is formed in binary64 (exact for these integers) and checked
        // against max_boxes before anything is narrowed to int32: coordinates in [-2^30,
        // 2^30 - 1] can span 2^31 boxes, one more than int32 holds.
        double c0[3], span[3];
        for (int i = 0; i < 3; ++i) {
            // floor is monotone, so min/max of floor(x/b) are floor(min x / b), floor(max x / b)
            c0[i] = floor(lo[i] / b);
            const double c1 = floor(hi[i] / b);
            if (!(c0[i] >= -1073741824.0 && c1 <= 1073741823.0)) {
                g->flags |= BDM_FLAG_NONFINITE;
                g->n = 0;
                return;
            }
            span[i] = c1 - c0[i] + 1.0;
        }
        if (span[0] * span[1] * span[2] > double(a.max_boxes) || span[0] > 2147483647.0 ||
            span[1] > 2147483647.0 || span[2] > 2147483647.0) {
            g->flags |= BDM_FLAG_BOXES;
            g->n = 0;
            return;
        }
        for (int i = 0; i < 3; ++i) {
            g->cmin[i] = int32_t(c0[i]);
            g->dims[i] = int32_t(span[i]);
        }
    }
    g->b = b;
    const double boxes = double(g->dims[0]) * double(g->dims[1]) * double(g->dims[2]);
    if (boxes > double(a.max_boxes)) {
        g->flags |= BDM_FLAG_BOXES;
        g->n = 0;
        return;
    }
    g->nboxes = int64_t(g->dims[0]) * g->dims[1] * g->dims[2];
    g->inv_b = 1.0 / g->b;
    g->div_nx = fastdiv_magic(uint32_t(g->dims[0]));
    g->div_ny = fastdiv_magic(uint32_t(g->dims[1]));
    // keys index the same boxes as in the last build only on the same lattice
    const bool same = g->b == prev_b && g->cmin[0] == prev_cmin[0] && g->cmin[1] == prev_cmin[1] &&
                      g->cmin[2] == prev_cmin[2] && g->dims[0] == prev_dims[0] && g->dims[1] == prev_dims[1] &&
                      g->dims[2] == prev_dims[2];
    g->skip_ok = marks && same;
    if (spec) {
        g->rekey = counted && same ? 0 : 1;
        g->rezero = counted && !same ? 1 : 0;
    }
    g->valid = 1;
}

// Box key of every agent and its arrival rank in its bucket (64 consecutive boxes of the packed
// box range).  Lanes of a wavefront with equal buckets in consecutive lanes (the usual case:
// the agents arrive in the box order of the previous step) share one atomic: the first lane
// of each run adds the run length and the others take their offsets from it.  A workgroup
// handles kKeyTiles tiles at once so that their atomics are in flight together.
constexpr int kKeyTiles = 4;

struct KeyLane {
    int64_t i;
    bool live;
    uint32_t k, bk, base;
    int head;
};

// The run of equal buckets the lane belongs to, and (on the run's first lane) the run's slots
// reserved in its bucket.
__device__ __forceinline__ void key_bucket_run(KeyLane &r, uint32_t *count) {
    const int lane = threadIdx.x & 63;
    r.head = lane;
    if (!r.live) r.bk = 0xFFFFFFFFu;
    const uint32_t prev = __shfl_up(r.bk, 1, 64);
    const unsigned long long heads = __ballot(r.live && (lane == 0 || prev != r.bk));
    // this lane's run head: highest head at or below the lane; the run ends at the next head
    // or at the first dead lane after the head (live lanes of a tile form a prefix)
    const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    if (upto) r.head = 63 - __clzll(static_cast<long long>(upto));
    const unsigned long long after = ~((2ull << r.head) - 1ull);
    const unsigned long long stop = (heads | ~__ballot(r.live)) & after;
    const int end = stop ? __ffsll(static_cast<long long>(stop)) - 1 : 64;
    if (r.live && lane == r.head) r.base = atomicAdd(&count[r.bk], uint32_t(end - r.head));
}

// What the key of an agent needs from its tile's slot.
struct KeyGrid {
    bool valid;
    bool per;
    int64_t n, agent_off, box_off;
    double b;
    int32_t cmin[3], dims[3];
};

__device__ __forceinline__ KeyGrid key_grid(const Slots &sl, int slot) {
    KeyGrid k{};
    if (slot < 0) return k;
    const GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    k.valid = g->valid != 0;
    k.per = S.periodic != 0;
    k.n = g->n;
    k.agent_off = S.agent_off;
    k.box_off = S.box_off;
    k.b = g->b;
    for (int a = 0; a < 3; ++a) {
        k.cmin[a] = g->cmin[a];
        k.dims[a] = g->dims[a];
    }
    return k;
}

// The kKeyTiles tiles of a group go through each phase together (grid records, then the
// coordinates, then the keys, then the atomics), so that their memory accesses are in flight
// together rather than one tile's chain of dependent accesses after another's.  A plain call
// reads its one grid record once per group.
// dirty / moved (plain calls that skip stationary agents, else NULL): the box of every agent
// that moved in the last step is marked (the box it entered; the step marked the one it left).
// gated (plain calls after k_key_spec): runs only when the build asked for the keys again.
__global__ __launch_bounds__(kBlock) void k_key_bucket(Slots sl, int64_t ntiles, const double *__restrict__ x,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ z, uint32_t *count,
                                                       uint32_t *__restrict__ key,
                                                       uint32_t *__restrict__ brank, uint8_t *dirty,
                                                       const uint8_t *__restrict__ moved, int32_t gated) {
    if (frozen_plain(&sl.grids[0], sl.table)) return;
    if (gated && !sl.grids[0].rekey) return;
    const int lane = threadIdx.x & 63;
    const bool mark = dirty && sl.grids[0].skip_ok;
    const int64_t ngroups = (ntiles + kKeyTiles - 1) / kKeyTiles;
    for (int64_t grp = xcd_tile(blockIdx.x, gridDim.x); grp < ngroups; grp += gridDim.x) {
        const int64_t tile = grp * kKeyTiles;
        KeyGrid kg[kKeyTiles];
        if (!sl.tilemap) {
            const KeyGrid k0 = key_grid(sl, 0);
#pragma unroll
            for (int u = 0; u < kKeyTiles; ++u) kg[u] = k0;
        } else {
#pragma unroll
            for (int u = 0; u < kKeyTiles; ++u) kg[u] = key_grid(sl, tile + u < ntiles ? slot_of_tile(sl, tile + u) : -1);
        }
        KeyLane r[kKeyTiles];
        double xv[kKeyTiles], yv[kKeyTiles], zv[kKeyTiles];
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            r[u] = KeyLane{};
            r[u].i = (tile + u) * kBlock + threadIdx.x;
            r[u].live = tile + u < ntiles && kg[u].valid && r[u].i - kg[u].agent_off < kg[u].n;
            xv[u] = r[u].live ? x[r[u].i] : 0.0;
            yv[u] = r[u].live ? y[r[u].i] : 0.0;
            zv[u] = r[u].live ? z[r[u].i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            if (!r[u].live) continue;
            const KeyGrid &k = kg[u];
            const int cx = box_coord(xv[u], k.b, k.cmin[0], k.dims[0], k.per);
            const int cy = box_coord(yv[u], k.b, k.cmin[1], k.dims[1], k.per);
            const int cz = box_coord(zv[u], k.b, k.cmin[2], k.dims[2], k.per);
            r[u].k = uint32_t(cx) + uint32_t(k.dims[0]) * (uint32_t(cy) + uint32_t(k.dims[1]) * uint32_t(cz));
            r[u].bk = uint32_t((uint64_t(k.box_off) + r[u].k) >> kBucketShift);
        }
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) key_bucket_run(r[u], count);
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            const uint32_t base = __shfl(r[u].base, r[u].head, 64);
            if (!r[u].live) continue;
            key[r[u].i] = r[u].k;
            brank[r[u].i] = base + uint32_t(lane - r[u].head);
            if (mark && moved[r[u].i]) dirty[r[u].k] = 1;
        }
    }
}

// A plain build's first pass: the bounds of the agents (one record per workgroup, as k_bounds
// writes them) and, on trust, every agent's key and bucket rank on the last build's lattice,
// counted into the histogram.  Agents move by at most the clamp in a step, so in a running
// simulation the lattice seldom changes, and the coordinates are then read once per build
// instead of twice.  k_finalize keeps the keys when the bounds give the same lattice (box edge,
// origin and dims; the keys depend on nothing else) and otherwise has the histogram cleared and
// the keys taken again.  Nothing is counted when the last build failed, had no boxes or there
// was none; a lane with a non-finite coordinate counts nothing either (its build fails).
// dirty / moved (skipping steps, else NULL): the box of every agent that moved in the last step
// is marked on the last lattice.  The marks count only when the build may skip (same lattice,
// marks ready); the bucket sort clears every box's mark in any case.
__global__ __launch_bounds__(kBlock) void k_key_spec(Slots sl, int64_t ntiles, const int64_t *n_ptr,
                                                     const double *__restrict__ x, const double *__restrict__ y,
                                                     const double *__restrict__ z, const double *__restrict__ d,
                                                     uint32_t *count, uint32_t *__restrict__ key,
                                                     uint32_t *__restrict__ brank, double *partials,
                                                     unsigned long long *tiles, int64_t max_tiles, uint8_t *dirty,
                                                     const uint8_t *__restrict__ moved) {
    GridDev *g = &sl.grids[0];
    if (frozen_plain(g, false)) return;
    if (blockIdx.x == 0) {  // reset the scan tiles of the coming histogram scan
        for (int64_t t = threadIdx.x; t < max_tiles; t += blockDim.x) tiles[t] = 0ull;
        if (threadIdx.x == 0) {
            g->scan_ticket = 0u;
            g->crowd_n = 0u;
        }
    }
    const int lane = threadIdx.x & 63;
    const SlotDev S = sl.one;
    const int64_t n = live_count(n_ptr, 0, S.capacity);
    const bool on_last = g->valid != 0 && g->nboxes > 0;  // a lattice with boxes to key into
    KeyGrid k{};
    k.per = S.periodic != 0;
    k.b = g->b;
    for (int a = 0; a < 3; ++a) {
        k.cmin[a] = g->cmin[a];
        k.dims[a] = g->dims[a];
    }
    double v[8];
    bounds_identity(v);
    bool bad = false;
    const int64_t ngroups = (ntiles + kKeyTiles - 1) / kKeyTiles;
    for (int64_t grp = xcd_tile(blockIdx.x, gridDim.x); grp < ngroups; grp += gridDim.x) {
        const int64_t tile = grp * kKeyTiles;
        KeyLane r[kKeyTiles];
        bool in[kKeyTiles];
        double xv[kKeyTiles], yv[kKeyTiles], zv[kKeyTiles], dv[kKeyTiles];
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            r[u] = KeyLane{};
            r[u].i = S.agent_off + (tile + u) * kBlock + threadIdx.x;
            in[u] = tile + u < ntiles && r[u].i - S.agent_off < n;
            xv[u] = in[u] ? x[r[u].i] : 0.0;
            yv[u] = in[u] ? y[r[u].i] : 0.0;
            zv[u] = in[u] ? z[r[u].i] : 0.0;
            dv[u] = in[u] && d ? d[r[u].i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            if (!in[u]) continue;
            const bool fin = __builtin_isfinite(xv[u]) && __builtin_isfinite(yv[u]) && __builtin_isfinite(zv[u]);
            bad |= !fin || !__builtin_isfinite(dv[u]);
            v[0] = fmin(v[0], xv[u]);
            v[3] = fmax(v[3], xv[u]);
            v[1] = fmin(v[1], yv[u]);
            v[4] = fmax(v[4], yv[u]);
            v[2] = fmin(v[2], zv[u]);
            v[5] = fmax(v[5], zv[u]);
            v[6] = fmax(v[6], dv[u]);
            r[u].live = on_last && fin;
            if (!r[u].live) continue;
            const int cx = box_coord(xv[u], k.b, k.cmin[0], k.dims[0], k.per);
            const int cy = box_coord(yv[u], k.b, k.cmin[1], k.dims[1], k.per);
            const int cz = box_coord(zv[u], k.b, k.cmin[2], k.dims[2], k.per);
            r[u].k = uint32_t(cx) + uint32_t(k.dims[0]) * (uint32_t(cy) + uint32_t(k.dims[1]) * uint32_t(cz));
            r[u].bk = uint32_t((uint64_t(S.box_off) + r[u].k) >> kBucketShift);
        }
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) key_bucket_run(r[u], count);
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            const uint32_t base = __shfl(r[u].base, r[u].head, 64);
            if (!r[u].live) continue;
            key[r[u].i] = r[u].k;
            brank[r[u].i] = base + uint32_t(lane - r[u].head);
            if (dirty && moved[r[u].i]) dirty[r[u].k] = 1;
        }
    }
    if (bad) v[7] = 1.0;
    bounds_store(v, partials + 8 * int64_t(blockIdx.x));
}

// Clears the histogram that k_key_spec counted into when the build did not keep its keys.
__global__ __launch_bounds__(kBlock) void k_count_clear(const GridDev *g, uint32_t *count, int64_t len) {
    if (frozen_plain(g, false) || !g->rezero) return;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x)
        count[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_scan_prepare(unsigned long long *tiles, int64_t max_tiles,
                                                         uint32_t *ticket) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < max_tiles) tiles[t] = 0ull;
    if (t == 0) *ticket = 0u;
}

// Exclusive scan of in[0, len) into out[0, len], out[len] = total; len read on the device (and
// clamped to len_fixed, the arrays' length) or fixed.
// Tiles are taken in launch order from a ticket, so a tile only ever waits on tiles that are
// already running.  Tile status word: value << 32 | flag (1 = tile aggregate, 2 = inclusive
// prefix).  Wavefront 0 looks back 64 predecessors at a time with ballots.
__global__ __launch_bounds__(kBlock) void k_scan(uint32_t *in, uint32_t *out, const int64_t *len_ptr,
                                                 int64_t len_fixed, unsigned long long *tiles,
                                                 uint32_t *ticket, int zero_in, GridDev *g, int32_t build) {
    if (build && g->frozen) return;  // the bucket scan of a plain build that changes nothing
    __shared__ uint32_t s_tile, s_prefix;
    __shared__ uint32_t s_wave[kBlock / 64];
    int64_t len = len_fixed;  // a device-resident length never exceeds the arrays' length
    if (len_ptr) {
        const int64_t v = *len_ptr;
        len = v < 0 ? 0 : (v < len_fixed ? v : len_fixed);
    }
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t ntiles = (len + kScanTile) / kScanTile;  // covers indices 0..len
    if (tile >= ntiles) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = tile * kScanTile + int64_t(threadIdx.x) * kScanItems;

    uint32_t v[kScanItems];
    if (base + kScanItems <= len) {
        const uint4 *src = reinterpret_cast<const uint4 *>(in + base);
        uint4 a = src[0], c = src[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < len) ? in[base + k] : 0u;
    }
    uint32_t tsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tsum += v[k];
    const uint32_t incl = wave_incl_scan(tsum);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t wave_off = 0, block_total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const uint32_t t = s_wave[w];
        if (w < wave) wave_off += t;
        block_total += t;
    }

    if (wave == 0) {
        uint32_t exclusive = 0;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&tiles[0], (static_cast<unsigned long long>(block_total) << 32) | 2ull,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&tiles[tile], (static_cast<unsigned long long>(block_total) << 32) | 1ull,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t look = tile - 1;
            uint32_t spins = 0;
            while (true) {
                const int64_t idx = look - lane;
                unsigned long long st = 2ull;  // below tile 0: a zero inclusive prefix
                if (idx >= 0)
                    st = __hip_atomic_load(&tiles[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t flag = uint32_t(st & 3ull);
                const unsigned long long not_ready = __ballot(flag == 0);
                const unsigned long long is_p = __ballot(flag == 2);
                const int first_p = is_p ? __ffsll(static_cast<long long>(is_p)) - 1 : 64;
                const unsigned long long need = first_p == 64 ? ~0ull : ((2ull << first_p) - 1ull);
                if (not_ready & need) {
                    if (++spins > kScanSpinLimit) {
                        if (lane == 0) atomicOr(&g->flags, BDM_FLAG_SCAN);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint32_t val = (lane <= first_p) ? uint32_t(st >> 32) : 0u;
                exclusive += wave_sum(val);
                if (first_p < 64) break;
                look -= 64;
            }
            if (lane == 0)
                __hip_atomic_store(&tiles[tile],
                                   (static_cast<unsigned long long>(exclusive + block_total) << 32) | 2ull,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_prefix = exclusive;
    }
    __syncthreads();
    uint32_t run = s_prefix + wave_off + (incl - tsum);
    if (base + kScanItems <= len) {
        uint32_t o[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            o[k] = run;
            run += v[k];
        }
        uint4 *dst = reinterpret_cast<uint4 *>(out + base);
        dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
        dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
        if (zero_in) {
            uint4 *src = reinterpret_cast<uint4 *>(in + base);
            src[0] = make_uint4(0u, 0u, 0u, 0u);
            src[1] = make_uint4(0u, 0u, 0u, 0u);
        }
        if (base + kScanItems == len) out[len] = run;  // total lands right after a full chunk
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t idx = base + k;
            if (idx <= len) out[idx] = run;
            if (zero_in && idx < len) in[idx] = 0u;
            run += v[k];
        }
    }
}

// Agent indices into their bucket's range of sorted positions, in arrival order (kKeyTiles
// tiles per workgroup at once, so that their dependent loads overlap; the workgroups stride
// over groups of tiles, so a simulation's tiles spread over all of them).
__global__ __launch_bounds__(kBlock) void k_bucket_scatter(Slots sl, int64_t ntiles,
                                                           const uint32_t *__restrict__ key,
                                                           const uint32_t *__restrict__ brank,
                                                           const uint32_t *__restrict__ bstart,
                                                           uint32_t *__restrict__ item, int64_t capacity) {
    if (frozen_plain(&sl.grids[0], sl.table)) return;
    const int64_t ngroups = (ntiles + kKeyTiles - 1) / kKeyTiles;
    for (int64_t grp = xcd_tile(blockIdx.x, gridDim.x); grp < ngroups; grp += gridDim.x) {
        const int64_t tile = grp * kKeyTiles, t1 = ntiles;
        int64_t iu[kKeyTiles];
        uint32_t bk[kKeyTiles], rk[kKeyTiles], pos[kKeyTiles], lim[kKeyTiles];
        GridDev *gu[kKeyTiles];
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            iu[u] = -1;
            const int64_t t = tile + u;
            if (t >= t1) continue;
            const int slot = slot_of_tile(sl, t);
            if (slot < 0) continue;
            GridDev *g = &sl.grids[slot];
            const SlotDev S = slot_record(sl, slot);
            const int64_t i = t * kBlock + threadIdx.x;
            if (!g->valid || i - S.agent_off >= g->n) continue;
            if (i == S.agent_off) g->sorted_base = bstart[S.box_off >> kBucketShift];
            iu[u] = i;
            gu[u] = g;
            bk[u] = uint32_t((uint64_t(S.box_off) + key[i]) >> kBucketShift);
            rk[u] = brank[i];
        }
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u)
            if (iu[u] >= 0) {
                pos[u] = bstart[bk[u]] + rk[u];
                lim[u] = bstart[bk[u] + 1];
            }
#pragma unroll
        for (int u = 0; u < kKeyTiles; ++u) {
            if (iu[u] < 0) continue;
            if (pos[u] >= uint64_t(capacity) || pos[u] >= lim[u]) {  // cannot happen with zeroed counts
                atomicOr(&gu[u]->flags, BDM_FLAG_SCAN);
                continue;
            }
            item[pos[u]] = uint32_t(iu[u]);
        }
    }
}

// One wavefront per bucket: order the bucket's agents by (box, id) and copy them into the sorted
// arrays; write the box starts of the bucket's 64 boxes.
//   1. histogram of the agents' boxes within the bucket (LDS);
//   2. exclusive scan over the 64 boxes (one box per lane): box starts;
//   3. each agent's id into its box's range (LDS cursor, arrival order; the ids themselves in
//      LDS up to kBucketLds agents, else in the scratch id array);
//   4. each agent counts the smaller ids of its box, which gives its final position, and copies
//      (x, y, z, r = d/2) packed as a double4 (halving and doubling a binary64 are exact, so d =
//      2r is recovered bit for bit), its pre-test records (the 8-byte one; the binary32 copy
//      relative to the lattice origin when asked for), adh, id and state there (the mechanics
//      finds an agent's box from its position, as the key was computed).
// A bucket holds any number of agents (the wavefront walks them 64 at a time).
struct SortOut {
    double4 *pos4;
    float4 *pos4f;  // binary32 copy for the crowded mechanics kernel (null: not written)
    uint2 *pos8;
    double *adh;
    uint32_t *id;
    uint8_t *state;
    uint32_t *tile_key;  // key of every tile's first agent (plain calls only)
    uint8_t *dirty;      // stationary skip (plain calls): box marks, folded into the starts
    double *fprev;       // stationary skip: the agents' last forces in the new sorted order
};

// One sorted agent as the bucket sort carries it.
struct BucketAgent {
    int64_t i;      // index in the input arrays
    int slot;       // its slot (-1: not a valid entry)
    uint32_t k;     // box key within its slot
    uint32_t kl;    // box within the bucket (>= 64: skip)
    uint32_t id;
    double x, y, z, rad, adh;
    uint8_t st;
};

// A bucket of at most 64 * K agents: K agents per lane held in registers through all phases.
template <int K, class Fetch, class Count, class Starts, class Group, class Settle, class Emit>
__device__ __forceinline__ void run_small(int lane, Fetch &fetch, Count &count, Starts &starts, Group &group,
                                          Settle &settle, Emit &emit) {
    BucketAgent a[K];
#pragma unroll
    for (int u = 0; u < K; ++u) a[u] = fetch(uint32_t(lane) + 64u * uint32_t(u), true);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < K; ++u) count(a[u]);
    starts();
#pragma unroll
    for (int u = 0; u < K; ++u) group(a[u]);
    settle();
#pragma unroll
    for (int u = 0; u < K; ++u) emit(a[u]);
}

// What the bucket sort reads and writes, for the helpers below.
// The lattice of the grid a wavefront's agents belong to (one slot per bucket), read once per
// wavefront for the pre-test records.
struct PreGrid {
    double b, inv_b;
    int32_t cmin[3];
    uint32_t nx, ny;
    unsigned long long div_nx, div_ny;
};

__device__ __forceinline__ PreGrid pre_grid(const GridDev *g) {
    PreGrid p;
    p.b = g->b;
    p.inv_b = g->inv_b;
    for (int a = 0; a < 3; ++a) p.cmin[a] = g->cmin[a];
    p.nx = uint32_t(g->dims[0]);
    p.ny = uint32_t(g->dims[1]);
    p.div_nx = g->div_nx;
    p.div_ny = g->div_ny;
    return p;
}

struct SortCtx {
    Slots sl;
    SoaIn s;
    const uint32_t *key;
    SortOut o;
    int periodic;
    int64_t capacity;
    PreGrid pg;  // the bucket's grid (open lattices only)
    bool fold;   // this build may skip stationary agents: carry the forces, mark the starts
};

// The agent at input index i, for a bucket whose first box is box0 (kl >= 64 marks an entry to
// skip: an index or key that cannot come from a valid build); `full` also loads what the copy
// needs.
__device__ __forceinline__ BucketAgent sort_agent(const SortCtx &c, int64_t box0, int64_t i, bool full) {
    BucketAgent a{};
    a.kl = 0xFFFFFFFFu;
    a.slot = -1;
    a.i = i;
    if (i < 0 || i >= c.capacity) return a;
    a.slot = slot_of_tile(c.sl, i / kBlock);
    if (a.slot < 0) return a;
    const SlotDev S = slot_record(c.sl, a.slot);
    a.k = c.key[i];
    a.kl = uint32_t(int64_t(S.box_off) + int64_t(a.k) - box0);
    a.id = c.s.id[i];
    if (full) {
        a.x = c.s.x[i];
        a.y = c.s.y[i];
        a.z = c.s.z[i];
        a.rad = c.s.d ? 0.5 * c.s.d[i] : 0.0;  // radius, exact
        a.adh = c.s.adh ? c.s.adh[i] : 0.0;
        a.st = c.s.state ? c.s.state[i] : 0;
    }
    return a;
}

// The sorted copy of agent a at sorted position dst.
__device__ __forceinline__ void sort_write(const SortCtx &c, const BucketAgent &a, uint32_t dst) {
    c.o.pos4[dst] = make_double4(a.x, a.y, a.z, a.rad);
    if (!c.periodic) {
        const PreGrid &g = c.pg;
        const uint32_t row = fastdiv(a.k, g.div_nx), zc = fastdiv(row, g.div_ny);
        const int cx = int(a.k - row * g.nx), cy = int(row - zc * g.ny), cz = int(zc);
        c.o.pos8[dst] = make_uint2(
            pre8_axis(a.x, g.inv_b, g.cmin[0] + cx) | pre8_axis(a.y, g.inv_b, g.cmin[1] + cy) << 16,
            pre8_axis(a.z, g.inv_b, g.cmin[2] + cz) | pre8_radius(a.rad, g.inv_b) << 16);
        if (c.o.pos4f)
            c.o.pos4f[dst] = make_float4(float(a.x - double(g.cmin[0]) * g.b), float(a.y - double(g.cmin[1]) * g.b),
                                         float(a.z - double(g.cmin[2]) * g.b), float(a.rad * kPretestRadius));
    }
    if (c.s.adh) c.o.adh[dst] = a.adh;
    c.o.id[dst] = a.id;
    if (c.s.state) c.o.state[dst] = a.st;
    if (c.o.tile_key && (dst & (kBlock - 1)) == 0) c.o.tile_key[dst / kBlock] = a.k;
    if (c.fold) {
        c.o.fprev[3 * size_t(dst)] = c.s.fx[a.i];
        c.o.fprev[3 * size_t(dst) + 1] = c.s.fy[a.i];
        c.o.fprev[3 * size_t(dst) + 2] = c.s.fz[a.i];
    }
}

// Six wavefronts per SIMD (at most 80 registers; the compiler's own choice of 81 allowed five):
// each wavefront's chain of dependent loads is short, so more of them in flight pay
// (measured at 2^24 agents: 428 -> 403 us).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_bucket_sort(
                                                        Slots sl, int64_t nbuckets, int64_t max_boxes,
                                                        SoaIn s, const uint32_t *__restrict__ key,
                                                        const uint32_t *__restrict__ bstart,
                                                        const uint32_t *__restrict__ item,
                                                        uint32_t *__restrict__ grouped, uint32_t *__restrict__ grouped_i,
                                                        uint32_t *__restrict__ start, SortOut o, int periodic,
                                                        int64_t capacity, uint32_t *__restrict__ crowd) {
    if (frozen_plain(&sl.grids[0], sl.table)) return;
    __shared__ uint32_t s_hist[kBlock / 64][kBucketBoxes];
    __shared__ uint32_t s_ls[kBlock / 64][kBucketBoxes];
    __shared__ uint32_t s_cur[kBlock / 64][kBucketBoxes];
    __shared__ uint32_t s_grp[kBlock / 64][kBucketLds];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (uniform)
    const int64_t bk = int64_t(xcd_tile(blockIdx.x, gridDim.x)) * (kBlock / 64) + wave;
    if (bk >= nbuckets) return;  // (the whole wavefront; no workgroup barrier below)
    if (sl.bucketmap && sl.bucketmap[bk] < 0) return;  // a batch bucket no simulation owns
    uint32_t *hist = s_hist[wave], *lst = s_ls[wave], *cur = s_cur[wave], *grp = s_grp[wave];
    const uint32_t b0 = bstart[bk];
    uint32_t b1 = bstart[bk + 1];
    if (b1 > uint64_t(capacity)) b1 = uint32_t(capacity);  // (only after a failed scan)
    const uint32_t m = b1 > b0 ? b1 - b0 : 0u;
    const bool in_lds = m <= uint32_t(kBucketLds);  // else the grouped ids go through memory
    const int64_t box0 = bk << kBucketShift;
    hist[lane] = 0u;

    const bool fold = o.dirty && sl.grids[0].skip_ok;  // (plain calls only)
    const SortCtx ctx{sl, s, key, o, periodic, capacity,
                      pre_grid(&sl.grids[sl.bucketmap ? sl.bucketmap[bk] : 0]), fold};
    auto from_index = [&](int64_t i, bool full) { return sort_agent(ctx, box0, i, full); };
    // the agent of item slot c
    auto fetch = [&](uint32_t c, bool full) {
        if (c >= m) {
            BucketAgent a{};
            a.kl = 0xFFFFFFFFu;
            a.slot = -1;
            return a;
        }
        return from_index(int64_t(item[b0 + c]), full);
    };
    auto count = [&](const BucketAgent &a) {
        if (a.kl < uint32_t(kBucketBoxes)) atomicAdd(&hist[a.kl], 1u);
    };
    auto group = [&](const BucketAgent &a) {
        if (a.kl >= uint32_t(kBucketBoxes)) return;
        const uint32_t p = atomicAdd(&cur[a.kl], 1u);
        if (in_lds) {
            grp[p] = a.id;
        } else {  // through L2 (bypassing L1), read back below by other lanes of this wavefront
            __hip_atomic_store(&grouped[b0 + p], a.id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&grouped_i[b0 + p], uint32_t(a.i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    auto write_out = [&](const BucketAgent &a, uint32_t dst) { sort_write(ctx, a, dst); };
    auto emit = [&](const BucketAgent &a) {  // rank among the ids of its box, kept in LDS
        if (a.kl >= uint32_t(kBucketBoxes)) return;
        const uint32_t l0 = lst[a.kl], gn = hist[a.kl];
        uint32_t r = 0;
        for (uint32_t j = 0; j < gn; ++j) r += grp[l0 + j] < a.id;
        if (r >= gn) return;  // duplicate ids (not a valid population)
        write_out(a, b0 + l0 + r);
    };
    auto starts = [&]() {  // exclusive scan over the bucket's 64 boxes (one per lane)
        __builtin_amdgcn_wave_barrier();
        const uint32_t h = hist[lane];
        const uint32_t ls = wave_incl_scan(h) - h;
        if (box0 + lane <= max_boxes) {
            uint32_t v = b0 + ls;
            if (o.dirty) {  // stationary skip: fold the box's mark into its start, clear the mark
                const int64_t bx = box0 + lane;
                if (fold && o.dirty[bx]) v |= kStartDirty;
                o.dirty[bx] = 0;
            }
            start[box0 + lane] = v;
        }
        // the first box start of the next bucket is this bucket's end: written here too, so that
        // a simulation whose box range ends at this bucket's end finds it even when no simulation
        // owns the next bucket (both writers write the same value).  Plain calls own every
        // bucket, and when they mark their starts only the owner may write one.
        if (!o.dirty && lane == 0 && box0 + kBucketBoxes <= max_boxes) start[box0 + kBucketBoxes] = b1;
        lst[lane] = ls;
        cur[lane] = ls;
        __builtin_amdgcn_wave_barrier();
    };
    auto settle = [&]() {  // grouped ids written above complete before they are read below
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        __builtin_amdgcn_wave_barrier();
    };

    if (m <= 128) {  // the usual bucket: up to two agents per lane, every load issued up front
        run_small<2>(lane, fetch, count, starts, group, settle, emit);
        return;
    }
    if (m <= 256) {
        run_small<4>(lane, fetch, count, starts, group, settle, emit);
        return;
    }
    __builtin_amdgcn_wave_barrier();
    for (uint32_t c = lane; c < m; c += 64) count(fetch(c, false));
    starts();
    for (uint32_t c = lane; c < m; c += 64) group(fetch(c, false));
    settle();
    if (in_lds) {
        for (uint32_t c = lane; c < m; c += 64) emit(fetch(c, true));
        return;
    }
    // a crowded bucket: its boxes are ranked by k_bucket_crowded, many wavefronts per bucket
    if (lane == 0) crowd[atomicAdd(&sl.grids[0].crowd_n, 1u)] = uint32_t(bk);
}

// The boxes of crowded buckets (more agents than the sort keeps in LDS), whose ids the bucket
// sort left grouped by box in `grouped` (agent indices in `grouped_i`): each wavefront takes
// whole boxes, 64 members at a time; the box's ids are staged in LDS, kBucketLds at a time, and
// each member counts the smaller ones, which gives its position.  A fixed grid strides over the
// listed buckets' boxes, so a few crowded buckets still spread over the whole device.
__global__ __launch_bounds__(kBlock) void k_bucket_crowded(Slots sl, int64_t max_boxes, SoaIn s,
                                                           const uint32_t *__restrict__ key,
                                                           const uint32_t *__restrict__ bstart,
                                                           const uint32_t *__restrict__ grouped,
                                                           const uint32_t *__restrict__ grouped_i,
                                                           const uint32_t *__restrict__ start, SortOut o,
                                                           int periodic, int64_t capacity,
                                                           const uint32_t *__restrict__ crowd) {
    if (frozen_plain(&sl.grids[0], sl.table)) return;
    __shared__ uint32_t s_grp[kBlock / 64][kBucketLds];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (uniform)
    uint32_t *grp = s_grp[wave];
    const uint32_t nc = sl.grids[0].crowd_n;
    SortCtx ctx{sl, s, key, o, periodic, capacity, {}, o.dirty && sl.grids[0].skip_ok};
    const int64_t nwaves = int64_t(gridDim.x) * (kBlock / 64);
    for (int64_t w = int64_t(blockIdx.x) * (kBlock / 64) + wave; w < int64_t(nc) * kBucketBoxes; w += nwaves) {
        const int64_t bk = crowd[w / kBucketBoxes];
        const int kl = int(w % kBucketBoxes);
        const int64_t box0 = bk << kBucketShift;
        if (box0 + kl + 1 > max_boxes) continue;
        const uint32_t b0 = bstart[bk], s0 = start[box0 + kl] & kStartMask, s1 = start[box0 + kl + 1] & kStartMask;
        if (s1 <= s0 || s0 < b0) continue;
        const uint32_t l0 = s0 - b0, gn = s1 - s0;
        ctx.pg = pre_grid(&sl.grids[sl.bucketmap ? sl.bucketmap[bk] : 0]);
        for (uint32_t m0 = 0; m0 < gn; m0 += 64) {
            const uint32_t pm = m0 + uint32_t(lane);
            const bool mine = pm < gn;
            const uint32_t me = mine ? grouped[b0 + l0 + pm] : 0u;
            uint32_t r = 0;
            for (uint32_t w0 = 0; w0 < gn; w0 += uint32_t(kBucketLds)) {
                const uint32_t wn = gn - w0 < uint32_t(kBucketLds) ? gn - w0 : uint32_t(kBucketLds);
                __builtin_amdgcn_wave_barrier();
                for (uint32_t e = uint32_t(lane); e < wn; e += 64) grp[e] = grouped[b0 + l0 + w0 + e];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (mine)
                    for (uint32_t e = 0; e < wn; ++e) r += grp[e] < me;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (!mine || r >= gn) continue;  // (r >= gn: duplicate ids, not a valid population)
            const BucketAgent a = sort_agent(ctx, box0, int64_t(grouped_i[b0 + l0 + pm]), true);
            if (a.kl == uint32_t(kl)) sort_write(ctx, a, b0 + l0 + r);
        }
    }
}

// Processing order of the mechanics tiles of a plain call: the tiles (256 consecutive sorted
// agents) sorted stably by (pencil of kPencilRows y-rows, z-plane) of their first agent.  Every
// order is correct (each tile is independent); this one keeps the three z-planes a tile reads
// within a small window.  The tiles' first keys are non-decreasing, so the tiles of one bin
// form one contiguous run, and the runs come in (z, pencil) order: the order is a permutation
// of runs, found from each run's ends, a scan over the bins and one write per tile.  Falls
// back to the identity when the grid has more than kOrderBins bins.
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

struct OrderGeom {
    int64_t ntile;
    uint32_t nx, ny, nz, nbins;
    bool ok;
    __device__ explicit OrderGeom(const GridDev *g) {
        ntile = g->valid ? (g->n + kBlock - 1) / kBlock : 0;
        nx = uint32_t(g->dims[0]);
        ny = uint32_t(g->dims[1]);
        nz = uint32_t(g->dims[2]);
        const int64_t bins = (int64_t(ny) + kPencilRows - 1) / kPencilRows * int64_t(nz);
        ok = ntile > 0 && nx > 0 && ny > 0 && bins > 0 && bins <= kOrderBins;
        nbins = ok ? uint32_t(bins) : 0u;
    }
    __device__ uint32_t bin(uint32_t k) const {
        const uint32_t row = k / nx, yy = row % ny, zz = row / ny;
        const uint32_t b = (yy / kPencilRows) * nz + zz;
        return b < nbins ? b : nbins - 1u;
    }
};

// First and last tile of every bin's run.
__global__ __launch_bounds__(kBlock) void k_order_runs(const GridDev *__restrict__ g,
                                                       const uint32_t *__restrict__ tile_key, uint32_t *first,
                                                       uint32_t *last) {
    if (g->frozen) return;
    const OrderGeom o(g);
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!o.ok || c >= o.ntile) return;
    const uint32_t b = o.bin(tile_key[c]);
    if (c == 0 || o.bin(tile_key[c - 1]) != b) first[b] = uint32_t(c);
    if (c == o.ntile - 1 || o.bin(tile_key[c + 1]) != b) last[b] = uint32_t(c);
}

// One workgroup: exclusive scan of the runs' lengths in (pencil, z) order; shift[b] is set so
// that tile c of bin b goes to position c + shift[b] (mod 2^32).  Clears the run ends for the
// next build.
// Only the bins below the grid's bin count can hold tiles (every entry is kNoTile between
// builds), so only those are read and reset; a small grid's scan skips the rest.
__global__ __launch_bounds__(1024) void k_order_scan(const GridDev *__restrict__ g, uint32_t *first,
                                                     uint32_t *last, uint32_t *shift) {
    if (g->frozen) return;
    __shared__ uint32_t s_part[1024 / 64];
    const OrderGeom o(g);
    const int t = threadIdx.x;
    const int per = (kOrderBins + 1023) / 1024;
    const int nbins = o.ok ? int(o.nbins) : 0;
    const int b0 = t * per;
    uint32_t len[per], sum = 0;
    for (int j = 0; j < per; ++j) {
        const int b = b0 + j;
        len[j] = 0;
        if (b < nbins && first[b] != kNoTile) len[j] = last[b] - first[b] + 1u;
        sum += len[j];
    }
    // exclusive scan of the threads' sums: within each wavefront, then over the 16 wavefronts
    const uint32_t incl = wave_incl_scan(sum);
    if ((t & 63) == 63) s_part[t >> 6] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < (t >> 6); ++w) run += s_part[w];
    for (int j = 0; j < per; ++j) {
        const int b = b0 + j;
        if (b >= nbins) break;
        if (len[j]) shift[b] = run - first[b];
        run += len[j];
        first[b] = kNoTile;
        last[b] = kNoTile;
    }
}

__global__ __launch_bounds__(kBlock) void k_order_write(const GridDev *__restrict__ g,
                                                        const uint32_t *__restrict__ tile_key,
                                                        const uint32_t *__restrict__ shift,
                                                        uint32_t *__restrict__ order, int64_t max_tiles) {
    if (g->frozen) return;
    const OrderGeom o(g);
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= o.ntile || c >= max_tiles) return;
    const uint32_t pos = o.ok ? uint32_t(c) + shift[o.bin(tile_key[c])] : uint32_t(c);
    if (pos < max_tiles) order[pos] = uint32_t(c);
}

__global__ __launch_bounds__(kBlock) void k_read_agents(const int64_t *n_ptr, const bdm_soa s,
                                                        ReadOut o) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, s.capacity);
    if (i >= n) return;
    const uint32_t id = s.id[i];
    if (id >= n) return;
    if (o.x) o.x[id] = s.x[i];
    if (o.y) o.y[id] = s.y[i];
    if (o.z) o.z[id] = s.z[i];
    if (o.d) o.d[id] = s.diam[i];
    if (o.fx) o.fx[id] = s.fx[i];
    if (o.fy) o.fy[id] = s.fy[i];
    if (o.fz) o.fz[id] = s.fz[i];
    if (o.state) o.state[id] = s.state[i];
}

// Whether a plain build and its step change nothing (stationary skip): the last step was a
// skipping step of this workspace that skipped every live agent, so no position moved; with the
// same live count, force law and requested box edge the lattice, the sorted agents and every
// force are what they are now.  Every later kernel of the build and of the step then returns at
// once.  A build that may not skip clears the flag.
__global__ void k_freeze_check(GridDev *g, SlotDev a, const int64_t *n_ptr, int32_t skip) {
    if (threadIdx.x != 0) return;
    const bool f = skip && g->kind == kGridOpenSkip && g->valid && g->consumed && g->mark_ready && g->skip_ok &&
                   g->skipped == g->n && n_ptr[0] == g->n && g->law_k == a.k && g->law_gamma == a.gamma &&
                   g->law_bits == a.force_bits && g->law_box == a.box;
    g->frozen = f ? 1 : 0;
}

// ---------------------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int64_t per = kBlock) {
    int64_t b = (n + per - 1) / per;
    return unsigned(b < 1 ? 1 : b);
}

// Workgroups of a per-tile launch: one per tile for a plain call; a batch strides over its
// tiles with at most grid_cap workgroups (0: 8192), so empty capacity costs a table read, not a
// dispatch, or (grid_cap -1) takes one workgroup per tile as well.
unsigned tile_grid(const Slots &sl, int64_t ntiles) {
    if (ntiles < 1) return 1;
    if (sl.grid_cap < 0) return unsigned(ntiles);
    const int64_t cap = sl.grid_cap > 0 ? sl.grid_cap : 8192;
    return unsigned(sl.table && ntiles > cap ? cap : ntiles);
}

void launch_grid_build(const bdm_soa &s, const Slots &sl, int64_t capacity, bool f32_copy, const Ws &w,
                       hipStream_t st, bool allow_freeze) {
    const bool has_d = sl.table ? true : sl.one.has_d != 0;
    const double *d = has_d ? s.diam : nullptr;
    const int64_t nbt = (capacity + kBoundsTile - 1) / kBoundsTile;
    // plain open-space mechanics that skips stationary agents (needs the forces of the last step)
    const bool skip = !sl.table && !sl.one.periodic && sl.one.skip && !f32_copy && s.fx && s.fy && s.fz;
    if (!sl.table)
        hipLaunchKernelGGL(k_freeze_check, dim3(1), dim3(64), 0, st, w.grid, sl.one, s.n, int32_t(skip && allow_freeze));
    const int32_t kind = (!sl.table && sl.one.periodic) ? kGridPeriodic
                         : f32_copy                     ? kGridOpenF32
                         : skip                         ? kGridOpenSkip
                                                        : kGridOpen;
    const int64_t nt = (capacity + kBlock - 1) / kBlock;
    const int64_t nkg = (nt + kKeyTiles - 1) / kKeyTiles;
    // Plain calls other than spheroid steps (whose box edge follows the growing cells) key the
    // agents on the last lattice in the bounds pass, and again only if the lattice moved.  A
    // plain call reduces its bounds into one record per workgroup (at most kBoundsGroups).
    const bool spec = !sl.table && !f32_copy;
    const unsigned nbg = sl.table ? tile_grid(sl, nbt)
                         : spec   ? unsigned(nkg < kBoundsGroups ? (nkg < 1 ? 1 : nkg) : kBoundsGroups)
                                  : unsigned(nbt < kBoundsGroups ? (nbt < 1 ? 1 : nbt) : kBoundsGroups);
    if (spec)
        hipLaunchKernelGGL(k_key_spec, dim3(nbg), dim3(kBlock), 0, st, sl, nt, s.n, s.x, s.y, s.z, d, w.count, w.key,
                           w.rank, w.partials, w.tiles, w.lay.max_tiles, skip ? w.dirty : nullptr, w.moved);
    else
        hipLaunchKernelGGL(k_bounds, dim3(nbg), dim3(kBlock), 0, st, sl, nbt, s.n, s.x, s.y, s.z, d, w.partials,
                           w.tiles, w.lay.max_tiles, int32_t(sl.table ? 0 : 1));
    hipLaunchKernelGGL(k_finalize, dim3(unsigned(sl.nslots)), dim3(kBlock), 0, st, sl, s.n, w.partials, kind,
                       int64_t(sl.table ? 0 : nbg), int32_t(spec));
    const unsigned nb = tile_grid(sl, nt);
    // keys and bucket ranks (rank array), bucket starts, agent indices by bucket
    if (spec) {
        hipLaunchKernelGGL(k_count_clear, dim3(64), dim3(kBlock), 0, st, w.grid, w.count, int64_t(w.lay.nbuckets));
        hipLaunchKernelGGL(k_key_bucket, dim3(nbg), dim3(kBlock), 0, st, sl, nt, s.x, s.y, s.z, w.count, w.key,
                           w.rank, skip ? w.dirty : nullptr, w.moved, int32_t(1));
    } else {
        hipLaunchKernelGGL(k_key_bucket, dim3(tile_grid(sl, nkg)), dim3(kBlock), 0, st, sl, nt, s.x, s.y, s.z,
                           w.count, w.key, w.rank, skip ? w.dirty : nullptr, w.moved, int32_t(0));
    }
    const unsigned nbk = tile_grid(sl, nkg);
    launch_scan(w.count, w.bstart, nullptr, w.lay.nbuckets, w, 1, false, st, !sl.table);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nbk), dim3(kBlock), 0, st, sl, nt, w.key, w.rank, w.bstart, w.item,
                       capacity);
    // per-bucket order; plain calls keep each tile's first key in the rank-by-id area; crowded
    // buckets group ids in the scratch id array and agent indices in the division-flag array
    // (free during the build: the tile order is written there afterwards)
    uint32_t *tile_key = sl.table ? nullptr : w.rankid;
    const int periodic = sl.table ? 0 : sl.one.periodic;
    SoaIn in{s.x, s.y, s.z, d, s.adh, s.id, s.state, s.fx, s.fy, s.fz};
    SortOut o{w.pos4, f32_copy ? w.pos4f : nullptr, w.pos8, w.adh, w.ids, w.state, tile_key,
              skip ? w.dirty : nullptr, w.fprev};
    const int64_t nwg = (w.lay.nbuckets + kBlock / 64 - 1) / (kBlock / 64);
    hipLaunchKernelGGL(k_bucket_sort, dim3(unsigned(nwg)), dim3(kBlock), 0, st, sl, w.lay.nbuckets,
                       w.lay.max_boxes, in, w.key, w.bstart, w.item, w.tmpid, w.flagid, w.start, o, periodic,
                       capacity, w.crowd);
    hipLaunchKernelGGL(k_bucket_crowded, dim3(kCrowdedGroups), dim3(kBlock), 0, st, sl, w.lay.max_boxes, in, w.key,
                       w.bstart, w.tmpid, w.flagid, w.start, o, periodic, capacity, w.crowd);
    if (!sl.table && !sl.one.periodic) {
        const unsigned nto = blocks_for(w.lay.ntiles);
        hipLaunchKernelGGL(k_order_runs, dim3(nto), dim3(kBlock), 0, st, w.grid, tile_key, w.order_first,
                           w.order_last);
        hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, st, w.grid, w.order_first, w.order_last,
                           w.order_shift);
        hipLaunchKernelGGL(k_order_write, dim3(nto), dim3(kBlock), 0, st, w.grid, tile_key, w.order_shift,
                           w.flagid, int64_t(w.lay.ntiles));
    }
}

void launch_scan(uint32_t *in, uint32_t *out, const int64_t *len_ptr, int64_t max_len, const Ws &w,
                 int zero_in, bool prepare, hipStream_t st, bool build) {
    const unsigned nt = unsigned((max_len + kScanTile) / kScanTile);
    if (prepare)
        hipLaunchKernelGGL(k_scan_prepare, dim3(blocks_for(w.lay.max_tiles)), dim3(kBlock), 0, st, w.tiles,
                           w.lay.max_tiles, &w.grid[0].scan_ticket);
    hipLaunchKernelGGL(k_scan, dim3(nt), dim3(kBlock), 0, st, in, out, len_ptr, max_len, w.tiles,
                       &w.grid[0].scan_ticket, zero_in, &w.grid[0], int32_t(build));
}

void launch_read_agents(const bdm_soa &s, const ReadOut &o, hipStream_t st) {
    hipLaunchKernelGGL(k_read_agents, dim3(blocks_for(s.capacity)), dim3(kBlock), 0, st, s.n, s, o);
}

}  // namespace bdm
