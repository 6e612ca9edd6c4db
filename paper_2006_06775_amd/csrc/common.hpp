// common.hpp -- internals shared by the gfx950 kernels and the C-ABI layer of libbdm.so.
//
// Workspace layout, the per-population ("slot") parameter record and grid record,
// Philox4x64-10 (Salmon et al., SC'11) and the box coordinate rule of the uniform grid (paper
// Sec. 2.1).
//
// Every kernel works on "slots": independent populations packed into one set of arrays.  A
// plain call is one slot whose record travels by value in the kernel arguments; the batched
// form keeps a table of slot records and a tile -> slot map in device memory.  Both run the
// same per-agent code, so an agent's arithmetic does not depend on the other slots.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdm.h"

namespace bdm {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts of 64) = agents per tile
constexpr int kBoundsTile = 1024;    // agents per workgroup of the bounds reduction
constexpr int kScanItems = 8;        // items per thread in the decoupled look-back scan
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kBucketShift = 6;       // 64 consecutive boxes per bucket of the two-level sort
constexpr int kBucketBoxes = 1 << kBucketShift;
constexpr int kOrderBins = 8192;      // largest (y-pencil x z-plane) count of the tile order

constexpr double kPretestRadius = 1.0006;  // radius scale of the binary32 pre-test copy of a record

// The 8-byte pre-test record of a sphere in an open lattice of box edge b, in units of
// b / 2^14.  Per axis 16 bits: the sphere's box index c (the key's) mod 4 (2 bits) above its
// offset within the box, q = floor((v / b - c) * 2^14) clamped to [0, 2^14 - 1] (14 bits; v / b
// is formed as v times the rounded 1/b, which for |v / b| < 2^31, the lattice's int32 range,
// is within 2^-7 units of it).  Two spheres whose boxes differ by at most one along the axis
// then differ in these 16 bits, modulo 2^16 and read as a signed 16-bit value, by exactly
// (c_j - c_i) * 2^14 + q_j - q_i: their offset in units to within 1 + 2^-6.  The radius is
// rounded up and one unit added (at most 2^13 + 2 for r <= b / 2).
__device__ __forceinline__ uint32_t pre8_axis(double v, double inv_b, int c) {
    const double u = (v * inv_b - double(c)) * 16384.0;
    uint32_t q = u > 0.0 ? uint32_t(u) : 0u;
    q = q > 16383u ? 16383u : q;
    return (uint32_t(c) & 3u) << 14 | q;
}
__device__ __forceinline__ uint32_t pre8_radius(double r, double inv_b) {
    const double u = ceil(r * inv_b * 16384.0) + 1.0;
    return u < 65535.0 ? uint32_t(u) : 65535u;
}
constexpr uint32_t kScanSpinLimit = 1u << 22;  // polls before a look-back gives up

// Bit 31 of a box start in builds that may skip stationary agents: an agent that moved in the
// last step left or entered the box.  Starts are below 2^31 (capacity), so the bit is free; every
// reader of such a build masks it off (kStartMask).
constexpr uint32_t kStartDirty = 0x80000000u, kStartMask = 0x7FFFFFFFu;

// Philox draw purposes: counter word 0 = purpose + (attempt << 8).
enum : uint64_t { kRngInit = 1, kRngMove = 2, kRngRec = 3, kRngInf = 4, kRngDiv = 5, kRngApo = 6, kRngMig = 7 };

// Grid description and step bookkeeping of one slot (device memory, 256 bytes).
struct GridDev {
    double b;                       // box edge
    int32_t cmin[3];                // lattice coordinate of box 0
    int32_t dims[3];                // boxes per axis
    int64_t nboxes;                 // dims product
    int64_t n;                      // agents binned by the last build
    int32_t valid;                  // 1 when the last build succeeded
    uint32_t flags;                 // sticky BDM_FLAG_* bits
    uint32_t scan_ticket;           // dynamic tile index of the running scan (slot 0 only)
    uint32_t crowd_n;               // crowded buckets listed by the bucket sort of the running build
    unsigned long long div_nx;      // fast-division multipliers of dims[0] and dims[1]
    unsigned long long div_ny;
    unsigned long long sir_counts[3];
    int64_t sorted_base;            // first sorted position of this slot (start[box_off])
    double inv_b;                   // 1 / b, rounded (the pre-test records' scale)
    int32_t kind;                   // what the last build wrote (kGrid*)
    int32_t consumed;               // 1 once a plain mechanical step has used the build
    int32_t mark_ready;             // the last plain step skipped stationary agents and marked its movers
    int32_t skip_ok;                // this build may skip stationary agents (same lattice, marks ready)
    int64_t skipped;                // agents the last skipping step skipped
    double law_k, law_gamma, law_box;  // force law and requested box edge of the last build
    int32_t law_bits;
    int32_t frozen;                 // this build and its step are skipped whole (nothing moved)
    unsigned long long skip_acc;    // a skipping step's skipped count while its workgroups sum it (0 between steps)
    uint32_t consume_ticket;        // workgroups of that sum done (0 between steps)
    unsigned long long sir_acc[3];  // a SIR step's S/I/R totals while its workgroups sum them (0 between steps)
    uint32_t sir_ticket;            // workgroups of that sum done (0 between steps)
    int32_t rekey;                  // a build whose keys on the last lattice do not stand: key again
    int32_t rezero;                 // ... and clear the histogram those keys counted into first
};
static_assert(sizeof(GridDev) <= 256, "grid record must fit its slot");

// What a grid build wrote, so that a step can refuse a build it cannot use: open space with the
// 8-byte pre-test records, the same plus the binary32 copies (spheroid steps), or the periodic
// (SIR) lattice, which writes no pre-test records.
enum : int32_t { kGridNone = 0, kGridOpen = 1, kGridOpenF32 = 2, kGridPeriodic = 3, kGridOpenSkip = 4 };

// A plain skipping build whose step changes nothing: the last step skipped every agent (so
// none moved), and the force law, requested box edge and live count are the same.  Every kernel
// of the build and of its mechanical step then leaves the workspace and the agents as they are.
__device__ __forceinline__ bool frozen_plain(const GridDev *g, bool table) { return !table && g->frozen; }

// Parameters and placement of one slot.
struct SlotDev {
    int64_t agent_off;   // first array index of the slot (multiple of kBoundsTile in a batch)
    int64_t capacity;    // agents the slot may hold
    int64_t box_off;     // first histogram entry of the slot
    int64_t max_boxes;   // histogram entries reserved for the slot
    int64_t steps_left;  // batch: steps still to run (the slot idles at 0); plain: 1
    double k, gamma, dt, max_disp;
    double box;          // requested box edge (<= 0: largest diameter)
    double L;            // periodic cube edge
    float kf, gf;        // binary32 copies of k and gamma
    int32_t force_bits;  // 64 or 32
    int32_t periodic;
    int32_t nb;          // periodic boxes per axis
    int32_t has_d;       // spheres (diameters present) or points
    int32_t skip;        // plain mechanics: skip agents in stationary regions
};

// Byte offsets of every workspace region (256-byte aligned).  `slots` = 0 is a plain
// workspace (one grid record, slot passed by value); > 0 is a batch of that many slots.
struct WsLayout {
    size_t grid, slots, tilemap, bucketmap, partials, count, bstart, start, tiles, key, rank, item, tmpid, pos4, pos4f, pos8,
        adh, ids, state, flagid, rankid, order_bins, crowd, dirty, moved, fprev, tileskip;
    size_t total;
    int64_t capacity, max_boxes, max_tiles, nslots, ntiles, nbuckets;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline bool ws_layout(int64_t capacity, int64_t max_boxes, int64_t slots, WsLayout *L) {
    if (capacity < 0 || max_boxes < 0 || slots < 0 || slots > BDM_MAX_SLOTS ||
        capacity > (int64_t(1) << 32) - 2 - kBoundsTile || max_boxes > (int64_t(1) << 32) - 2)
        return false;
    size_t cap = size_t(capacity), mb = size_t(max_boxes);
    const size_t nbk = (mb >> kBucketShift) + 1;  // buckets covering box indices 0..max_boxes
    size_t longest = cap > nbk ? cap : nbk;       // longest scan: bucket counts or division flags
    size_t tiles = (longest + 1 + kScanTile - 1) / kScanTile + 1;
    size_t ngrid = slots > 0 ? size_t(slots) : 1;
    size_t ntile = (cap + kBlock - 1) / kBlock;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    L->grid = take(256 * ngrid);
    L->slots = take(slots > 0 ? sizeof(SlotDev) * size_t(slots) : 0);
    L->tilemap = take(slots > 0 ? 4 * ntile : 0);
    L->bucketmap = take(slots > 0 ? 4 * nbk : 0);
    L->partials = take(64 * ((cap + kBoundsTile - 1) / kBoundsTile + 1));
    L->count = take(4 * (nbk + 1));
    L->bstart = take(4 * (nbk + 1));
    L->start = take(4 * (mb + 3)) + 4;  // one spare entry on each side (16-byte reads of kb - 1 .. kb + 2)
    L->tiles = take(8 * tiles);
    L->key = take(4 * cap);
    L->rank = take(4 * cap);
    L->item = take(4 * cap);
    L->tmpid = take(4 * cap);
    L->pos4 = take(32 * cap);
    L->pos4f = take(16 * cap);
    L->pos8 = take(8 * cap);
    L->adh = take(8 * cap);
    L->ids = take(4 * cap);
    L->state = take(cap);
    L->flagid = take(4 * (cap + 1));
    L->rankid = take(4 * (cap + 1));
    L->order_bins = take(3 * 4 * size_t(kOrderBins));
    L->crowd = take(4 * (nbk + 1));  // buckets the bucket sort hands to the crowded-box ranking
    L->dirty = take(mb + 1);         // stationary skip: boxes a mover left or entered
    L->moved = take(cap);            // stationary skip: agents that moved in the last step
    L->fprev = take(24 * cap);       // stationary skip: the last step's force, in the new sorted order
    L->tileskip = take(4 * (kBlock / 64) * ntile);  // stationary skip: agents skipped per wavefront of a tile
    L->total = off;
    L->capacity = capacity;
    L->max_boxes = max_boxes;
    L->max_tiles = int64_t(tiles);
    L->nslots = slots;
    L->ntiles = int64_t(ntile);
    L->nbuckets = int64_t(nbk);
    return true;
}

// Typed views of one workspace.
struct Ws {
    GridDev *grid;       // [max(1, nslots)]
    SlotDev *slots;      // batch only
    int32_t *tilemap;    // batch only: tile -> slot (-1 = none)
    int32_t *bucketmap;  // batch only: bucket of 64 boxes -> slot owning it (-1 = none)
    double *partials;    // bounds reduction: 8 values per kBoundsTile agents
    uint32_t *count;     // agents per bucket of 64 boxes (scan input, kept zero between builds)
    uint32_t *bstart;    // first sorted position of each bucket
    uint32_t *start;     // first sorted position of each box
    unsigned long long *tiles;
    uint32_t *key, *rank, *item, *tmpid;
    double4 *pos4;
    float4 *pos4f;       // binary32 filter copy of pos4 (crowded mechanics: spheroid steps)
    uint2 *pos8;         // 8-byte fixed-point filter record (mechanics slots)
    double *adh;
    uint32_t *ids;
    uint8_t *state;
    uint32_t *flagid, *rankid;
    uint32_t *order_first, *order_last, *order_shift;  // tile-order runs per bin (plain calls)
    uint32_t *crowd;     // crowded buckets of the running build (bucket sort -> crowded-box ranking)
    uint8_t *dirty;      // stationary skip: per box, a mover left or entered it since the last build
    uint8_t *moved;      // stationary skip: per agent (sorted order of the last build), it moved
    double *fprev;       // stationary skip: fx, fy, fz of the last step, in this build's sorted order
    uint32_t *tileskip;  // stationary skip: agents skipped per tile of the last step
    WsLayout lay;
};

inline Ws ws_view(void *base, const WsLayout &L) {
    char *p = static_cast<char *>(base);
    Ws w;
    w.grid = reinterpret_cast<GridDev *>(p + L.grid);
    w.slots = L.nslots > 0 ? reinterpret_cast<SlotDev *>(p + L.slots) : nullptr;
    w.tilemap = L.nslots > 0 ? reinterpret_cast<int32_t *>(p + L.tilemap) : nullptr;
    w.bucketmap = L.nslots > 0 ? reinterpret_cast<int32_t *>(p + L.bucketmap) : nullptr;
    w.partials = reinterpret_cast<double *>(p + L.partials);
    w.count = reinterpret_cast<uint32_t *>(p + L.count);
    w.bstart = reinterpret_cast<uint32_t *>(p + L.bstart);
    w.start = reinterpret_cast<uint32_t *>(p + L.start);
    w.tiles = reinterpret_cast<unsigned long long *>(p + L.tiles);
    w.key = reinterpret_cast<uint32_t *>(p + L.key);
    w.rank = reinterpret_cast<uint32_t *>(p + L.rank);
    w.item = reinterpret_cast<uint32_t *>(p + L.item);
    w.tmpid = reinterpret_cast<uint32_t *>(p + L.tmpid);
    w.pos4 = reinterpret_cast<double4 *>(p + L.pos4);
    w.pos4f = reinterpret_cast<float4 *>(p + L.pos4f);
    w.pos8 = reinterpret_cast<uint2 *>(p + L.pos8);
    w.adh = reinterpret_cast<double *>(p + L.adh);
    w.ids = reinterpret_cast<uint32_t *>(p + L.ids);
    w.state = reinterpret_cast<uint8_t *>(p + L.state);
    w.flagid = reinterpret_cast<uint32_t *>(p + L.flagid);
    w.rankid = reinterpret_cast<uint32_t *>(p + L.rankid);
    w.crowd = reinterpret_cast<uint32_t *>(p + L.crowd);
    w.dirty = reinterpret_cast<uint8_t *>(p + L.dirty);
    w.moved = reinterpret_cast<uint8_t *>(p + L.moved);
    w.fprev = reinterpret_cast<double *>(p + L.fprev);
    w.tileskip = reinterpret_cast<uint32_t *>(p + L.tileskip);
    w.order_first = reinterpret_cast<uint32_t *>(p + L.order_bins);
    w.order_last = w.order_first + kOrderBins;
    w.order_shift = w.order_last + kOrderBins;
    w.lay = L;
    return w;
}

// Slot addressing handed to every kernel by value.
struct Slots {
    const SlotDev *table;      // batch: slot records; plain: nullptr (use `one`)
    const int32_t *tilemap;    // batch: tile -> slot; plain: nullptr (every tile is slot 0)
    const int32_t *bucketmap;  // batch: bucket -> owning slot or -1; plain: nullptr (all owned)
    GridDev *grids;            // grid record per slot
    int64_t nslots;            // 1 for a plain call
    SlotDev one;               // the plain call's slot record
    int32_t grid_cap;          // batch: workgroups of the per-tile launches (they stride over the tiles)
};

__device__ __forceinline__ int slot_of_tile(const Slots &sl, int64_t tile) {
    return sl.tilemap ? sl.tilemap[tile] : 0;
}

__device__ __forceinline__ SlotDev slot_record(const Slots &sl, int slot) {
    return sl.table ? sl.table[slot] : sl.one;
}

// Live count of a slot clamped to its capacity (a corrupted count must not index out of bounds).
__device__ __forceinline__ int64_t live_count(const int64_t *n_ptr, int slot, int64_t capacity) {
    const int64_t n = n_ptr[slot];
    return n < 0 ? 0 : (n > capacity ? capacity : n);
}

// ---------------------------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------------------------

// Philox4x64-10: per round, words 0 and 2 are multiplied (64x64 -> 128) by the two round
// multipliers; the new block is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
// lo(M0*c0)); the key advances by the two Weyl increments before every round but the first.
struct Block4 {
    uint64_t w[4];
};

__device__ __forceinline__ Block4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                         uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return Block4{{c0, c1, c2, c3}};
}

__device__ __forceinline__ Block4 draw(uint64_t seed, uint64_t salt, uint64_t purpose,
                                       uint64_t attempt, uint64_t id, uint64_t step) {
    return philox(purpose + (attempt << 8), id, step, 0, seed, salt);
}

// Uniform binary64 in [0, 1) from the top 53 bits of a word (exact).
__device__ __forceinline__ double u01(uint64_t w) {
    return double(w >> 11) * 0x1.0p-53;
}

// Bernoulli threshold prepared on the host: mode 0 never, 1 compare, 2 always.
struct Threshold {
    uint64_t t;
    int32_t mode;
};

__device__ __forceinline__ bool bernoulli(uint64_t w, Threshold th) {
    return th.mode == 2 || (th.mode == 1 && w < th.t);
}

// Box coordinate along one axis: floor(v / b) relative to the grid origin (open space) or as
// is (periodic cube), clamped into [0, nb - 1].  In open space the clamp never binds (the
// origin and dims come from the min/max of the same positions) and only guards memory.
__device__ __forceinline__ int box_coord(double v, double b, int cmin, int nb, bool periodic) {
    double f = floor(v / b);
    if (!periodic) f -= double(cmin);
    if (f < 0.0) f = 0.0;
    if (f > double(nb - 1)) f = double(nb - 1);
    return int(f);
}

// Division of a 32-bit value by a 32-bit divisor d >= 1 through the multiplier M = (2^64 - 1)/d
// + 1 (Lemire, Kaser and Kurz, "Faster remainder by direct computation", 2019): a / d is the
// high 64 bits of M * a, exact for every 32-bit a; d = 1 (M wraps to 0) is handled apart.
__host__ __device__ __forceinline__ unsigned long long fastdiv_magic(uint32_t d) {
    return d <= 1 ? 0ull : ~0ull / d + 1ull;
}
__device__ __forceinline__ uint32_t fastdiv(uint32_t a, unsigned long long m) {
    return m ? uint32_t(__umul64hi(m, a)) : a;
}

// Wavefront-wide inclusive prefix sum (64 lanes).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, uint32_t(__shfl_xor(int(v), d, 64)));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, uint32_t(__shfl_xor(int(v), d, 64)));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Workgroup `bid` of `nblocks` is dispatched to XCD bid % 8; give every XCD one contiguous
// eighth of the tiles so that neighbouring rows of the box-sorted arrays share its L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nblocks) {
    const uint32_t per = nblocks / 8, rem = nblocks % 8, x = bid % 8, idx = bid / 8;
    return x * per + (x < rem ? x : rem) + idx;
}


// Conservative contact pre-test in binary32 (every real contact passes; see pretest_slack).
__device__ __forceinline__ bool maybe_touch(const float4 &a, const float4 &c, float slack) {
    const float dx = a.x - c.x, dy = a.y - c.y, dz = a.z - c.z;
    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    const float s = a.w + c.w;  // scaled radii
    return d2 < __builtin_fmaf(s, s, slack);
}

// Absolute slack of the binary32 pre-test of a slot.  Stored coordinates are relative to the
// lattice origin o and lie within M = (largest dims + 1) * b of it (plus the rounding of x / b
// at the lattice edges), so each is off by at most 2^-24 M and a difference by at most
// e = 2^-23 (M + b) (with b >= r_i + r_j >= the distance of any contact).  Then the binary32
// squared distance, one product and two fused multiply-adds, exceeds the true one by at most
// (1 + 2^-24)^3 (2 sqrt(3) d e + 3 e^2); with e doubled, 4 (b + e) e bounds that.  The copy's
// radii are scaled by 1.0006, so after the rounding of the radii, of their sum and of the fused
// square-and-add the threshold is at least 1.0012 (r_i + r_j)^2 + slack: the relative margin
// covers the rounding of every exact law's own contact test.  So no pair that the exact law
// counts as a contact can fail the pre-test.
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

}  // namespace bdm
