// k_mech.hip -- mechanical step on gfx950: 27-box gather, sphere-sphere force, adherence gate,
// clamp and synchronous integration in one kernel (paper Sec. 2.1 "calculate mechanical forces"
// agent operation; Zubler & Douglas force model shared with Cortex3D, Sec. 3.4).
//
// One lane per agent in box-sorted order.  The 27 neighbour boxes are 9 contiguous key runs
// (dz, dy in {-1, 0, 1}; dx = -1..+1 adjacent in key space because x varies fastest), so
// candidates arrive in ascending (key, id) order -- the canonical summation order.  For agents
// in sparsely filled boxes, boxes that no sphere in them can reach are dropped from the ends of
// these runs (about a third of the 27 at uniform density; see load_runs), which removes only
// non-contacts.
//
// The work is split in two so that the wavefront does not pay the expensive exact law for
// every candidate of every lane:
//   1. candidate stream: each lane walks its runs as one flattened stream (run table in LDS)
//      and keeps the candidates that pass a cheap conservative squared-distance test in a small
//      per-lane queue in LDS;
//   2. exact pass: the queued candidates, still in canonical order, are re-read and evaluated
//      exactly as the definition spells the law (binary64 or binary32) and summed.  At the end
//      of the stream the wavefront evaluates all its lanes' queued pairs together, one pair per
//      lane (exact_packed); each lane still adds its own terms in its own order.
// The packed record holds (x, y, z, r) with r = d/2.
//
// Schedule: a tile is 256 consecutive sorted agents.  A plain call processes its tiles in the
// pencil order built with the grid (rows grouped 16 at a time and swept along z) and gives each
// XCD one contiguous part of that sequence, so the three z-planes a tile reads stay in that
// XCD's L2.  Outputs are written with non-temporal stores: they are not read again in the step.
#include "kernels.hpp"
#include "record8.hpp"

namespace bdm {

constexpr int kQueue = 8;          // queued candidates per lane before an exact pass
constexpr int kQueueCrowded = 6;   // the same for crowded populations (must differ from kQueue)
constexpr uint32_t kCullMaxBox = 8;  // agents in a box up to which its agents drop out-of-reach boxes

// The pair law for agent i with record p and a candidate j at offset (dx, dy, dz) = p - q with
// radius rj: whether the spheres overlap and, if so, the term (tx, ty, tz) that j adds to the
// force on i.  A non-contact adds nothing.  Coincident centres add nothing either; kCoincident
// (the traced kernels) reports them as the contact they are, with a term of +0 (a running sum
// that starts at +0 never becomes -0, so adding +0 changes no bit).
template <bool F32, bool kCoincident = false>
__device__ __forceinline__ bool pair_term(const double4 &p, double dx, double dy, double dz, double rj, float rif,
                                          const SlotDev &a, double &tx, double &ty, double &tz) {
    const double ri = p.w;
    if constexpr (!F32) {
        const double s = ri + rj;
        const double dist = __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
        const double delta = s - dist;
        if constexpr (kCoincident) {
            if (delta > 0.0 && dist == 0.0) {
                tx = ty = tz = 0.0;
                return true;
            }
        }
        if (!(delta > 0.0) || dist == 0.0) return false;
        const double rhat = (ri * rj) / s;
        const double F = a.k * delta - a.gamma * __builtin_sqrt(rhat * delta);
        const double sc = F / dist;
        tx = sc * dx;
        ty = sc * dy;
        tz = sc * dz;
    } else {
        const float dxf = float(dx), dyf = float(dy), dzf = float(dz);
        const float dist = __builtin_sqrtf((dxf * dxf + dyf * dyf) + dzf * dzf);
        const float rjf = float(rj);
        const float sf = rif + rjf;
        const float delta = sf - dist;
        if constexpr (kCoincident) {
            if (delta > 0.0f && dist == 0.0f) {
                tx = ty = tz = 0.0;
                return true;
            }
        }
        if (!(delta > 0.0f) || dist == 0.0f) return false;
        const float rhat = (rif * rjf) / sf;
        const float F = a.kf * delta - a.gf * __builtin_sqrtf(rhat * delta);
        const float sc = F / dist;
        tx = double(sc * dxf);
        ty = double(sc * dyf);
        tz = double(sc * dzf);
    }
    return true;
}

template <bool F32, bool kCoincident>
__device__ __forceinline__ bool exact_pair(const double4 &p, double dx, double dy, double dz, double rj, float rif,
                                           const SlotDev &a, double &fx, double &fy, double &fz) {
    double tx, ty, tz;
    if (pair_term<F32, kCoincident>(p, dx, dy, dz, rj, rif, a, tx, ty, tz)) {
        fx = fx + tx;
        fy = fy + ty;
        fz = fz + tz;
        return true;
    }
    return false;
}

// Contact record of a traced step (a test hook): every contact the step adds, in the order it
// is added, as a count and an order-sensitive hash of the partners' sorted positions within the
// slot (h = h * 0x9E3779B1 + position + 1, modulo 2^32).  NoTrace compiles to nothing; the
// traced kernels are separate instantiations of the same code, so their contact decisions are
// the step's own.
struct NoTrace {
    static constexpr bool kOn = false;
    __device__ __forceinline__ void hit(uint32_t) {}
};
struct Trace {
    static constexpr bool kOn = true;
    uint32_t unit, base, n, h;  // candidate offsets are unit * (base + position)
    __device__ __forceinline__ void hit(uint32_t u) {
        n += 1u;
        h = h * 0x9E3779B1u + (u / unit - base + 1u);
    }
};

// Key range [lo, hi) of row r (dz = r / 3 - 1, dy = r % 3 - 1) of the 27 boxes around the box
// (cx, cy, cz): boxes x0..x1 of that row, clipped to the lattice; an empty range off it.
__device__ __forceinline__ void row_range(const GridDev *__restrict__ g, const uint32_t *__restrict__ start, int cx,
                                          int cy, int cz, int r, uint32_t &lo, uint32_t &hi) {
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    const int zz = cz + r / 3 - 1, yy = cy + r % 3 - 1;
    lo = hi = 0;
    if (zz < 0 || zz >= nz || yy < 0 || yy >= ny) return;
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < nx - 1 ? cx + 1 : nx - 1;
    const uint32_t kb = uint32_t(x0) + uint32_t(nx) * (uint32_t(yy) + uint32_t(ny) * uint32_t(zz));
    lo = start[kb] & kStartMask;
    hi = start[kb + uint32_t(x1 - x0) + 1u] & kStartMask;
}

// The candidate runs of the agent with record p in box (cx, cy, cz), in canonical order, into
// column t of s_run as (first record offset in units of kUnit, length), the non-empty runs
// first, then (0, 0); returns the candidate count.
//
// A box of the 27 is dropped when no sphere in it can reach the agent: every sphere has
// r <= b / 2 (the box edge is at least the largest diameter), so a contact needs a centre
// within r_p + b / 2 of p, and the box's nearest point is farther than that.  The distance to a
// box follows from the gaps between p and the faces of its own box (a candidate's key puts its
// centre beyond the shared face).  The test keeps a relative margin of 1e-3 on the squared
// reach, far above the rounding of the gaps and of either exact contact test, so every box
// holding a contact is kept.  Dropped boxes sit at the ends of a row (a row's middle box is the
// nearest of the three) or are the whole row, so each row stays one contiguous run, and the
// kept candidates keep their order.  Dropping them changes no sum: a non-contact adds nothing.
// Where the lanes of a wavefront walk nearly the same runs (agents packed into a few crowded
// boxes), they walk the union of their runs together instead: row r's union is
// [lo[r], hi[r]) in record indices, and `coop` says the wavefront does so (uniform).
struct RowUnion {
    uint32_t lo[9], hi[9];
    bool coop;
};

// kSkip (a build that skips stationary agents): the starts carry the boxes' marks in bit 31
// (kStartDirty); they are masked off, and `dirty` says whether any box the agent keeps (any box
// that can hold a sphere touching it) is marked.
template <uint32_t kUnit, bool kCoop, bool kSkip = false>
__device__ __forceinline__ uint32_t load_runs(const GridDev *__restrict__ g, const uint32_t *__restrict__ start,
                                              int cx, int cy, int cz, const double4 &p, bool live,
                                              uint2 (*s_run)[kBlock], int t, RowUnion &un, bool *dirty = nullptr) {
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    const double b = g->b;
    const double ox = double(g->cmin[0]) + double(cx), oy = double(g->cmin[1]) + double(cy),
                 oz = double(g->cmin[2]) + double(cz);
    const double gxl = fmax(p.x - ox * b, 0.0), gxr = fmax((ox + 1.0) * b - p.x, 0.0);
    const double gyl = fmax(p.y - oy * b, 0.0), gyr = fmax((oy + 1.0) * b - p.y, 0.0);
    const double gzl = fmax(p.z - oz * b, 0.0), gzr = fmax((oz + 1.0) * b - p.z, 0.0);
    const double gx2l = gxl * gxl, gx2r = gxr * gxr;
    // every row loads its bounds (a row off the lattice reads a clamped, valid box and is then
    // emptied), so the loads are issued together, without branches: one 16-byte load of the
    // starts of boxes kb - 1 .. kb + 2 per row, through a range-checked buffer resource based
    // one entry before the slot's starts (the workspace holds memory on both sides of them)
    const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t *>(start - 1), 0, uint32_t(g->nboxes + 3) * 4u, 0x00020000);
    __attribute__((ext_vector_type(4))) uint32_t v[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const int yc = min(max(cy + r % 3 - 1, 0), ny - 1), zc = min(max(cz + r / 3 - 1, 0), nz - 1);
        const uint32_t kb = uint32_t(cx) + uint32_t(nx) * (uint32_t(yc) + uint32_t(ny) * uint32_t(zc));
        v[r] = __builtin_amdgcn_raw_buffer_load_b128(srs, kb * 4u, 0, 0);  // kb - 1 .. kb + 2
    }
    uint32_t marks[9];  // (kSkip) row r: bit 0, 1, 2 = box kb - 1, kb, kb + 1 marked
    if constexpr (kSkip) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            marks[r] = (v[r][0] >> 31) | (v[r][1] >> 31) << 1 | (v[r][2] >> 31) << 2;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[r][e] &= kStartMask;
        }
    }
    // Dropping boxes pays where an agent shares its box with few others.  Agents of one box walk
    // the same runs in step when none are dropped, so a wavefront's lanes read the same records
    // together; dropping boxes per agent breaks that, which costs more than it saves in crowded
    // boxes (measured: at about one agent per box dropping is faster even for boxes of four; at
    // a few hundred per box it is a third slower).
    const double reach = p.w + 0.5 * b;
    const double T = v[4][2] - v[4][1] <= kCullMaxBox ? (reach * reach) * 1.001 : __builtin_inf();
    uint32_t lo[9], hi[9];
    bool any_mark = false;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const int dz = r / 3 - 1, dy = r % 3 - 1;
        const int zz = cz + dz, yy = cy + dy;
        const double gy = dy < 0 ? gyl : gyr, gz = dz < 0 ? gzl : gzr;
        const double gyz = (dy != 0 ? gy * gy : 0.0) + (dz != 0 ? gz * gz : 0.0);
        const bool in = zz >= 0 && zz < nz && yy >= 0 && yy < ny && gyz < T;
        const bool left = cx > 0 && gyz + gx2l < T, right = cx < nx - 1 && gyz + gx2r < T;
        lo[r] = in && live ? (left ? v[r][0] : v[r][1]) : 0u;
        hi[r] = in && live ? (right ? v[r][3] : v[r][2]) : 0u;
        if constexpr (kSkip) {
            const uint32_t kept = in ? (2u | (left ? 1u : 0u) | (right ? 4u : 0u)) : 0u;
            any_mark |= (marks[r] & kept) != 0u;
        }
    }
    if constexpr (kSkip) *dirty = any_mark;
    un.coop = false;
    if constexpr (kCoop) {
        // every lane takes part (the wavefront's lanes are all active here)
        uint32_t own = 0, total = 0;
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const bool ne = hi[r] > lo[r];
            un.lo[r] = wave_min(ne ? lo[r] : 0xFFFFFFFFu);
            un.hi[r] = wave_max(ne ? hi[r] : 0u);
            own += hi[r] - lo[r];
            total += un.hi[r] > un.lo[r] ? un.hi[r] - un.lo[r] : 0u;
        }
        // together when the union is at most twice the longest own stream
        un.coop = total <= 2u * wave_max(own);
        if (un.coop) {  // the table holds each row in place: (first, end) record indices
#pragma unroll
            for (int r = 0; r < 9; ++r) s_run[r][t] = make_uint2(lo[r], hi[r]);
            return own;
        }
    }
    // non-empty runs to the front in order, empty ones to the back: a permutation of the 9 rows
    uint32_t cnt = 0, k = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const uint32_t len = hi[r] - lo[r];
        const bool ne = len != 0u;
        const uint32_t pos = ne ? k : 8u - (uint32_t(r) - k);
        s_run[pos][t] = ne ? make_uint2(lo[r] * kUnit, len) : make_uint2(0u, 0u);
        k += ne ? 1u : 0u;
        cnt += len;
    }
    return cnt;
}

// Coarse all-pairs pre-test of a cooperative walk on the matrix cores: for the 64 agents of a
// wavefront and a chunk of 64 candidate records, which pairs may pass maybe_touch.  With
// coordinates relative to the wavefront's origin o (lane 0's record), a' = a - o, c' = c - o,
// the test value is the dot product of the agent vector (a'x, a'y, a'z, a.w, 1, A) and the
// candidate vector (-2c'x, -2c'y, -2c'z, -2c.w, C, 1), with
//   A = |a'|^2 - a.w^2 - slack - k (|a'|^2 + a.w^2 + slack),  C = |c'|^2 - c.w^2 - k (|c'|^2 + c.w^2),
// which is |a' - c'|^2 - (a.w + c.w)^2 - slack - k (|a'|^2 + a.w^2 + |c'|^2 + c.w^2 + slack):
// maybe_touch's condition less a margin.  A pair is kept when the value is negative.  Each
// rounding on either side (the shift, maybe_touch's own arithmetic, the matrix product, which
// adds each pair of products with one rounding, measured) is below 2^-23 of these magnitudes,
// and about 32 of them add up, so the margin k = 2^-14 keeps every pair maybe_touch passes; it
// widens the kept shell by about k (|a'|^2 + |c'|^2) / (a.w + c.w)^2, below 0.1 % here.  The
// survivors still go through maybe_touch, so the queue holds exactly what the plain walk puts
// there, in the same order.
// v_mfma_f32_32x32x2f32: lane l gives A[l % 32][l / 32] and B[l / 32][l % 32]; output element v
// of lane l is D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].  Candidates are the rows (two blocks
// of 32), agents the columns (two blocks of 32); K = 6 takes three products per block.
constexpr float kCoarseMargin = 0x1p-14f;
typedef float mfma16f __attribute__((ext_vector_type(16)));

struct CoarseAgents {
    float ox, oy, oz;  // wavefront origin
    float b[2][3];     // B operand of agent block ab, product s: component 2s + (lane / 32)
};

__device__ __forceinline__ float first_lane(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// (every lane of the wavefront takes part)
__device__ __forceinline__ CoarseAgents coarse_agents(const float4 &pf, float slack, int lane) {
    CoarseAgents ca;
    ca.ox = first_lane(pf.x);
    ca.oy = first_lane(pf.y);
    ca.oz = first_lane(pf.z);
    const float ax = pf.x - ca.ox, ay = pf.y - ca.oy, az = pf.z - ca.oz, aw = pf.w;
    const float a2 = __builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax)), w2 = aw * aw;
    const float aA = ((a2 - w2) - slack) - kCoarseMargin * ((a2 + w2) + slack);
    const bool hi = lane >= 32;
#pragma unroll
    for (int ab = 0; ab < 2; ++ab) {
        const int src = ab * 32 + (lane & 31);
        const float sx = __shfl(ax, src, 64), sy = __shfl(ay, src, 64), sz = __shfl(az, src, 64);
        const float sw = __shfl(aw, src, 64), sa = __shfl(aA, src, 64);
        ca.b[ab][0] = hi ? sy : sx;
        ca.b[ab][1] = hi ? sw : sz;
        ca.b[ab][2] = hi ? sa : 1.0f;
    }
    return ca;
}

// Bit e of the result: candidate e of the chunk staged at stage[0..63] may touch this lane's
// agent (every lane of the wavefront takes part; entries past the chunk's end give bits that
// the caller masks off).
__device__ __forceinline__ uint64_t coarse_mask(const CoarseAgents &ca, const float4 *stage, int lane) {
    const int h = lane >> 5;
    uint32_t mine[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const float4 c = stage[cb * 32 + (lane & 31)];
        const float cx = c.x - ca.ox, cy = c.y - ca.oy, cz = c.z - ca.oz, cw = c.w;
        const float c2 = __builtin_fmaf(cz, cz, __builtin_fmaf(cy, cy, cx * cx)), w2 = cw * cw;
        const float cC = (c2 - w2) - kCoarseMargin * (c2 + w2);
        const float a0 = -2.0f * (h ? cy : cx), a1 = -2.0f * (h ? cw : cz), a2 = h ? 1.0f : cC;
        uint32_t w[2];
#pragma unroll
        for (int ab = 0; ab < 2; ++ab) {
            mfma16f acc = {};
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, ca.b[ab][0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, ca.b[ab][1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, ca.b[ab][2], acc, 0, 0, 0);
            uint32_t bits = 0u;
#pragma unroll
            for (int v = 0; v < 16; ++v) {  // the sign bit: negative values are kept
                const float x = acc[v];  // (a bit cast of acc[v] itself would read element 0)
                bits |= (__float_as_uint(x) >> 31) << (8 * (v / 4) + (v % 4));
            }
            w[ab] = bits << (4 * h);
        }
        // this lane's agent is column lane % 32 of block lane / 32: its rows of the other half
        // are with lane ^ 32, which sends its block-(1 - its half) word
        const uint32_t other = uint32_t(__shfl_xor(int(h ? w[0] : w[1]), 32, 64));
        mine[cb] = (h ? w[1] : w[0]) | other;
    }
    return uint64_t(mine[0]) | (uint64_t(mine[1]) << 32);
}

__device__ __forceinline__ uint64_t low_bits(uint32_t n) { return n >= 64u ? ~0ull : (1ull << n) - 1ull; }

// Packed-record loads by candidate offset u in units of kUnit.  RecBuf: raw buffer resources
// with 32-bit byte offsets when the sorted arrays are below 4 GiB (u is 16 times the sorted
// position: the binary64 record sits at byte 2u, the 8-byte record at u / 2); out-of-range
// offsets read zero.  RecGlobal: plain indices.  full() reads the binary64 record (x, y, z, r),
// pre() the 8-byte pre-test record.
struct RecBuf {
    static constexpr uint32_t kUnit = 16;
    static constexpr bool kF32Copy = false;
    using Pre = uint2;
    void *base, *base8;
    uint32_t bytes;  // of the binary64 records (the 8-byte records are a quarter of it)
    __device__ __forceinline__ double4 full(uint32_t u) const {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, 0x00020000);
        const uint32_t off = u * 2u;
        const auto lo = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const auto hi = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
        const double2 a = __builtin_bit_cast(double2, lo), c = __builtin_bit_cast(double2, hi);
        return make_double4(a.x, a.y, c.x, c.y);
    }
    __device__ __forceinline__ uint2 pre(uint32_t u) const {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base8, 0, bytes / 4u, 0x00020000);
        return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, u / 2u, 0, 0));
    }
    static __device__ __forceinline__ bool touch(const uint2 &a, const uint2 &c, float) { return touch8i(own8(a), c); }
};
// The binary32 copies instead (the crowded kernel: its walk is bound by VALU, not by memory).
struct RecBuf4 {
    static constexpr uint32_t kUnit = 16;
    static constexpr bool kF32Copy = true;
    using Pre = float4;
    void *base, *basef;
    uint32_t bytes;  // of the binary64 records (the binary32 copy is half as long)
    __device__ __forceinline__ double4 full(uint32_t u) const {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, 0x00020000);
        const uint32_t off = u * 2u;
        const auto lo = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const auto hi = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
        const double2 a = __builtin_bit_cast(double2, lo), c = __builtin_bit_cast(double2, hi);
        return make_double4(a.x, a.y, c.x, c.y);
    }
    __device__ __forceinline__ float4 pre(uint32_t u) const {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(basef, 0, bytes / 2u, 0x00020000);
        return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, u, 0, 0));
    }
    static __device__ __forceinline__ bool touch(const float4 &a, const float4 &c, float slack) {
        return maybe_touch(a, c, slack);
    }
};
struct RecGlobal {
    static constexpr uint32_t kUnit = 1;
    static constexpr bool kF32Copy = false;
    using Pre = uint2;
    const double4 *__restrict__ p;
    const uint2 *__restrict__ p8;
    __device__ __forceinline__ double4 full(uint32_t u) const { return p[u]; }
    __device__ __forceinline__ uint2 pre(uint32_t u) const { return p8[u]; }
    static __device__ __forceinline__ bool touch(const uint2 &a, const uint2 &c, float) { return touch8i(own8(a), c); }
};
struct RecGlobal4 {
    static constexpr uint32_t kUnit = 1;
    static constexpr bool kF32Copy = true;
    using Pre = float4;
    const double4 *__restrict__ p;
    const float4 *__restrict__ pf;
    __device__ __forceinline__ double4 full(uint32_t u) const { return p[u]; }
    __device__ __forceinline__ float4 pre(uint32_t u) const { return pf[u]; }
    static __device__ __forceinline__ bool touch(const float4 &a, const float4 &c, float slack) {
        return maybe_touch(a, c, slack);
    }
};


// Walk over a lane's packed runs (column col of s_run): next() returns the offset of the next
// candidate in canonical order.  It has no branch: the following run is read from LDS on
// every call and taken when the current one ends.  The run index stops at the last row, so
// the reads stay in the table after the stream's end (candidates produced past the end are
// only prefetched, never tested).
struct Walker {
    uint32_t off, left, row;
    uint2 nxt;
    template <uint32_t kUnit>
    __device__ __forceinline__ uint32_t next(const uint2 (*s_run)[kBlock], int col) {
        const uint32_t u = off;
        const bool sw = left == 1u;
        off = sw ? nxt.x : off + kUnit;
        left = sw ? nxt.y : left - 1u;
        row = sw ? min(row + 1u, 8u) : row;
        nxt = s_run[row][col];
        return u;
    }
};

// Orders the LDS accesses of one wavefront: the lanes' writes before the barrier are seen by the
// reads after it (the LDS serves a wavefront's accesses in issue order; this keeps the compiler
// from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Final exact pass of a whole wavefront at once.  The lanes' queued candidates are laid out one
// after another (lane order, each lane's queue order kept) and evaluated 64 at a time, one pair
// per lane, instead of each lane walking its own queue while the lanes with shorter queues idle.
// Each lane then adds the terms of its own pairs in its queue order, so its sum is the one its
// own walk would give.  The run table is no longer needed here; in the wavefront's columns,
// The scratch is 9 rows of 64 8-byte entries, one per lane of the wavefront: entry (row, lane)
// at scr[row * stride + cbase + lane]; rows 0-2 hold a round's terms, rows 3 and 6-8 every
// lane's own record (r, x, y, z), rows 4-5 the layout (lane | slot << 6 per pair, at most 512;
// bit 15 set once the pair is a contact).  Every lane of the wavefront must take part.
template <bool F32, int kQ, class Rec, class Tr>
__device__ __forceinline__ void exact_packed(const SlotDev &S, const double4 &p, const Rec &rec, uint32_t qn,
                                             uint2 *scr, int stride, int cbase, const uint32_t (*s_q)[kBlock],
                                             int t, double &fx, double &fy, double &fz, Tr &tr) {
    static_assert(kQ <= 8, "the layout holds 64 lanes x 8 slots");
    const int lane = t & 63, w0 = t - lane;
    const uint32_t incl = wave_incl_scan(qn), excl = incl - qn;
    const uint32_t total = uint32_t(__shfl(int(incl), 63, 64));
    if (total == 0) return;
    auto at = [&](int row, int c) -> uint2 & { return scr[row * stride + cbase + c]; };
    auto layout = [&](uint32_t e) -> uint16_t * {
        return reinterpret_cast<uint16_t *>(&at(4 + int(e >> 8), 0)) + (e & 255u);
    };
    at(3, lane) = __builtin_bit_cast(uint2, p.w);
    at(6, lane) = __builtin_bit_cast(uint2, p.x);
    at(7, lane) = __builtin_bit_cast(uint2, p.y);
    at(8, lane) = __builtin_bit_cast(uint2, p.z);
    for (uint32_t k = 0; k < qn; ++k) *layout(excl + k) = uint16_t(uint32_t(lane) | (k << 6));
    for (uint32_t base = 0; base < total; base += 64) {
        wave_lds_sync();
        const uint32_t e = base + uint32_t(lane);
        double tx = 0.0, ty = 0.0, tz = 0.0;
        if (e < total) {
            uint16_t *le = layout(e);
            const uint32_t m = *le, o = m & 63u;
            const double4 po = make_double4(
                __builtin_bit_cast(double, at(6, int(o))), __builtin_bit_cast(double, at(7, int(o))),
                __builtin_bit_cast(double, at(8, int(o))), __builtin_bit_cast(double, at(3, int(o))));
            const double4 r = rec.full(s_q[m >> 6][w0 + o]);
            if (pair_term<F32, Tr::kOn>(po, po.x - r.x, po.y - r.y, po.z - r.z, r.w, float(po.w), S, tx, ty, tz))
                *le = uint16_t(m | 0x8000u);
        }
        at(0, lane) = __builtin_bit_cast(uint2, tx);
        at(1, lane) = __builtin_bit_cast(uint2, ty);
        at(2, lane) = __builtin_bit_cast(uint2, tz);
        wave_lds_sync();
        const uint32_t lo = excl > base ? excl : base, hi = incl < base + 64u ? incl : base + 64u;
        for (uint32_t f = lo; f < hi; ++f) {
            const uint32_t m = *layout(f);
            if (m & 0x8000u) {
                const int c = int(f - base);
                fx = fx + __builtin_bit_cast(double, at(0, c));
                fy = fy + __builtin_bit_cast(double, at(1, c));
                fz = fz + __builtin_bit_cast(double, at(2, c));
                if constexpr (Tr::kOn) tr.hit(s_q[(m >> 6) & 7u][t]);
            }
        }
    }
}

// Summed force on the agent with record p at sorted position q whose `cnt` candidates are the
// runs in column t of s_run (canonical order); the queue uses the same column.
// The candidates are tested two per iteration, each pre-test record loaded two candidates
// ahead.  Survivors of the pre-test go to the queue (written unconditionally, kept when they
// pass), which the exact law empties in order, with the next record always in flight.
// With the normal queue the pairs run while the queue has room for two; the exact law then
// empties it with every lane of the wavefront together (a lane whose queue fills early waits
// for the others instead of running its own exact pass alone), and the last pass is the
// packed one.  In crowded populations nearly every lane fills its own queue within a few
// candidates of the others, and each lane empties it where it fills (measured faster there).
template <bool F32, int kQ, class Rec, class Pre, class Tr>
__device__ __forceinline__ void mech_forces(const SlotDev &S, uint32_t q, const double4 &p,
                                            const Rec &rec, float slack, uint2 (*s_run)[kBlock], uint32_t cnt,
                                            uint32_t (*s_q)[kBlock], int t, const Pre &pre_final,
                                            const RowUnion &un, typename Rec::Pre *s_stage, double &fx, double &fy,
                                            double &fz, Tr &tr) {
    constexpr uint32_t U = Rec::kUnit;
    constexpr bool kSync = kQ == kQueue;
    const uint32_t qu = q * U;
    const float rif = float(p.w);
    const typename Rec::Pre pf = rec.pre(qu);
    fx = 0.0;
    fy = 0.0;
    fz = 0.0;
    uint32_t qn = 0;
    // the record of the next queued candidate is loaded while the current one is evaluated
    // (its registers are free once the differences are taken)
    auto flush = [&]() {
        if (qn > 0) {
            if constexpr (kSync) {
                double4 r = rec.full(s_q[0][t]);
                for (uint32_t k = 0; k < qn; ++k) {
                    const double dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z, rj = r.w;
                    r = rec.full(s_q[k + 1u < qn ? k + 1u : k][t]);
                    const bool hit = exact_pair<F32, Tr::kOn>(p, dx, dy, dz, rj, rif, S, fx, fy, fz);
                    if constexpr (Tr::kOn) {
                        if (hit) tr.hit(s_q[k][t]);
                    }
                }
            } else {  // the crowded kernel's exact pass keeps two records ahead
                const uint32_t last = qn - 1u;
                double4 r = rec.full(s_q[0][t]);
                double4 r1 = rec.full(s_q[min(1u, last)][t]);
                for (uint32_t k = 0; k < qn; ++k) {
                    const double dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z, rj = r.w;
                    r = r1;
                    r1 = rec.full(s_q[min(k + 2u, last)][t]);
                    const bool hit = exact_pair<F32, Tr::kOn>(p, dx, dy, dz, rj, rif, S, fx, fy, fz);
                    if constexpr (Tr::kOn) {
                        if (hit) tr.hit(s_q[k][t]);
                    }
                }
            }
        }
        qn = 0;
    };
    auto push = [&](uint32_t u, const typename Rec::Pre &c) {
        s_q[qn][t] = u;
        qn += (Rec::touch(pf, c, slack) && u != qu) ? 1u : 0u;
        if constexpr (!kSync) {
            if (qn == uint32_t(kQ)) flush();
        }
    };
    if (un.coop) {
        // The wavefront walks the union of its lanes' runs row by row, 64 records at a time:
        // lane k loads record base + k (one coalesced load for the wavefront, the next chunk in
        // flight while this one is tested), the chunk goes through LDS, and every lane tests
        // each record that lies in its own run, in order.  A lane's candidates thus come in its
        // canonical order.  The queues are emptied together when one of them could fill.
        const int lane = t & 63, w0 = t - lane;
        [[maybe_unused]] CoarseAgents ca{};
        if constexpr (Rec::kF32Copy) ca = coarse_agents(pf, slack, lane);
#pragma unroll 1
        for (int r = 0; r < 9; ++r) {
            const uint32_t ulo = un.lo[r], uhi = un.hi[r];
            if (ulo >= uhi) continue;
            const uint2 own = s_run[r][t];
            typename Rec::Pre nxt = rec.pre(min(ulo + uint32_t(lane), uhi - 1u) * U);
            for (uint32_t base = ulo; base < uhi; base += 64u) {
                wave_lds_sync();
                s_stage[t] = nxt;
                if (base + 64u < uhi) nxt = rec.pre(min(base + 64u + uint32_t(lane), uhi - 1u) * U);
                wave_lds_sync();
                if constexpr (Rec::kF32Copy) {
                    // the matrix cores pick the pairs that may touch, and those go to the queue in
                    // ascending order within the lane's run (a pair that does not touch adds
                    // nothing in the exact law)
                    const uint32_t kn = min(64u, uhi - base);
                    const uint32_t a = own.x > base ? min(own.x - base, kn) : 0u;
                    const uint32_t b = own.y > base ? min(own.y - base, kn) : 0u;
                    uint64_t m = coarse_mask(ca, &s_stage[w0], lane) & low_bits(b) & ~low_bits(a);
                    if constexpr (Tr::kOn) {  // the traced kernels leave the agent itself out
                        const uint32_t self = qu / U - base;
                        if (self < 64u) m &= ~(1ull << self);
                    }
                    uint32_t lo = uint32_t(m), hi = uint32_t(m >> 32);
                    uint32_t pc = uint32_t(__builtin_popcount(lo) + __builtin_popcount(hi));
                    while (__any(pc != 0u)) {
                        if (__any(qn == uint32_t(kQ))) flush();
                        const uint32_t take = min(pc, uint32_t(kQ) - qn);
                        for (uint32_t k = 0; k < take; ++k) {
                            const bool low = lo != 0u;
                            const uint32_t word = low ? lo : hi;
                            const uint32_t e = uint32_t(__builtin_ctz(word)) + (low ? 0u : 32u);
                            if (low)
                                lo &= lo - 1u;
                            else
                                hi &= hi - 1u;
                            s_q[qn + k][t] = (base + e) * U;
                        }
                        qn += take;
                        pc -= take;
                    }
                    continue;
                }
                // four records per step, read from LDS together; the queues are emptied first
                // when one of them could fill within the step.  [a, b) is the lane's own run
                // within the chunk (entries past the chunk's end are valid LDS and outside it).
                // The agent itself may enter its queue: the law adds nothing at zero distance
                // (the traced kernels, which count coincident centres as contacts, skip it).
                const uint32_t kn = min(64u, uhi - base);
                const uint32_t a = own.x > base ? min(own.x - base, kn) : 0u;
                const uint32_t b = own.y > base ? min(own.y - base, kn) : 0u;
                for (uint32_t k = 0; k < kn; k += 4u) {
                    if (__any(qn > uint32_t(kQ - 4))) flush();
                    typename Rec::Pre cand[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) cand[i] = s_stage[w0 + int(k) + i];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t e = k + uint32_t(i);
                        const uint32_t u = (base + e) * U;
                        s_q[qn][t] = u;
                        qn += ((e >= a) & (e < b) & (!Tr::kOn || u != qu) & Rec::touch(pf, cand[i], slack)) ? 1u : 0u;
                    }
                }
            }
        }
        pre_final();
        flush();
        return;
    }
    const uint2 r0 = s_run[0][t];
    Walker w{r0.x, r0.y, 1u, s_run[1][t]};
    uint32_t ua = w.next<U>(s_run, t);
    typename Rec::Pre ca = rec.pre(ua);
    uint32_t ub = w.next<U>(s_run, t);
    typename Rec::Pre cb = rec.pre(ub);
    uint32_t c = 0;
    const uint32_t pairs_end = cnt ? cnt - 1u : 0u;  // a pair starts at c while c < cnt - 1
    for (;;) {
        while (c < pairs_end && (!kSync || qn <= uint32_t(kQ - 2))) {
            push(ua, ca);
            ua = w.next<U>(s_run, t);
            ca = rec.pre(ua);
            push(ub, cb);
            ub = w.next<U>(s_run, t);
            cb = rec.pre(ub);
            c += 2u;
        }
        if (c >= pairs_end) break;
        flush();
        ca = rec.pre(ua);  // reloaded rather than held in registers across the exact pass
        cb = rec.pre(ub);
    }
    if (c < cnt) {  // odd count: the last candidate
        if (qn == uint32_t(kQ)) flush();
        push(ua, ca);
    }
    pre_final();
    if constexpr (kSync)
        exact_packed<F32, kQ>(S, p, rec, qn, &s_run[0][0], kBlock, t - (t & 63), s_q, t, fx, fy, fz, tr);
    else
        flush();
}

// One tile: 256 agents of one slot, one lane per agent.  precision: 64 or 32 for a plain call;
// 0 = per slot.
// Stationary skip (paper Sec. 2.3 (iv)), plain calls: an agent whose kept boxes (every box that
// can hold a sphere touching it, its own included) are unmarked -- no agent left or entered them
// in the last step, so it did not move either -- on an unchanged lattice has the same candidates,
// contacts and force as in the last step, where it was gated: it keeps that force (carried by the
// sort into fprev) and its position, without a walk.  Every agent records whether it moves and
// marks the box it leaves; the next build marks the box it enters.
struct SkipIO {
    const double *fprev;  // the last step's force of each sorted agent
    uint8_t *moved;       // per output slot: the agent moves in this step
    uint8_t *dirty;       // per box: a mover leaves it
    uint32_t *tileskip;   // per wavefront of each tile: agents skipped
};

template <int kPrec, int kQ, class Tr, bool kSkip = false, class Rec>
__device__ __forceinline__ void mech_tile(const Slots &sl, int64_t tile, const Rec &rec,
                                          const double *__restrict__ adh_s, const uint32_t *__restrict__ id_s,
                                          const uint8_t *__restrict__ state_s,
                                          const uint32_t *__restrict__ start_all, const bdm_soa &out,
                                          uint2 (*s_run)[kBlock], uint32_t (*s_q)[kBlock], typename Rec::Pre *s_stage,
                                          const TraceOut &tout, const SkipIO &sk = SkipIO{}) {
    const int t = threadIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    const GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    const int64_t l0 = tile * kBlock - S.agent_off;  // local (sorted) index of the tile's first agent
    if (!g->valid || l0 >= g->n) return;
    // Lanes past the slot's agents stay, with no candidates, because the final exact pass needs
    // every lane of the wavefront; they read the last agent's inputs and write nothing.
    const int64_t l = l0 + t;
    const bool live = l < g->n && l < S.capacity;
    const bool f32 = kPrec == 32 || (kPrec == 0 && S.force_bits == 32);
    const uint32_t q = uint32_t(g->sorted_base + (l < g->n ? l : g->n - 1));
    const double4 p = rec.full(q * Rec::kUnit);
    // the agent's box from its position, as the build computed its key (binary64 division and
    // floor, clamped to the lattice): no sorted key array is written or read
    const int cx = box_coord(p.x, g->b, g->cmin[0], g->dims[0], false);
    const int cy = box_coord(p.y, g->b, g->cmin[1], g->dims[1], false);
    const int cz = box_coord(p.z, g->b, g->cmin[2], g->dims[2], false);
    [[maybe_unused]] const uint32_t key =
        uint32_t(cx) + uint32_t(g->dims[0]) * (uint32_t(cy) + uint32_t(g->dims[1]) * uint32_t(cz));
    RowUnion un;
    bool marked = false;
    uint32_t cnt = load_runs<Rec::kUnit, kQ == kQueueCrowded, kSkip>(g, start_all + S.box_off, cx, cy, cz, p, live,
                                                                    s_run, t, un, &marked);
    bool skip = false;
    if constexpr (kSkip) {
        skip = g->skip_ok && live && !marked;
        if (skip) cnt = 0;
        const unsigned long long m = __ballot(skip);
        if ((t & 63) == 0) sk.tileskip[tile * (kBlock / 64) + (t >> 6)] = uint32_t(__popcll(m));
    }
    double fx, fy, fz;
    // the agent's remaining inputs are loaded before the last exact pass, which hides their latency
    double adh;
    uint32_t id;
    uint8_t state = 0;
    auto pre = [&]() {
        adh = adh_s[q];
        id = id_s[q];
        if (out.state) state = state_s[q];
    };
    Tr tr{};
    if constexpr (Tr::kOn) tr = Tr{Rec::kUnit, uint32_t(g->sorted_base), 0u, 0u};
    if (f32)
        mech_forces<true, kQ>(S, q, p, rec, pretest_slack(g), s_run, cnt, s_q, t, pre, un, s_stage, fx, fy, fz, tr);
    else
        mech_forces<false, kQ>(S, q, p, rec, pretest_slack(g), s_run, cnt, s_q, t, pre, un, s_stage, fx, fy, fz, tr);
    if (!live) return;
    if constexpr (Tr::kOn) {
        tout.counts[S.agent_off + l] = tr.n;
        tout.hashes[S.agent_off + l] = tr.h;
    }
    if constexpr (kSkip) {
        if (skip) {
            fx = sk.fprev[3 * size_t(q)];
            fy = sk.fprev[3 * size_t(q) + 1];
            fz = sk.fprev[3 * size_t(q) + 2];
        }
    }

    // adherence gate, clamp, integrate (binary64)
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
    if constexpr (kSkip) {
        const bool moves = !(fn < adh);
        sk.moved[o] = moves ? 1 : 0;
        if (moves) sk.dirty[key] = 1;
    }
    __builtin_nontemporal_store(nxp, &out.x[o]);
    __builtin_nontemporal_store(nyp, &out.y[o]);
    __builtin_nontemporal_store(nzp, &out.z[o]);
    __builtin_nontemporal_store(2.0 * p.w, &out.diam[o]);
    __builtin_nontemporal_store(adh, &out.adh[o]);
    __builtin_nontemporal_store(id, &out.id[o]);
    if (out.state) out.state[o] = state;
    if (out.fx) __builtin_nontemporal_store(fx, &out.fx[o]);
    if (out.fy) __builtin_nontemporal_store(fy, &out.fy[o]);
    if (out.fz) __builtin_nontemporal_store(fz, &out.fz[o]);
}

// Plain call: the tiles in the pencil order, one contiguous part of it per XCD.
template <int kPrec, int kQ, class Tr, bool kSkip = false, class Rec>
__device__ __forceinline__ void mech_plain(const Slots &sl, const uint32_t *__restrict__ order, const Rec &rec,
                                           const double *__restrict__ adh_s, const uint32_t *__restrict__ id_s,
                                           const uint8_t *__restrict__ state_s,
                                           const uint32_t *__restrict__ start, const bdm_soa &out,
                                           const TraceOut &tout, const SkipIO &sk = SkipIO{}) {
    __shared__ uint2 s_run[9][kBlock];
    __shared__ uint32_t s_q[kQ][kBlock];
    __shared__ typename Rec::Pre s_stage[kQ == kQueueCrowded ? kBlock : 1];  // records of a cooperative walk
    GridDev *g0 = &sl.grids[0];
    if (frozen_plain(g0, sl.table)) return;  // nothing moved since the last step: nothing changes
    // no usable grid of these agents: never built, its build failed, already used by a step,
    // or built for another model (the periodic lattice has no pre-test records; the crowded
    // kernel reads the binary32 copies only spheroid builds write)
    // (a build that skips stationary agents marks its starts: only the skipping kernel reads it)
    const bool usable = g0->valid && !g0->consumed &&
                        (kQ == kQueueCrowded ? g0->kind == kGridOpenF32
                         : kSkip             ? g0->kind == kGridOpenSkip
                                             : (g0->kind == kGridOpen || g0->kind == kGridOpenF32));
    if (!usable) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&g0->flags, BDM_FLAG_NOGRID);
        return;
    }
    const uint32_t live_tiles = uint32_t((g0->n + kBlock - 1) / kBlock);
    if (blockIdx.x >= live_tiles) return;
    mech_tile<kPrec, kQ, Tr, kSkip>(sl, order[xcd_tile(blockIdx.x, live_tiles)], rec, adh_s, id_s, state_s,
                                    start, out, s_run, s_q, s_stage, tout, sk);
}

// The normal queue: six wavefronts per SIMD (80 registers), which is also what the LDS of a
// workgroup allows.
template <int kPrec, class Tr, class Rec>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_mech(
    Slots sl, const uint32_t *__restrict__ order, Rec rec, const double *__restrict__ adh_s,
    const uint32_t *__restrict__ id_s, const uint8_t *__restrict__ state_s,
    const uint32_t *__restrict__ start, bdm_soa out, TraceOut tout) {
    mech_plain<kPrec, kQueue, Tr>(sl, order, rec, adh_s, id_s, state_s, start, out, tout);
}

// The same with the stationary skip.
template <int kPrec, class Tr, class Rec>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_mech_skip(
    Slots sl, const uint32_t *__restrict__ order, Rec rec, const double *__restrict__ adh_s,
    const uint32_t *__restrict__ id_s, const uint8_t *__restrict__ state_s,
    const uint32_t *__restrict__ start, bdm_soa out, TraceOut tout, SkipIO sk) {
    mech_plain<kPrec, kQueue, Tr, true>(sl, order, rec, adh_s, id_s, state_s, start, out, tout, sk);
}

// The crowded queue.  Its LDS (28 KB per workgroup with a queue of 6) allows five wavefronts per
// SIMD, as the registers do.  With the cooperative walk's pre-test on the matrix cores, queues of
// 5, 6, 7 and 10 took the 60-step spheroid 0.075, 0.077, 0.080 and 0.087 s and the 122 steps to
// 4.1 M cells 2.35, 2.33, 2.33-2.34 and 2.32-2.34 s: shorter queues leave fewer lanes idle in
// each exact pass.
template <int kPrec, class Tr, class Rec>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_mech_crowded(
    Slots sl, const uint32_t *__restrict__ order, Rec rec, const double *__restrict__ adh_s,
    const uint32_t *__restrict__ id_s, const uint8_t *__restrict__ state_s,
    const uint32_t *__restrict__ start, bdm_soa out, TraceOut tout) {
    mech_plain<kPrec, kQueueCrowded, Tr>(sl, order, rec, adh_s, id_s, state_s, start, out, tout);
}

// Batch (precision per slot): the workgroups stride over the tiles (a simulation's tiles spread
// over all of them), neighbouring tiles of a round going to workgroups of one XCD.
template <class Tr, class Rec>
__global__ __launch_bounds__(kBlock) void k_mech_batch(Slots sl, int64_t ntiles, Rec rec,
                                                       const double *__restrict__ adh_s,
                                                       const uint32_t *__restrict__ id_s,
                                                       const uint8_t *__restrict__ state_s,
                                                                                                              const uint32_t *__restrict__ start, bdm_soa out,
                                                       TraceOut tout) {
    __shared__ uint2 s_run[9][kBlock];
    __shared__ uint32_t s_q[kQueue][kBlock];
    for (int64_t tile = xcd_tile(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x)
        mech_tile<0, kQueue, Tr>(sl, tile, rec, adh_s, id_s, state_s, start, out, s_run, s_q, nullptr, tout);
}

// Batch, one workgroup per tile (the work split that deals every tile its own workgroup): without
// the striding loop the kernel needs 76 registers and runs six wavefronts per SIMD; the striding
// form needs 113 and runs four.
template <class Tr, class Rec>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_mech_batch_tile(
    Slots sl, int64_t ntiles, Rec rec, const double *__restrict__ adh_s, const uint32_t *__restrict__ id_s,
    const uint8_t *__restrict__ state_s, const uint32_t *__restrict__ start,
    bdm_soa out, TraceOut tout) {
    __shared__ uint2 s_run[9][kBlock];
    __shared__ uint32_t s_q[kQueue][kBlock];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile < ntiles)
        mech_tile<0, kQueue, Tr>(sl, tile, rec, adh_s, id_s, state_s, start, out, s_run, s_q, nullptr, tout);
}

// Test hook: contact lists per sorted slot in force-sum order (mechanical contact, plain calls).
__global__ __launch_bounds__(kBlock) void k_contacts_mech(Slots sl, const double4 *__restrict__ pos4,
                                                          const uint32_t *__restrict__ id_s,
                                                          const uint32_t *__restrict__ start, int f32,
                                                          uint32_t *counts, const int64_t *offsets,
                                                          uint32_t *ids) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const GridDev *g = &sl.grids[0];
    if (!g->valid || s >= g->n) return;
    const double b = g->b;
    const double4 p = pos4[s];
    const int cx = box_coord(p.x, b, g->cmin[0], g->dims[0], false);
    const int cy = box_coord(p.y, b, g->cmin[1], g->dims[1], false);
    const int cz = box_coord(p.z, b, g->cmin[2], g->dims[2], false);
    const double ri = p.w;
    const float rif = float(ri);
    uint32_t c = 0;
    for (int r = 0; r < 9; ++r) {
        uint32_t lo, hi;
        row_range(g, start, cx, cy, cz, r, lo, hi);
        for (uint32_t j = lo; j < hi; ++j) {
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

template <class Tr, class Rec>
static void launch_mech_rec(const bdm_soa &s, const Slots &sl, int64_t ntiles, unsigned nb, int precision,
                            const uint32_t *order, const Rec &rec, const Ws &w, const TraceOut &tout, hipStream_t st) {
#define BDM_MECH(K, P)                                                                                     \
    hipLaunchKernelGGL((K<P, Tr, Rec>), dim3(nb), dim3(kBlock), 0, st, sl, order, rec, w.adh, w.ids, w.state, \
                       w.start, s, tout)
    if constexpr (Rec::kF32Copy) {  // the crowded kernel
        if (precision == 32)
            BDM_MECH(k_mech_crowded, 32);
        else
            BDM_MECH(k_mech_crowded, 64);
    } else if (!sl.table && sl.one.skip) {
        const SkipIO sk{w.fprev, w.moved, w.dirty, w.tileskip};
        if (precision == 32)
            hipLaunchKernelGGL((k_mech_skip<32, Tr, Rec>), dim3(nb), dim3(kBlock), 0, st, sl, order, rec, w.adh, w.ids,
                               w.state, w.start, s, tout, sk);
        else
            hipLaunchKernelGGL((k_mech_skip<64, Tr, Rec>), dim3(nb), dim3(kBlock), 0, st, sl, order, rec, w.adh, w.ids,
                               w.state, w.start, s, tout, sk);
    } else if (precision == 32) {
        BDM_MECH(k_mech, 32);
    } else if (precision == 64) {
        BDM_MECH(k_mech, 64);
    } else if (int64_t(nb) >= ntiles) {  // a workgroup for every tile
        hipLaunchKernelGGL((k_mech_batch_tile<Tr, Rec>), dim3(nb), dim3(kBlock), 0, st, sl, ntiles, rec, w.adh,
                           w.ids, w.state, w.start, s, tout);
    } else {
        hipLaunchKernelGGL((k_mech_batch<Tr, Rec>), dim3(nb), dim3(kBlock), 0, st, sl, ntiles, rec, w.adh, w.ids,
                           w.state, w.start, s, tout);
    }
#undef BDM_MECH
}

template <class Rec>
static void launch_mech_traced(const bdm_soa &s, const Slots &sl, int64_t ntiles, unsigned nb, int precision,
                               const uint32_t *order, const Rec &rec, const Ws &w, const TraceOut *trace,
                               hipStream_t st) {
    if (trace)
        launch_mech_rec<Trace>(s, sl, ntiles, nb, precision, order, rec, w, *trace, st);
    else
        launch_mech_rec<NoTrace>(s, sl, ntiles, nb, precision, order, rec, w, TraceOut{nullptr, nullptr}, st);
}

// A plain mechanical step has used its grid build: the next step needs a new one.  After a step
// that skips stationary agents, its marks are ready for the next build, and the agents skipped
// are summed from the per-wavefront counts of the tiles it ran, by kConsumeGroups workgroups:
// each adds its share to an accumulator, and the last one to finish (a ticket) records the total
// and resets the accumulator and the ticket for the next step.  (One workgroup took 110 us for
// the 262 144 counts of 2^24 agents.)
// A build that found nothing to do (frozen) holds for its force law only: a step that asked for
// another one was refused (it needs a new build; its kernel left the agents as they are).
constexpr unsigned kConsumeGroups = 64;
__global__ __launch_bounds__(1024) void k_grid_consume(GridDev *g, const uint32_t *tileskip, int32_t skip, SlotDev a) {
    __shared__ unsigned long long s_part[1024 / 64];
    if (g->frozen) {
        if (blockIdx.x == 0 && threadIdx.x == 0 &&
            (g->law_k != a.k || g->law_gamma != a.gamma || g->law_bits != a.force_bits))
            atomicOr(&g->flags, BDM_FLAG_NOGRID);
        return;
    }
    if (!skip) {
        if (blockIdx.x == 0 && threadIdx.x == 0) g->consumed = 1;
        return;
    }
    const bool ran = g->valid && g->kind == kGridOpenSkip && !g->consumed;
    const int64_t nw = ran ? (g->n + kBlock - 1) / kBlock * (kBlock / 64) : 0;
    unsigned long long c = 0;
    if (g->skip_ok)
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nw; i += int64_t(gridDim.x) * blockDim.x)
            c += tileskip[i];
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x != 0) return;
    unsigned long long sum = 0;
    for (int k = 0; k < 1024 / 64; ++k) sum += s_part[k];
    atomicAdd(&g->skip_acc, sum);
    __threadfence();
    if (atomicAdd(&g->consume_ticket, 1u) != gridDim.x - 1) return;
    __threadfence();
    const unsigned long long total = atomicAdd(&g->skip_acc, 0ull);
    g->skip_acc = 0ull;
    g->consume_ticket = 0u;
    if (ran) {
        g->skipped = int64_t(total);
        g->mark_ready = 1;
    }
    g->consumed = 1;
}

// crowded: a population packed so densely that agents have tens of contacts (the growing
// spheroid): the kernel with the cooperative walk and its own queue length.
void launch_mech(const bdm_soa &s, const Slots &sl, int64_t capacity, int precision, bool crowded, const Ws &w,
                 hipStream_t st, const TraceOut *trace) {
    const int64_t ntiles = (capacity + kBlock - 1) / kBlock;
    const unsigned nb = tile_grid(sl, ntiles);
    const uint32_t *order = sl.table ? nullptr : w.flagid;  // plain: order built with the grid
    const uint64_t bytes = uint64_t(w.lay.capacity) * 32u;
    if (bytes <= 0xFFFFFFE0ull) {
        if (crowded)
            launch_mech_traced(s, sl, ntiles, nb, precision, order,
                               RecBuf4{static_cast<void *>(w.pos4), static_cast<void *>(w.pos4f), uint32_t(bytes)}, w,
                               trace, st);
        else
            launch_mech_traced(s, sl, ntiles, nb, precision, order,
                               RecBuf{static_cast<void *>(w.pos4), static_cast<void *>(w.pos8), uint32_t(bytes)}, w,
                               trace, st);
    } else if (crowded) {
        launch_mech_traced(s, sl, ntiles, nb, precision, order, RecGlobal4{w.pos4, w.pos4f}, w, trace, st);
    } else {
        launch_mech_traced(s, sl, ntiles, nb, precision, order, RecGlobal{w.pos4, w.pos8}, w, trace, st);
    }
    if (!sl.table)
        hipLaunchKernelGGL(k_grid_consume, dim3(kConsumeGroups), dim3(1024), 0, st, w.grid, w.tileskip,
                           int32_t(sl.one.skip), sl.one);
}

void launch_contacts_mech(int f32, const Slots &sl, const Ws &w, uint32_t *counts, const int64_t *offsets,
                          uint32_t *ids, hipStream_t st) {
    int64_t nb = (w.lay.capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_contacts_mech, dim3(unsigned(nb)), dim3(kBlock), 0, st, sl, w.pos4, w.ids, w.start, f32,
                       counts, offsets, ids);
}

}  // namespace bdm
