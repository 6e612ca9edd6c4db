// k_grid.hip -- uniform-grid build on gfx950 (paper Sec. 2.1: equal boxes, agents binned by
// centre, box edge from the largest agent, 27-box neighbourhood).
//
// Pipeline for every slot at once (one launch each, all device-resident, no host read-back):
//   bounds     min/max of x, y, z and max diameter per 1024 agents (one partial record each)
//   finalize   one workgroup per slot: reduce its partials, box edge, lattice origin and dims,
//              box count check
//   key_count  box key per agent and its arrival rank in the box (integer atomics)
//   scan       single-pass decoupled look-back exclusive scan of the packed histogram
//   scatter    ids into their box range in arrival order
//   canon      each agent counts the smaller ids in its box (ascending-id order inside a box)
//              and copies itself into the sorted copy: (x, y, z, r = d/2) packed as double4
//              (halving and doubling a binary64 are exact, so d = 2r is recovered bit for bit)
//              plus its box key, and for mechanics a binary32 copy (x - o, y - o, z - o, r)
//              relative to the lattice origin o that only the conservative contact pre-test reads
//   order      one workgroup: the processing order of the mechanics tiles (pencils of rows
//              swept along z, so that the three z-planes a tile reads stay in one XCD's L2)
#include "kernels.hpp"

namespace bdm {

constexpr int kPencilRows = 16;       // y-rows per pencil of the processing order
constexpr int kOrderBins = 8192;      // largest pencil x z-plane count the order kernel sorts

// Per workgroup of kBoundsTile agents: min/max of x, y, z, max diameter and a non-finite flag,
// written as one 8-value partial record (no atomics).
__device__ __forceinline__ void bounds_tile(const Slots &sl, int64_t btile, const int64_t *n_ptr,
                                            const double *__restrict__ x, const double *__restrict__ y,
                                            const double *__restrict__ z, const double *__restrict__ d,
                                            double *partials) {
    const int64_t base = btile * kBoundsTile;
    const int slot = slot_of_tile(sl, base / kBlock);
    if (slot < 0) return;
    const SlotDev S = slot_record(sl, slot);
    const int64_t n = live_count(n_ptr, slot, S.capacity);
    const int64_t l0 = base - S.agent_off;  // local index of the workgroup's first agent
    if (l0 >= n) return;
    double v[8];
    for (int a = 0; a < 3; ++a) {
        v[a] = __builtin_inf();
        v[3 + a] = -__builtin_inf();
    }
    v[6] = 0.0;
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
    v[7] = bad ? 1.0 : 0.0;
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
        partials[btile * 8 + a] = r;
    }
    __syncthreads();  // s_red is reused by the next tile of this workgroup
}

__global__ __launch_bounds__(kBlock) void k_bounds(Slots sl, int64_t nbtiles, const int64_t *n_ptr,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ d, double *partials,
                                                   unsigned long long *tiles, int64_t max_tiles) {
    if (blockIdx.x == 0) {  // reset the scan tiles of the coming histogram scan
        for (int64_t t = threadIdx.x; t < max_tiles; t += blockDim.x) tiles[t] = 0ull;
        if (threadIdx.x == 0) sl.grids[0].scan_ticket = 0u;
    }
    for (int64_t bt = blockIdx.x; bt < nbtiles; bt += gridDim.x) bounds_tile(sl, bt, n_ptr, x, y, z, d, partials);
}

// One workgroup per slot: reduce the slot's bounds partials, then box edge, lattice, box count.
__global__ __launch_bounds__(kBlock) void k_finalize(Slots sl, const int64_t *n_ptr, const double *partials) {
    const int slot = int(blockIdx.x);
    if (slot >= sl.nslots) return;
    const SlotDev a = slot_record(sl, slot);
    GridDev *g = &sl.grids[slot];
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
        const int64_t b0 = a.agent_off / kBoundsTile, nb = (n + kBoundsTile - 1) / kBoundsTile;
        for (int64_t k = threadIdx.x; k < nb; k += blockDim.x) {
            const double *p = partials + (b0 + k) * 8;
            for (int i = 0; i < 3; ++i) {
                v[i] = fmin(v[i], p[i]);
                v[3 + i] = fmax(v[3 + i], p[3 + i]);
            }
            v[6] = fmax(v[6], p[6]);
            v[7] = fmax(v[7], p[7]);
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
    g->sir_counts[0] = g->sir_counts[1] = g->sir_counts[2] = 0ull;
    g->valid = 0;
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
        for (int i = 0; i < 3; ++i) {
            // floor is monotone, so min/max of floor(x/b) are floor(min x / b), floor(max x / b)
            const double c0 = floor(lo[i] / b), c1 = floor(hi[i] / b);
            if (!(c0 >= -1073741824.0 && c1 <= 1073741823.0)) {
                g->flags |= BDM_FLAG_NONFINITE;
                g->n = 0;
                return;
            }
            g->cmin[i] = int32_t(c0);
            g->dims[i] = int32_t(c1) - int32_t(c0) + 1;
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
    g->div_nx = fastdiv_magic(uint32_t(g->dims[0]));
    g->div_ny = fastdiv_magic(uint32_t(g->dims[1]));
    g->valid = 1;
}

__device__ __forceinline__ void key_count_tile(const Slots &sl, int64_t tile, const double *__restrict__ x,
                                               const double *__restrict__ y, const double *__restrict__ z,
                                               uint32_t *count, uint32_t *__restrict__ key,
                                               uint32_t *__restrict__ rank) {
    const int64_t i = tile * kBlock + threadIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    const GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    if (!g->valid || i - S.agent_off >= g->n) return;
    const double b = g->b;
    const bool per = S.periodic != 0;
    const int cx = box_coord(x[i], b, g->cmin[0], g->dims[0], per);
    const int cy = box_coord(y[i], b, g->cmin[1], g->dims[1], per);
    const int cz = box_coord(z[i], b, g->cmin[2], g->dims[2], per);
    const uint32_t k = uint32_t(cx) + uint32_t(g->dims[0]) * (uint32_t(cy) + uint32_t(g->dims[1]) * uint32_t(cz));
    key[i] = k;
    rank[i] = atomicAdd(&count[S.box_off + k], 1u);
}

__global__ __launch_bounds__(kBlock) void k_key_count(Slots sl, int64_t ntiles, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, uint32_t *count,
                                                      uint32_t *__restrict__ key,
                                                      uint32_t *__restrict__ rank) {
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        key_count_tile(sl, tile, x, y, z, count, key, rank);
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
                                                 uint32_t *ticket, int zero_in, GridDev *g) {
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

__device__ __forceinline__ void scatter_tile(const Slots &sl, int64_t tile, const uint32_t *__restrict__ key,
                                             const uint32_t *__restrict__ rank,
                                             const uint32_t *__restrict__ start,
                                             const uint32_t *__restrict__ id, uint32_t *__restrict__ tmpid) {
    const int64_t i = tile * kBlock + threadIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    if (!g->valid || i - S.agent_off >= g->n) return;
    const uint32_t base = start[S.box_off];
    if (i == S.agent_off) g->sorted_base = base;
    const uint32_t pos = start[S.box_off + key[i]] + rank[i];
    if (pos - base >= uint32_t(g->n)) {  // cannot happen with a zeroed histogram; guards memory
        atomicOr(&g->flags, BDM_FLAG_SCAN);
        return;
    }
    tmpid[pos] = id[i];
}

__global__ __launch_bounds__(kBlock) void k_scatter_id(Slots sl, int64_t ntiles, const uint32_t *__restrict__ key,
                                                       const uint32_t *__restrict__ rank,
                                                       const uint32_t *__restrict__ start,
                                                       const uint32_t *__restrict__ id,
                                                       uint32_t *__restrict__ tmpid) {
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        scatter_tile(sl, tile, key, rank, start, id, tmpid);
}

__device__ __forceinline__ void canon_tile(const Slots &sl, int64_t tile, const SoaIn &s,
                                           const uint32_t *__restrict__ key, const uint32_t *__restrict__ start,
                                           const uint32_t *__restrict__ tmpid, double4 *__restrict__ pos4,
                                           float4 *__restrict__ pos4f, double *__restrict__ adh_s,
                                           uint32_t *__restrict__ id_s, uint8_t *__restrict__ state_s,
                                           uint32_t *__restrict__ key_s, uint32_t *__restrict__ tile_key) {
    const int64_t i = tile * kBlock + threadIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    const GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    if (!g->valid || i - S.agent_off >= g->n) return;
    const uint32_t k = key[i];
    const uint32_t end = start[S.box_off] + uint32_t(g->n);
    const uint32_t s0 = start[S.box_off + k];
    const uint32_t s1 = min(start[S.box_off + k + 1], end);
    const uint32_t me = s.id[i];
    uint32_t r = 0;
    for (uint32_t j = s0; j < s1; ++j) r += tmpid[j] < me;
    const uint32_t dst = s0 + r;
    if (dst >= s1) return;
    const double x = s.x[i], y = s.y[i], z = s.z[i], rad = s.d ? 0.5 * s.d[i] : 0.0;  // radius, exact
    pos4[dst] = make_double4(x, y, z, rad);
    if (!S.periodic) {  // binary32 copy relative to the lattice origin, for the contact pre-test
        const double b = g->b;
        pos4f[dst] = make_float4(float(x - double(g->cmin[0]) * b), float(y - double(g->cmin[1]) * b),
                                 float(z - double(g->cmin[2]) * b), float(rad));
    }
    if (s.adh) adh_s[dst] = s.adh[i];
    id_s[dst] = me;
    key_s[dst] = k;
    if (s.state) state_s[dst] = s.state[i];
    if (tile_key) {  // key of every tile's first agent (plain calls only: one slot, base 0)
        if ((dst & (kBlock - 1)) == 0) tile_key[dst / kBlock] = k;
    }
}

__global__ __launch_bounds__(kBlock) void k_canon(Slots sl, int64_t ntiles, SoaIn s, const uint32_t *__restrict__ key,
                                                  const uint32_t *__restrict__ start,
                                                  const uint32_t *__restrict__ tmpid,
                                                  double4 *__restrict__ pos4, float4 *__restrict__ pos4f,
                                                  double *__restrict__ adh_s, uint32_t *__restrict__ id_s,
                                                  uint8_t *__restrict__ state_s, uint32_t *__restrict__ key_s,
                                                  uint32_t *__restrict__ tile_key) {
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        canon_tile(sl, tile, s, key, start, tmpid, pos4, pos4f, adh_s, id_s, state_s, key_s, tile_key);
}

// Processing order of the mechanics tiles of a plain call: counting sort of the tiles (256
// consecutive sorted agents) by (pencil of kPencilRows y-rows, z-plane) of their first agent.
// Every order is correct (each tile is independent); this one keeps the three z-planes a tile
// reads within a small window.  Falls back to the identity when the grid has too many pencils.
__global__ __launch_bounds__(1024) void k_tile_order(const GridDev *__restrict__ g,
                                                     const uint32_t *__restrict__ tile_key,
                                                     uint32_t *__restrict__ order, int64_t max_tiles) {
    __shared__ uint32_t s_bin[kOrderBins];
    __shared__ uint32_t s_part[1024];
    const int t = threadIdx.x;
    const int64_t ntile = g->valid ? (g->n + kBlock - 1) / kBlock : 0;
    const int ny = g->dims[1], nz = g->dims[2], nx = g->dims[0];
    const int64_t pencils = (int64_t(ny) + kPencilRows - 1) / kPencilRows;
    const int64_t nbins = pencils * int64_t(nz);
    if (ntile == 0) return;
    if (nbins > kOrderBins || nbins <= 0) {
        for (int64_t c = t; c < ntile && c < max_tiles; c += blockDim.x) order[c] = uint32_t(c);
        return;
    }
    for (int b = t; b < nbins; b += blockDim.x) s_bin[b] = 0u;
    __syncthreads();
    auto bin_of = [&](uint32_t k) -> uint32_t {
        const uint32_t row = k / uint32_t(nx);
        const uint32_t yy = row % uint32_t(ny), zz = row / uint32_t(ny);
        return (yy / kPencilRows) * uint32_t(nz) + zz;
    };
    for (int64_t c = t; c < ntile; c += blockDim.x) atomicAdd(&s_bin[bin_of(tile_key[c])], 1u);
    __syncthreads();
    // exclusive scan of the bins: each thread owns a contiguous chunk
    const int per = int((nbins + blockDim.x - 1) / blockDim.x);
    const int b0 = t * per, b1 = min(int(nbins), b0 + per);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += s_bin[b];
    s_part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan of the chunk sums
        const uint32_t v = t >= off ? s_part[t - off] : 0u;
        __syncthreads();
        s_part[t] += v;
        __syncthreads();
    }
    uint32_t run = s_part[t] - sum;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = s_bin[b];
        s_bin[b] = run;
        run += c;
    }
    __syncthreads();
    for (int64_t c = t; c < ntile; c += blockDim.x) {
        const uint32_t pos = atomicAdd(&s_bin[bin_of(tile_key[c])], 1u);
        if (pos < max_tiles) order[pos] = uint32_t(c);
    }
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

// ---------------------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int64_t per = kBlock) {
    int64_t b = (n + per - 1) / per;
    return unsigned(b < 1 ? 1 : b);
}

// Workgroups of a per-tile launch: one per tile for a plain call; a batch strides over its
// tiles with at most kBatchGrid workgroups, so empty capacity costs a table read, not a dispatch.
unsigned tile_grid(const Slots &sl, int64_t ntiles) {
    const int64_t cap = 8192;
    if (ntiles < 1) return 1;
    return unsigned(sl.table && ntiles > cap ? cap : ntiles);
}

void launch_grid_build(const bdm_soa &s, const Slots &sl, int64_t capacity, const Ws &w, hipStream_t st) {
    const bool has_d = sl.table ? true : sl.one.has_d != 0;
    const double *d = has_d ? s.diam : nullptr;
    const int64_t nbt = (capacity + kBoundsTile - 1) / kBoundsTile;
    hipLaunchKernelGGL(k_bounds, dim3(tile_grid(sl, nbt)), dim3(kBlock), 0, st, sl, nbt, s.n, s.x, s.y, s.z, d,
                       w.partials, w.tiles, w.lay.max_tiles);
    hipLaunchKernelGGL(k_finalize, dim3(unsigned(sl.nslots)), dim3(kBlock), 0, st, sl, s.n, w.partials);
    const int64_t nt = (capacity + kBlock - 1) / kBlock;
    const unsigned nb = tile_grid(sl, nt);
    hipLaunchKernelGGL(k_key_count, dim3(nb), dim3(kBlock), 0, st, sl, nt, s.x, s.y, s.z, w.count, w.key, w.rank);
    launch_scan(w.count, w.start, nullptr, w.lay.max_boxes, w, 1, false, st);
    hipLaunchKernelGGL(k_scatter_id, dim3(nb), dim3(kBlock), 0, st, sl, nt, w.key, w.rank, w.start, s.id, w.tmpid);
    SoaIn in{s.x, s.y, s.z, d, s.adh, s.id, s.state};
    uint32_t *tile_key = sl.table ? nullptr : w.rankid;  // plain calls reuse the rank-by-id area
    // the sorted agents' keys go to the rank array, which nothing reads after the scatter
    hipLaunchKernelGGL(k_canon, dim3(nb), dim3(kBlock), 0, st, sl, nt, in, w.key, w.start, w.tmpid, w.pos4, w.pos4f,
                       w.adh, w.ids, w.state, w.rank, tile_key);
    if (!sl.table && !sl.one.periodic)
        hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, st, w.grid, tile_key, w.flagid,
                           int64_t(w.lay.ntiles));
}

void launch_scan(uint32_t *in, uint32_t *out, const int64_t *len_ptr, int64_t max_len, const Ws &w,
                 int zero_in, bool prepare, hipStream_t st) {
    const unsigned nt = unsigned((max_len + kScanTile) / kScanTile);
    if (prepare)
        hipLaunchKernelGGL(k_scan_prepare, dim3(blocks_for(w.lay.max_tiles)), dim3(kBlock), 0, st, w.tiles,
                           w.lay.max_tiles, &w.grid[0].scan_ticket);
    hipLaunchKernelGGL(k_scan, dim3(nt), dim3(kBlock), 0, st, in, out, len_ptr, max_len, w.tiles,
                       &w.grid[0].scan_ticket, zero_in, &w.grid[0]);
}

void launch_read_agents(const bdm_soa &s, const ReadOut &o, hipStream_t st) {
    hipLaunchKernelGGL(k_read_agents, dim3(blocks_for(s.capacity)), dim3(kBlock), 0, st, s.n, s, o);
}

}  // namespace bdm
