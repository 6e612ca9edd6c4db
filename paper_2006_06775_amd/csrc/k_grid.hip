// k_grid.hip -- uniform-grid build on gfx950 (paper Sec. 2.1: equal boxes, agents binned by
// centre, box edge from the largest agent, 27-box neighbourhood).
//
// Pipeline for every slot at once (one launch each, all device-resident, no host read-back):
//   bounds     min/max of x, y, z and max diameter over each slot's live agents
//              (order-encoded 64-bit atomics, one per workgroup and quantity)
//   finalize   one lane per slot: box edge, lattice origin and dims, box count check
//   key_count  box key per agent and its arrival rank in the box (integer atomics)
//   scan       single-pass decoupled look-back exclusive scan of the packed histogram
//   scatter    ids into their box range in arrival order
//   canon      each agent counts the smaller ids in its box (ascending-id order inside a box)
//              and copies itself into the sorted copy: (x, y, z, r = d/2) packed as double4
//              (halving and doubling a binary64 are exact, so d = 2r is recovered bit for bit)
//   order      one workgroup: the processing order of the mechanics tiles (pencils of rows
//              swept along z, so that the three z-planes a tile reads stay in one XCD's L2)
#include "kernels.hpp"

namespace bdm {

constexpr int kPencilRows = 16;       // y-rows per pencil of the processing order
constexpr int kOrderBins = 8192;      // largest pencil x z-plane count the order kernel sorts

__global__ __launch_bounds__(kBlock) void k_bounds(Slots sl, const int64_t *n_ptr,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ d,
                                                   unsigned long long *tiles, int64_t max_tiles) {
    const int64_t base = int64_t(blockIdx.x) * kBoundsTile;
    if (blockIdx.x == 0) {  // reset the scan tiles of the coming histogram scan
        for (int64_t t = threadIdx.x; t < max_tiles; t += blockDim.x) tiles[t] = 0ull;
        if (threadIdx.x == 0) sl.grids[0].scan_ticket = 0u;
    }
    const int slot = slot_of_tile(sl, base / kBlock);
    if (slot < 0) return;
    const SlotDev S = slot_record(sl, slot);
    GridDev *g = &sl.grids[slot];
    const int64_t n = live_count(n_ptr, slot, S.capacity);
    const int64_t l0 = base - S.agent_off;  // local index of the workgroup's first agent
    if (l0 >= n) return;
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    double dmax = 0.0;
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
        lo[0] = fmin(lo[0], px[u]);
        hi[0] = fmax(hi[0], px[u]);
        lo[1] = fmin(lo[1], py[u]);
        hi[1] = fmax(hi[1], py[u]);
        lo[2] = fmin(lo[2], pz[u]);
        hi[2] = fmax(hi[2], pz[u]);
        dmax = fmax(dmax, pd[u]);
    }
    uint32_t badw = bad ? 1u : 0u;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], s, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], s, 64));
        }
        dmax = fmax(dmax, __shfl_xor(dmax, s, 64));
        badw |= __shfl_xor(badw, s, 64);
    }
    __shared__ double s_red[kBlock / 64][8];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        for (int a = 0; a < 3; ++a) {
            s_red[wave][a] = lo[a];
            s_red[wave][3 + a] = hi[a];
        }
        s_red[wave][6] = dmax;
        s_red[wave][7] = badw ? 1.0 : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(lo[a], s_red[w][a]);
                hi[a] = fmax(hi[a], s_red[w][3 + a]);
            }
            dmax = fmax(dmax, s_red[w][6]);
            badw |= s_red[w][7] != 0.0;
        }
        if (badw) atomicOr(&g->red_bad, 1u);
        for (int a = 0; a < 3; ++a) {
            atomicMin(&g->red_min[a], ord_enc(lo[a]));
            atomicMax(&g->red_max[a], ord_enc(hi[a]));
        }
        if (d) atomicMax(&g->red_dmax, ord_enc(dmax));
    }
}

// One lane per slot: box edge, lattice, box count; resets the reductions for the next build.
__global__ void k_finalize(Slots sl, const int64_t *n_ptr) {
    const int slot = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (slot >= sl.nslots) return;
    const SlotDev a = slot_record(sl, slot);
    GridDev *g = &sl.grids[slot];
    const int64_t n_raw = n_ptr[slot];
    const int64_t n = live_count(n_ptr, slot, a.capacity);
    const double dmax = a.has_d ? ord_dec(g->red_dmax) : 0.0;
    double lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        lo[i] = ord_dec(g->red_min[i]);
        hi[i] = ord_dec(g->red_max[i]);
    }
    const uint32_t bad = g->red_bad;
    for (int i = 0; i < 3; ++i) {
        g->red_min[i] = ~0ull;
        g->red_max[i] = 0ull;
    }
    g->red_dmax = 0ull;
    g->red_bad = 0u;
    g->sir_counts[0] = g->sir_counts[1] = g->sir_counts[2] = 0ull;
    g->valid = 0;
    g->n = 0;
    g->nboxes = 0;
    if (a.steps_left <= 0) return;  // idle batch slot
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
    g->valid = 1;
}

__global__ __launch_bounds__(kBlock) void k_key_count(Slots sl, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, uint32_t *count,
                                                      uint32_t *__restrict__ key,
                                                      uint32_t *__restrict__ rank) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int slot = slot_of_tile(sl, blockIdx.x);
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

__global__ __launch_bounds__(kBlock) void k_scatter_id(Slots sl, const uint32_t *__restrict__ key,
                                                       const uint32_t *__restrict__ rank,
                                                       const uint32_t *__restrict__ start,
                                                       const uint32_t *__restrict__ id,
                                                       uint32_t *__restrict__ tmpid) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int slot = slot_of_tile(sl, blockIdx.x);
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

__global__ __launch_bounds__(kBlock) void k_canon(Slots sl, SoaIn s, const uint32_t *__restrict__ key,
                                                  const uint32_t *__restrict__ start,
                                                  const uint32_t *__restrict__ tmpid,
                                                  double4 *__restrict__ pos4, double *__restrict__ adh_s,
                                                  uint32_t *__restrict__ id_s, uint8_t *__restrict__ state_s,
                                                  uint32_t *__restrict__ tile_key) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int slot = slot_of_tile(sl, blockIdx.x);
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
    pos4[dst] = make_double4(s.x[i], s.y[i], s.z[i], s.d ? 0.5 * s.d[i] : 0.0);  // radius, exact
    if (s.adh) adh_s[dst] = s.adh[i];
    id_s[dst] = me;
    if (s.state) state_s[dst] = s.state[i];
    if (tile_key) {  // key of every tile's first agent (plain calls only: one slot, base 0)
        if ((dst & (kBlock - 1)) == 0) tile_key[dst / kBlock] = k;
    }
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

void launch_grid_build(const bdm_soa &s, const Slots &sl, int64_t capacity, const Ws &w, hipStream_t st) {
    const bool has_d = sl.table ? true : sl.one.has_d != 0;
    const double *d = has_d ? s.diam : nullptr;
    hipLaunchKernelGGL(k_bounds, dim3(blocks_for(capacity, kBoundsTile)), dim3(kBlock), 0, st, sl, s.n,
                       s.x, s.y, s.z, d, w.tiles, w.lay.max_tiles);
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(sl.nslots, 64)), dim3(64), 0, st, sl, s.n);
    const unsigned nb = blocks_for(capacity);
    hipLaunchKernelGGL(k_key_count, dim3(nb), dim3(kBlock), 0, st, sl, s.x, s.y, s.z, w.count, w.key, w.rank);
    launch_scan(w.count, w.start, nullptr, w.lay.max_boxes, w, 1, false, st);
    hipLaunchKernelGGL(k_scatter_id, dim3(nb), dim3(kBlock), 0, st, sl, w.key, w.rank, w.start, s.id, w.tmpid);
    SoaIn in{s.x, s.y, s.z, d, s.adh, s.id, s.state};
    uint32_t *tile_key = sl.table ? nullptr : w.rankid;  // plain calls reuse the rank-by-id area
    hipLaunchKernelGGL(k_canon, dim3(nb), dim3(kBlock), 0, st, sl, in, w.key, w.start, w.tmpid, w.pos4, w.adh,
                       w.ids, w.state, tile_key);
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
