// k_grid.hip -- uniform-grid build on gfx950 (paper Sec. 2.1: equal boxes, agents binned by
// centre, box edge from the largest agent, 27-box neighbourhood).
//
// Pipeline (one launch each, all device-resident, no host read-back):
//   bounds     min/max of x, y, z and max diameter over the live agents (order-encoded
//              64-bit atomics, one per workgroup and quantity); also resets the scan tiles
//   finalize   one wavefront: box edge, lattice origin and dims, box count check
//   key_count  box key per agent and its arrival rank in the box (integer atomics)
//   scan       single-pass decoupled look-back exclusive scan of the histogram into start[]
//   scatter    ids into their box range in arrival order
//   canon      each agent counts the smaller ids in its box (ascending-id order inside a box)
//              and copies itself into the sorted SoA copy (x, y, z, d packed as double4)
#include "kernels.hpp"

namespace bdm {

__global__ __launch_bounds__(kBlock) void k_bounds(const int64_t *n_ptr, int64_t capacity,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ d, GridDev *g,
                                                   unsigned long long *tiles, int64_t max_tiles) {
    const int64_t n = live_count(n_ptr, capacity);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t t = gi; t < max_tiles; t += stride) tiles[t] = 0ull;
    if (gi == 0) g->scan_ticket = 0u;

    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    double dmax = 0.0;
    uint32_t bad = 0;
    for (int64_t i = gi; i < n; i += stride) {
        double p[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            bad |= !__builtin_isfinite(p[a]);
            lo[a] = fmin(lo[a], p[a]);
            hi[a] = fmax(hi[a], p[a]);
        }
        if (d) {
            double v = d[i];
            bad |= !__builtin_isfinite(v);
            dmax = fmax(dmax, v);
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], s, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], s, 64));
        }
        dmax = fmax(dmax, __shfl_xor(dmax, s, 64));
        bad |= __shfl_xor(bad, s, 64);
    }
    __shared__ double s_red[kBlock / 64][8];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        for (int a = 0; a < 3; ++a) {
            s_red[wave][a] = lo[a];
            s_red[wave][3 + a] = hi[a];
        }
        s_red[wave][6] = dmax;
        s_red[wave][7] = bad ? 1.0 : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(lo[a], s_red[w][a]);
                hi[a] = fmax(hi[a], s_red[w][3 + a]);
            }
            dmax = fmax(dmax, s_red[w][6]);
            bad |= s_red[w][7] != 0.0;
        }
        if (bad) atomicOr(&g->red_bad, 1u);
        if (lo[0] <= hi[0]) {  // this workgroup saw at least one finite agent
            for (int a = 0; a < 3; ++a) {
                atomicMin(&g->red_min[a], ord_enc(lo[a]));
                atomicMax(&g->red_max[a], ord_enc(hi[a]));
            }
        }
        if (d) atomicMax(&g->red_dmax, ord_enc(dmax));
    }
}

__global__ void k_finalize(const int64_t *n_ptr, int64_t capacity, GridDev *g, FinalizeArgs a) {
    if (threadIdx.x != 0) return;
    const int64_t n_raw = *n_ptr;
    const int64_t n = live_count(n_ptr, capacity);
    const double dmax = a.has_d ? ord_dec(g->red_dmax) : 0.0;
    double lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        lo[i] = ord_dec(g->red_min[i]);
        hi[i] = ord_dec(g->red_max[i]);
    }
    const uint32_t bad = g->red_bad;
    // reset the reductions for the next build
    for (int i = 0; i < 3; ++i) {
        g->red_min[i] = ~0ull;
        g->red_max[i] = 0ull;
    }
    g->red_dmax = 0ull;
    g->red_bad = 0u;
    g->sir_counts[0] = g->sir_counts[1] = g->sir_counts[2] = 0ull;
    g->valid = 0;
    g->n = n;
    g->nboxes = 0;
    if (n_raw != n) {
        g->flags |= BDM_FLAG_BADCOUNT;
        return;
    }
    if (bad) {
        g->flags |= BDM_FLAG_NONFINITE;
        return;
    }
    double b;
    if (a.periodic) {
        if (a.box < dmax) {
            g->flags |= BDM_FLAG_BOXSMALL;
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
            return;
        }
        for (int i = 0; i < 3; ++i) {
            // floor is monotone, so min/max of floor(x/b) are floor(min x / b), floor(max x / b)
            double c0 = floor(lo[i] / b), c1 = floor(hi[i] / b);
            if (!(c0 >= -1073741824.0 && c1 <= 1073741823.0)) {
                g->flags |= BDM_FLAG_NONFINITE;
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
        return;
    }
    g->nboxes = int64_t(g->dims[0]) * g->dims[1] * g->dims[2];
    g->valid = 1;
}

__global__ __launch_bounds__(kBlock) void k_key_count(const GridDev *__restrict__ g,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z,
                                                      uint32_t *count, uint32_t *__restrict__ key,
                                                      uint32_t *__restrict__ rank, int periodic) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!g->valid || i >= g->n) return;
    const double b = g->b;
    const int cx = box_coord(x[i], b, g->cmin[0], g->dims[0], periodic);
    const int cy = box_coord(y[i], b, g->cmin[1], g->dims[1], periodic);
    const int cz = box_coord(z[i], b, g->cmin[2], g->dims[2], periodic);
    const uint32_t k = uint32_t(cx) + uint32_t(g->dims[0]) * (uint32_t(cy) + uint32_t(g->dims[1]) * uint32_t(cz));
    key[i] = k;
    rank[i] = atomicAdd(&count[k], 1u);
}

__global__ __launch_bounds__(kBlock) void k_scan_prepare(unsigned long long *tiles, int64_t max_tiles,
                                                         uint32_t *ticket) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < max_tiles) tiles[t] = 0ull;
    if (t == 0) *ticket = 0u;
}

// Exclusive scan of in[0, len) into out[0, len], out[len] = total; len read on the device.
// Tiles are taken in launch order from a ticket, so a tile only ever waits on tiles that are
// already running.  Tile status word: value << 32 | flag (1 = tile aggregate, 2 = inclusive
// prefix).  Wavefront 0 looks back 64 predecessors at a time with ballots.
__global__ __launch_bounds__(kBlock) void k_scan(uint32_t *in, uint32_t *out, const int64_t *len_ptr,
                                                 const int32_t *gate, unsigned long long *tiles,
                                                 uint32_t *ticket, int zero_in, GridDev *g) {
    __shared__ uint32_t s_tile, s_prefix;
    __shared__ uint32_t s_wave[kBlock / 64];
    if (gate && *gate == 0) return;
    const int64_t len = *len_ptr;
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
    if (base + kScanItems <= len + 1 && base + kScanItems <= len) {
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

__global__ __launch_bounds__(kBlock) void k_scatter_id(GridDev *__restrict__ g,
                                                       const uint32_t *__restrict__ key,
                                                       const uint32_t *__restrict__ rank,
                                                       const uint32_t *__restrict__ start,
                                                       const uint32_t *__restrict__ id,
                                                       uint32_t *__restrict__ tmpid) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!g->valid || i >= g->n) return;
    const uint32_t slot = start[key[i]] + rank[i];
    if (slot >= g->n) {  // cannot happen with a zeroed histogram; guards memory all the same
        atomicOr(&g->flags, BDM_FLAG_SCAN);
        return;
    }
    tmpid[slot] = id[i];
}

__global__ __launch_bounds__(kBlock) void k_canon(const GridDev *__restrict__ g, SoaIn s,
                                                  const uint32_t *__restrict__ key,
                                                  const uint32_t *__restrict__ start,
                                                  const uint32_t *__restrict__ tmpid,
                                                  double4 *__restrict__ pos4, double *__restrict__ adh_s,
                                                  uint32_t *__restrict__ id_s,
                                                  uint8_t *__restrict__ state_s) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!g->valid || i >= g->n) return;
    const uint32_t k = key[i];
    const uint32_t s0 = start[k];
    const uint32_t s1 = min(start[k + 1], uint32_t(g->n));
    const uint32_t me = s.id[i];
    uint32_t r = 0;
    for (uint32_t j = s0; j < s1; ++j) r += tmpid[j] < me;
    const uint32_t dst = s0 + r;
    if (dst >= s1) return;
    pos4[dst] = make_double4(s.x[i], s.y[i], s.z[i], s.d ? s.d[i] : 0.0);
    if (s.adh) adh_s[dst] = s.adh[i];
    id_s[dst] = me;
    if (s.state) state_s[dst] = s.state[i];
}

__global__ __launch_bounds__(kBlock) void k_read_agents(const int64_t *n_ptr, const bdm_soa s,
                                                        ReadOut o) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, s.capacity);
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
static inline unsigned blocks_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return unsigned(b < 1 ? 1 : b);
}

void launch_grid_build(const bdm_soa &s, const FinalizeArgs &fa, const Ws &w, hipStream_t st) {
    const int64_t cap = s.capacity;
    unsigned nb_bounds = blocks_for(cap);
    if (nb_bounds > 2048) nb_bounds = 2048;
    hipLaunchKernelGGL(k_bounds, dim3(nb_bounds), dim3(kBlock), 0, st, s.n, s.capacity, s.x, s.y, s.z,
                       fa.has_d ? s.diam : nullptr, w.grid, w.tiles, w.lay.max_tiles);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, s.n, s.capacity, w.grid, fa);
    const unsigned nb = blocks_for(cap);
    hipLaunchKernelGGL(k_key_count, dim3(nb), dim3(kBlock), 0, st, w.grid, s.x, s.y, s.z, w.count,
                       w.key, w.rank, int(fa.periodic));
    launch_scan(w.count, w.start, &w.grid->nboxes, &w.grid->valid, w.lay.max_boxes, w, 1, false, st);
    hipLaunchKernelGGL(k_scatter_id, dim3(nb), dim3(kBlock), 0, st, w.grid, w.key, w.rank, w.start,
                       s.id, w.tmpid);
    SoaIn in{s.x, s.y, s.z, fa.has_d ? s.diam : nullptr, s.adh, s.id, s.state};
    hipLaunchKernelGGL(k_canon, dim3(nb), dim3(kBlock), 0, st, w.grid, in, w.key, w.start, w.tmpid,
                       w.pos4, w.adh, w.ids, w.state);
}

void launch_scan(uint32_t *in, uint32_t *out, const int64_t *len_ptr, const int32_t *gate,
                 int64_t max_len, const Ws &w, int zero_in, bool prepare, hipStream_t st) {
    const unsigned nt = unsigned((max_len + kScanTile) / kScanTile);
    if (prepare)
        hipLaunchKernelGGL(k_scan_prepare, dim3(blocks_for(w.lay.max_tiles)), dim3(kBlock), 0, st,
                           w.tiles, w.lay.max_tiles, &w.grid->scan_ticket);
    hipLaunchKernelGGL(k_scan, dim3(nt), dim3(kBlock), 0, st, in, out, len_ptr, gate, w.tiles,
                       &w.grid->scan_ticket, zero_in, w.grid);
}

void launch_read_agents(const bdm_soa &s, const ReadOut &o, hipStream_t st) {
    hipLaunchKernelGGL(k_read_agents, dim3(blocks_for(s.capacity)), dim3(kBlock), 0, st, s.n, s, o);
}

}  // namespace bdm
