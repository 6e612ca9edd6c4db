// k_sir.hip -- SIR epidemiology step on gfx950 (paper Sec. 3.3: infection with a probability
// when an infected agent is within the infection radius, recovery with a probability each
// step, bounded random movement, agents counted per group).
//
// One lane per agent in box-sorted order on the periodic grid of positions at t.  Everything
// reads state/positions at t (the sorted copies in the workspace) and writes t+1 into the
// caller's arrays, so the update is synchronous.  The infected neighbours of each susceptible
// agent are counted from the infected side (k_sir_seed) before the step.  Random numbers are Philox blocks keyed by
// (seed, salt) at counter (purpose + attempt*2^8, agent id, step, 0): the outcome of every agent
// depends only on its id and the step, never on the order of the lanes.
#include "kernels.hpp"

namespace bdm {

__device__ __forceinline__ double min_image(double v, double L, double half) {
    if (v > half) return v - L;
    if (v < -half) return v + L;
    return v;
}

__device__ __forceinline__ double wrap(double v, double L) {
    if (v < 0.0) v += L;
    if (v >= L) v -= L;
    if (v == L) v = 0.0;
    return v;
}

// Contact counts of the susceptible agents, zeroed before they are gathered.
__global__ __launch_bounds__(kBlock) void k_sir_zero(Slots sl, uint32_t *__restrict__ m) {
    const int64_t tile = blockIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    const GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    const int64_t l = tile * kBlock + threadIdx.x - S.agent_off;
    if (g->valid && l < g->n) m[g->sorted_base + l] = 0u;
}

// Every infected agent adds one to the count m of each susceptible agent within the infection
// radius (inclusive, periodic minimum image) among its 27 boxes.  This is the count each
// susceptible agent would find among its own 27 boxes: the periodic box neighbourhood is
// symmetric (at least 3 boxes per axis), and the differences are taken as susceptible minus
// infected, exactly as the susceptible agent takes them.  The count is an integer, so the order
// of the additions does not matter.  The work is proportional to the infected agents.  Each
// wavefront takes its infected agents one at a time, one of its lanes per box of the agent's 27,
// so an infected agent costs one box's chain of dependent loads, not 27 of them in a row.
__global__ __launch_bounds__(kBlock) void k_sir_seed(Slots sl, const double4 *__restrict__ pos4,
                                                     const uint8_t *__restrict__ state_s,
                                                     const uint32_t *__restrict__ start_all, SirArgs a,
                                                     uint32_t *m) {
    const int64_t tile = blockIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    const GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    const int64_t l = tile * kBlock + threadIdx.x - S.agent_off;
    const bool live = g->valid && l < g->n && l < S.capacity;
    const uint32_t q = live ? uint32_t(g->sorted_base + l) : 0u;
    unsigned long long inf = __ballot(live && state_s[q] == 1);
    if (!inf) return;  // (the whole wavefront)
    const uint32_t *start = start_all + S.box_off;
    const int nb = g->dims[0];
    const double b = g->b;
    const int lane = threadIdx.x & 63;
    const int ox = lane % 3 - 1, oy = (lane / 3) % 3 - 1, oz = lane / 9 - 1;  // lanes 0-26
    while (inf) {
        const int k = __ffsll(static_cast<long long>(inf)) - 1;
        inf &= inf - 1ull;
        const uint32_t qi = uint32_t(__shfl(int(q), k, 64));
        if (lane >= 27) continue;
        const double4 p = pos4[qi];
        const int xx = (box_coord(p.x, b, 0, nb, true) + ox + nb) % nb;
        const int yy = (box_coord(p.y, b, 0, nb, true) + oy + nb) % nb;
        const int zz = (box_coord(p.z, b, 0, nb, true) + oz + nb) % nb;
        const uint32_t kb = uint32_t(xx) + uint32_t(nb) * (uint32_t(yy) + uint32_t(nb) * uint32_t(zz));
        const uint32_t j1 = start[kb + 1];
        for (uint32_t j = start[kb]; j < j1; ++j) {
            if (state_s[j] != 0) continue;
            const double4 c = pos4[j];
            const double dx = min_image(c.x - p.x, a.L, a.half);
            const double dy = min_image(c.y - p.y, a.L, a.half);
            const double dz = min_image(c.z - p.z, a.L, a.half);
            if (((dx * dx + dy * dy) + dz * dz) <= a.r2) atomicAdd(&m[j], 1u);
        }
    }
}

// Five wavefronts per SIMD (96 registers, a few spilled; the Philox draws take many) instead of
// the four that the compiler's 110 allow: 2 % faster per SIR step.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_sir(Slots sl, const double4 *__restrict__ pos4,
                                                const uint8_t *__restrict__ state_s,
                                                const uint32_t *__restrict__ id_s,
                                                const uint32_t *__restrict__ m_s, SirArgs a,
                                                bdm_soa out, uint32_t *__restrict__ tile_counts) {
    const int64_t tile = blockIdx.x;
    const int slot = slot_of_tile(sl, tile);
    if (slot < 0) return;
    GridDev *g = &sl.grids[slot];
    const SlotDev S = slot_record(sl, slot);
    const int64_t l = tile * kBlock + threadIdx.x - S.agent_off;
    const bool live = g->valid && l < g->n && l < S.capacity;
    uint8_t ns = 3;  // no agent
    if (live) {
        const uint32_t q = uint32_t(g->sorted_base + l);
        const double4 p = pos4[q];
        const uint8_t st = state_s[q];
        const uint32_t me = id_s[q];
        ns = st;
        if (st == 0) {
            const uint32_t m = m_s[q];  // infected agents within the radius (k_sir_seed)
            for (uint32_t c = 0; c < m; ++c) {
                if (bernoulli(draw(a.seed, a.salt, kRngInf, c, me, a.step).w[0], a.tinf)) {
                    ns = 1;
                    break;
                }
            }
        } else if (st == 1) {
            if (bernoulli(draw(a.seed, a.salt, kRngRec, 0, me, a.step).w[0], a.trec)) ns = 2;
        }
        const Block4 w = draw(a.seed, a.salt, kRngMove, 0, me, a.step);
        const int64_t o = S.agent_off + l;
        out.x[o] = wrap(p.x + a.walk * (2.0 * u01(w.w[0]) - 1.0), a.L);
        out.y[o] = wrap(p.y + a.walk * (2.0 * u01(w.w[1]) - 1.0), a.L);
        out.z[o] = wrap(p.z + a.walk * (2.0 * u01(w.w[2]) - 1.0), a.L);
        out.state[o] = ns;
        out.id[o] = me;
    }
    // S/I/R totals of the tile, summed over the tiles by k_sir_total.  (Atomics from every
    // wavefront onto the three totals serialised at the memory side: about 2 ms per step at
    // 10^7 agents.)
    __shared__ uint32_t s_cnt[kBlock / 64][3];
    const uint32_t cs = wave_sum(ns == 0), ci = wave_sum(ns == 1), cr = wave_sum(ns == 2);
    if ((threadIdx.x & 63) == 0) {
        s_cnt[threadIdx.x >> 6][0] = cs;
        s_cnt[threadIdx.x >> 6][1] = ci;
        s_cnt[threadIdx.x >> 6][2] = cr;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t v = 0;
        for (int w = 0; w < kBlock / 64; ++w) v += s_cnt[w][threadIdx.x];
        tile_counts[4 * tile + threadIdx.x] = v;
    }
}

// The S/I/R totals of a plain step: the tiles' counts summed by kTotalGroups workgroups.  Each
// adds its share to an accumulator, and the last one to finish (a ticket) records the totals and
// resets the accumulator and the ticket for the next step.  (One workgroup took 18 us for the
// 39 063 tiles of 10^7 agents.)
constexpr int kTotalThreads = 1024;
constexpr unsigned kTotalGroups = 64;
__global__ __launch_bounds__(kTotalThreads) void k_sir_total(GridDev *g, const uint32_t *__restrict__ tile_counts,
                                                             int64_t ntiles) {
    __shared__ unsigned long long s_part[kTotalThreads / 64][3];
    unsigned long long v[3] = {0ull, 0ull, 0ull};
    for (int64_t t = int64_t(blockIdx.x) * kTotalThreads + threadIdx.x; t < ntiles;
         t += int64_t(gridDim.x) * kTotalThreads)
        for (int k = 0; k < 3; ++k) v[k] += tile_counts[4 * t + k];
    for (int d = 32; d >= 1; d >>= 1)
        for (int k = 0; k < 3; ++k) v[k] += __shfl_xor(v[k], d, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 3; ++k) s_part[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 3; ++k) {
        unsigned long long sum = 0ull;
        for (int w = 0; w < kTotalThreads / 64; ++w) sum += s_part[w][k];
        atomicAdd(&g->sir_acc[k], sum);
    }
    __threadfence();
    if (atomicAdd(&g->sir_ticket, 1u) != gridDim.x - 1) return;
    __threadfence();
    for (int k = 0; k < 3; ++k) {
        g->sir_counts[k] = atomicAdd(&g->sir_acc[k], 0ull);
        g->sir_acc[k] = 0ull;
    }
    g->sir_ticket = 0u;
}

// Test hook: SIR contacts (any state) per sorted slot, boxes visited in (dz, dy, dx) order.
__global__ __launch_bounds__(kBlock) void k_contacts_periodic(Slots sl, const double4 *__restrict__ pos4,
                                                              const uint32_t *__restrict__ id_s,
                                                              const uint32_t *__restrict__ start,
                                                              ContactArgs a, uint32_t *counts,
                                                              const int64_t *offsets, uint32_t *ids) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const GridDev *g = &sl.grids[0];
    if (!g->valid || s >= g->n) return;
    const double4 p = pos4[s];
    const int nb = g->dims[0];
    const double b = g->b;
    const int cx = box_coord(p.x, b, 0, nb, true);
    const int cy = box_coord(p.y, b, 0, nb, true);
    const int cz = box_coord(p.z, b, 0, nb, true);
    uint32_t c = 0;
    for (int oz = -1; oz <= 1; ++oz) {
        const int zz = (cz + oz + nb) % nb;
        for (int oy = -1; oy <= 1; ++oy) {
            const int yy = (cy + oy + nb) % nb;
            for (int ox = -1; ox <= 1; ++ox) {
                const int xx = (cx + ox + nb) % nb;
                const uint32_t kb = uint32_t(xx) + uint32_t(nb) * (uint32_t(yy) + uint32_t(nb) * uint32_t(zz));
                for (uint32_t j = start[kb]; j < start[kb + 1]; ++j) {
                    if (j == uint32_t(s)) continue;
                    const double4 q = pos4[j];
                    const double dx = min_image(p.x - q.x, a.L, a.half);
                    const double dy = min_image(p.y - q.y, a.L, a.half);
                    const double dz = min_image(p.z - q.z, a.L, a.half);
                    if (((dx * dx + dy * dy) + dz * dz) <= a.r2) {
                        if (ids) ids[offsets[s] + c] = id_s[j];
                        ++c;
                    }
                }
            }
        }
    }
    counts[s] = c;
}

void launch_sir(const bdm_soa &s, const Slots &sl, int64_t capacity, const SirArgs &a, const Ws &w,
                hipStream_t st) {
    int64_t nb = (capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    // the contact counts live in the division-flag array, free once the grid is built
    hipLaunchKernelGGL(k_sir_zero, dim3(unsigned(nb)), dim3(kBlock), 0, st, sl, w.flagid);
    hipLaunchKernelGGL(k_sir_seed, dim3(unsigned(nb)), dim3(kBlock), 0, st, sl, w.pos4, w.state, w.start, a,
                       w.flagid);
    // the tiles' S/I/R counts go to the bounds partials (free once the grid is built; 16 bytes
    // per 256 agents fit in their 64 bytes per 1024)
    uint32_t *tile_counts = reinterpret_cast<uint32_t *>(w.partials);
    hipLaunchKernelGGL(k_sir, dim3(unsigned(nb)), dim3(kBlock), 0, st, sl, w.pos4, w.state, w.ids, w.flagid, a, s,
                       tile_counts);
    hipLaunchKernelGGL(k_sir_total, dim3(kTotalGroups), dim3(kTotalThreads), 0, st, sl.grids, tile_counts, nb);
}

void launch_contacts(const ContactArgs &a, const Slots &sl, const Ws &w, uint32_t *counts,
                     const int64_t *offsets, uint32_t *ids, hipStream_t st) {
    if (a.mode != 2) {
        launch_contacts_mech(a.mode == 1, sl, w, counts, offsets, ids, st);
        return;
    }
    int64_t nb = (w.lay.capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_contacts_periodic, dim3(unsigned(nb)), dim3(kBlock), 0, st, sl, w.pos4, w.ids,
                       w.start, a, counts, offsets, ids);
}

}  // namespace bdm
