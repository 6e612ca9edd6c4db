// k_gen.hip -- seeded initial state, workspace and slot-table maintenance, and the IEEE probe.
//
// Generator: agent i draws Philox4x64-10 blocks at counter (INIT + attempt*2^8, i, 0, 0) keyed
// by (seed, salt); u = (word >> 11) * 2^-53.  Cube: words 0..2 give x, y, z = L*u, word 3 the
// diameter dlo + (dhi - dlo)*u.  Ball: v = 2u - 1 per axis, accepted when |v|^2 <= 1 (at most 64
// attempts, else the origin), position L*v.  SIR: cube positions, state 1 for id < n_infected.
// Soma: cube positions and diameters, cell type (state) id mod 2.
// The paper places tumour cells in a ball (Sec. 3.2) and persons at random in a cube (Sec. 3.3).
#include "kernels.hpp"

namespace bdm {

__global__ __launch_bounds__(kBlock) void k_generate(bdm_soa s, GenArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) *s.n = a.n;
    if (i >= a.n) return;
    double x = 0.0, y = 0.0, z = 0.0, u3 = 0.0;
    if (a.kind == BDM_GEN_BALL) {
        for (uint64_t attempt = 0; attempt < 64; ++attempt) {
            const Block4 w = draw(a.seed, a.salt, kRngInit, attempt, uint64_t(i), 0);
            const double vx = 2.0 * u01(w.w[0]) - 1.0;
            const double vy = 2.0 * u01(w.w[1]) - 1.0;
            const double vz = 2.0 * u01(w.w[2]) - 1.0;
            if ((vx * vx + vy * vy) + vz * vz <= 1.0) {
                x = a.L * vx;
                y = a.L * vy;
                z = a.L * vz;
                u3 = u01(w.w[3]);
                break;
            }
        }
    } else {
        const Block4 w = draw(a.seed, a.salt, kRngInit, 0, uint64_t(i), 0);
        x = a.L * u01(w.w[0]);
        y = a.L * u01(w.w[1]);
        z = a.L * u01(w.w[2]);
        u3 = u01(w.w[3]);
    }
    s.x[i] = x;
    s.y[i] = y;
    s.z[i] = z;
    if (s.diam) s.diam[i] = a.dlo + (a.dhi - a.dlo) * u3;
    if (s.adh) s.adh[i] = a.adh;
    if (s.fx) s.fx[i] = 0.0;
    if (s.fy) s.fy[i] = 0.0;
    if (s.fz) s.fz[i] = 0.0;
    s.id[i] = uint32_t(i);
    if (s.state) {
        uint8_t st = 0;
        if (a.kind == BDM_GEN_SIR && i < a.n_infected) st = 1;
        if (a.kind == BDM_GEN_SOMA) st = uint8_t(i & 1);
        s.state[i] = st;
    }
}

__global__ __launch_bounds__(kBlock) void k_fp_probe(const double *a, const double *b, int64_t n,
                                                     double *os, double *od, float *osf, float *odf) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = a[i], y = b[i];
    if (os) os[i] = __builtin_sqrt(x);
    if (od) od[i] = x / y;
    if (osf) osf[i] = __builtin_sqrtf(float(x));
    if (odf) odf[i] = float(x) / float(y);
}

__device__ void clear_grid(GridDev *g) {
    g->b = 0.0;
    for (int a = 0; a < 3; ++a) {
        g->cmin[a] = 0;
        g->dims[a] = 0;
        g->sir_counts[a] = 0ull;
    }
    g->nboxes = 0;
    g->n = 0;
    g->valid = 0;
    g->flags = 0u;
    g->scan_ticket = 0u;
    g->crowd_n = 0u;
    g->sorted_base = 0;
    g->kind = kGridNone;
    g->consumed = 0;
    g->mark_ready = 0;
    g->law_k = g->law_gamma = g->law_box = 0.0;
    g->law_bits = 0;
    g->frozen = 0;
    g->skip_ok = 0;
    g->skipped = 0;
    g->skip_acc = 0ull;
    g->consume_ticket = 0u;
    g->sir_acc[0] = g->sir_acc[1] = g->sir_acc[2] = 0ull;
    g->sir_ticket = 0u;
    g->rekey = 0;
    g->rezero = 0;
}

// Zero the grid records, the histogram and the scan tiles; empty the batch slot table.
__global__ __launch_bounds__(kBlock) void k_ws_init(GridDev *g, int64_t ngrid, uint32_t *count, int64_t ncount,
                                                    unsigned long long *tiles, int64_t ntiles, SlotDev *slots,
                                                    int32_t *tilemap, int64_t ntilemap, int32_t *bucketmap,
                                                    int64_t nbucketmap, uint32_t *runs, int64_t nruns) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t k = i; k < ncount; k += stride) count[k] = 0u;
    for (int64_t k = i; k < ntiles; k += stride) tiles[k] = 0ull;
    for (int64_t k = i; k < ntilemap; k += stride) tilemap[k] = -1;
    for (int64_t k = i; k < nbucketmap; k += stride) bucketmap[k] = -1;
    for (int64_t k = i; k < nruns; k += stride) runs[k] = 0xFFFFFFFFu;  // no run in any bin
    for (int64_t k = i; k < ngrid; k += stride) {
        clear_grid(&g[k]);
        if (slots) {
            SlotDev z{};
            slots[k] = z;
        }
    }
}

// Write one slot record and point its tiles and buckets at it (rec.capacity < 0 clears the
// slot: its tiles point nowhere and its record is zeroed).  Runs on the stream, so replays see
// it in order.
__global__ __launch_bounds__(kBlock) void k_set_slot(SlotDev *slots, int32_t *tilemap, int32_t *bucketmap,
                                                     GridDev *grids, int32_t slot, SlotDev rec, int64_t first_tile,
                                                     int64_t ntile, int64_t first_bucket, int64_t nbucket,
                                                     int32_t value) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < ntile) tilemap[first_tile + i] = value;
    if (i < nbucket) bucketmap[first_bucket + i] = value;
    if (i == 0) {
        slots[slot] = rec;
        clear_grid(&grids[slot]);
    }
}

// Release the buckets the slot's current record owns (before the record is rewritten).
__global__ __launch_bounds__(kBlock) void k_unmap_buckets(const SlotDev *slots, int32_t *bucketmap, int64_t nbuckets,
                                                          int32_t slot) {
    const SlotDev r = slots[slot];
    if (r.capacity <= 0 || r.max_boxes <= 0) return;
    const int64_t b0 = r.box_off >> kBucketShift, b1 = (r.box_off + r.max_boxes - 1) >> kBucketShift;
    for (int64_t b = b0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; b <= b1 && b < nbuckets;
         b += int64_t(gridDim.x) * blockDim.x)
        if (bucketmap[b] == slot) bucketmap[b] = -1;
}

// One step done for every slot that was running.
__global__ void k_batch_advance(SlotDev *slots, int64_t nslots) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s < nslots && slots[s].steps_left > 0) slots[s].steps_left -= 1;
}

static inline unsigned nblocks(int64_t n, int64_t cap_blocks) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (cap_blocks > 0 && b > cap_blocks) b = cap_blocks;
    return unsigned(b);
}

void launch_generate(const bdm_soa &s, const GenArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_generate, dim3(nblocks(a.n, 0)), dim3(kBlock), 0, st, s, a);
}

void launch_fp_probe(const double *a, const double *b, int64_t n, double *os, double *od, float *osf,
                     float *odf, hipStream_t st) {
    hipLaunchKernelGGL(k_fp_probe, dim3(nblocks(n, 0)), dim3(kBlock), 0, st, a, b, n, os, od, osf, odf);
}

void launch_ws_init(const Ws &w, hipStream_t st) {
    const int64_t ncount = w.lay.nbuckets + 1;
    const int64_t ngrid = w.lay.nslots > 0 ? w.lay.nslots : 1;
    const int64_t nmap = w.lay.nslots > 0 ? w.lay.ntiles : 0;
    const int64_t nbmap = w.lay.nslots > 0 ? w.lay.nbuckets : 0;
    int64_t most = ncount > w.lay.max_tiles ? ncount : w.lay.max_tiles;
    if (nmap > most) most = nmap;
    if (nbmap > most) most = nbmap;
    if (2 * kOrderBins > most) most = 2 * kOrderBins;
    hipLaunchKernelGGL(k_ws_init, dim3(nblocks(most, 4096)), dim3(kBlock), 0, st, w.grid, ngrid, w.count, ncount,
                       w.tiles, w.lay.max_tiles, w.slots, w.tilemap, nmap, w.bucketmap, nbmap, w.order_first,
                       int64_t(2 * kOrderBins));
}

void launch_set_slot(const Ws &w, int32_t slot, const SlotDev &rec, int64_t first_tile, int64_t ntile,
                     int32_t value, hipStream_t st) {
    // release the buckets of the record being replaced, then map the new record's buckets
    hipLaunchKernelGGL(k_unmap_buckets, dim3(64), dim3(kBlock), 0, st, w.slots, w.bucketmap, w.lay.nbuckets, slot);
    int64_t first_bucket = 0, nbucket = 0;
    if (value >= 0 && rec.max_boxes > 0) {
        first_bucket = rec.box_off >> kBucketShift;
        nbucket = ((rec.box_off + rec.max_boxes - 1) >> kBucketShift) - first_bucket + 1;
    }
    const int64_t most = ntile > nbucket ? ntile : nbucket;
    hipLaunchKernelGGL(k_set_slot, dim3(nblocks(most, 0)), dim3(kBlock), 0, st, w.slots, w.tilemap, w.bucketmap,
                       w.grid, slot, rec, first_tile, ntile, first_bucket, nbucket, value);
}

// Box starts as a reader sees them: without the stationary-skip marks of bit 31.
__global__ __launch_bounds__(kBlock) void k_mask_starts(uint32_t *p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] &= kStartMask;
}

void launch_mask_starts(uint32_t *p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_mask_starts, dim3(nblocks(n, 0)), dim3(kBlock), 0, st, p, n);
}

// The status bits of a plain workspace's grid record into a caller's device word.
__global__ void k_copy_flags(const GridDev *g, uint32_t *out) {
    if (threadIdx.x == 0) out[0] = g->flags;
}

void launch_copy_flags(const Ws &w, uint32_t *out, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_flags, dim3(1), dim3(64), 0, st, w.grid, out);
}

void launch_batch_advance(const Ws &w, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_advance, dim3(nblocks(w.lay.nslots, 0)), dim3(kBlock), 0, st, w.slots,
                       w.lay.nslots);
}

}  // namespace bdm
