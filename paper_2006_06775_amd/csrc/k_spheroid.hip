// k_spheroid.hip -- tumour-spheroid behaviour on gfx950 (paper Sec. 3.2: cell growth, duplication,
// apoptosis and Brownian migration; the cell growth & division benchmark of Sec. 3.4).  Plain
// calls (one slot).
//
//   apo_flag   survival flag by agent id: dies iff word 0 of (APO, id, step) is below the
//              threshold floor(p_apo * 2^64)
//   scan       exclusive scan of the survival flags in id order: the new id of each survivor
//   apo_stage  survivor -> staging slot (its new id), in the workspace's sorted-copy arrays
//              (position and diameter, adherence, and the state when the caller keeps one)
//   apo_commit staging -> slots 0 .. n'-1 of the caller's arrays, id = slot
//   apo_count  n = n'
//   migrate    every live agent moves by walk * (2u - 1) per axis, u from (MIG, id, step)
//
//   grow_flag  diam *= grow for every live agent; division flag by agent id (diam >= div_d);
//              also clears the scan tiles for the rank scan that follows
//   scan       exclusive scan of the flags in id order: rank of each dividing mother by id
//   divide     mother of rank r puts its daughter in slot n + r (id n + r) when that is below
//              capacity; random axis by rejection from Philox (DIV, attempt, id, step)
//   append     n += number of daughters that fitted
// The live count stays on the device; nothing is read back to the host.
#include "kernels.hpp"

namespace bdm {

__global__ __launch_bounds__(kBlock) void k_grow_flag(const int64_t *n_ptr, int64_t capacity,
                                                      double *diam, const uint32_t *__restrict__ id,
                                                      DivArgs a, uint32_t *flagid,
                                                      unsigned long long *tiles, int64_t max_tiles,
                                                      uint32_t *ticket, GridDev *g) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < max_tiles) tiles[i] = 0ull;
    if (i == 0) *ticket = 0u;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n) return;
    const double d = diam[i] * a.grow;
    diam[i] = d;
    const uint32_t me = id[i];
    if (me >= n) {
        atomicOr(&g->flags, BDM_FLAG_BADID);
        return;
    }
    flagid[me] = d >= a.div_d ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_divide(const int64_t *n_ptr, int64_t capacity, bdm_soa s,
                                                   const uint32_t *__restrict__ rankid, DivArgs a,
                                                   GridDev *g) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n) return;
    const double d = s.diam[i];
    if (!(d >= a.div_d)) return;
    const uint32_t me = s.id[i];
    if (me >= n) return;
    const int64_t slot = n + int64_t(rankid[me]);
    if (slot >= capacity) {
        atomicOr(&g->flags, BDM_FLAG_CAPACITY);
        return;
    }
    double ux = 1.0, uy = 0.0, uz = 0.0;
    for (uint64_t attempt = 0; attempt < 64; ++attempt) {
        const Block4 w = draw(a.seed, a.salt, kRngDiv, attempt, me, a.step);
        const double vx = 2.0 * u01(w.w[0]) - 1.0;
        const double vy = 2.0 * u01(w.w[1]) - 1.0;
        const double vz = 2.0 * u01(w.w[2]) - 1.0;
        const double q = (vx * vx + vy * vy) + vz * vz;
        if (q > 0.0 && q <= 1.0) {
            const double norm = __builtin_sqrt(q);
            ux = vx / norm;
            uy = vy / norm;
            uz = vz / norm;
            break;
        }
    }
    const double dp = d * a.half_cbrt;
    const double qd = 0.25 * dp;
    const double ox = qd * ux, oy = qd * uy, oz = qd * uz;
    const double x = s.x[i], y = s.y[i], z = s.z[i];
    s.x[slot] = x + ox;
    s.y[slot] = y + oy;
    s.z[slot] = z + oz;
    s.diam[slot] = dp;
    s.adh[slot] = s.adh[i];
    if (s.state) s.state[slot] = s.state[i];
    s.id[slot] = uint32_t(slot);
    s.x[i] = x - ox;
    s.y[i] = y - oy;
    s.z[i] = z - oz;
    s.diam[i] = dp;
}

__global__ void k_append(int64_t *n_ptr, int64_t capacity, const uint32_t *rankid) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t n = live_count(n_ptr, 0, capacity);
    int64_t nn = n + int64_t(rankid[n]);
    if (nn > capacity) nn = capacity;
    *n_ptr = nn;
}

__global__ __launch_bounds__(kBlock) void k_apo_flag(const int64_t *n_ptr, int64_t capacity,
                                                     const uint32_t *__restrict__ id, ApoArgs a,
                                                     uint32_t *flagid, GridDev *g) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n) return;
    const uint32_t me = id[i];
    if (me >= n) {
        atomicOr(&g->flags, BDM_FLAG_BADID);
        return;
    }
    flagid[me] = bernoulli(draw(a.seed, a.salt, kRngApo, 0, me, a.step).w[0], a.tapo) ? 0u : 1u;
}

// Survivors to the staging arrays at their new ids.  The bounds checks only guard memory when
// the ids were not a permutation of 0 .. n-1 (BDM_FLAG_BADID is then set).
__global__ __launch_bounds__(kBlock) void k_apo_stage(const int64_t *n_ptr, int64_t capacity, bdm_soa s,
                                                      const uint32_t *__restrict__ flagid,
                                                      const uint32_t *__restrict__ rankid, double4 *pos,
                                                      double *adh, uint8_t *state) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n) return;
    const uint32_t me = s.id[i];
    if (me >= n || flagid[me] == 0u) return;
    const int64_t j = rankid[me];
    if (j >= n) return;
    pos[j] = make_double4(s.x[i], s.y[i], s.z[i], s.diam[i]);
    adh[j] = s.adh[i];
    if (s.state) state[j] = s.state[i];
}

__global__ __launch_bounds__(kBlock) void k_apo_commit(const int64_t *n_ptr, int64_t capacity, bdm_soa s,
                                                       const uint32_t *__restrict__ rankid,
                                                       const double4 *__restrict__ pos,
                                                       const double *__restrict__ adh,
                                                       const uint8_t *__restrict__ state) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    int64_t kept = rankid[n];
    if (kept > n) kept = n;
    if (j >= kept) return;
    const double4 p = pos[j];
    s.x[j] = p.x;
    s.y[j] = p.y;
    s.z[j] = p.z;
    s.diam[j] = p.w;
    s.adh[j] = adh[j];
    if (s.state) s.state[j] = state[j];
    s.id[j] = uint32_t(j);
}

__global__ void k_apo_count(int64_t *n_ptr, int64_t capacity, const uint32_t *rankid) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t n = live_count(n_ptr, 0, capacity);
    int64_t kept = rankid[n];
    if (kept > n) kept = n;
    *n_ptr = kept;
}

__global__ __launch_bounds__(kBlock) void k_migrate(const int64_t *n_ptr, int64_t capacity, bdm_soa s,
                                                    MigArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n) return;
    const Block4 w = draw(a.seed, a.salt, kRngMig, 0, s.id[i], a.step);
    s.x[i] = s.x[i] + a.walk * (2.0 * u01(w.w[0]) - 1.0);
    s.y[i] = s.y[i] + a.walk * (2.0 * u01(w.w[1]) - 1.0);
    s.z[i] = s.z[i] + a.walk * (2.0 * u01(w.w[2]) - 1.0);
}

void launch_apoptosis(const bdm_soa &s, int64_t capacity, const ApoArgs &a, const Ws &w, hipStream_t st) {
    int64_t nb = (capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_apo_flag, dim3(unsigned(nb)), dim3(kBlock), 0, st, s.n, capacity, s.id, a, w.flagid,
                       &w.grid[0]);
    launch_scan(w.flagid, w.rankid, s.n, capacity, w, 0, true, st);
    hipLaunchKernelGGL(k_apo_stage, dim3(unsigned(nb)), dim3(kBlock), 0, st, s.n, capacity, s, w.flagid, w.rankid,
                       w.pos4, w.adh, w.state);
    hipLaunchKernelGGL(k_apo_commit, dim3(unsigned(nb)), dim3(kBlock), 0, st, s.n, capacity, s, w.rankid, w.pos4,
                       w.adh, w.state);
    hipLaunchKernelGGL(k_apo_count, dim3(1), dim3(64), 0, st, s.n, capacity, w.rankid);
}

void launch_migrate(const bdm_soa &s, int64_t capacity, const MigArgs &a, hipStream_t st) {
    int64_t nb = (capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_migrate, dim3(unsigned(nb)), dim3(kBlock), 0, st, s.n, capacity, s, a);
}

void launch_grow_divide(const bdm_soa &s, const Slots &sl, int64_t capacity, const DivArgs &a, const Ws &w,
                        hipStream_t st) {
    (void)sl;
    const int64_t cap = capacity;  // daughters must land inside the caller's arrays
    int64_t nb = (cap + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    const int64_t need = w.lay.max_tiles;
    int64_t nb_flag = nb;
    if (nb_flag * kBlock < need) nb_flag = (need + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_grow_flag, dim3(unsigned(nb_flag)), dim3(kBlock), 0, st, s.n, cap, s.diam, s.id, a,
                       w.flagid, w.tiles, w.lay.max_tiles, &w.grid[0].scan_ticket, &w.grid[0]);
    launch_scan(w.flagid, w.rankid, s.n, cap, w, 0, false, st);
    hipLaunchKernelGGL(k_divide, dim3(unsigned(nb)), dim3(kBlock), 0, st, s.n, cap, s, w.rankid, a, &w.grid[0]);
    hipLaunchKernelGGL(k_append, dim3(1), dim3(64), 0, st, s.n, cap, w.rankid);
}

}  // namespace bdm
