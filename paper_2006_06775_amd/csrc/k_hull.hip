// k_hull.hip -- the device half of the spheroid-diameter observable on gfx950 (paper Sec. 3.2:
// the spheroid diameter is derived from the volume of the convex hull around all cells).
//
// The hull of N cell centres has few vertices, and almost every centre lies inside a polytope
// spanned by a handful of extreme centres.  Two passes over the agents do the O(N) part:
//
//   extreme   for each direction u_k, the agent maximising u_k . x (ties: the smallest slot);
//             a wavefront reduces each direction's key with cross-lane maxima, one atomic per
//             wavefront and direction, then a second pass finds the smallest slot holding it
//   keep      every agent that is not strictly inside all given half-spaces (planes of the
//             polytope spanned by the extreme agents, with a margin) is appended to a list,
//             one atomic per wavefront
//
// Dropping centres strictly inside a polytope whose vertices are centres does not change the
// hull, so the hull of the kept centres is the hull of all of them.  The host builds both
// hulls (of the extreme agents, then of the kept ones); the agents never leave the device.
#include "kernels.hpp"

namespace bdm {

static inline unsigned hull_blocks(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return unsigned(b < 1 ? 1 : b);
}

constexpr int kMaxDirs = BDM_HULL_MAX_DIRS;
constexpr int kMaxPlanes = BDM_HULL_MAX_PLANES;

// Total order of binary64 values as unsigned keys (negative values reversed).
__device__ __forceinline__ uint64_t order_key(double v) {
    const uint64_t b = uint64_t(__double_as_longlong(v));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double support(double ux, double uy, double uz, double x, double y, double z) {
    return (ux * x + uy * y) + uz * z;
}

__global__ void k_extreme_init(int32_t ndir, unsigned long long *work, int32_t *out_slot) {
    const int k = int(threadIdx.x);
    if (k < ndir) {
        work[k] = 0ull;
        out_slot[k] = 0x7fffffff;
    }
}

__global__ __launch_bounds__(kBlock) void k_extreme_max(const int64_t *n_ptr, int64_t capacity, const double *x,
                                                        const double *y, const double *z,
                                                        const double *__restrict__ dirs, int32_t ndir,
                                                        unsigned long long *work) {
    __shared__ double s_dir[3 * kMaxDirs];
    for (int t = threadIdx.x; t < 3 * ndir; t += blockDim.x) s_dir[t] = dirs[t];
    __syncthreads();
    const int64_t n = live_count(n_ptr, 0, capacity);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (int64_t(blockIdx.x) * blockDim.x >= n) return;  // whole block idle (uniform)
    const bool live = i < n;
    const double px = live ? x[i] : 0.0, py = live ? y[i] : 0.0, pz = live ? z[i] : 0.0;
    const int lane = int(threadIdx.x & 63);
    for (int k = 0; k < ndir; ++k) {
        unsigned long long key =
            live ? order_key(support(s_dir[3 * k], s_dir[3 * k + 1], s_dir[3 * k + 2], px, py, pz)) : 0ull;
        for (int m = 32; m >= 1; m >>= 1) {
            const unsigned long long o = __shfl_xor(key, m, 64);
            key = o > key ? o : key;
        }
        if (lane == 0 && key != 0ull) atomicMax(&work[k], key);
    }
}

__global__ __launch_bounds__(kBlock) void k_extreme_arg(const int64_t *n_ptr, int64_t capacity, const double *x,
                                                        const double *y, const double *z,
                                                        const double *__restrict__ dirs, int32_t ndir,
                                                        const unsigned long long *__restrict__ work,
                                                        int32_t *out_slot) {
    __shared__ double s_dir[3 * kMaxDirs];
    __shared__ unsigned long long s_best[kMaxDirs];
    for (int t = threadIdx.x; t < 3 * ndir; t += blockDim.x) s_dir[t] = dirs[t];
    for (int t = threadIdx.x; t < ndir; t += blockDim.x) s_best[t] = work[t];
    __syncthreads();
    const int64_t n = live_count(n_ptr, 0, capacity);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double px = x[i], py = y[i], pz = z[i];
    for (int k = 0; k < ndir; ++k) {
        const uint64_t key = order_key(support(s_dir[3 * k], s_dir[3 * k + 1], s_dir[3 * k + 2], px, py, pz));
        if (key == s_best[k]) atomicMin(&out_slot[k], int32_t(i));
    }
}

__global__ void k_keep_init(int64_t *out_count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out_count = 0;
}

__global__ __launch_bounds__(kBlock) void k_hull_keep(const int64_t *n_ptr, int64_t capacity, const double *x,
                                                      const double *y, const double *z,
                                                      const double *__restrict__ planes, int32_t nplane,
                                                      double tol, int32_t *out_slot, int64_t max_out,
                                                      unsigned long long *out_count) {
    __shared__ double s_pl[4 * kMaxPlanes];
    for (int t = threadIdx.x; t < 4 * nplane; t += blockDim.x) s_pl[t] = planes[t];
    __syncthreads();
    const int64_t n = live_count(n_ptr, 0, capacity);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (int64_t(blockIdx.x) * blockDim.x >= n) return;  // whole block idle (uniform)
    bool keep = false;
    if (i < n) {
        const double px = x[i], py = y[i], pz = z[i];
        for (int k = 0; k < nplane && !keep; ++k) {
            const double v = support(s_pl[4 * k], s_pl[4 * k + 1], s_pl[4 * k + 2], px, py, pz) + s_pl[4 * k + 3];
            keep = !(v < -tol);  // on or outside a face (or not finite): a hull-vertex candidate
        }
    }
    const uint64_t mask = __ballot(keep);
    if (mask == 0ull) return;
    const int lane = int(threadIdx.x & 63);
    const int leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0ull;
    if (lane == leader) base = atomicAdd(out_count, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (keep) {
        const int64_t at = int64_t(base) + __popcll(mask & ((1ull << lane) - 1ull));
        if (at < max_out) out_slot[at] = int32_t(i);
    }
}

void launch_extreme_points(const bdm_soa &s, const double *dirs, int32_t ndir, unsigned long long *work,
                           int32_t *out_slot, hipStream_t st) {
    const unsigned nb = hull_blocks(s.capacity);
    hipLaunchKernelGGL(k_extreme_init, dim3(1), dim3(kMaxDirs), 0, st, ndir, work, out_slot);
    hipLaunchKernelGGL(k_extreme_max, dim3(nb), dim3(kBlock), 0, st, s.n, s.capacity, s.x, s.y, s.z, dirs, ndir,
                       work);
    hipLaunchKernelGGL(k_extreme_arg, dim3(nb), dim3(kBlock), 0, st, s.n, s.capacity, s.x, s.y, s.z, dirs, ndir,
                       work, out_slot);
}

void launch_hull_keep(const bdm_soa &s, const double *planes, int32_t nplane, double tol, int32_t *out_slot,
                      int64_t max_out, int64_t *out_count, hipStream_t st) {
    const unsigned nb = hull_blocks(s.capacity);
    hipLaunchKernelGGL(k_keep_init, dim3(1), dim3(64), 0, st, out_count);
    hipLaunchKernelGGL(k_hull_keep, dim3(nb), dim3(kBlock), 0, st, s.n, s.capacity, s.x, s.y, s.z, planes, nplane,
                       tol, out_slot, max_out, reinterpret_cast<unsigned long long *>(out_count));
}

}  // namespace bdm
