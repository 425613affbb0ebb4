// Device kernels of the DMK Stokeslet path (gfx950, double precision).
#include "dmk_kernels.hpp"


#include <algorithm>
#include <type_traits>
#include <mutex>

namespace dmk {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kInv8Pi = 1.0 / (8.0 * kPi);
constexpr double k3Over4Pi = 3.0 / (4.0 * kPi);
// largest grid.y of a launch
constexpr int kMaxGridY = 65535;

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
}  // namespace

// Far-field storage: double (FP64 plans) or float (mixed-precision plans).
// Arithmetic is FP64 either way; loads widen and stores round.
template <typename S>
struct Store;
template <>
struct Store<double> {
    using cx = double2;
};
template <>
struct Store<float> {
    using cx = float2;
};

// =============================================================================
// tree construction
// =============================================================================
__global__ __launch_bounds__(256) void k_bbox(const double* __restrict__ pts, int64_t n, double* __restrict__ part)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    double bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            const double v = pts[3 * i + d];
            if (!isfinite(v))
                bad += 1;
            else {
                lo[d] = fmin(lo[d], v);
                hi[d] = fmax(hi[d], v);
            }
        }
    }
    __shared__ double sh[7][256];
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    sh[6][threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + s]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + s]);
            }
            sh[6][threadIdx.x] += sh[6][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 7)
        part[blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

void launch_bbox(const double* pts, int64_t n, double* partial, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_bbox, dim3(nblk), dim3(256), 0, s, pts, n, partial);
}

// One block per problem: bounding box and non-finite count of the points
// [off[b], off[b+1]), written to part[8b .. 8b+6].
__global__ __launch_bounds__(256) void k_bbox_seg(const double* __restrict__ pts, const int64_t* __restrict__ off,
                                                  double* __restrict__ part)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    double bad = 0;
    const int64_t a = off[blockIdx.x], b = off[blockIdx.x + 1];
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x)
        for (int d = 0; d < 3; ++d) {
            const double v = pts[3 * i + d];
            if (!isfinite(v))
                bad += 1;
            else {
                lo[d] = fmin(lo[d], v);
                hi[d] = fmax(hi[d], v);
            }
        }
    __shared__ double sh[7][256];
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    sh[6][threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + st]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + st]);
            }
            sh[6][threadIdx.x] += sh[6][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < 7)
        part[blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

void launch_bbox_seg(const double* pts, const int64_t* off, int nprob, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_bbox_seg, dim3(nprob), dim3(256), 0, s, pts, off, partial);
}

// Problem index of every point: the b with off[b] <= i < off[b+1].
__global__ __launch_bounds__(256) void k_fill_pid(const int64_t* __restrict__ off, int nprob, int64_t n,
                                                  int* __restrict__ pid)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    pid[i] = lo;
}

void launch_fill_pid(const int64_t* off, int nprob, int64_t n, int* pid, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_pid, dim3(nblocks(n, 256)), dim3(256), 0, s, off, nprob, n, pid);
}

__device__ inline uint64_t spread3(uint64_t v)
{
    // bit b of v -> bit 3b
    uint64_t r = 0;
    for (int b = 0; b < 19; ++b)
        r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

__global__ __launch_bounds__(256) void k_morton(const double* __restrict__ pts, int64_t n,
                                                const int* __restrict__ pid, const double* __restrict__ geo,
                                                uint64_t* __restrict__ keys, int* __restrict__ idx)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double* g = geo + 4 * (pid ? pid[i] : 0);
    const double c[3] = {g[0], g[1], g[2]};
    const double inv_len = g[3];
    uint64_t q[3];
    for (int d = 0; d < 3; ++d) {
        const double u = (pts[3 * i + d] - c[d]) * inv_len + 0.5;  // [0,1)
        double g = floor(u * 524288.0);                            // 2^19 cells
        g = fmin(fmax(g, 0.0), 524287.0);
        q[d] = (uint64_t)g;
    }
    keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    idx[i] = (int)i;
}

void launch_morton(const double* pts, int64_t n, const int* pid, const double* geo, uint64_t* keys, int* idx,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_morton, dim3(nblocks(n, 256)), dim3(256), 0, s, pts, n, pid, geo, keys, idx);
}

__global__ __launch_bounds__(256) void k_gather_points(const double* __restrict__ pts, int64_t n,
                                                       const int* __restrict__ perm, const int* __restrict__ pid,
                                                       const double* __restrict__ geo, double* __restrict__ x,
                                                       double* __restrict__ y, double* __restrict__ z)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t o = perm[i];
    // sorting is per problem, so sorted position i lies in the same problem as input position i
    const double* g = geo + 4 * (pid ? pid[i] : 0);
    x[i] = (pts[3 * o] - g[0]) * g[3];
    y[i] = (pts[3 * o + 1] - g[1]) * g[3];
    z[i] = (pts[3 * o + 2] - g[2]) * g[3];
}

void launch_gather_points(const double* pts, int64_t n, const int* perm, const int* pid, const double* geo,
                          double* x, double* y, double* z, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_points, dim3(nblocks(n, 256)), dim3(256), 0, s, pts, n, perm, pid, geo, x, y, z);
}

// ---- compact point groups inside leaves -------------------------------------
// One block per segment (at most kKdCap points, LDS resident).  Level by
// level, every segment of more than 8 points is sorted along the longest side
// of its bounding box and cut after a whole number of 64-point chunks (above
// 64 points) or 8-point groups (at most 64); children take the ids 2k and
// 2k + 1, so ids stay in position order and below 2^depth <= kKdCap / 8
// (at most 8 cut levels for 2048 points).  A sort key is (segment id: 9 bits |
// coordinate quantised to 11 bits | local index: 12 bits); keys are distinct,
// so the bitonic sort gives one order.
namespace {
constexpr int kKdMaxSeg = kKdCap / 8;
constexpr int kKdThreads = 512;  // 8 waves: twice the blocks per CU of 1024 threads, whose stages are latency bound

__global__ __launch_bounds__(kKdThreads) void k_leaf_kd(const KdSeg* __restrict__ segs, const double* __restrict__ x,
                                                 const double* __restrict__ y, const double* __restrict__ z,
                                                 int* __restrict__ src)
{
    __shared__ float c[3][kKdCap];
    __shared__ uint32_t key[kKdCap];
    __shared__ int t_lo[2][kKdMaxSeg], t_len[2][kKdMaxSeg];
    __shared__ float s_min[kKdMaxSeg], s_inv[kKdMaxSeg];
    __shared__ int s_ax[kKdMaxSeg];
    __shared__ int seg_max;   // longest segment of the current level
    const KdSeg S = segs[blockIdx.x];
    const int len = S.len;
    if (len <= 8 || len > kKdCap)
        return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const double ox = x[S.start], oy = y[S.start], oz = z[S.start];
    int P2 = 1;
    while (P2 < len)
        P2 <<= 1;
    for (int i = tid; i < P2; i += kKdThreads) {
        if (i < len) {
            c[0][i] = (float)(x[S.start + i] - ox);
            c[1][i] = (float)(y[S.start + i] - oy);
            c[2][i] = (float)(z[S.start + i] - oz);
        }
        key[i] = i < len ? (uint32_t)i : 0xffffffffu;
    }
    if (tid == 0) {
        t_lo[0][0] = 0;
        t_len[0][0] = len;
        seg_max = len;
    }
    __syncthreads();
    for (int depth = 0, cur = 0; depth < 10; ++depth, cur ^= 1) {
        const int nid = 1 << depth;
        // bounding box, cut axis and quantisation of every segment to cut
        for (int k = wid; k < nid; k += kKdThreads / 64) {
            const int lo = t_lo[cur][k], sl = t_len[cur][k];
            if (sl <= 8)
                continue;
            float mn[3] = {3e38f, 3e38f, 3e38f}, mx[3] = {-3e38f, -3e38f, -3e38f};
            for (int i = lo + lane; i < lo + sl; i += 64) {
                const int p = (int)(key[i] & 0xfffu);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    mn[d] = fminf(mn[d], c[d][p]);
                    mx[d] = fmaxf(mx[d], c[d][p]);
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    mn[d] = fminf(mn[d], __shfl_xor(mn[d], off));
                    mx[d] = fmaxf(mx[d], __shfl_xor(mx[d], off));
                }
            if (lane == 0) {
                int ax = 0;
                if (mx[1] - mn[1] > mx[ax] - mn[ax])
                    ax = 1;
                if (mx[2] - mn[2] > mx[ax] - mn[ax])
                    ax = 2;
                const float ext = mx[ax] - mn[ax];
                s_ax[k] = ax;
                s_min[k] = mn[ax];
                s_inv[k] = ext > 0.f ? 2047.f / ext : 0.f;
            }
        }
        __syncthreads();
        // keys of this level
        for (int k = wid; k < nid; k += kKdThreads / 64) {
            const int lo = t_lo[cur][k], sl = t_len[cur][k];
            const bool cut = sl > 8;
            const int ax = cut ? s_ax[k] : 0;
            const float mn = cut ? s_min[k] : 0.f, inv = cut ? s_inv[k] : 0.f;
            for (int i = lo + lane; i < lo + sl; i += 64) {
                const uint32_t p = key[i] & 0xfffu;
                uint32_t q = 0;
                if (cut)
                    q = (uint32_t)min(2047, max(0, (int)((c[ax][p] - mn) * inv)));
                key[i] = ((uint32_t)k << 23) | (q << 12) | p;
            }
        }
        __syncthreads();
        // bitonic sort of key[0, P2) (padding keys sort last); once every
        // segment has at most 64 points it lies inside one aligned 64-block
        // (cuts above 64 points fall on chunk boundaries), and sorting each
        // block on its own, ascending, is enough
        const int kmax = seg_max <= 64 ? min(64, P2) : P2;
        for (int kk = 2; kk <= kmax; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int t = tid; t < P2 / 2; t += kKdThreads) {
                    const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                    const int l = i + j;
                    const uint32_t a = key[i], b = key[l];
                    if ((a > b) == (kk == kmax || (i & kk) == 0)) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
                __syncthreads();
            }
        // cut: children 2k and 2k + 1 of the next level
        __syncthreads();
        if (tid == 0)
            seg_max = 0;
        __syncthreads();
        for (int k = tid; k < nid; k += kKdThreads) {
            const int lo = t_lo[cur][k], sl = t_len[cur][k];
            int left = sl;
            if (sl > 8) {
                const int unit = sl > 64 ? 64 : 8;
                left = unit * (((sl + unit - 1) / unit) / 2);
            }
            if (2 * k + 1 < kKdMaxSeg) {
                t_lo[cur ^ 1][2 * k] = lo;
                t_len[cur ^ 1][2 * k] = left;
                t_lo[cur ^ 1][2 * k + 1] = lo + left;
                t_len[cur ^ 1][2 * k + 1] = sl - left;
            }
            atomicMax(&seg_max, max(left, sl - left));
        }
        __syncthreads();
        if (seg_max <= 8 || 2 * nid > kKdMaxSeg)
            break;
    }
    for (int i = tid; i < len; i += kKdThreads)
        src[S.start + i] = (int)(S.start + (key[i] & 0xfffu));
}

__global__ __launch_bounds__(256) void k_iota(int* __restrict__ v, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n)
        v[i] = (int)i;
}

__global__ __launch_bounds__(256) void k_compose(const int* __restrict__ perm, const int* __restrict__ src,
                                                 int64_t n, int* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = perm[src[i]];
}
}  // namespace

void launch_leaf_order(const KdSeg* segs, int nseg, const int* perm, const double* x, const double* y,
                       const double* z, int64_t n, int* src, int* perm_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota, dim3(nblocks(n, 256)), dim3(256), 0, s, src, n);
    if (nseg > 0)
        hipLaunchKernelGGL(k_leaf_kd, dim3(nseg), dim3(kKdThreads), 0, s, segs, x, y, z, src);
    hipLaunchKernelGGL(k_compose, dim3(nblocks(n, 256)), dim3(256), 0, s, perm, src, n, perm_out);
}


__global__ __launch_bounds__(256) void k_chunk_bbox(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, const int64_t* __restrict__ cstart,
                                                    const int* __restrict__ clen, int nchunk,
                                                    double* __restrict__ bbox)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchunk)
        return;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    const int64_t s = cstart[c];
    for (int k = 0; k < clen[c]; ++k) {
        const double v[3] = {x[s + k], y[s + k], z[s + k]};
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], v[d]);
            hi[d] = fmax(hi[d], v[d]);
        }
    }
    for (int d = 0; d < 3; ++d) {
        bbox[6 * c + d] = lo[d];
        bbox[6 * c + 3 + d] = hi[d];
    }
}

void launch_chunk_bbox(const double* x, const double* y, const double* z, const int64_t* cstart, const int* clen,
                       int nchunk, double* bbox, hipStream_t s)
{
    if (nchunk == 0)
        return;
    hipLaunchKernelGGL(k_chunk_bbox, dim3(nblocks(nchunk, 256)), dim3(256), 0, s, x, y, z, cstart, clen, nchunk,
                       bbox);
}

// =============================================================================
// per evaluation
// =============================================================================
// Sorted forces: points with input index < nsrc are sources (force f[o]),
// the rest are targets only (zero force).
__global__ __launch_bounds__(256) void k_gather_forces(const double* __restrict__ f, int64_t n, int64_t nsrc,
                                                       const int* __restrict__ perm, double* __restrict__ fs)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t o = perm[i];
    const bool src = o < nsrc;
    fs[i] = src ? f[3 * o] : 0.0;
    fs[n + i] = src ? f[3 * o + 1] : 0.0;
    fs[2 * n + i] = src ? f[3 * o + 2] : 0.0;
}

void launch_gather_forces(const double* f, int64_t n, int64_t nsrc, const int* perm, double* fs, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_forces, dim3(nblocks(n, 256)), dim3(256), 0, s, f, n, nsrc, perm, fs);
}

// Stresslet sources: the symmetric double-layer density of f n^T for the far
// field, rho[6][n] = (f1 n1, f2 n2, f3 n3, f1 n2 + f2 n1, f1 n3 + f3 n1,
// f2 n3 + f3 n2) (the kernel is symmetric in its last two indices, so the
// off-diagonal pairs enter summed), and f, n themselves for the near field,
// fn[6][n].  Points with input index >= nsrc carry zero strength.
__global__ __launch_bounds__(256) void k_gather_stresslet(const double* __restrict__ f, const double* __restrict__ nv,
                                                          int64_t n, int64_t nsrc, const int* __restrict__ perm,
                                                          double* __restrict__ rho, double* __restrict__ fn)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t o = perm[i];
    const bool src = o < nsrc;
    const double f1 = src ? f[3 * o] : 0.0, f2 = src ? f[3 * o + 1] : 0.0, f3 = src ? f[3 * o + 2] : 0.0;
    const double n1 = src ? nv[3 * o] : 0.0, n2 = src ? nv[3 * o + 1] : 0.0, n3 = src ? nv[3 * o + 2] : 0.0;
    rho[i] = f1 * n1;
    rho[n + i] = f2 * n2;
    rho[2 * n + i] = f3 * n3;
    rho[3 * n + i] = f1 * n2 + f2 * n1;
    rho[4 * n + i] = f1 * n3 + f3 * n1;
    rho[5 * n + i] = f2 * n3 + f3 * n2;
    fn[i] = f1;
    fn[n + i] = f2;
    fn[2 * n + i] = f3;
    fn[3 * n + i] = n1;
    fn[4 * n + i] = n2;
    fn[5 * n + i] = n3;
}

void launch_gather_stresslet(const double* f, const double* nv, int64_t n, int64_t nsrc, const int* perm, double* rho,
                             double* fn, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_stresslet, dim3(nblocks(n, 256)), dim3(256), 0, s, f, nv, n, nsrc, perm, rho, fn);
}

// Barycentric Lagrange basis on first-kind Chebyshev nodes.
template <int P>
__device__ inline void lagrange(double xi, const double* __restrict__ t, const double* __restrict__ w, double* L)
{
    int hit = -1;
    double den = 0;
#pragma unroll
    for (int a = 0; a < P; ++a) {
        const double d = xi - t[a];
        if (d == 0.0)
            hit = a;
        const double v = w[a] / (d == 0.0 ? 1.0 : d);
        L[a] = v;
        den += v;
    }
    const double id = 1.0 / den;
#pragma unroll
    for (int a = 0; a < P; ++a)
        L[a] = hit >= 0 ? (a == hit ? 1.0 : 0.0) : L[a] * id;
}

// ---- block order ----------------------------------------------------------------
// Workgroups are handed to the 8 XCDs round-robin, and each XCD has its own L2.
// xcd_block() renumbers the blocks of a 1D grid of xcd_grid(total) so that each
// XCD runs a contiguous range of [0, total): neighbouring work items (here,
// receivers adjacent in Morton order) then read shared data through the same
// L2.  Padding blocks get -1 and must return.  Only for work of even cost per
// block: on the point kernels a contiguous range puts whole clusters on one
// XCD and the imbalance outweighs the cache gain.
__device__ inline int xcd_block(int total)
{
    const int per = (total + 7) / 8;
    const int lg = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    return lg < total ? lg : -1;
}
inline unsigned xcd_grid(int total) { return (unsigned)(((total + 7) / 8) * 8); }

// ---- point <-> proxy grid (MFMA) ---------------------------------------------------
// Lagrange values of every point on its leaf's proxy grid, computed once per
// plan: Ltab[i][d][0..PA) (d = x, y, z; PA = p rounded up to 4, zero padded).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int P>
struct MCfg {
    static constexpr int PA = (P + 3) / 4 * 4;   // K padding for 16x16x4 steps
    static constexpr int NK = PA / 4;
    static constexpr int NT = (P + 15) / 16;     // 16-row tiles over a grid axis
    static constexpr int RS = PA + 1;            // LDS row stride (odd: conflict-free column reads)
};

template <int P, typename LT>
__global__ __launch_bounds__(256) void k_lagrange_table(const LeafDesc* __restrict__ leaves,
                                                        const double* __restrict__ x, const double* __restrict__ y,
                                                        const double* __restrict__ z, const double* __restrict__ ct,
                                                        const double* __restrict__ cw, LT* __restrict__ Ltab)
{
    // The rows of CP consecutive points (3 PA values each, contiguous in the
    // table) are formed in LDS, one (point, axis) row per thread, then
    // written out as one contiguous run with 16-byte stores.
    constexpr int PA = MCfg<P>::PA;
    constexpr int ROW = 3 * PA;
    constexpr int CP = PA <= 24 ? 128 : 64;  // points per chunk (at most 72 KB of LDS)
    constexpr int V = 16 / sizeof(LT);       // values per 16-byte store
    static_assert(ROW % V == 0, "rows are a whole number of 16-byte words");
    __shared__ __align__(16) LT tile[CP * ROW];
    const LeafDesc L = leaves[blockIdx.x];
    const double sc = (double)(2ll << L.level);
    const double cen[3] = {L.cx, L.cy, L.cz};
    const double* crd[3] = {x, y, z};
    for (int64_t c0 = L.start; c0 < L.end; c0 += CP) {
        const int np = (int)min((int64_t)CP, L.end - c0);
        for (int w = threadIdx.x; w < 3 * np; w += 256) {
            const int pt = w / 3, d = w - 3 * pt;
            double Lv[PA];
            lagrange<P>((crd[d][c0 + pt] - cen[d]) * sc, ct, cw, Lv);
#pragma unroll
            for (int a = P; a < PA; ++a)
                Lv[a] = 0.0;
            LT* o = tile + pt * ROW + d * PA;
#pragma unroll
            for (int a = 0; a < PA; ++a)
                o[a] = (LT)Lv[a];
        }
        __syncthreads();
        // 16-byte words of the chunk's rows, contiguous in the table
        using W = typename std::conditional<sizeof(LT) == 8, double2, float4>::type;
        const W* src = reinterpret_cast<const W*>(tile);
        W* dst = reinterpret_cast<W*>(Ltab + (size_t)c0 * ROW);
        for (int e = threadIdx.x; e < np * ROW / V; e += 256)
            dst[e] = src[e];
        __syncthreads();
    }
}

// Far-field potential at the points (final interpolation) as MFMA GEMMs:
// for every z index c, D[b][pt] = sum_a V[j][c][b][a] Lx[pt][a] (V z-major),
// then u_j[pt] += Lz[pt][c] sum_b Ly[pt][b] D[b][pt].  A block takes 64 points
// of one leaf (16 per wave); the z-slab of V sits in LDS.
// points per leaf-evaluation block (4 lanes per point): 128 unless 256 are
// asked for, and 256 only where the kernel fits the 128 registers of a
// 1024-thread block.  128-point blocks (two per CU, each waiting at its own
// slab barriers) measured faster at p = 23: 1.66 against 1.86 ms (FP64) and
// 1.35 against 1.71 ms (FP32) on 10^6 clustered points.
constexpr bool eval256_fits(int p) { return p <= 16 || p == 23 || p == 30; }
int eval_chunk_points(int p, int request)
{
    if (request == 256 && eval256_fits(p))
        return 256;
    return 128;
}

template <int P, typename S, int PTS>
__global__ __launch_bounds__(PTS * 4) void k_leaf_eval(const EvalChunk* __restrict__ chunks, int nchunk,
                                                              const double* __restrict__ Ltab,
                                                              const S* __restrict__ V, int64_t n,
                                                              double* __restrict__ u)
{
    constexpr int PA = MCfg<P>::PA, NK = MCfg<P>::NK, RS = MCfg<P>::RS;
    // the A rows are the (component j, b) pairs rho = j P + b of the slab,
    // packed into NTP tiles of 16 (5 instead of 6 at P = 23, 7 instead of 9
    // at P = 36); rows past 3 P are zero
    constexpr int NR = 3 * P;
    constexpr int NTP = (NR + 15) / 16;
    constexpr int PB = 16 * NTP;
    constexpr int NTH = PTS * 4;
    constexpr int NPRE = (3 * P * P + NTH - 1) / NTH;  // slab elements per thread
    __shared__ double slab[2][PB][RS];                  // double-buffered c-slabs
    const EvalChunk C = chunks[blockIdx.x];
    const S* v = V + (size_t)C.fid * 3 * P * P * P;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int lr = l & 15, lk = l >> 4;
    const int64_t i = C.start + 16 * w + lr;
    const bool valid = i < C.end;
    const double* Li = Ltab + (size_t)(valid ? i : C.start) * 3 * PA;
    double bx[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s)
        bx[s] = valid ? Li[4 * s + lk] : 0.0;
    // b weights of this lane's output rows rho = 16 T + lk + 4 r
    double wy[NTP][4];
#pragma unroll
    for (int T = 0; T < NTP; ++T)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rho = 16 * T + lk + 4 * r;
            wy[T][r] = (valid && rho < NR) ? Li[PA + rho % P] : 0.0;
        }
    // the padding rows / columns of both buffers stay zero
    for (int e = tid; e < 2 * PB * RS; e += NTH)
        (&slab[0][0][0])[e] = 0.0;
    // slab c+1 is loaded into registers while slab c is used from LDS
    double pre[NPRE];
    auto fetch = [&](int c) {
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int e = tid + k * NTH;
            if (e < 3 * P * P) {
                const int j = e / (P * P), r = e % (P * P);
                pre[k] = (double)v[(size_t)j * P * P * P + (size_t)c * P * P + r];
            }
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int e = tid + k * NTH;
            if (e < 3 * P * P) {
                // e = (j P + b) P + a
                slab[buf][e / P][e % P] = pre[k];
            }
        }
    };
    __syncthreads();
    fetch(0);
    put(0);
    __syncthreads();
    double u0 = 0, u1 = 0, u2 = 0;
    // a wave whose 16 points all lie past the chunk's end (the tail chunk of
    // a leaf) only helps to stage the slabs
    const bool busy = __ballot(valid) != 0ull;
#pragma unroll 1
    for (int c = 0; c < P; ++c) {
        const int cur = c & 1;
        if (c + 1 < P)
            fetch(c + 1);
        if (busy) {
            const double lz = valid ? Li[2 * PA + c] : 0.0;
            double X[3] = {0, 0, 0};
            // every tile's chain first (independent chains the scheduler can
            // interleave), then the b-weighted sums of their results
            mfma_d4 acc[NTP];
#pragma unroll
            for (int T = 0; T < NTP; ++T)
                acc[T] = mfma_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < NK; ++s)
#pragma unroll
                for (int T = 0; T < NTP; ++T)
                    acc[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(slab[cur][16 * T + lr][4 * s + lk], bx[s], acc[T], 0, 0, 0);
#pragma unroll
            for (int T = 0; T < NTP; ++T) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // rows 16 T + 4 r + (0..3) over the lanes: one component,
                    // or two where a component ends among them
                    const int j0 = (16 * T + 4 * r) / P, j1 = (16 * T + 4 * r + 3) / P;
                    if (j0 >= 3)
                        continue;  // padding rows
                    const double t = wy[T][r] * acc[T][r];
                    if (j0 == j1 || j1 >= 3) {
                        X[j0] += t;
                    } else {
                        const bool hi = 16 * T + 4 * r + lk >= j1 * P;
                        X[j0] += hi ? 0.0 : t;
                        X[j1] += hi ? t : 0.0;
                    }
                }
            }
            u0 = fma(lz, X[0], u0);
            u1 = fma(lz, X[1], u1);
            u2 = fma(lz, X[2], u2);
        }
        // the other buffer was last read before the previous barrier
        if (c + 1 < P)
            put(cur ^ 1);
        __syncthreads();
    }
    // the four lanes of a point hold disjoint rows
    u0 += __shfl_xor(u0, 16);
    u1 += __shfl_xor(u1, 16);
    u2 += __shfl_xor(u2, 16);
    u0 += __shfl_xor(u0, 32);
    u1 += __shfl_xor(u1, 32);
    u2 += __shfl_xor(u2, 32);
    if (valid && lk == 0) {
        u[i] += u0;
        u[n + i] += u1;
        u[2 * n + i] += u2;
    }
}

// The same evaluation for plans whose far field is stored in FP32: the
// contractions over a run on v_mfma_f32_16x16x4f32 (twice the FP64 MFMA rate)
// with the proxy potentials and Lagrange values in FP32; the b and c weights
// and the accumulation at the points stay FP64.  The f32 MFMA returns row
// 4 (l/16) + r of its 16 x 16 tile in register r of lane l.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int P, int PTS>
__global__ __launch_bounds__(PTS * 4) void k_leaf_eval32(const EvalChunk* __restrict__ chunks,
                                                                     int nchunk, const float* __restrict__ Ltab,
                                                                     const float* __restrict__ V, int64_t n,
                                                                     double* __restrict__ u)
{
    constexpr int PA = MCfg<P>::PA, NK = MCfg<P>::NK, NT = MCfg<P>::NT, RS = MCfg<P>::RS;
    constexpr int PB = 16 * NT;
    constexpr int NTH = PTS * 4;
    constexpr int NPRE = (3 * P * P + NTH - 1) / NTH;  // slab elements per thread
    __shared__ float slab[2][3][PB][RS];                // double-buffered c-slabs
    const EvalChunk C = chunks[blockIdx.x];
    const float* v = V + (size_t)C.fid * 3 * P * P * P;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int lr = l & 15, lk = l >> 4;
    const int64_t i = C.start + 16 * w + lr;
    const bool valid = i < C.end;
    const float* Li = Ltab + (size_t)(valid ? i : C.start) * 3 * PA;
    float bx[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s)
        bx[s] = valid ? Li[4 * s + lk] : 0.0f;
    double wy[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = 16 * t + 4 * lk + r;
            wy[t][r] = (valid && b < P) ? (double)Li[PA + b] : 0.0;
        }
    for (int e = tid; e < 2 * 3 * PB * RS; e += NTH)
        (&slab[0][0][0][0])[e] = 0.0f;
    float pre[NPRE];
    auto fetch = [&](int c) {
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int e = tid + k * NTH;
            if (e < 3 * P * P) {
                const int j = e / (P * P), r = e % (P * P);
                pre[k] = v[(size_t)j * P * P * P + (size_t)c * P * P + r];
            }
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int e = tid + k * NTH;
            if (e < 3 * P * P) {
                const int j = e / (P * P), r = e % (P * P);
                slab[buf][j][r / P][r % P] = pre[k];
            }
        }
    };
    __syncthreads();
    fetch(0);
    put(0);
    __syncthreads();
    double u0 = 0, u1 = 0, u2 = 0;
    const bool busy = __ballot(valid) != 0ull;
#pragma unroll 1
    for (int c = 0; c < P; ++c) {
        const int cur = c & 1;
        if (c + 1 < P)
            fetch(c + 1);
        if (busy) {
            const double lz = valid ? (double)Li[2 * PA + c] : 0.0;
            double X[3] = {0, 0, 0};
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    mfma_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int s = 0; s < NK; ++s)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(slab[cur][j][16 * t + lr][4 * s + lk], bx[s], acc,
                                                                   0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        X[j] = fma(wy[t][r], (double)acc[r], X[j]);
                }
            u0 = fma(lz, X[0], u0);
            u1 = fma(lz, X[1], u1);
            u2 = fma(lz, X[2], u2);
        }
        if (c + 1 < P)
            put(cur ^ 1);
        __syncthreads();
    }
    u0 += __shfl_xor(u0, 16);
    u1 += __shfl_xor(u1, 16);
    u2 += __shfl_xor(u2, 16);
    u0 += __shfl_xor(u0, 32);
    u1 += __shfl_xor(u1, 32);
    u2 += __shfl_xor(u2, 32);
    if (valid && lk == 0) {
        u[i] += u0;
        u[n + i] += u1;
        u[2 * n + i] += u2;
    }
}

// Proxy charges (Step 2a) as MFMA contractions over the points:
//   Q[j][a][n] = sum_pt Lx[pt][a] f_j[pt] W[pt][n],  W[pt][n] = Ly[pt][b] Lz[pt][c],  n = b P + c,
// with v_mfma_f64_16x16x4f64: rows = the NC P pairs (j, a) in Q's order,
// packed into 16-row tiles across the components (69 rows in 5 tiles at
// p = 23, not 3 x 2), columns = 16-tiles of the flattened (b, c) index (Q's
// rows stored contiguously), K = 4 points.  A row (j, a) is Q's row j P + a,
// so the output stores run along n.  The A operand carries the force,
// Lx[pt][a] f_j[pt]; the B operand W is shared by the components.
template <int P>
struct AMCfg {
    static constexpr int PA = MCfg<P>::PA;
    static constexpr int NTOT = (P * P + 15) / 16;   // n-tiles
};
template <int P, int NC>
struct AMPack {
    static constexpr int ROWS = NC * P;                      // (j, a) rows
    static constexpr int RT = (ROWS + 15) / 16;              // row tiles
    // at most 8 row tiles per wave (their A operands share each B operand);
    // 3 n-tiles per wave where the row tiles are few enough for the registers
    static constexpr int RG = (RT + 7) / 8;                  // row-tile groups
    static constexpr int TPW = (RT + RG - 1) / RG;           // row tiles per wave
    static constexpr int NN = NC == 6 && TPW <= 5 ? 3 : 2;   // n-tiles per wave
    static constexpr int NG = (AMCfg<P>::NTOT + NN - 1) / NN;  // n-tile groups
    static constexpr int TASKS = RG * NG;                    // waves per leaf
};

// The FP32 kernel's tiling: its FP64 fold sums double the registers per
// accumulator tile, so the six stresslet densities go in groups of two row
// tiles with three n-tiles each.
template <int P, int NC>
struct AMPack32 {
    static constexpr int ROWS = NC * P;
    static constexpr int RT = (ROWS + 15) / 16;
    static constexpr int MAXT = NC == 6 ? 2 : 8;
    static constexpr int RG = (RT + MAXT - 1) / MAXT;
    static constexpr int TPW = (RT + RG - 1) / RG;
    static constexpr int NN = NC == 6 ? 3 : 2;
    static constexpr int NG = (AMCfg<P>::NTOT + NN - 1) / NN;
    static constexpr int TASKS = RG * NG;
};

template <int P, int NC, typename S>
__global__ __launch_bounds__(64) void k_anterp_mfma(const LeafDesc* __restrict__ leaves, int nleaf,
                                                    const double* __restrict__ Ltab,
                                                    const double* __restrict__ fs, int64_t n, S* __restrict__ Q)
{
    using C = AMCfg<P>;
    using K = AMPack<P, NC>;
    constexpr int PA = C::PA, NN = K::NN, TPW = K::TPW;
    // workgroups go to the 8 XCDs in turn: leaf k runs all its waves on XCD
    // k % 8, so its Lagrange rows and forces are read into one L2 only
    const int xcd = blockIdx.x % 8, sx = blockIdx.x / 8;
    const int task = sx % K::TASKS;
    const int leaf = xcd + 8 * (sx / K::TASKS);
    if (leaf >= nleaf)
        return;
    const LeafDesc L = leaves[leaf];
    const int rg = task % K::RG, ng = task / K::RG;
    const int l = threadIdx.x;
    const int li = l & 15, lk = l >> 4;
    // row tiles 16 (TPW rg + T) ...: this lane's A rows (j, a); rows past
    // NC P read a valid entry and are never stored
    const int t0 = TPW * rg;
    int arow[TPW], frow[TPW];
#pragma unroll
    for (int T = 0; T < TPW; ++T) {
        const int row = min(16 * (t0 + T) + li, K::ROWS - 1);
        arow[T] = row % P;
        frow[T] = row / P;
    }
    int bcol[NN], ccol[NN];
    bool n_ok[NN];
#pragma unroll
    for (int t = 0; t < NN; ++t) {
        const int nn = 16 * (NN * ng + t) + li;
        n_ok[t] = nn < P * P;
        bcol[t] = n_ok[t] ? nn / P : 0;
        ccol[t] = n_ok[t] ? nn % P : 0;
    }
    mfma_d4 acc[TPW][NN];
#pragma unroll
    for (int T = 0; T < TPW; ++T)
#pragma unroll
        for (int t = 0; t < NN; ++t)
            acc[T][t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    // The leaf's points go in blocks of KB: the block's Lagrange rows (one
    // contiguous run of the table) and forces are loaded by the whole wave
    // with 16-byte loads into registers while the previous block's products
    // run, then written to LDS, from which each lane reads its operands.
    // Rows (j, a) past NC P and columns n >= P^2 are never stored, so only
    // the forces past the leaf's end need to be zero.  The workgroup is one
    // wave: its LDS accesses complete in order.
    constexpr int ROW = 3 * PA;           // doubles per point of the table
    constexpr int KB = ROW <= 72 ? 16 : 8;  // points per block (4 or 2 MFMA steps; fewer registers at large P)
    constexpr int BLK2 = KB * ROW / 2;    // 16-byte words per block of rows
    constexpr int PER = (BLK2 + 63) / 64;
    constexpr int FPER = (NC * KB + 63) / 64;
    __shared__ double2 sL[BLK2];
    __shared__ double sF[NC * KB];
    const int npt = (int)(L.end - L.start);
    const double* Lb = Ltab + (size_t)L.start * ROW;
    double st0[PER], st1[PER];  // the next block (the two halves of its 16-byte words)
    double sf[FPER], sm[FPER];  // its forces and their 0/1 masks (applied at the LDS store)
    // unconditional loads from clamped indices: a row past the table's end
    // repeats its last row (finite, and its force is zero), and a leaf
    // without sources (a target-only leaf) reads its first row and force,
    // which exist as the leaf is not empty; the forces are
    // masked by a product at the LDS store (a select would turn the load into
    // a branch, and an early product would wait for the load)
#define DMK_AM_GLOAD(I0)                                                                     \
    {                                                                                        \
        const int i0_ = (I0);                                                                \
        const double2* src = (const double2*)(Lb + (size_t)i0_ * ROW);                       \
        const int64_t rows = n - (L.start + i0_);                                            \
        const int lim = (int)min((int64_t)BLK2, rows * (ROW / 2)) - 1;                       \
        _Pragma("unroll") for (int u = 0; u < PER; ++u)                                      \
        {                                                                                    \
            const double2 v = src[min(l + 64 * u, lim)];                                     \
            st0[u] = v.x;                                                                    \
            st1[u] = v.y;                                                                    \
        }                                                                                    \
        _Pragma("unroll") for (int u = 0; u < FPER; ++u)                                     \
        {                                                                                    \
            const int e = l + 64 * u;                                                        \
            const int j = min(e / KB, NC - 1), k = e % KB;                                   \
            sf[u] = fs[(size_t)j * n + L.start + max(min(i0_ + k, npt - 1), 0)];             \
            sm[u] = (e < NC * KB && i0_ + k < npt) ? 1.0 : 0.0;                              \
        }                                                                                    \
    }
#define DMK_AM_LSTORE()                                                                      \
    {                                                                                        \
        _Pragma("unroll") for (int u = 0; u < PER; ++u) if (l + 64 * u < BLK2) sL[l + 64 * u] = make_double2(st0[u], st1[u]); \
        _Pragma("unroll") for (int u = 0; u < FPER; ++u) if (l + 64 * u < NC * KB) sF[l + 64 * u] = sf[u] * sm[u]; \
    }
    const double* sLd = (const double*)sL;
    const int nblk = (npt + KB - 1) / KB;
    // a wave of the last row group may own fewer than TPW tiles
    const int tv = min(TPW, K::RT - t0);
    DMK_AM_GLOAD(0)
    DMK_AM_LSTORE()
    for (int blk = 0; blk < nblk; ++blk) {
        const bool more = blk + 1 < nblk;
        if (more)
            DMK_AM_GLOAD((blk + 1) * KB)
#pragma unroll
        for (int ks = 0; ks < KB / 4; ++ks) {
            const int pl = 4 * ks + lk;
            const double* row = sLd + pl * ROW;
            double w[NN];
#pragma unroll
            for (int t = 0; t < NN; ++t)
                w[t] = row[PA + bcol[t]] * row[2 * PA + ccol[t]];
#pragma unroll
            for (int T = 0; T < TPW; ++T)
                if (T < tv) {
                    const double af = row[arow[T]] * sF[frow[T] * KB + pl];
#pragma unroll
                    for (int t = 0; t < NN; ++t)
                        acc[T][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, w[t], acc[T][t], 0, 0, 0);
                }
        }
        if (more)
            DMK_AM_LSTORE()
    }
#undef DMK_AM_GLOAD
#undef DMK_AM_LSTORE
    // D[row = lk + 4 r][col = li] of tile (T, t): Q row 16 (t0 + T) + lk + 4 r, n = 16 (NN ng + t) + li
    S* q = Q + (size_t)L.fid * NC * P * P * P;
#pragma unroll
    for (int t = 0; t < NN; ++t) {
        if (!n_ok[t])
            continue;
        const int nn = 16 * (NN * ng + t) + li;
#pragma unroll
        for (int T = 0; T < TPW; ++T)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = 16 * (t0 + T) + lk + 4 * r;
                if (rr < K::ROWS)
                    q[(size_t)rr * P * P + nn] = (S)acc[T][t][r];
            }
    }
}

// Proxy charges for plans whose far field is stored in FP32: the same
// packed contraction on v_mfma_f32_16x16x4f32 with FP32 Lagrange values and
// forces.  The FP32 accumulators are folded into FP64 sums every 64 points
// (blocked summation: the rounding error grows with 64 terms, not with the
// leaf's size), and the FP64 sums are rounded once to the stored FP32 charges.
template <int P, int NC>
__global__ __launch_bounds__(64) void k_anterp_mfma32(const LeafDesc* __restrict__ leaves, int nleaf,
                                                      const float* __restrict__ Ltab, const double* __restrict__ fs,
                                                      int64_t n, float* __restrict__ Q)
{
    using C = AMCfg<P>;
    using K = AMPack32<P, NC>;
    constexpr int PA = C::PA, NN = K::NN, TPW = K::TPW;
    const int xcd = blockIdx.x % 8, sx = blockIdx.x / 8;
    const int task = sx % K::TASKS;
    const int leaf = xcd + 8 * (sx / K::TASKS);
    if (leaf >= nleaf)
        return;
    const LeafDesc L = leaves[leaf];
    const int rg = task % K::RG, ng = task / K::RG;
    const int l = threadIdx.x;
    const int li = l & 15, lk = l >> 4;
    const int t0 = TPW * rg;
    int arow[TPW], frow[TPW];
#pragma unroll
    for (int T = 0; T < TPW; ++T) {
        const int row = min(16 * (t0 + T) + li, K::ROWS - 1);
        arow[T] = row % P;
        frow[T] = row / P;
    }
    int bcol[NN], ccol[NN];
    bool n_ok[NN];
#pragma unroll
    for (int t = 0; t < NN; ++t) {
        const int nn = 16 * (NN * ng + t) + li;
        n_ok[t] = nn < P * P;
        bcol[t] = n_ok[t] ? nn / P : 0;
        ccol[t] = n_ok[t] ? nn % P : 0;
    }
    mfma_f4 acc[TPW][NN];
    double sum[TPW][NN][4];
#pragma unroll
    for (int T = 0; T < TPW; ++T)
#pragma unroll
        for (int t = 0; t < NN; ++t) {
            acc[T][t] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sum[T][t][r] = 0.0;
        }
    auto fold = [&]() {
#pragma unroll
        for (int T = 0; T < TPW; ++T)
#pragma unroll
            for (int t = 0; t < NN; ++t) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    sum[T][t][r] += (double)acc[T][t][r];
                acc[T][t] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
            }
    };
    // Blocks of KB points staged through LDS as in the FP64 kernel (16-byte
    // loads of the block's table rows and forces while the previous block's
    // products run; the force on the A side; indices clamped, forces past
    // the leaf's end masked at the LDS store).
    constexpr int ROW = 3 * PA;          // floats per point of the table
    constexpr int KB = 16;               // points per block (4 MFMA steps)
    constexpr int BLK4 = KB * ROW / 4;   // 16-byte words per block of rows
    constexpr int PER = (BLK4 + 63) / 64;
    constexpr int FPER = (NC * KB + 63) / 64;
    constexpr int FOLD = 64 / KB;        // blocks per FP64 fold (64 points)
    __shared__ float4 sL[BLK4];
    __shared__ float sF[NC * KB];
    const int npt = (int)(L.end - L.start);
    const float* Lb = Ltab + (size_t)L.start * ROW;
    float st0[PER], st1[PER], st2[PER], st3[PER];
    double sf[FPER], sm[FPER];
#define DMK_AM_GLOAD(I0)                                                                     \
    {                                                                                        \
        const int i0_ = (I0);                                                                \
        const float4* src = (const float4*)(Lb + (size_t)i0_ * ROW);                         \
        const int64_t rows = n - (L.start + i0_);                                            \
        const int lim = (int)min((int64_t)BLK4, rows * (ROW / 4)) - 1;                       \
        _Pragma("unroll") for (int u = 0; u < PER; ++u)                                      \
        {                                                                                    \
            const float4 v = src[min(l + 64 * u, lim)];                                      \
            st0[u] = v.x;                                                                    \
            st1[u] = v.y;                                                                    \
            st2[u] = v.z;                                                                    \
            st3[u] = v.w;                                                                    \
        }                                                                                    \
        _Pragma("unroll") for (int u = 0; u < FPER; ++u)                                     \
        {                                                                                    \
            const int e = l + 64 * u;                                                        \
            const int j = min(e / KB, NC - 1), k = e % KB;                                   \
            sf[u] = fs[(size_t)j * n + L.start + max(min(i0_ + k, npt - 1), 0)];             \
            sm[u] = (e < NC * KB && i0_ + k < npt) ? 1.0 : 0.0;                              \
        }                                                                                    \
    }
#define DMK_AM_LSTORE()                                                                      \
    {                                                                                        \
        _Pragma("unroll") for (int u = 0; u < PER; ++u) if (l + 64 * u < BLK4)               \
            sL[l + 64 * u] = make_float4(st0[u], st1[u], st2[u], st3[u]);                    \
        _Pragma("unroll") for (int u = 0; u < FPER; ++u) if (l + 64 * u < NC * KB)           \
            sF[l + 64 * u] = (float)(sf[u] * sm[u]);                                         \
    }
    const float* sLf = (const float*)sL;
    const int nblk = (npt + KB - 1) / KB;
    const int tv = min(TPW, K::RT - t0);
    DMK_AM_GLOAD(0)
    DMK_AM_LSTORE()
    for (int blk = 0; blk < nblk; ++blk) {
        const bool more = blk + 1 < nblk;
        if (more)
            DMK_AM_GLOAD((blk + 1) * KB)
#pragma unroll
        for (int ks = 0; ks < KB / 4; ++ks) {
            const int pl = 4 * ks + lk;
            const float* row = sLf + pl * ROW;
            float w[NN];
#pragma unroll
            for (int t = 0; t < NN; ++t)
                w[t] = row[PA + bcol[t]] * row[2 * PA + ccol[t]];
#pragma unroll
            for (int T = 0; T < TPW; ++T)
                if (T < tv) {
                    const float af = row[arow[T]] * sF[frow[T] * KB + pl];
#pragma unroll
                    for (int t = 0; t < NN; ++t)
                        acc[T][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, w[t], acc[T][t], 0, 0, 0);
                }
        }
        if (blk % FOLD == FOLD - 1)
            fold();
        if (more)
            DMK_AM_LSTORE()
    }
    fold();
#undef DMK_AM_GLOAD
#undef DMK_AM_LSTORE
    // D[row = 4 lk + r][col = li] of tile (T, t): Q row 16 (t0 + T) + 4 lk + r, n = 16 (NN ng + t) + li
    float* q = Q + (size_t)L.fid * NC * P * P * P;
#pragma unroll
    for (int t = 0; t < NN; ++t) {
        if (!n_ok[t])
            continue;
        const int nn = 16 * (NN * ng + t) + li;
#pragma unroll
        for (int T = 0; T < TPW; ++T)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = 16 * (t0 + T) + 4 * lk + r;
                if (rr < K::ROWS)
                    q[(size_t)rr * P * P + nn] = (float)sum[T][t][r];
            }
    }
}

// Chebyshev orders with compiled point kernels: the Table tab:params values
// (prolate and Gaussian columns) plus intermediate orders for explicit
// parameter choices.
#define DMK_P_DISPATCH(p, MACRO) \
    switch (p) {                 \
    case 11: MACRO(11); break;   \
    case 12: MACRO(12); break;   \
    case 14: MACRO(14); break;   \
    case 16: MACRO(16); break;   \
    case 20: MACRO(20); break;   \
    case 22: MACRO(22); break;   \
    case 23: MACRO(23); break;   \
    case 26: MACRO(26); break;   \
    case 28: MACRO(28); break;   \
    case 30: MACRO(30); break;   \
    case 33: MACRO(33); break;   \
    case 36: MACRO(36); break;   \
    case 40: MACRO(40); break;   \
    case 43: MACRO(43); break;   \
    case 44: MACRO(44); break;   \
    case 48: MACRO(48); break;   \
    default: break;              \
    }

bool p_supported(int p)
{
    switch (p) {
    case 11: case 12: case 14: case 16: case 20: case 22: case 23: case 26: case 28: case 30: case 33: case 36:
    case 40: case 43: case 44: case 48: return true;
    default: return false;
    }
}

int lagrange_pad(int p) { return (p + 3) / 4 * 4; }

void launch_lagrange_table(int p, const LeafDesc* leaves, int nleaf, const double* x, const double* y,
                           const double* z, const double* cheb_t, const double* cheb_w, void* Ltab, bool f32,
                           hipStream_t s)
{
    if (nleaf == 0)
        return;
#define L_LT(P)                                                                                              \
    if (f32)                                                                                                 \
        hipLaunchKernelGGL((k_lagrange_table<P, float>), dim3(nleaf), dim3(256), 0, s, leaves, x, y, z, cheb_t, \
                           cheb_w, (float*)Ltab);                                                            \
    else                                                                                                     \
        hipLaunchKernelGGL((k_lagrange_table<P, double>), dim3(nleaf), dim3(256), 0, s, leaves, x, y, z,      \
                           cheb_t, cheb_w, (double*)Ltab)
    DMK_P_DISPATCH(p, L_LT)
#undef L_LT
}

void launch_anterp(int p, int nc, const LeafDesc* leaves, int nleaf, const void* Ltab, const double* fs, int64_t n,
                   void* Q, bool f32, hipStream_t s)
{
    if (nleaf == 0)
        return;
    const int nleaf8 = (nleaf + 7) / 8 * 8;
#define L_ANTERP_NC(P, NC)                                                                                       \
    if (f32) {                                                                                                   \
        hipLaunchKernelGGL((k_anterp_mfma32<P, NC>), dim3(nleaf8 * AMPack32<P, NC>::TASKS), dim3(64), 0, s,    \
                           leaves, nleaf, (const float*)Ltab, fs, n, (float*)Q);                                 \
    } else {                                                                                                     \
        hipLaunchKernelGGL((k_anterp_mfma<P, NC, double>), dim3(nleaf8 * AMPack<P, NC>::TASKS), dim3(64), 0, s,  \
                           leaves, nleaf, (const double*)Ltab, fs, n, (double*)Q);                               \
    }
#define L_ANTERP(P)               \
    if (nc == 6) {                \
        L_ANTERP_NC(P, 6);        \
    } else {                      \
        L_ANTERP_NC(P, 3);        \
    }
    DMK_P_DISPATCH(p, L_ANTERP)
#undef L_ANTERP
#undef L_ANTERP_NC
}

void launch_leaf_eval(int p, int pts, const EvalChunk* chunks, int nchunk, const void* Ltab, const void* V,
                      int64_t n, double* u, bool f32, hipStream_t s)
{
    if (nchunk == 0)
        return;
#define L_EVAL_T(P, PTS)                                                                                    \
    if (f32)                                                                                                \
        hipLaunchKernelGGL((k_leaf_eval32<P, PTS>), dim3(nchunk), dim3(PTS * 4), 0, s, chunks, nchunk,      \
                           (const float*)Ltab, (const float*)V, n, u);                                      \
    else                                                                                                    \
        hipLaunchKernelGGL((k_leaf_eval<P, double, PTS>), dim3(nchunk), dim3(PTS * 4), 0, s, chunks, nchunk, \
                           (const double*)Ltab, (const double*)V, n, u)
#define L_EVAL(P)                                      \
    if constexpr (eval256_fits(P)) {                   \
        if (pts == 256) {                              \
            L_EVAL_T(P, 256);                          \
        } else {                                       \
            L_EVAL_T(P, 128);                          \
        }                                              \
    } else {                                           \
        L_EVAL_T(P, 128);                              \
    }
    DMK_P_DISPATCH(p, L_EVAL)
#undef L_EVAL
#undef L_EVAL_T
}

// x / d for 0 <= x < 2^20 and d >= 1 given inv_d = 1/d (rounded to float):
// (x + 1/2) / d is at least 1/(2d) from an integer, and the float error is at
// most about 2^-22 (x / d) < 1/(4d), so truncation gives the exact quotient.
__device__ inline int div_small(int x, float inv_d) { return (int)(((float)x + 0.5f) * inv_d); }

// ---- separable tensor stages ---------------------------------------------------
template <int MODE>
struct StageTraits {
    static constexpr bool xc = (MODE == ST_OUT_FULL || MODE == ST_IN_FULL || MODE == ST_IN_HALF_REAL);
    static constexpr bool yc = (MODE == ST_OUT_HALF || MODE == ST_OUT_FULL || MODE == ST_IN_FULL);
    static constexpr bool fold = (MODE != ST_IN_HALF_REAL);
};

// 256 threads per RT-row tile (RT = 64 or 32): the input slab
// X[0..Nin)[r0..r0+RT) is staged in LDS with all loads in flight, thread
// (row, g) accumulates the half outputs g, g+NG, ... (NG = 256/RT groups)
// from it, and the output tile Y[r0..r0+RT)[0..Nout) is staged in LDS again
// and written as one contiguous block (or scatter-added to the children's
// grids, one contiguous run of p per row and child).  Long axes take RT = 32:
// half the LDS and half the accumulators per thread, twice the workgroups per
// CU to keep loads in flight.
template <int MODE, int IO, int NI, int RT, typename S>
__global__ __launch_bounds__(256) void k_stage(StageArgs a)
{
    constexpr int NG = 256 / RT;
    using Tr = StageTraits<MODE>;
    constexpr int XE = Tr::xc ? 2 : 1;
    constexpr int YE = Tr::yc ? 2 : 1;
    extern __shared__ double smem[];
    const int nm = a.Nh * a.Kh;
    double2* smat = (double2*)smem;
    double* tile = smem + 2 * nm;
    const int tid = threadIdx.x;
    for (int k = tid; k < nm; k += 256)
        smat[k] = make_double2(a.mat[2 * k], a.mat[2 * k + 1]);
    const int nc = a.ncomp;
    const int slot = a.slot0 + (int)blockIdx.y / nc, comp = blockIdx.y % nc;
    const int R = a.R, Nin = a.Nin, Nout = a.Nout, p = a.p;
    const int r0 = blockIdx.x * RT;
    const int nrow = min(RT, R - r0);
    const size_t p3 = (size_t)p * p * p;
    // ---- input slab ----
    if (IO == IO_GATHER8) {
        // the children's 2p x 2p x 2p grid: with e = tid + 256 i the row
        // rr = tid % RT (= (B, C), B and C in [0, 2p)) is the thread's own and
        // k = tid / RT + NG i, so the row's child offsets are found once
        const int rr = tid % RT;
        const int r = r0 + rr;
        const int B = div_small(r, 1.0f / (float)(2 * p)), C = r - 2 * p * B;
        const int bh = B >= p, ch = C >= p;
        const size_t bc = (size_t)(B - p * bh) * p + (C - p * ch);
        const int* cf = a.child_fid + slot * 8 + 2 * bh + ch;
        for (int k = tid / RT; k < Nin; k += NG) {
            double v0 = 0.0;
            if (rr < nrow) {
                const int kh = k >= p;
                const int f = cf[4 * kh];
                if (f >= 0)
                    v0 = (double)((const S*)a.X)[((size_t)f * nc + comp) * p3 + (size_t)(k - p * kh) * p * p + bc];
            }
            tile[k * RT + rr] = v0;
        }
    } else {
        const size_t xoff = ((size_t)(a.xmap ? a.xmap[slot] : slot - a.xbase) * nc + comp) * a.xstride;
        for (int e = tid; e < Nin * RT; e += 256) {
            const int k = e / RT, rr = e % RT;
            const int r = r0 + rr;
            double v0 = 0.0, v1 = 0.0;
            if (rr < nrow) {
                if (XE == 2) {
                    const typename Store<S>::cx v = ((const typename Store<S>::cx*)a.X)[xoff + (size_t)k * R + r];
                    v0 = (double)v.x;
                    v1 = (double)v.y;
                } else {
                    v0 = (double)((const S*)a.X)[xoff + (size_t)k * R + r];
                }
            }
            if (XE == 2)
                ((double2*)tile)[e] = make_double2(v0, v1);
            else
                tile[e] = v0;
        }
    }
    __syncthreads();
    const int lane = tid % RT, g = tid / RT;
    double Ur[NI], Ui[NI], Wr[NI], Wi[NI];
#pragma unroll
    for (int t = 0; t < NI; ++t)
        Ur[t] = Ui[t] = Wr[t] = Wi[t] = 0.0;
    for (int j = 0; j < a.Kh; ++j) {
        const int k1 = j + a.in_off;
        const int k2 = Nin - 1 - k1;
        double x1r, x1i = 0, x2r = 0, x2i = 0;
        if (XE == 2) {
            const double2 v1 = ((const double2*)tile)[k1 * RT + lane];
            x1r = v1.x;
            x1i = v1.y;
            if (Tr::fold && k2 != k1) {
                const double2 v2 = ((const double2*)tile)[k2 * RT + lane];
                x2r = v2.x;
                x2i = v2.y;
            }
        } else {
            x1r = tile[k1 * RT + lane];
            if (k2 != k1)
                x2r = tile[k2 * RT + lane];
        }
        double er, ei, orr, oi;
        if (Tr::fold) {
            er = x1r + x2r;
            ei = x1i + x2i;
            orr = x1r - x2r;
            oi = x1i - x2i;
        } else {  // half modes: even part <- real, odd part <- imaginary
            er = x1r;
            ei = 0;
            orr = x1i;
            oi = 0;
        }
#pragma unroll
        for (int t = 0; t < NI; ++t) {
            const int i = g + NG * t;
            if (i < a.Nh) {
                const double2 m = smat[i * a.Kh + j];
                Ur[t] = fma(m.x, er, Ur[t]);
                Wr[t] = fma(m.y, orr, Wr[t]);
                if (Tr::xc && Tr::fold) {
                    Ui[t] = fma(m.x, ei, Ui[t]);
                    Wi[t] = fma(m.y, oi, Wi[t]);
                }
            }
        }
    }
    __syncthreads();  // input slab consumed; the tile now holds outputs [row][n]
#pragma unroll
    for (int t = 0; t < NI; ++t) {
        const int i = g + NG * t;
        if (i >= a.Nh)
            continue;
        const int n1 = i + a.out_off;
        const int n2 = Nout - 1 - n1;
        double y1r, y1i = 0, y2r, y2i = 0;
        bool two = (n2 != n1);
        if (MODE == ST_SYM_REAL) {
            y1r = Ur[t] + Wr[t];
            y2r = Ur[t] - Wr[t];
        } else if (MODE == ST_OUT_HALF) {
            y1r = Ur[t];
            y1i = -Wr[t];
            y2r = 0;
            two = false;
        } else if (MODE == ST_OUT_FULL) {
            y1r = Ur[t] + Wi[t];  // U - iW
            y1i = Ui[t] - Wr[t];
            y2r = Ur[t] - Wi[t];  // U + iW
            y2i = Ui[t] + Wr[t];
        } else if (MODE == ST_IN_FULL) {
            y1r = Ur[t] - Wi[t];  // U + iW
            y1i = Ui[t] + Wr[t];
            y2r = Ur[t] + Wi[t];  // U - iW
            y2i = Ui[t] - Wr[t];
        } else {                  // ST_IN_HALF_REAL
            y1r = Ur[t] - Wr[t];
            y2r = Ur[t] + Wr[t];
        }
        if (YE == 2) {
            ((double2*)tile)[lane * Nout + n1] = make_double2(y1r, y1i);
            if (two)
                ((double2*)tile)[lane * Nout + n2] = make_double2(y2r, y2i);
        } else {
            tile[lane * Nout + n1] = y1r;
            if (two)
                tile[lane * Nout + n2] = y2r;
        }
    }
    __syncthreads();
    if (IO == IO_SCATTER8) {
        // rows r = (C, B) of the child grid, output axis A; child (A/p, B/p, C/p)
        S* Yd = (S*)a.Y;
        const float inv_out = 1.0f / (float)Nout, inv_2p = 1.0f / (float)(2 * p);
        for (int e = tid; e < nrow * Nout; e += 256) {
            const int rr = div_small(e, inv_out), A = e - Nout * rr;
            const int r = r0 + rr;
            const int C = div_small(r, inv_2p), B = r - 2 * p * C;
            const int ah = A >= p, bh = B >= p, ch = C >= p;
            const int f = a.child_fid[slot * 8 + 4 * ah + 2 * bh + ch];
            if (f >= 0) {
                S& y = Yd[((size_t)f * nc + comp) * p3 + ((size_t)(C - p * ch) * p + (B - p * bh)) * p + (A - p * ah)];
                y = (S)((double)y + tile[e]);
            }
        }
    } else {
        const size_t yoff = ((size_t)(a.ymap ? a.ymap[slot] : slot - a.ybase) * nc + comp) * a.ystride * YE +
                            (size_t)r0 * Nout * YE;
        S* Yd = (S*)a.Y + yoff;
        const int cnt = nrow * Nout * YE;
        if (a.accumulate) {
            for (int e = tid; e < cnt; e += 256)
                Yd[e] = (S)((double)Yd[e] + tile[e]);
        } else {
            for (int e = tid; e < cnt; e += 256)
                Yd[e] = (S)tile[e];
        }
    }
}

template <int MODE, int IO, int NI, int RT, typename S>
static void stage_launch_t(dim3 grid, size_t shm, const StageArgs& a, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_stage<MODE, IO, NI, RT, S>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((k_stage<MODE, IO, NI, RT, S>), grid, dim3(256), shm, s, a);
}

template <int MODE, int IO, int NI, int RT>
static void stage_launch(dim3 grid, size_t shm, const StageArgs& a, hipStream_t s)
{
    if (a.f32)
        stage_launch_t<MODE, IO, NI, RT, float>(grid, shm, a, s);
    else
        stage_launch_t<MODE, IO, NI, RT, double>(grid, shm, a, s);
}

// LDS of a 64-row tile above which the stage runs 32-row tiles, and above
// which 16-row tiles (the grids of tol 1e-9 and tighter)
constexpr size_t kStageLdsSplit = 16 * 1024;
constexpr size_t kStageLdsSplit16 = 45 * 1024;

template <int MODE, int IO>
static void stage_ni(const StageArgs& a, hipStream_t s)
{
    using Tr = StageTraits<MODE>;
    auto lds = [&](int rt) {
        const size_t tile =
            std::max((size_t)a.Nin * rt * (Tr::xc ? 2 : 1), (size_t)a.Nout * rt * (Tr::yc ? 2 : 1));
        return (size_t)a.Nh * a.Kh * sizeof(double2) + tile * sizeof(double);
    };
    int rt = lds(64) > kStageLdsSplit16 ? 16 : (lds(64) > kStageLdsSplit ? 32 : 64);
    // a requested tile height where the compiled accumulator counts and the
    // LDS allow it (NI <= 4 at 16 rows, <= 8 at 32, <= 12 at 64)
    if (a.rt_request == 16 || a.rt_request == 32 || a.rt_request == 64) {
        const int r = a.rt_request;
        const int nir = (a.Nh + 256 / r - 1) / (256 / r);
        if (nir <= (r == 16 ? 4 : r == 32 ? 8 : 12) && lds(r) <= 150 * 1024)
            rt = r;
    }
    const size_t shm = lds(rt);
    const int ni = (a.Nh + 256 / rt - 1) / (256 / rt);
    // grid.y (slot, component) stays within 65535: large slot counts go in chunks
    const int chunk = kMaxGridY / a.ncomp;
    for (int s0 = a.slot0; s0 < a.nslots; s0 += chunk) {
        StageArgs b = a;
        b.slot0 = s0;
        const dim3 grid(nblocks(a.R, rt), std::min(chunk, a.nslots - s0) * a.ncomp);
        if (rt == 16) {
            stage_launch<MODE, IO, 4, 16>(grid, shm, b, s);  // ni <= 3: at most 48 half outputs
        } else if (rt == 32) {
            if (ni <= 4)
                stage_launch<MODE, IO, 4, 32>(grid, shm, b, s);
            else
                stage_launch<MODE, IO, 8, 32>(grid, shm, b, s);
        } else if (ni <= 4) {
            stage_launch<MODE, IO, 4, 64>(grid, shm, b, s);
        } else if (ni <= 8) {
            stage_launch<MODE, IO, 8, 64>(grid, shm, b, s);
        } else {
            stage_launch<MODE, IO, 12, 64>(grid, shm, b, s);
        }
    }
}

void launch_stage(int mode, int io, const StageArgs& a, hipStream_t s)
{
    if (a.nslots == 0 || a.R == 0)
        return;
    switch (mode) {
    case ST_SYM_REAL:
        if (io == IO_GATHER8)
            stage_ni<ST_SYM_REAL, IO_GATHER8>(a, s);
        else if (io == IO_SCATTER8)
            stage_ni<ST_SYM_REAL, IO_SCATTER8>(a, s);
        else
            stage_ni<ST_SYM_REAL, IO_PLAIN>(a, s);
        break;
    case ST_OUT_HALF: stage_ni<ST_OUT_HALF, IO_PLAIN>(a, s); break;
    case ST_OUT_FULL: stage_ni<ST_OUT_FULL, IO_PLAIN>(a, s); break;
    case ST_IN_FULL: stage_ni<ST_IN_FULL, IO_PLAIN>(a, s); break;
    default: stage_ni<ST_IN_HALF_REAL, IO_PLAIN>(a, s); break;
    }
}

// ---- translation --------------------------------------------------------------
// One block per (m_y slab, receiver).  The sender side is x-major
// (Phi[m_x][m_y][m_z]) and the receiver side z-major (Psi[m_z][m_y][m_x]); a
// slab of fixed m_y is read as q runs of n1 contiguous modes, transposed in LDS
// and written as n1 runs of q contiguous modes, so both sides stay coalesced.
// An entry is packed as 32 * (sender slot) + 9 (o_x + 1) + 3 (o_y + 1) + (o_z + 1)
// with the colleague offset o in {-1, 0, 1}^3.  Its phase exp(-2 pi i m.o / 3)
// depends on m only through m mod 3: each thread keeps 2 (m_k mod 3) and reads
// the phase index from a 2-bit table.
template <typename S, bool PLAIN>
__global__ __launch_bounds__(256) void k_translate(int q, int n1, int nparts, int nrecv,
                                                   const RecvDesc* __restrict__ recv, const int* __restrict__ e_pk,
                                                   const typename Store<S>::cx* __restrict__ Phi,
                                                   const double* __restrict__ wdiff,
                                                   typename Store<S>::cx* __restrict__ Psi)
{
    using cx = typename Store<S>::cx;
    extern __shared__ cplx tile[];  // [3][m_z][m_x] over this block's m_z range
    const int H = q * n1 * n1;
    // Blocks go round-robin over the 8 XCDs; give each XCD a contiguous run
    // of (part, slab, receiver) triples with the receiver fastest, so that
    // receivers adjacent in Morton order -- which share most of their
    // colleagues -- read the same sender slabs through the same L2.  A slab
    // is split into nparts ranges of m_z where its LDS tile would be large.
    const int total = nparts * n1 * nrecv;
    const int lg = xcd_block(total);
    if (lg < 0)
        return;
    const int part = lg / (n1 * nrecv);
    const int rem = lg - part * (n1 * nrecv);
    const int iy = rem / nrecv;
    const RecvDesc rd = recv[rem - iy * nrecv];
    const int h3 = (n1 + nparts - 1) / nparts;
    const int z0 = part * h3, nz = min(h3, n1 - z0);
    const int NS = q * nz;          // modes of the slab in this block
    const int m2 = iy - (q - 1);
    const double s3 = 0.86602540378443864676;
    const double lscale = (double)(1ll << rd.level);
    const int w2 = 2 * (((m2 % 3) + 3) % 3);
    const size_t H3 = (size_t)3 * H;
    for (int idx = threadIdx.x; idx < NS; idx += blockDim.x) {
        const int m1 = idx / nz;
        const int i3 = z0 + idx - m1 * nz;
        const int m3 = i3 - (q - 1);
        const cx* base = Phi + ((size_t)m1 * n1 + iy) * n1 + i3;
        const int w1 = 2 * (m1 % 3), w3 = 2 * (((m3 % 3) + 3) % 3);
        double F[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        cx va[3], vb[3];
        // sums one entry: F += exp(-2 pi i m.o / 3) v
        auto add = [&](int pk, const cx (&v)[3]) {
            const int c = pk & 31;
            const int sh = w1 * (c / 9 - 1) + w2 * ((c / 3) % 3 - 1) + w3 * (c % 3 - 1) + 12;
            // (k mod 3) at bits 2k, k = 0..12
            const int ph = (0x924924 >> sh) & 3;
            const double pr = ph ? -0.5 : 1.0;
            const double pi = ph == 0 ? 0.0 : (ph == 1 ? -s3 : s3);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double vr = (double)v[j].x, vi = (double)v[j].y;
                F[j][0] = fma(-pi, vi, fma(pr, vr, F[j][0]));
                F[j][1] = fma(pi, vr, fma(pr, vi, F[j][1]));
            }
        };
        auto load = [&](int pk, cx (&v)[3]) {
            const cx* ps = base + (size_t)(pk >> 5) * H3;
#pragma unroll
            for (int j = 0; j < 3; ++j)
                v[j] = ps[(size_t)j * H];
        };
        // two entries' loads in flight: each sum waits only for the older
        // one.  The loop body has no branch and its loads are unconditional
        // (indices past the end re-read the last entry), so the compiler's
        // wait before a sum never has to cover the newer loads.
        const int ne = rd.eend - rd.ebeg;
        if (ne > 0) {
            const int* ep = e_pk + rd.ebeg;
            int pa = ep[0];
            load(pa, va);
            int pb = ep[min(1, ne - 1)];
            load(pb, vb);
            for (int k = 0; k + 1 < ne; k += 2) {
                add(pa, va);
                pa = ep[min(k + 2, ne - 1)];
                load(pa, va);
                add(pb, vb);
                pb = ep[min(k + 3, ne - 1)];
                load(pb, vb);
            }
            if (ne & 1)
                add(pa, va);
        }
        if (PLAIN) {
            // the symbol was applied on the sending side (stresslet)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                tile[(j * nz + i3 - z0) * q + m1] = cplx{F[j][0], F[j][1]};
        } else {
            const int mm = m1 * m1 + m2 * m2 + m3 * m3;
            const double w = mm > 0 ? wdiff[mm] * lscale : 0.0;
            const double inv = mm > 0 ? 1.0 / mm : 0.0;
            const double dr = (m1 * F[0][0] + m2 * F[1][0] + m3 * F[2][0]) * inv;
            const double di = (m1 * F[0][1] + m2 * F[1][1] + m3 * F[2][1]) * inv;
            const int mv[3] = {m1, m2, m3};
#pragma unroll
            for (int j = 0; j < 3; ++j)
                tile[(j * nz + i3 - z0) * q + m1] = cplx{w * (F[j][0] - mv[j] * dr), w * (F[j][1] - mv[j] * di)};
        }
    }
    __syncthreads();
    typename Store<S>::cx* out = Psi + (size_t)rd.slot * 3 * H;
    for (int idx = threadIdx.x; idx < 3 * NS; idx += blockDim.x) {
        const int j = idx / NS;
        const int r = idx - j * NS;
        const int i3 = z0 + r / q;
        const int m1 = r - (i3 - z0) * q;
        const cplx t = tile[idx];
        out[(size_t)j * H + ((size_t)i3 * n1 + iy) * q + m1] = {(S)t.re, (S)t.im};
    }
}

void launch_translate(int q, int n1, const RecvDesc* recv, int nrecv, const int* e_pk, const void* Phi,
                      const double* wdiff, void* Psi, bool f32, bool plain, hipStream_t s)
{
    if (nrecv == 0)
        return;
    // two m_z ranges per slab where one tile would exceed 32 KB of LDS
    const int nparts = (size_t)3 * q * n1 * sizeof(cplx) > 32 * 1024 ? 2 : 1;
    const size_t lds = (size_t)3 * q * ((n1 + nparts - 1) / nparts) * sizeof(cplx);
    const int total = nparts * n1 * nrecv;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_translate<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipFuncSetAttribute((const void*)k_translate<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipFuncSetAttribute((const void*)k_translate<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipFuncSetAttribute((const void*)k_translate<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
#define L_TR(T2, S, PL)                                                                                        \
    hipLaunchKernelGGL((k_translate<S, PL>), dim3(xcd_grid(total)), dim3(256), lds, s, q, n1, nparts, nrecv, recv, e_pk, \
                       (const T2*)Phi, wdiff, (T2*)Psi)
    if (f32) {
        if (plain)
            L_TR(float2, float, true);
        else
            L_TR(float2, float, false);
    } else {
        if (plain)
            L_TR(double2, double, true);
        else
            L_TR(double2, double, false);
    }
#undef L_TR
}

// Stresslet difference symbol applied on the sending side (the 6 -> 3
// contraction, eq. moll_stresslet): for each sender slot and mode m (x-major
// half spectrum), u_j = i w [m^2 (2 (rho m)_j + m_j tr rho) - 2 m_j m.rho.m],
// w = 4^level wdiff_t(|m|^2), rho the symmetric density with the
// off-diagonal pairs stored summed.
template <typename S>
__global__ __launch_bounds__(256) void k_stress_symbol(int q, int n1, const int* __restrict__ send_level,
                                                       const typename Store<S>::cx* __restrict__ Phi6,
                                                       const double* __restrict__ wdiff_t,
                                                       typename Store<S>::cx* __restrict__ Phi3)
{
    const int H = q * n1 * n1;
    const int mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= H)
        return;
    const int snd = blockIdx.y;
    const int m1 = mi / (n1 * n1);
    const int rem = mi - m1 * n1 * n1;
    const int m2 = rem / n1 - (q - 1), m3 = rem % n1 - (q - 1);
    const int mm = m1 * m1 + m2 * m2 + m3 * m3;
    const double w = mm > 0 ? wdiff_t[mm] * (double)(1ll << (2 * send_level[snd])) : 0.0;
    const typename Store<S>::cx* in = Phi6 + (size_t)snd * 6 * H + mi;
    double rr[6], ri[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const typename Store<S>::cx v = in[(size_t)c * H];
        rr[c] = (double)v.x;
        ri[c] = (double)v.y;
    }
    const double m[3] = {(double)m1, (double)m2, (double)m3};
    auto apply = [&](const double* g, double* u) {
        // symmetric matrix from (11, 22, 33, 12+21, 13+31, 23+32)
        const double a11 = g[0], a22 = g[1], a33 = g[2], a12 = 0.5 * g[3], a13 = 0.5 * g[4], a23 = 0.5 * g[5];
        const double rm0 = a11 * m[0] + a12 * m[1] + a13 * m[2];
        const double rm1 = a12 * m[0] + a22 * m[1] + a23 * m[2];
        const double rm2 = a13 * m[0] + a23 * m[1] + a33 * m[2];
        const double tr = a11 + a22 + a33;
        const double mrm = m[0] * rm0 + m[1] * rm1 + m[2] * rm2;
        u[0] = mm * (2.0 * rm0 + m[0] * tr) - 2.0 * m[0] * mrm;
        u[1] = mm * (2.0 * rm1 + m[1] * tr) - 2.0 * m[1] * mrm;
        u[2] = mm * (2.0 * rm2 + m[2] * tr) - 2.0 * m[2] * mrm;
    };
    double ur[3], ui[3];
    apply(rr, ur);
    apply(ri, ui);
    typename Store<S>::cx* out = Phi3 + (size_t)snd * 3 * H + mi;
    // multiplication by i w: (re, im) -> (-w im, w re)
#pragma unroll
    for (int j = 0; j < 3; ++j)
        out[(size_t)j * H] = {(S)(-w * ui[j]), (S)(w * ur[j])};
}

void launch_stress_symbol(int q, int n1, int nsend, const int* send_level, const void* Phi6, const double* wdiff_t,
                          void* Phi3, bool f32, hipStream_t s)
{
    if (nsend == 0)
        return;
    const size_t H = (size_t)q * n1 * n1;
    for (int s0 = 0; s0 < nsend; s0 += kMaxGridY) {
        const dim3 grid(nblocks((int64_t)H, 256), std::min(kMaxGridY, nsend - s0));
        if (f32)
            hipLaunchKernelGGL(k_stress_symbol<float>, grid, dim3(256), 0, s, q, n1, send_level + s0,
                               (const float2*)Phi6 + (size_t)s0 * 6 * H, wdiff_t, (float2*)Phi3 + (size_t)s0 * 3 * H);
        else
            hipLaunchKernelGGL(k_stress_symbol<double>, grid, dim3(256), 0, s, q, n1, send_level + s0,
                               (const double2*)Phi6 + (size_t)s0 * 6 * H, wdiff_t,
                               (double2*)Phi3 + (size_t)s0 * 3 * H);
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_root_symbol(int mh, int mf, const typename Store<S>::cx* __restrict__ Phi,
                                                     const double* __restrict__ w,
                                                     typename Store<S>::cx* __restrict__ Psi)
{
    const int H = mh * mf * mf;
    const int mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= H)
        return;
    Phi += (size_t)blockIdx.y * 3 * H;  // one root per grid row
    Psi += (size_t)blockIdx.y * 3 * H;
    const int M = (mf - 1) / 2;
    const int m1 = mi / (mf * mf);
    const int rem = mi - m1 * mf * mf;
    const int m2 = rem / mf - M, m3 = rem % mf - M;
    const int mm = m1 * m1 + m2 * m2 + m3 * m3;
    double Fr[3], Fi[3];
    for (int j = 0; j < 3; ++j) {
        const typename Store<S>::cx v = Phi[(size_t)j * H + mi];
        Fr[j] = (double)v.x;
        Fi[j] = (double)v.y;
    }
    const double ww = mm > 0 ? w[mm] : 0.0;
    const double inv = mm > 0 ? 1.0 / mm : 0.0;
    const double dr = (m1 * Fr[0] + m2 * Fr[1] + m3 * Fr[2]) * inv;
    const double di = (m1 * Fi[0] + m2 * Fi[1] + m3 * Fi[2]) * inv;
    const int mv[3] = {m1, m2, m3};
    const size_t mo = ((size_t)(m3 + M) * mf + (m2 + M)) * mh + m1;
    for (int j = 0; j < 3; ++j)
        Psi[(size_t)j * H + mo] = {(S)(ww * (Fr[j] - mv[j] * dr)), (S)(ww * (Fi[j] - mv[j] * di))};
}

void launch_root_symbol(int mh, int mf, int nroot, const void* Phi, const double* w, void* Psi, bool f32,
                        hipStream_t s)
{
    const size_t H = (size_t)mh * mf * mf;
    for (int r0 = 0; r0 < nroot; r0 += kMaxGridY) {
        const dim3 grid(nblocks((int64_t)H, 256), std::min(kMaxGridY, nroot - r0));
        if (f32)
            hipLaunchKernelGGL(k_root_symbol<float>, grid, dim3(256), 0, s, mh, mf,
                               (const float2*)Phi + (size_t)r0 * 3 * H, w, (float2*)Psi + (size_t)r0 * 3 * H);
        else
            hipLaunchKernelGGL(k_root_symbol<double>, grid, dim3(256), 0, s, mh, mf,
                               (const double2*)Phi + (size_t)r0 * 3 * H, w, (double2*)Psi + (size_t)r0 * 3 * H);
    }
}

// Stresslet root symbol (truncated kernel, eq. moll_stresslet with Bhat^R):
// Phi6 x-major [6][mx][my][mz] -> Psi3 z-major [3][mz][my][mx],
// u_j = i w(|m|^2) [k^2 (2 (rho k)_j + k_j tr rho) - 2 k_j k.rho.k], k = kscale m.
template <typename S>
__global__ __launch_bounds__(256) void k_root_symbol_t(int mh, int mf, const typename Store<S>::cx* __restrict__ Phi,
                                                       const double* __restrict__ w, double kscale,
                                                       typename Store<S>::cx* __restrict__ Psi)
{
    const int H = mh * mf * mf;
    const int mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= H)
        return;
    Phi += (size_t)blockIdx.y * 6 * H;
    Psi += (size_t)blockIdx.y * 3 * H;
    const int M = (mf - 1) / 2;
    const int m1 = mi / (mf * mf);
    const int rem = mi - m1 * mf * mf;
    const int m2 = rem / mf - M, m3 = rem % mf - M;
    const int mm = m1 * m1 + m2 * m2 + m3 * m3;
    const double ww = mm > 0 ? w[mm] : 0.0;
    const double k[3] = {kscale * m1, kscale * m2, kscale * m3};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    double gr[6], gi[6];
    for (int c = 0; c < 6; ++c) {
        const typename Store<S>::cx v = Phi[(size_t)c * H + mi];
        gr[c] = (double)v.x;
        gi[c] = (double)v.y;
    }
    auto apply = [&](const double* g, double* u) {
        const double a11 = g[0], a22 = g[1], a33 = g[2], a12 = 0.5 * g[3], a13 = 0.5 * g[4], a23 = 0.5 * g[5];
        const double rk0 = a11 * k[0] + a12 * k[1] + a13 * k[2];
        const double rk1 = a12 * k[0] + a22 * k[1] + a23 * k[2];
        const double rk2 = a13 * k[0] + a23 * k[1] + a33 * k[2];
        const double tr = a11 + a22 + a33;
        const double krk = k[0] * rk0 + k[1] * rk1 + k[2] * rk2;
        u[0] = k2 * (2.0 * rk0 + k[0] * tr) - 2.0 * k[0] * krk;
        u[1] = k2 * (2.0 * rk1 + k[1] * tr) - 2.0 * k[1] * krk;
        u[2] = k2 * (2.0 * rk2 + k[2] * tr) - 2.0 * k[2] * krk;
    };
    double ur[3], ui[3];
    apply(gr, ur);
    apply(gi, ui);
    const size_t mo = ((size_t)(m3 + M) * mf + (m2 + M)) * mh + m1;
    for (int j = 0; j < 3; ++j)
        Psi[(size_t)j * H + mo] = {(S)(-ww * ui[j]), (S)(ww * ur[j])};
}

void launch_root_symbol_t(int mh, int mf, int nroot, const void* Phi, const double* w, double kscale, void* Psi,
                          bool f32, hipStream_t s)
{
    const size_t H = (size_t)mh * mf * mf;
    for (int r0 = 0; r0 < nroot; r0 += kMaxGridY) {
        const dim3 grid(nblocks((int64_t)H, 256), std::min(kMaxGridY, nroot - r0));
        if (f32)
            hipLaunchKernelGGL(k_root_symbol_t<float>, grid, dim3(256), 0, s, mh, mf,
                               (const float2*)Phi + (size_t)r0 * 6 * H, w, kscale,
                               (float2*)Psi + (size_t)r0 * 3 * H);
        else
            hipLaunchKernelGGL(k_root_symbol_t<double>, grid, dim3(256), 0, s, mh, mf,
                               (const double2*)Phi + (size_t)r0 * 6 * H, w, kscale,
                               (double2*)Psi + (size_t)r0 * 3 * H);
    }
}

// ---- near field -----------------------------------------------------------------
// Residual Stokeslet at scale r_l (r < r_l):
//   S_R(y) f = f/(8 pi r) + (y.f) y/(8 pi r^3) - [P(s) f + Q(s) (y.f) y / r_l^2]/(4 pi r_l),
// s = r^2 / r_l^2, with P and Q polynomials in t = 2s - 1 (monomial
// coefficients, Horner; their signs alternate so Horner is as stable as the
// Chebyshev form).
__device__ inline double rsqrt_f64(double x)
{
    // hardware estimate refined by one second-order Newton step:
    // e = 1 - x y^2,  y <- y + y e (1/2 + 3/8 e)
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

template <int ND>
__device__ inline double horner(const double* __restrict__ m, double t)
{
    double p = m[ND - 1];
#pragma unroll
    for (int k = ND - 2; k >= 0; --k)
        p = fma(p, t, m[k]);
    return p;
}

// The same with the leading coefficient already in a vector register (a
// fused multiply-add reads at most one scalar register).
template <int ND>
__device__ inline double horner_v(const double* __restrict__ m, double top, double t)
{
    double p = top;
#pragma unroll
    for (int k = ND - 2; k >= 0; --k)
        p = fma(p, t, m[k]);
    return p;
}

// The same pair for NR force vectors: the geometry, the square root and both
// radial polynomials are shared, only the projections onto the forces repeat.
// v holds the source as (x, y, z, f_0, ..., f_{NR-1}) (already shifted) with
// the forces pre-scaled by 1/(8 pi), so that with c2 = 8 pi cP = 2 / r_l and
// c3 = 8 pi cQ = 2 / r_l^3 the pair adds
//   a f' + (d.f') b d,   a = 1/r - c2 P(s),   b = 1/r^3 - c3 Q(s).
// pt, qt: the leading coefficients of P and Q in vector registers.  RF = false
// uses the hardware reciprocal square root unrefined (relative error below
// 6e-8, measured on gfx950), enough for tolerances of 1e-6 and above.
// NZ: no two distinct points of the plan coincide, so the only pair at r = 0
// is a target with itself; such pairs are skipped here and the kernel adds
// the self term -S_M(0) f separately (saving the r = 0 select on every pair).
template <int ND, int NR, bool RF, bool NZ = false>
__device__ inline void residual_pair_multi(double xt, double yt, double zt, const double* v, double rl2, double tw,
                                           double c2, double c3, double pt, double qt, const RadialPoly& poly,
                                           double (&u)[NR][3])
{
    const double dx = xt - v[0], dy = yt - v[1], dz = zt - v[2];
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (NZ ? (r2 < rl2 && r2 > 0.0) : (r2 < rl2)) {
        const double rq = RF ? rsqrt_f64(r2) : __builtin_amdgcn_rsq(r2);
        const double rinv = NZ ? rq : (r2 > 0.0 ? rq : 0.0);
        const double t = fma(r2, tw, -1.0);
        const double P = horner_v<ND>(poly.P, pt, t);
        const double Q = horner_v<ND>(poly.Q, qt, t);
        const double a = fma(-c2, P, rinv);
        const double bq = fma(-c3, Q, rinv * rinv * rinv);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double fx = v[3 + 3 * r], fy = v[4 + 3 * r], fz = v[5 + 3 * r];
            const double b = fma(dx, fx, fma(dy, fy, dz * fz)) * bq;
            u[r][0] = fma(a, fx, fma(b, dx, u[r][0]));
            u[r][1] = fma(a, fy, fma(b, dy, u[r][1]));
            u[r][2] = fma(a, fz, fma(b, dz, u[r][2]));
        }
    }
}

// Residual stresslet pair (eq. res_stresslet with R_Tdiag, R_Toffd of eq.
// T-offd, rearranged around the free-space stresslet): with d = x_t - x_s,
// s = |d|^2 / r_lambda^2, A and D the radial polynomials (poly.P, poly.Q),
//   u += [-(3/4pi) (d.f)(d.n)/|d|^5 + cA A(s) (d.f)(d.n) + cD D(s) (f.n)] d
//        + cD D(s) [(d.n) f + (d.f) n],
// cA = 3/(2 pi r_lambda^5), cD = 1/(4 pi r_lambda^3).  v holds the source as
// (x, y, z, f, n, f.n).  Every term is proportional to d, so a pair at r = 0
// contributes nothing (the stresslet has no self term).
template <int ND>
__device__ inline void residual_pair_stresslet(double xt, double yt, double zt, const double* v, double rl2,
                                               double tw, double cA, double cD, double pt, double qt,
                                               const RadialPoly& poly, double (&u)[1][3])
{
    const double dx = xt - v[0], dy = yt - v[1], dz = zt - v[2];
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (r2 < rl2) {
        const double rinv = r2 > 0.0 ? rsqrt_f64(r2) : 0.0;
        const double rinv2 = rinv * rinv;
        const double t = fma(r2, tw, -1.0);
        const double A = horner_v<ND>(poly.P, pt, t);
        const double D = horner_v<ND>(poly.Q, qt, t);
        const double df = fma(dx, v[3], fma(dy, v[4], dz * v[5]));
        const double dn = fma(dx, v[6], fma(dy, v[7], dz * v[8]));
        const double c2 = cD * D;
        const double c1 = df * dn * fma(cA, A, -k3Over4Pi * rinv2 * rinv2 * rinv);
        const double cy = fma(c2, v[9], c1);
        const double a = c2 * dn, b = c2 * df;
        u[0][0] = fma(cy, dx, fma(a, v[3], fma(b, v[6], u[0][0])));
        u[0][1] = fma(cy, dy, fma(a, v[4], fma(b, v[7], u[0][1])));
        u[0][2] = fma(cy, dz, fma(a, v[5], fma(b, v[8], u[0][2])));
    }
}

// One wave per target group of TG = 64/SG points of a leaf; lane (t, s) handles
// target t against every SG-th queued source.  Source leaves of the near list
// are walked in 64-point chunks: a chunk whose bounding box lies farther than
// r_lambda from the group's box is skipped, and of the rest each source is kept
// only if it lies within r_lambda of that box.  Kept sources (with the periodic
// image shift applied, and the NR force vectors of the batch) are packed into
// LDS and evaluated at once.  Every batch size visits sources in the same
// order, so a force vector's result does not depend on how it was batched.
// The SG partial sums of a target are combined by cross-lane shuffles.
// Forces and outputs are [NR][3][n].  KER = 1: the stresslet (NR = 1), with
// the sources' f and n as fs[6][n].  RF: refined reciprocal square root (the
// Stokeslet pair routine).  The packed tile is padded with up to SG - 1 far
// away dummy sources, so every lane runs the same number of pair steps.
template <int ND, int SG, int NR, int KER, bool RF, bool NZ>
__global__ __launch_bounds__(64) void k_near(const NearWork* __restrict__ work, int nwork,
                                             const NearLeaf* __restrict__ leaves,
                                             const NearEntryDev* __restrict__ entries, const double* __restrict__ cbbox,
                                             const double* __restrict__ x, const double* __restrict__ y,
                                             const double* __restrict__ z, const double* __restrict__ fs, int64_t n,
                                             RadialPoly poly, int self_term, double* __restrict__ u)
{
    constexpr int TG = 64 / SG;
    constexpr int NV = KER == 1 ? 7 : 3 * NR;  // staged values per source beyond its position
    constexpr int W2 = (3 + NV + 1) / 2;       // double2 per staged source
    __shared__ double2 S[64 + SG - 1][W2];
    const NearWork w = work[blockIdx.x];
    if (w.leaf < 0)  // padding of the per-XCD work lists
        return;
    const NearLeaf T = leaves[w.leaf];
    const int lane = threadIdx.x;
    const int tl = lane / SG, sl = lane % SG;
    const int64_t g0 = T.tstart + (int64_t)w.chunk * TG;
    const int64_t i = g0 + tl;
    const bool valid = i < T.tend;
    const double xt = valid ? x[i] : 0.0, yt = valid ? y[i] : 0.0, zt = valid ? z[i] : 0.0;
    // bounding box of the target group (wave reduction)
    double tlo[3] = {valid ? xt : 1e300, valid ? yt : 1e300, valid ? zt : 1e300};
    double thi[3] = {valid ? xt : -1e300, valid ? yt : -1e300, valid ? zt : -1e300};
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            tlo[d] = fmin(tlo[d], __shfl_xor(tlo[d], off));
            thi[d] = fmax(thi[d], __shfl_xor(thi[d], off));
        }
    double acc[NR][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
        acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
    // leading radial coefficients, held in vector registers
    double pt = poly.P[ND - 1], qt = poly.Q[ND - 1];
    asm volatile("" : "+v"(pt), "+v"(qt));
    for (int e = T.ebeg; e < T.eend; ++e) {
        const NearEntryDev E = entries[e];
        // powers of two of the level: exact, and equal to the quotients
        // 1 / r_l, 1 / (4 pi r_l), ... rounded once
        const int lam = E.lambda;
        const double rl2 = ldexp(1.0, -2 * lam);
        const double tw = ldexp(2.0, 2 * lam);
        // Stokeslet (forces staged times 1/(8 pi)): c2 = 2 / r_l, c3 = 2 / r_l^3;
        // stresslet: cA = 3/(2 pi r_l^5), cD = 1/(4 pi r_l^3)
        const double cP = KER == 1 ? ldexp(3.0 / (2.0 * kPi), 5 * lam) : ldexp(2.0, lam);
        const double cQ = KER == 1 ? ldexp(1.0 / (4.0 * kPi), 3 * lam) : ldexp(2.0, 3 * lam);
        const double sh[3] = {(double)E.sx, (double)E.sy, (double)E.sz};
        const int nch = (int)((E.send - E.sstart + 63) / 64);
        for (int kb = 0; kb < nch; kb += 64) {
            // the lanes test 64 chunks of the entry against the group's box at
            // once; the wave then visits the chunks within r_lambda in order
            bool cnear = false;
            if (kb + lane < nch) {
                const double* sb = cbbox + 6 * (size_t)(E.cbase + kb + lane);
                double gap2 = 0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double g = fmax(0.0, fmax(sb[d] + sh[d] - thi[d], tlo[d] - (sb[3 + d] + sh[d])));
                    gap2 += g * g;
                }
                cnear = gap2 < rl2;
            }
            for (unsigned long long cm = __ballot(cnear); cm != 0; cm &= cm - 1) {
                const int k = kb + __ffsll((long long)cm) - 1;
                const int64_t s0 = E.sstart + 64 * (int64_t)k;
                const int ccnt = (int)min((int64_t)64, E.send - s0);
                double sx = 0, sy = 0, sz = 0;
                bool keep = false;
                if (lane < ccnt) {
                    const int64_t j = s0 + lane;
                    sx = x[j] + sh[0];
                    sy = y[j] + sh[1];
                    sz = z[j] + sh[2];
                    const double gx = fmax(0.0, fmax(tlo[0] - sx, sx - thi[0]));
                    const double gy = fmax(0.0, fmax(tlo[1] - sy, sy - thi[1]));
                    const double gz = fmax(0.0, fmax(tlo[2] - sz, sz - thi[2]));
                    keep = fma(gx, gx, fma(gy, gy, gz * gz)) < rl2;
                }
                const unsigned long long mask = __ballot(keep);
                const int kept = __popcll(mask);
                if (kept == 0)
                    continue;
                const int pos = __popcll(mask & ((1ull << lane) - 1ull));
                __syncthreads();
                if (keep) {
                    const int64_t j = s0 + lane;
                    double v[2 * W2];
                    v[0] = sx;
                    v[1] = sy;
                    v[2] = sz;
                    if (KER == 1) {
#pragma unroll
                        for (int c = 0; c < 6; ++c)
                            v[3 + c] = fs[(size_t)c * n + j];
                        v[9] = fma(v[3], v[6], fma(v[4], v[7], v[5] * v[8]));
                    } else {
#pragma unroll
                        for (int c = 0; c < 3 * NR; ++c)
                            v[3 + c] = fs[(size_t)c * n + j] * kInv8Pi;
                    }
                    if (2 * W2 > 3 + NV)
                        v[2 * W2 - 1] = 0.0;
#pragma unroll
                    for (int c = 0; c < W2; ++c)
                        S[pos][c] = make_double2(v[2 * c], v[2 * c + 1]);
                }
                if (SG > 1 && lane < SG - 1) {
                    // dummies far outside every support: r^2 >= r_lambda^2
                    S[kept + lane][0] = make_double2(1e100, 1e100);
#pragma unroll
                    for (int c = 1; c < W2; ++c)
                        S[kept + lane][c] = make_double2(1e100, 0.0);
                }
                __syncthreads();
                const int steps = (kept + SG - 1) / SG;
#pragma unroll 2
                for (int it = 0; it < steps; ++it) {
                    const int jj = it * SG + sl;
                    double v[2 * W2];
#pragma unroll
                    for (int c = 0; c < W2; ++c) {
                        const double2 t2 = S[jj][c];
                        v[2 * c] = t2.x;
                        v[2 * c + 1] = t2.y;
                    }
                    if constexpr (KER == 1)
                        residual_pair_stresslet<ND>(xt, yt, zt, v, rl2, tw, cP, cQ, pt, qt, poly, acc);
                    else
                        residual_pair_multi<ND, NR, RF, NZ>(xt, yt, zt, v, rl2, tw, cP, cQ, pt, qt, poly, acc);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int off = 1; off < SG; off <<= 1) {
            acc[r][0] += __shfl_xor(acc[r][0], off);
            acc[r][1] += __shfl_xor(acc[r][1], off);
            acc[r][2] += __shfl_xor(acc[r][2], off);
        }
    if (NZ && self_term && valid && sl == 0) {
        // the pair of the target with itself (eq. S_self at the leaf's scale):
        // -(2 / r_l) P(-1) f / (8 pi)
        const double a = -ldexp(2.0 * poly.p_self, T.level);
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                acc[r][c] = fma(a, fs[(size_t)(3 * r + c) * n + i] * kInv8Pi, acc[r][c]);
    }
    if (valid && sl == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            u[(size_t)(3 * r) * n + i] += acc[r][0];
            u[(size_t)(3 * r + 1) * n + i] += acc[r][1];
            u[(size_t)(3 * r + 2) * n + i] += acc[r][2];
        }
    }
}

#define DMK_ND_DISPATCH(nd, MACRO) \
    if (nd <= 14) {                \
        MACRO(14);                 \
    } else if (nd <= 18) {         \
        MACRO(18);                 \
    } else if (nd <= 21) {         \
        MACRO(21);                 \
    } else {                       \
        MACRO(24);                 \
    }

void launch_near(int kernel, int sg, int nr, bool refine, bool no_coincident, bool self_term, const NearWork* work,
                 int nwork, const NearLeaf* leaves, const NearEntryDev* entries, const double* cbbox, const double* x,
                 const double* y, const double* z, const double* fs, int64_t n, const RadialPoly& poly, double* u,
                 hipStream_t s)
{
    if (nwork == 0)
        return;
#define L_NEAR_KZ(ND, SG, NR, KER, RF, NZ)                                                                             \
    hipLaunchKernelGGL((k_near<ND, SG, NR, KER, RF, NZ>), dim3(nwork), dim3(64), 0, s, work, nwork, leaves, entries, \
                       cbbox, x, y, z, fs, n, poly, self_term ? 1 : 0, u)
#define L_NEAR_KK(ND, SG, NR, KER, RF)             \
    do {                                           \
        if (KER == 0 && no_coincident)             \
            L_NEAR_KZ(ND, SG, NR, KER, RF, true);  \
        else                                       \
            L_NEAR_KZ(ND, SG, NR, KER, RF, false); \
    } while (0)
    // batches of several force vectors always use 4 source lanes per target
#define L_STOKES(ND, RF)                     \
    if (nr == 2) {                           \
        L_NEAR_KK(ND, 4, 2, 0, RF);          \
    } else if (nr == 4) {                    \
        L_NEAR_KK(ND, 4, 4, 0, RF);          \
    } else if (nr == 8) {                    \
        L_NEAR_KK(ND, 4, 8, 0, RF);          \
    } else if (sg == 1) {                    \
        L_NEAR_KK(ND, 1, 1, 0, RF);          \
    } else if (sg == 2) {                    \
        L_NEAR_KK(ND, 2, 1, 0, RF);          \
    } else if (sg == 4) {                    \
        L_NEAR_KK(ND, 4, 1, 0, RF);          \
    } else {                                 \
        L_NEAR_KK(ND, 8, 1, 0, RF);          \
    }
    // the unrefined square root only with the shortest fits (tol >= 1e-6)
#define L_NEAR(ND)                           \
    if (kernel == 1) {                       \
        if (sg == 1)                         \
            L_NEAR_KK(ND, 1, 1, 1, true);    \
        else if (sg == 2)                    \
            L_NEAR_KK(ND, 2, 1, 1, true);    \
        else if (sg == 4)                    \
            L_NEAR_KK(ND, 4, 1, 1, true);    \
        else                                 \
            L_NEAR_KK(ND, 8, 1, 1, true);    \
    } else if (ND == 14 && !refine) {        \
        L_STOKES(14, false);                 \
    } else {                                 \
        L_STOKES(ND, true);                  \
    }
    DMK_ND_DISPATCH(poly.nd, L_NEAR)
#undef L_NEAR
#undef L_STOKES
#undef L_NEAR_KK
#undef L_NEAR_KZ
}

template <int SG>
__global__ __launch_bounds__(64) void k_near_count(const NearWork* __restrict__ work, int nwork,
                                                   const NearLeaf* __restrict__ leaves,
                                                   const NearEntryDev* __restrict__ entries,
                                                   const double* __restrict__ cbbox, const double* __restrict__ x,
                                                   const double* __restrict__ y, const double* __restrict__ z,
                                                   unsigned long long* __restrict__ out)
{
    constexpr int TG = 64 / SG;
    const NearWork w = work[blockIdx.x];
    if (w.leaf < 0)  // padding of the per-XCD work lists
        return;
    const NearLeaf T = leaves[w.leaf];
    const int lane = threadIdx.x;
    const int tl = lane / SG, sl = lane % SG;
    const int64_t g0 = T.tstart + (int64_t)w.chunk * TG;
    const int64_t i = g0 + tl;
    const bool valid = i < T.tend;
    const int nt = (int)min((int64_t)TG, T.tend - g0);
    const double xt = valid ? x[i] : 0.0, yt = valid ? y[i] : 0.0, zt = valid ? z[i] : 0.0;
    double tlo[3] = {valid ? xt : 1e300, valid ? yt : 1e300, valid ? zt : 1e300};
    double thi[3] = {valid ? xt : -1e300, valid ? yt : -1e300, valid ? zt : -1e300};
    for (int off = 32; off >= 1; off >>= 1)
        for (int d = 0; d < 3; ++d) {
            tlo[d] = fmin(tlo[d], __shfl_xor(tlo[d], off));
            thi[d] = fmax(thi[d], __shfl_xor(thi[d], off));
        }
    unsigned long long ev = 0, in = 0;
    for (int e = T.ebeg; e < T.eend; ++e) {
        const NearEntryDev E = entries[e];
        const double rl = 1.0 / (double)(1ll << E.lambda);
        const double rl2 = rl * rl;
        const double sh[3] = {(double)E.sx, (double)E.sy, (double)E.sz};
        const int nch = (int)((E.send - E.sstart + 63) / 64);
        for (int k = 0; k < nch; ++k) {
            const double* sb = cbbox + 6 * (size_t)(E.cbase + k);
            double gap2 = 0;
            for (int d = 0; d < 3; ++d) {
                const double g = fmax(0.0, fmax(sb[d] + sh[d] - thi[d], tlo[d] - (sb[3 + d] + sh[d])));
                gap2 += g * g;
            }
            if (gap2 >= rl2)
                continue;
            const int64_t s0 = E.sstart + 64 * (int64_t)k;
            const int64_t s1 = min(s0 + 64, E.send);
            bool keep = false;
            if (s0 + lane < s1) {
                const int64_t j = s0 + lane;
                const double sx = x[j] + sh[0], sy = y[j] + sh[1], sz = z[j] + sh[2];
                const double gx = fmax(0.0, fmax(tlo[0] - sx, sx - thi[0]));
                const double gy = fmax(0.0, fmax(tlo[1] - sy, sy - thi[1]));
                const double gz = fmax(0.0, fmax(tlo[2] - sz, sz - thi[2]));
                keep = fma(gx, gx, fma(gy, gy, gz * gz)) < rl2;
            }
            const int kept = __popcll(__ballot(keep));
            if (lane == 0)
                ev += (unsigned long long)kept * nt;
            for (int64_t j = s0 + sl; j < s1 && valid; j += SG) {
                const double dx = xt - (x[j] + sh[0]), dy = yt - (y[j] + sh[1]), dz = zt - (z[j] + sh[2]);
                const double r2 = dx * dx + dy * dy + dz * dz;
                in += (r2 < rl2 && r2 > 0.0) ? 1ull : 0ull;
            }
        }
    }
    atomicAdd(&out[0], ev);
    atomicAdd(&out[1], in);
}

void launch_near_count(int sg, const NearWork* work, int nwork, const NearLeaf* leaves, const NearEntryDev* entries,
                       const double* cbbox, const double* x, const double* y, const double* z,
                       unsigned long long* out, hipStream_t s)
{
    if (nwork == 0)
        return;
    if (sg == 1)
        hipLaunchKernelGGL(k_near_count<1>, dim3(nwork), dim3(64), 0, s, work, nwork, leaves, entries, cbbox,
                           x, y, z, out);
    else if (sg == 2)
        hipLaunchKernelGGL(k_near_count<2>, dim3(nwork), dim3(64), 0, s, work, nwork, leaves, entries, cbbox,
                           x, y, z, out);
    else if (sg == 4)
        hipLaunchKernelGGL(k_near_count<4>, dim3(nwork), dim3(64), 0, s, work, nwork, leaves, entries, cbbox,
                           x, y, z, out);
    else
        hipLaunchKernelGGL(k_near_count<8>, dim3(nwork), dim3(64), 0, s, work, nwork, leaves, entries, cbbox,
                           x, y, z, out);
}

// Brute-force residual sums over all sources with the near field's own pair
// routine and source staging: forces scaled by 1/(8 pi) as they are read, the
// leading radial coefficients in vector registers, c2 = 2 / r_l and
// c3 = 2 / r_l^3 (powers of two when r_l is), and the same choice RF of the
// reciprocal square root as the near field of a plan at this tolerance.
template <int ND, bool RF>
__global__ __launch_bounds__(64) void k_residual_direct(const double* __restrict__ tx, const double* __restrict__ ty,
                                                        const double* __restrict__ tz, int64_t m,
                                                        const double* __restrict__ sx, const double* __restrict__ sy,
                                                        const double* __restrict__ sz, const double* __restrict__ sf,
                                                        int64_t ns, double rl, RadialPoly poly, double* __restrict__ u)
{
    const int64_t i = blockIdx.x * (int64_t)64 + threadIdx.x;
    const bool valid = i < m;
    const double xt = valid ? tx[i] : 0.0, yt = valid ? ty[i] : 0.0, zt = valid ? tz[i] : 0.0;
    const double rl2 = rl * rl, tw = 2.0 / rl2;
    const double c2 = 2.0 / rl, c3 = c2 / rl2;
    double pt = poly.P[ND - 1], qt = poly.Q[ND - 1];
    asm volatile("" : "+v"(pt), "+v"(qt));
    double acc[1][3] = {{0, 0, 0}};
    for (int64_t j = 0; j < ns; ++j) {
        const double v[6] = {sx[j], sy[j], sz[j], sf[j] * kInv8Pi, sf[ns + j] * kInv8Pi, sf[2 * ns + j] * kInv8Pi};
        residual_pair_multi<ND, 1, RF>(xt, yt, zt, v, rl2, tw, c2, c3, pt, qt, poly, acc);
    }
    if (valid) {
        u[3 * i] = acc[0][0];
        u[3 * i + 1] = acc[0][1];
        u[3 * i + 2] = acc[0][2];
    }
}

// stresslet: sf = (f, n) as [6][ns]
template <int ND>
__global__ __launch_bounds__(64) void k_residual_direct_t(const double* __restrict__ tx,
                                                          const double* __restrict__ ty,
                                                          const double* __restrict__ tz, int64_t m,
                                                          const double* __restrict__ sx,
                                                          const double* __restrict__ sy,
                                                          const double* __restrict__ sz,
                                                          const double* __restrict__ sf, int64_t ns, double rl,
                                                          RadialPoly poly, double* __restrict__ u)
{
    const int64_t i = blockIdx.x * (int64_t)64 + threadIdx.x;
    const bool valid = i < m;
    const double xt = valid ? tx[i] : 0.0, yt = valid ? ty[i] : 0.0, zt = valid ? tz[i] : 0.0;
    const double rl2 = rl * rl;
    const double cA = 3.0 / (2.0 * kPi * rl2 * rl2 * rl), cD = 1.0 / (4.0 * kPi * rl2 * rl);
    double acc[1][3] = {{0, 0, 0}};
    for (int64_t j = 0; j < ns; ++j) {
        double v[10] = {sx[j], sy[j], sz[j]};
        for (int c = 0; c < 6; ++c)
            v[3 + c] = sf[(size_t)c * ns + j];
        v[9] = fma(v[3], v[6], fma(v[4], v[7], v[5] * v[8]));
        residual_pair_stresslet<ND>(xt, yt, zt, v, rl2, 2.0 / rl2, cA, cD, poly.P[ND - 1], poly.Q[ND - 1], poly, acc);
    }
    if (valid) {
        u[3 * i] = acc[0][0];
        u[3 * i + 1] = acc[0][1];
        u[3 * i + 2] = acc[0][2];
    }
}

void launch_residual_direct_t(const double* tx, const double* ty, const double* tz, int64_t m, const double* sx,
                              const double* sy, const double* sz, const double* sf, int64_t ns, double r_lambda,
                              const RadialPoly& poly, double* u, hipStream_t s)
{
    if (m == 0)
        return;
#define L_RES(ND)                                                                                                 \
    hipLaunchKernelGGL(k_residual_direct_t<ND>, dim3(nblocks(m, 64)), dim3(64), 0, s, tx, ty, tz, m, sx, sy, sz, \
                       sf, ns, r_lambda, poly, u)
    DMK_ND_DISPATCH(poly.nd, L_RES)
#undef L_RES
}

void launch_residual_direct(const double* tx, const double* ty, const double* tz, int64_t m, const double* sx,
                            const double* sy, const double* sz, const double* sf, int64_t ns, double r_lambda,
                            bool refine, const RadialPoly& poly, double* u, hipStream_t s)
{
    if (m == 0)
        return;
#define L_RES_RF(ND, RF)                                                                                      \
    hipLaunchKernelGGL((k_residual_direct<ND, RF>), dim3(nblocks(m, 64)), dim3(64), 0, s, tx, ty, tz, m, sx, sy, \
                       sz, sf, ns, r_lambda, poly, u)
    // the same rule as launch_near: the unrefined estimate only with the shortest fits
#define L_RES(ND)                    \
    if (ND == 14 && !refine) {       \
        L_RES_RF(14, false);         \
    } else {                         \
        L_RES_RF(ND, true);          \
    }
    DMK_ND_DISPATCH(poly.nd, L_RES)
#undef L_RES
#undef L_RES_RF
}

// ---- finishing --------------------------------------------------------------------
// One block per root: out[3r + j] = coef * sum of root r's proxy charges of component j.
template <typename S>
__global__ __launch_bounds__(256) void k_sum_root(const S* __restrict__ Q, const int* __restrict__ root_fid, int p3,
                                                  double coef, double* __restrict__ out)
{
    __shared__ double sh[256];
    const S* q = Q + (size_t)root_fid[blockIdx.x] * 3 * p3;
    for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int k = threadIdx.x; k < p3; k += 256)
            s += (double)q[(size_t)j * p3 + k];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st)
                sh[threadIdx.x] += sh[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            out[3 * blockIdx.x + j] = coef * sh[0];
        __syncthreads();
    }
}

void launch_sum_root(const void* Q, const int* root_fid, int nroot, int p3, double coef, double* out, bool f32,
                     hipStream_t s)
{
    if (f32)
        hipLaunchKernelGGL(k_sum_root<float>, dim3(nroot), dim3(256), 0, s, (const float*)Q, root_fid, p3, coef, out);
    else
        hipLaunchKernelGGL(k_sum_root<double>, dim3(nroot), dim3(256), 0, s, (const double*)Q, root_fid, p3, coef,
                           out);
}

// Moments of the stresslet densities of each root (one block per root) for
// the k = 0 term of the periodic stresslet sum: out[4r] = sum_s f_s . n_s,
// out[4r + 1 + d] = sum_s x_{s,d} (f_s . n_s), both read off the root's proxy
// densities (their traces), which reproduce the constant and linear moments
// of the point densities exactly (the Lagrange basis reproduces polynomials
// of degree < p).  The root is the unit box centred at the origin (the
// coordinates of the sorted points): node a sits at t_a / 2.  The k = 0 term
// depends on positions only through differences, so the centring is free.
template <typename S>
__global__ __launch_bounds__(256) void k_stress_moment(const S* __restrict__ Q, const int* __restrict__ root_fid,
                                                       int p, const double* __restrict__ cheb_t,
                                                       double* __restrict__ out)
{
    __shared__ double sh[4][256];
    const size_t p3 = (size_t)p * p * p;
    const S* q = Q + (size_t)root_fid[blockIdx.x] * 6 * p3;
    double m[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < (int)p3; k += 256) {
        const int a = k / (p * p), b = (k / p) % p, c = k % p;
        const double tr = (double)q[k] + (double)q[p3 + k] + (double)q[2 * p3 + k];
        m[0] += tr;
        m[1] += 0.5 * cheb_t[a] * tr;
        m[2] += 0.5 * cheb_t[b] * tr;
        m[3] += 0.5 * cheb_t[c] * tr;
    }
    for (int j = 0; j < 4; ++j)
        sh[j][threadIdx.x] = m[j];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int j = 0; j < 4; ++j)
                sh[j][threadIdx.x] += sh[j][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4)
        out[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

void launch_stress_moment(const void* Q, const int* root_fid, int nroot, int p, const double* cheb_t, double* out,
                          bool f32, hipStream_t s)
{
    if (f32)
        hipLaunchKernelGGL(k_stress_moment<float>, dim3(nroot), dim3(256), 0, s, (const float*)Q, root_fid, p,
                           cheb_t, out);
    else
        hipLaunchKernelGGL(k_stress_moment<double>, dim3(nroot), dim3(256), 0, s, (const double*)Q, root_fid, p,
                           cheb_t, out);
}

// vel (caller's order) = scale_b (u + c_b), b the point's problem: scale_b
// undoes that problem's unit-box map, c_b its free-space constant (or none).
// lin (periodic stresslet): adds lin[4b+1+d] - x_d lin[4b] at the sorted
// (centred unit-box) coordinates x: the k = 0 term, in a unit box that is the
// unit cell.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ u, int64_t n, const int* __restrict__ perm,
                                                  int64_t tofs, const int* __restrict__ pid,
                                                  const double* __restrict__ scale, int sq,
                                                  const double* __restrict__ cst, const double* __restrict__ lin,
                                                  const double* __restrict__ x, const double* __restrict__ y,
                                                  const double* __restrict__ z, double* __restrict__ vel)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    // input indices below tofs are sources without a velocity output
    const int64_t o = perm[i] - tofs;
    if (o < 0)
        return;
    const int b = pid ? pid[i] : 0;
    const double sc = sq ? scale[b] * scale[b] : scale[b];
    double c0 = cst ? cst[3 * b] : 0.0, c1 = cst ? cst[3 * b + 1] : 0.0, c2 = cst ? cst[3 * b + 2] : 0.0;
    if (lin) {
        const double m0 = lin[4 * b];
        c0 += lin[4 * b + 1] - x[i] * m0;
        c1 += lin[4 * b + 2] - y[i] * m0;
        c2 += lin[4 * b + 3] - z[i] * m0;
    }
    vel[3 * o] = sc * (u[i] + c0);
    vel[3 * o + 1] = sc * (u[n + i] + c1);
    vel[3 * o + 2] = sc * (u[2 * n + i] + c2);
}

void launch_finalize(const double* u, int64_t n, const int* perm, int64_t tofs, const int* pid, const double* scale,
                     int sq, const double* cst, const double* lin, const double* x, const double* y, const double* z,
                     double* vel, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(nblocks(n, 256)), dim3(256), 0, s, u, n, perm, tofs, pid, scale, sq, cst,
                       lin, x, y, z, vel);
}

__global__ __launch_bounds__(256) void k_zero(uint32_t* __restrict__ p, size_t count)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const size_t count = bytes / 4;
    if (count == 0)
        return;
    const unsigned nb = (unsigned)std::min<size_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, s, (uint32_t*)p, count);
}

// ---- fixed device workspace ---------------------------------------------------------
// Staging of the entry point for callers that cannot allocate
// (dmk_stokes_residual_sum_noalloc): targets, sources and forces as SoA, at
// most kScratchDoubles values.  Every GPU holds its own copy until the process
// ends; calls on one GPU share it.
constexpr size_t kScratchDoubles = (size_t)1 << 21;  // 16 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

size_t scratch_doubles()
{
    return kScratchDoubles;
}

hipError_t scratch_address(double** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // the array's name in host code is only a stand-in for the symbol;
        // its device address on the current GPU comes from the runtime
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace dmk
