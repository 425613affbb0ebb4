// Device kernels of the DMK Stokeslet path (gfx950, double precision).
#include "dmk_kernels.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>

namespace dmk {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kInv8Pi = 1.0 / (8.0 * kPi);

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
}  // namespace

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

__device__ inline uint64_t spread3(uint64_t v)
{
    // bit b of v -> bit 3b
    uint64_t r = 0;
    for (int b = 0; b < 19; ++b)
        r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

__global__ __launch_bounds__(256) void k_morton(const double* __restrict__ pts, int64_t n, double cx, double cy,
                                                double cz, double inv_len, uint64_t* __restrict__ keys,
                                                int* __restrict__ idx)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double c[3] = {cx, cy, cz};
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

void launch_morton(const double* pts, int64_t n, double cx, double cy, double cz, double inv_len, uint64_t* keys,
                   int* idx, hipStream_t s)
{
    hipLaunchKernelGGL(k_morton, dim3(nblocks(n, 256)), dim3(256), 0, s, pts, n, cx, cy, cz, inv_len, keys, idx);
}

__global__ __launch_bounds__(256) void k_gather_points(const double* __restrict__ pts, int64_t n,
                                                       const int* __restrict__ perm, double cx, double cy,
                                                       double cz, double inv_len, double* __restrict__ x,
                                                       double* __restrict__ y, double* __restrict__ z)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t o = perm[i];
    x[i] = (pts[3 * o] - cx) * inv_len;
    y[i] = (pts[3 * o + 1] - cy) * inv_len;
    z[i] = (pts[3 * o + 2] - cz) * inv_len;
}

void launch_gather_points(const double* pts, int64_t n, const int* perm, double cx, double cy, double cz,
                          double inv_len, double* x, double* y, double* z, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_points, dim3(nblocks(n, 256)), dim3(256), 0, s, pts, n, perm, cx, cy, cz, inv_len,
                       x, y, z);
}

size_t sort_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                       (const int*)nullptr, (int*)nullptr, (int)n, 0, 57);
    return bytes;
}

void launch_sort(void* temp, size_t temp_bytes, const uint64_t* kin, uint64_t* kout, const int* vin, int* vout,
                 int64_t n, int end_bit, hipStream_t s)
{
    (void)hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, kin, kout, vin, vout, (int)n, 0, end_bit, s);
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
__global__ __launch_bounds__(256) void k_gather_forces(const double* __restrict__ f, int64_t n,
                                                       const int* __restrict__ perm, double* __restrict__ fs)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t o = perm[i];
    fs[i] = f[3 * o];
    fs[n + i] = f[3 * o + 1];
    fs[2 * n + i] = f[3 * o + 2];
}

void launch_gather_forces(const double* f, int64_t n, const int* perm, double* fs, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_forces, dim3(nblocks(n, 256)), dim3(256), 0, s, f, n, perm, fs);
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

// Proxy charges of one leaf per block; each thread owns output rows (b, c).
template <int P>
__global__ __launch_bounds__(256) void k_anterp(const LeafDesc* __restrict__ leaves, const double* __restrict__ x,
                                                const double* __restrict__ y, const double* __restrict__ z,
                                                const double* __restrict__ fs, int64_t n,
                                                const double* __restrict__ ct, const double* __restrict__ cw,
                                                double* __restrict__ Q)
{
    constexpr int CH = P > 36 ? 32 : 64;
    __shared__ double sL[3][CH][P];
    __shared__ double sf[CH][3];
    const LeafDesc L = leaves[blockIdx.x];
    const double sc = (double)(2ll << L.level);  // 1 / (half box length)
    const double cen[3] = {L.cx, L.cy, L.cz};
    const double* crd[3] = {x, y, z};
    const int tid = threadIdx.x;
    constexpr int NPAIR = P * P;
    for (int round = 0; round * 256 < NPAIR; ++round) {
        const int pair = round * 256 + tid;
        const bool valid = pair < NPAIR;
        const int b = valid ? pair / P : 0;
        const int c = valid ? pair % P : 0;
        double acc[P][3];
#pragma unroll
        for (int a = 0; a < P; ++a)
            acc[a][0] = acc[a][1] = acc[a][2] = 0.0;
        for (int64_t cs = L.start; cs < L.end; cs += CH) {
            __syncthreads();
            for (int task = tid; task < 3 * CH; task += 256) {
                const int pt = task % CH, d = task / CH;
                const int64_t i = cs + pt;
                double Lv[P];
                if (i < L.end) {
                    lagrange<P>((crd[d][i] - cen[d]) * sc, ct, cw, Lv);
                } else {
#pragma unroll
                    for (int a = 0; a < P; ++a)
                        Lv[a] = 0.0;
                }
#pragma unroll
                for (int a = 0; a < P; ++a)
                    sL[d][pt][a] = Lv[a];
                sf[pt][d] = i < L.end ? fs[d * n + i] : 0.0;
            }
            __syncthreads();
            if (valid) {
                for (int pt = 0; pt < CH; ++pt) {
                    const double wbc = sL[1][pt][b] * sL[2][pt][c];
                    const double w0 = wbc * sf[pt][0], w1 = wbc * sf[pt][1], w2 = wbc * sf[pt][2];
#pragma unroll
                    for (int a = 0; a < P; ++a) {
                        const double la = sL[0][pt][a];
                        acc[a][0] = fma(la, w0, acc[a][0]);
                        acc[a][1] = fma(la, w1, acc[a][1]);
                        acc[a][2] = fma(la, w2, acc[a][2]);
                    }
                }
            }
        }
        if (valid) {
            double* q = Q + (size_t)L.fid * 3 * P * P * P;
#pragma unroll
            for (int a = 0; a < P; ++a)
                for (int j = 0; j < 3; ++j)
                    q[((size_t)j * P + a) * P * P + b * P + c] = acc[a][j];
        }
    }
}

// Far-field potential at the points of one leaf per block.
template <int P>
__global__ __launch_bounds__(128) void k_leaf_eval(const LeafDesc* __restrict__ leaves, const double* __restrict__ x,
                                                   const double* __restrict__ y, const double* __restrict__ z,
                                                   int64_t n, const double* __restrict__ ct,
                                                   const double* __restrict__ cw, const double* __restrict__ V,
                                                   double* __restrict__ u)
{
    __shared__ double sLy[128][P];
    const LeafDesc L = leaves[blockIdx.x];
    const double sc = (double)(2ll << L.level);
    const double* v = V + (size_t)L.fid * 3 * P * P * P;
    const int tid = threadIdx.x;
    for (int64_t ts = L.start; ts < L.end; ts += 128) {
        const int64_t i = ts + tid;
        const bool valid = i < L.end;
        // V is stored z-major (V[c][b][a]); the outer sum runs over z
        const double xi = valid ? (z[i] - L.cz) * sc : 0.0;
        const double eta = valid ? (y[i] - L.cy) * sc : 0.0;
        const double zeta = valid ? (x[i] - L.cx) * sc : 0.0;
        double Lx[P], Lz[P], Ly[P];
        lagrange<P>(xi, ct, cw, Lx);
        lagrange<P>(eta, ct, cw, Ly);
        lagrange<P>(zeta, ct, cw, Lz);
#pragma unroll
        for (int b = 0; b < P; ++b)
            sLy[tid][b] = Ly[b];
        // Lx to LDS as well (reuse the row after y is consumed per a)
        double u0 = 0, u1 = 0, u2 = 0;
        for (int a = 0; a < P; ++a) {
            double la = 0;
#pragma unroll
            for (int aa = 0; aa < P; ++aa)
                la = (aa == a) ? Lx[aa] : la;
            double t0 = 0, t1 = 0, t2 = 0;
            for (int b = 0; b < P; ++b) {
                const double* v0 = v + ((size_t)a * P + b) * P;
                double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    s0 = fma(v0[c], Lz[c], s0);
                    s1 = fma(v0[(size_t)P * P * P + c], Lz[c], s1);
                    s2 = fma(v0[(size_t)2 * P * P * P + c], Lz[c], s2);
                }
                const double lb = sLy[tid][b];
                t0 = fma(lb, s0, t0);
                t1 = fma(lb, s1, t1);
                t2 = fma(lb, s2, t2);
            }
            u0 = fma(la, t0, u0);
            u1 = fma(la, t1, u1);
            u2 = fma(la, t2, u2);
        }
        if (valid) {
            u[i] = u0;
            u[n + i] = u1;
            u[2 * n + i] = u2;
        }
    }
}

#define DMK_P_DISPATCH(p, MACRO) \
    switch (p) {                 \
    case 12: MACRO(12); break;   \
    case 23: MACRO(23); break;   \
    case 33: MACRO(33); break;   \
    case 44: MACRO(44); break;   \
    default: break;              \
    }

bool p_supported(int p) { return p == 12 || p == 23 || p == 33 || p == 44; }

void launch_anterp(int p, const LeafDesc* leaves, int nleaf, const double* x, const double* y, const double* z,
                   const double* fs, int64_t n, const double* cheb_t, const double* cheb_w, double* Q,
                   hipStream_t s)
{
    if (nleaf == 0)
        return;
#define L_ANTERP(P) \
    hipLaunchKernelGGL(k_anterp<P>, dim3(nleaf), dim3(256), 0, s, leaves, x, y, z, fs, n, cheb_t, cheb_w, Q)
    DMK_P_DISPATCH(p, L_ANTERP)
#undef L_ANTERP
}

void launch_leaf_eval(int p, const LeafDesc* leaves, int nleaf, const double* x, const double* y, const double* z,
                      int64_t n, const double* cheb_t, const double* cheb_w, const double* V, double* u,
                      hipStream_t s)
{
    if (nleaf == 0)
        return;
#define L_EVAL(P) hipLaunchKernelGGL(k_leaf_eval<P>, dim3(nleaf), dim3(128), 0, s, leaves, x, y, z, n, cheb_t, cheb_w, V, u)
    DMK_P_DISPATCH(p, L_EVAL)
#undef L_EVAL
}

// ---- separable tensor stages ---------------------------------------------------
template <int MODE>
struct StageTraits {
    static constexpr bool xc = (MODE == ST_OUT_FULL || MODE == ST_IN_FULL || MODE == ST_IN_HALF_REAL);
    static constexpr bool yc = (MODE == ST_OUT_HALF || MODE == ST_OUT_FULL || MODE == ST_IN_FULL);
    static constexpr bool fold = (MODE != ST_IN_HALF_REAL);
};

// 256 threads per 64-row tile: the input slab X[0..Nin)[r0..r0+64) is staged
// in LDS with all loads in flight, thread (row, g) accumulates the half
// outputs g, g+4, ... from it, and the output tile Y[r0..r0+64)[0..Nout) is
// staged in LDS again and written as one contiguous block (or scatter-added to
// the children's grids, one contiguous run of p per row and child).
template <int MODE, int IO, int NI>
__global__ __launch_bounds__(256) void k_stage(StageArgs a)
{
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
    const int slot = blockIdx.y / 3, comp = blockIdx.y % 3;
    const int R = a.R, Nin = a.Nin, Nout = a.Nout, p = a.p;
    const int r0 = blockIdx.x * 64;
    const int nrow = min(64, R - r0);
    const size_t p3 = (size_t)p * p * p;
    // ---- input slab ----
    {
        const size_t xoff = ((size_t)(a.xmap ? a.xmap[slot] : slot) * 3 + comp) * a.xstride;
        for (int e = tid; e < Nin * 64; e += 256) {
            const int k = e >> 6, rr = e & 63;
            const int r = r0 + rr;
            double v0 = 0.0, v1 = 0.0;
            if (rr < nrow) {
                if (IO == IO_GATHER8) {
                    const int B = r / (2 * p), C = r % (2 * p);
                    const int f = a.child_fid[slot * 8 + 4 * (k / p) + 2 * (B / p) + (C / p)];
                    if (f >= 0)
                        v0 = ((const double*)a.X)[((size_t)f * 3 + comp) * p3 + ((size_t)(k % p) * p + (B % p)) * p +
                                                  (C % p)];
                } else if (XE == 2) {
                    const double2 v = ((const double2*)a.X)[xoff + (size_t)k * R + r];
                    v0 = v.x;
                    v1 = v.y;
                } else {
                    v0 = ((const double*)a.X)[xoff + (size_t)k * R + r];
                }
            }
            if (XE == 2)
                ((double2*)tile)[e] = make_double2(v0, v1);
            else
                tile[e] = v0;
        }
    }
    __syncthreads();
    const int lane = tid & 63, g = tid >> 6;
    double Ur[NI], Ui[NI], Wr[NI], Wi[NI];
#pragma unroll
    for (int t = 0; t < NI; ++t)
        Ur[t] = Ui[t] = Wr[t] = Wi[t] = 0.0;
    for (int j = 0; j < a.Kh; ++j) {
        const int k1 = j + a.in_off;
        const int k2 = Nin - 1 - k1;
        double x1r, x1i = 0, x2r = 0, x2i = 0;
        if (XE == 2) {
            const double2 v1 = ((const double2*)tile)[k1 * 64 + lane];
            x1r = v1.x;
            x1i = v1.y;
            if (Tr::fold && k2 != k1) {
                const double2 v2 = ((const double2*)tile)[k2 * 64 + lane];
                x2r = v2.x;
                x2i = v2.y;
            }
        } else {
            x1r = tile[k1 * 64 + lane];
            if (k2 != k1)
                x2r = tile[k2 * 64 + lane];
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
            const int i = g + 4 * t;
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
        const int i = g + 4 * t;
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
        double* Yd = (double*)a.Y;
        for (int e = tid; e < nrow * Nout; e += 256) {
            const int rr = e / Nout, A = e % Nout;
            const int r = r0 + rr;
            const int C = r / (2 * p), B = r % (2 * p);
            const int f = a.child_fid[slot * 8 + 4 * (A / p) + 2 * (B / p) + (C / p)];
            if (f >= 0)
                Yd[((size_t)f * 3 + comp) * p3 + ((size_t)(C % p) * p + (B % p)) * p + (A % p)] += tile[e];
        }
    } else {
        const size_t yoff = ((size_t)(a.ymap ? a.ymap[slot] : slot) * 3 + comp) * a.ystride * YE +
                            (size_t)r0 * Nout * YE;
        double* Yd = (double*)a.Y + yoff;
        const int cnt = nrow * Nout * YE;
        if (a.accumulate) {
            for (int e = tid; e < cnt; e += 256)
                Yd[e] += tile[e];
        } else {
            for (int e = tid; e < cnt; e += 256)
                Yd[e] = tile[e];
        }
    }
}

template <int MODE, int IO, int NI>
static void stage_launch(dim3 grid, size_t shm, const StageArgs& a, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_stage<MODE, IO, NI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((k_stage<MODE, IO, NI>), grid, dim3(256), shm, s, a);
}

template <int MODE, int IO>
static void stage_ni(const StageArgs& a, hipStream_t s)
{
    using Tr = StageTraits<MODE>;
    dim3 grid(nblocks(a.R, 64), a.nslots * 3);
    const size_t tile = std::max((size_t)a.Nin * 64 * (Tr::xc ? 2 : 1), (size_t)a.Nout * 64 * (Tr::yc ? 2 : 1));
    const size_t shm = (size_t)a.Nh * a.Kh * sizeof(double2) + tile * sizeof(double);
    const int ni = (a.Nh + 3) / 4;
    if (ni <= 4)
        stage_launch<MODE, IO, 4>(grid, shm, a, s);
    else if (ni <= 8)
        stage_launch<MODE, IO, 8>(grid, shm, a, s);
    else
        stage_launch<MODE, IO, 12>(grid, shm, a, s);
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
__global__ __launch_bounds__(256) void k_translate(int q, int n1, const RecvDesc* __restrict__ recv,
                                                   const int* __restrict__ e_src, const int8_t* __restrict__ e_off,
                                                   const cplx* __restrict__ Phi, const double* __restrict__ wdiff,
                                                   cplx* __restrict__ Psi)
{
    const int H = q * n1 * n1;
    const int mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= H)
        return;
    const RecvDesc rd = recv[blockIdx.y];
    const int m1 = mi / (n1 * n1);
    const int rem = mi - m1 * n1 * n1;
    const int m2 = rem / n1 - (q - 1);
    const int m3 = rem % n1 - (q - 1);
    const double s3 = 0.86602540378443864676;
    double F[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int e = rd.ebeg; e < rd.eend; ++e) {
        const int src = e_src[e];
        const int t = m1 * e_off[3 * e] + m2 * e_off[3 * e + 1] + m3 * e_off[3 * e + 2];
        const int tm = ((t % 3) + 3) % 3;
        // exp(-i 2 pi t / 3)
        const double pr = tm == 0 ? 1.0 : -0.5;
        const double pi = tm == 0 ? 0.0 : (tm == 1 ? -s3 : s3);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const cplx v = Phi[((size_t)src * 3 + j) * H + mi];
            F[j][0] += pr * v.re - pi * v.im;
            F[j][1] += pr * v.im + pi * v.re;
        }
    }
    const int mm = m1 * m1 + m2 * m2 + m3 * m3;
    double w = 0;
    if (mm > 0)
        w = wdiff[mm] * (double)(1ll << rd.level);
    const double inv = mm > 0 ? 1.0 / mm : 0.0;
    const double dr = (m1 * F[0][0] + m2 * F[1][0] + m3 * F[2][0]) * inv;
    const double di = (m1 * F[0][1] + m2 * F[1][1] + m3 * F[2][1]) * inv;
    const int mv[3] = {m1, m2, m3};
    // incoming side is stored z-major: Psi[mz][my][mx]
    const size_t mo = ((size_t)(m3 + q - 1) * n1 + (m2 + q - 1)) * q + m1;
#pragma unroll
    for (int j = 0; j < 3; ++j)
        Psi[((size_t)rd.slot * 3 + j) * H + mo] = cplx{w * (F[j][0] - mv[j] * dr), w * (F[j][1] - mv[j] * di)};
}

void launch_translate(int q, int n1, const RecvDesc* recv, int nrecv, const int* e_src, const int8_t* e_off,
                      const cplx* Phi, const double* wdiff, cplx* Psi, hipStream_t s)
{
    if (nrecv == 0)
        return;
    const int H = q * n1 * n1;
    hipLaunchKernelGGL(k_translate, dim3(nblocks(H, 256), nrecv), dim3(256), 0, s, q, n1, recv, e_src, e_off, Phi,
                       wdiff, Psi);
}

__global__ __launch_bounds__(256) void k_root_symbol(int mh, int mf, const cplx* __restrict__ Phi,
                                                     const double* __restrict__ w, cplx* __restrict__ Psi)
{
    const int H = mh * mf * mf;
    const int mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= H)
        return;
    const int M = (mf - 1) / 2;
    const int m1 = mi / (mf * mf);
    const int rem = mi - m1 * mf * mf;
    const int m2 = rem / mf - M, m3 = rem % mf - M;
    const int mm = m1 * m1 + m2 * m2 + m3 * m3;
    cplx F[3];
    for (int j = 0; j < 3; ++j)
        F[j] = Phi[(size_t)j * H + mi];
    const double ww = mm > 0 ? w[mm] : 0.0;
    const double inv = mm > 0 ? 1.0 / mm : 0.0;
    const double dr = (m1 * F[0].re + m2 * F[1].re + m3 * F[2].re) * inv;
    const double di = (m1 * F[0].im + m2 * F[1].im + m3 * F[2].im) * inv;
    const int mv[3] = {m1, m2, m3};
    const size_t mo = ((size_t)(m3 + M) * mf + (m2 + M)) * mh + m1;
    for (int j = 0; j < 3; ++j)
        Psi[(size_t)j * H + mo] = cplx{ww * (F[j].re - mv[j] * dr), ww * (F[j].im - mv[j] * di)};
}

void launch_root_symbol(int mh, int mf, const cplx* Phi, const double* w, cplx* Psi, hipStream_t s)
{
    const int H = mh * mf * mf;
    hipLaunchKernelGGL(k_root_symbol, dim3(nblocks(H, 256)), dim3(256), 0, s, mh, mf, Phi, w, Psi);
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

template <int ND>
__device__ inline void residual_pair(double dx, double dy, double dz, double fx, double fy, double fz, double rl2,
                                     double tw, double cP, double cQ, const RadialPoly& poly, double& u0,
                                     double& u1, double& u2)
{
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (r2 < rl2 && r2 > 0.0) {
        const double rinv = rsqrt_f64(r2);
        const double t = fma(r2, tw, -1.0);
        const double P = horner<ND>(poly.P, t);
        const double Q = horner<ND>(poly.Q, t);
        const double dot = fma(dx, fx, fma(dy, fy, dz * fz));
        const double cr = kInv8Pi * rinv;
        const double a = fma(-cP, P, cr);
        const double b = dot * fma(-cQ, Q, cr * rinv * rinv);
        u0 = fma(a, fx, fma(b, dx, u0));
        u1 = fma(a, fy, fma(b, dy, u1));
        u2 = fma(a, fz, fma(b, dz, u2));
    }
}

// One wave per 64 targets of a leaf.  Each non-pruned 64-point source chunk of
// every near-list entry is staged in LDS (periodic shift applied) and read
// back by broadcast.
template <int ND>
__global__ __launch_bounds__(64) void k_near(const NearWork* __restrict__ work, const NearLeaf* __restrict__ leaves,
                                             const NearEntryDev* __restrict__ entries, const double* __restrict__ cbbox,
                                             const double* __restrict__ x, const double* __restrict__ y,
                                             const double* __restrict__ z, const double* __restrict__ fs, int64_t n,
                                             RadialPoly poly, double self_coef, double* __restrict__ u)
{
    __shared__ double2 S[64][3];
    const NearWork w = work[blockIdx.x];
    const NearLeaf T = leaves[w.leaf];
    const int lane = threadIdx.x;
    const int64_t i = T.tstart + (int64_t)w.chunk * 64 + lane;
    const bool valid = i < T.tend;
    const double xt = valid ? x[i] : 0.0, yt = valid ? y[i] : 0.0, zt = valid ? z[i] : 0.0;
    const double* tb = cbbox + 6 * (size_t)(T.cbase + w.chunk);
    const double tlo[3] = {tb[0], tb[1], tb[2]}, thi[3] = {tb[3], tb[4], tb[5]};
    double u0 = 0, u1 = 0, u2 = 0;
    for (int e = T.ebeg; e < T.eend; ++e) {
        const NearEntryDev E = entries[e];
        const double rl = 1.0 / (double)(1ll << E.lambda);
        const double rl2 = rl * rl, inv_rl2 = 1.0 / rl2;
        const double cP = 1.0 / (4.0 * kPi * rl), cQ = cP * inv_rl2;
        const double tw = 2.0 * inv_rl2;
        const double sh[3] = {(double)E.sx, (double)E.sy, (double)E.sz};
        const int nch = (int)((E.send - E.sstart + 63) / 64);
        for (int k = 0; k < nch; ++k) {
            const double* sb = cbbox + 6 * (size_t)(E.cbase + k);
            double gap2 = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double g = fmax(0.0, fmax(sb[d] + sh[d] - thi[d], tlo[d] - (sb[3 + d] + sh[d])));
                gap2 += g * g;
            }
            if (gap2 >= rl2)
                continue;
            const int64_t s0 = E.sstart + 64 * (int64_t)k;
            const int cnt = (int)min((int64_t)64, E.send - s0);
            __syncthreads();
            if (lane < cnt) {
                const int64_t j = s0 + lane;
                S[lane][0] = make_double2(x[j] + sh[0], y[j] + sh[1]);
                S[lane][1] = make_double2(z[j] + sh[2], fs[j]);
                S[lane][2] = make_double2(fs[n + j], fs[2 * n + j]);
            }
            __syncthreads();
            for (int jj = 0; jj < cnt; ++jj) {
                const double2 a = S[jj][0], b = S[jj][1], c = S[jj][2];
                residual_pair<ND>(xt - a.x, yt - a.y, zt - b.x, b.y, c.x, c.y, rl2, tw, cP, cQ, poly, u0, u1, u2);
            }
        }
    }
    if (valid) {
        const double sc = self_coef * (double)(1ll << T.level);
        u[i] += u0 + sc * fs[i];
        u[n + i] += u1 + sc * fs[n + i];
        u[2 * n + i] += u2 + sc * fs[2 * n + i];
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

void launch_near(const NearWork* work, int nwork, const NearLeaf* leaves, const NearEntryDev* entries,
                 const double* cbbox, const double* x, const double* y, const double* z, const double* fs, int64_t n,
                 const RadialPoly& poly, double self_coef, double* u, hipStream_t s)
{
    if (nwork == 0)
        return;
#define L_NEAR(ND)                                                                                               \
    hipLaunchKernelGGL(k_near<ND>, dim3(nwork), dim3(64), 0, s, work, leaves, entries, cbbox, x, y, z, fs, n, poly, \
                       self_coef, u)
    DMK_ND_DISPATCH(poly.nd, L_NEAR)
#undef L_NEAR
}

__global__ __launch_bounds__(64) void k_near_count(const NearWork* __restrict__ work,
                                                   const NearLeaf* __restrict__ leaves,
                                                   const NearEntryDev* __restrict__ entries,
                                                   const double* __restrict__ cbbox, const double* __restrict__ x,
                                                   const double* __restrict__ y, const double* __restrict__ z,
                                                   unsigned long long* __restrict__ out)
{
    const NearWork w = work[blockIdx.x];
    const NearLeaf T = leaves[w.leaf];
    const int64_t i = T.tstart + (int64_t)w.chunk * 64 + threadIdx.x;
    const bool valid = i < T.tend;
    const int nt = (int)min((int64_t)64, T.tend - (T.tstart + (int64_t)w.chunk * 64));
    const double xt = valid ? x[i] : 0.0, yt = valid ? y[i] : 0.0, zt = valid ? z[i] : 0.0;
    const double* tb = cbbox + 6 * (size_t)(T.cbase + w.chunk);
    const double tlo[3] = {tb[0], tb[1], tb[2]}, thi[3] = {tb[3], tb[4], tb[5]};
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
            if (threadIdx.x == 0)
                ev += (unsigned long long)(s1 - s0) * nt;
            for (int64_t j = s0; j < s1 && valid; ++j) {
                const double dx = xt - (x[j] + sh[0]), dy = yt - (y[j] + sh[1]), dz = zt - (z[j] + sh[2]);
                const double r2 = dx * dx + dy * dy + dz * dz;
                in += (r2 < rl2 && r2 > 0.0) ? 1ull : 0ull;
            }
        }
    }
    atomicAdd(&out[0], ev);
    atomicAdd(&out[1], in);
}

void launch_near_count(const NearWork* work, int nwork, const NearLeaf* leaves, const NearEntryDev* entries,
                       const double* cbbox, const double* x, const double* y, const double* z,
                       unsigned long long* out, hipStream_t s)
{
    if (nwork == 0)
        return;
    hipLaunchKernelGGL(k_near_count, dim3(nwork), dim3(64), 0, s, work, leaves, entries, cbbox, x, y, z, out);
}

template <int ND>
__global__ __launch_bounds__(64) void k_residual_direct(const double* __restrict__ tx, const double* __restrict__ ty,
                                                        const double* __restrict__ tz, int64_t m,
                                                        const double* __restrict__ sx, const double* __restrict__ sy,
                                                        const double* __restrict__ sz, const double* __restrict__ sf,
                                                        int64_t ns, double rl, RadialPoly poly, double* __restrict__ u)
{
    const int64_t i = blockIdx.x * (int64_t)64 + threadIdx.x;
    const bool valid = i < m;
    const double xt = valid ? tx[i] : 0.0, yt = valid ? ty[i] : 0.0, zt = valid ? tz[i] : 0.0;
    const double rl2 = rl * rl, inv_rl2 = 1.0 / rl2;
    const double cP = 1.0 / (4.0 * kPi * rl), cQ = cP * inv_rl2;
    double u0 = 0, u1 = 0, u2 = 0;
    for (int64_t j = 0; j < ns; ++j)
        residual_pair<ND>(xt - sx[j], yt - sy[j], zt - sz[j], sf[j], sf[ns + j], sf[2 * ns + j], rl2, 2.0 * inv_rl2,
                          cP, cQ, poly, u0, u1, u2);
    if (valid) {
        u[3 * i] = u0;
        u[3 * i + 1] = u1;
        u[3 * i + 2] = u2;
    }
}

void launch_residual_direct(const double* tx, const double* ty, const double* tz, int64_t m, const double* sx,
                            const double* sy, const double* sz, const double* sf, int64_t ns, double r_lambda,
                            const RadialPoly& poly, double* u, hipStream_t s)
{
    if (m == 0)
        return;
#define L_RES(ND)                                                                                               \
    hipLaunchKernelGGL(k_residual_direct<ND>, dim3(nblocks(m, 64)), dim3(64), 0, s, tx, ty, tz, m, sx, sy, sz, sf, \
                       ns, r_lambda, poly, u)
    DMK_ND_DISPATCH(poly.nd, L_RES)
#undef L_RES
}

// ---- finishing --------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sum_root(const double* __restrict__ Q, int p3, double coef,
                                                  double* __restrict__ out)
{
    __shared__ double sh[256];
    for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int k = threadIdx.x; k < p3; k += 256)
            s += Q[(size_t)j * p3 + k];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st)
                sh[threadIdx.x] += sh[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            out[j] = coef * sh[0];
        __syncthreads();
    }
}

void launch_sum_root(const double* Qroot, int p3, double coef, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_root, dim3(1), dim3(256), 0, s, Qroot, p3, coef, out);
}

__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ u, int64_t n, const int* __restrict__ perm,
                                                  double scale, const double* __restrict__ cst,
                                                  double* __restrict__ vel)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t o = perm[i];
    const double c0 = cst ? cst[0] : 0.0, c1 = cst ? cst[1] : 0.0, c2 = cst ? cst[2] : 0.0;
    vel[3 * o] = scale * (u[i] + c0);
    vel[3 * o + 1] = scale * (u[n + i] + c1);
    vel[3 * o + 2] = scale * (u[2 * n + i] + c2);
}

void launch_finalize(const double* u, int64_t n, const int* perm, double scale, const double* cst, double* vel,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(nblocks(n, 256)), dim3(256), 0, s, u, n, perm, scale, cst, vel);
}

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ p, size_t count)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

void launch_zero(double* p, size_t count, hipStream_t s)
{
    if (count == 0)
        return;
    const unsigned nb = (unsigned)std::min<size_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, s, p, count);
}

}  // namespace dmk
