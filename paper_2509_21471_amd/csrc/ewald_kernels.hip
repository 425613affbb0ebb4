// Spreading, Fourier-space scaling and interpolation of the single-level
// spectral Ewald variant on the periodic unit cell.
#include "ewald_kernels.hpp"

#include <algorithm>

namespace dmk {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0xFF0000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}

// Morton code of a tile (digit 4 bx + 2 by + bz, as the point keys)
__device__ inline uint32_t tile_code(int tx, int ty, int tz)
{
    return (spread3((uint32_t)tx) << 2) | (spread3((uint32_t)ty) << 1) | spread3((uint32_t)tz);
}

// Blocks go round-robin over the 8 XCDs, each with its own L2; this gives
// every XCD a contiguous Morton range of tiles instead, so the regions and
// neighbour points that adjacent tiles share are read through one L2.
// Padding blocks get -1.
__device__ inline int xcd_tile(int total)
{
    const int per = (total + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    return t < total ? t : -1;
}

// gridding kernel, Clenshaw in v = 2 t^2 - 1 over the zero-padded series
// (fixed length, so the coefficients sit in scalar registers); 0 for |t| >= 1
__device__ inline double gker(const GridPoly& g, double t)
{
    if (!(fabs(t) < 1.0))
        return 0.0;
    const double v = fma(2.0 * t, t, -1.0);
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = kGridTerms - 1; k >= 1; --k) {
        const double b0 = fma(2.0 * v, b1, -b2) + g.a[k];
        b2 = b1;
        b1 = b0;
    }
    return fma(v, b1, -b2) + g.a[0];
}

// grid coordinate of a point of tile coordinate tc, kept inside that tile
// (its Morton key and its coordinate agree up to rounding)
__device__ inline double grid_coord(double x, int M, int B, int tc)
{
    const double t0 = (double)(tc * B);
    const double X = (x + 0.5) * (double)M;
    return fmin(fmax(X, t0), nextafter(t0 + (double)B, 0.0));
}

constexpr int kSpreadChunk = 128;

// One block per tile.  The block walks the points of the 27 neighbouring
// tiles (periodic images included) in chunks: every candidate whose stencil
// overlaps this tile gets its B weights per axis at this tile's grid lines,
// and the survivors are packed, in candidate order, into LDS.  Each thread
// then accumulates its own grid points over the packed candidates, so every
// grid value is summed in a fixed order and written once.
template <int B>
__global__ __launch_bounds__(256) void k_ewald_spread(int M, int Lt, int w, GridPoly g,
                                                      const int64_t* __restrict__ tile_start,
                                                      const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, const double* __restrict__ fs,
                                                      int64_t n, double* __restrict__ grid)
{
    constexpr int B3 = B * B * B;
    constexpr int NO = (B3 + 255) / 256;  // owned grid points per thread
    __shared__ double wt[kSpreadChunk][3][B];
    __shared__ double ff[kSpreadChunk][3];
    __shared__ double xs[kSpreadChunk][3];
    __shared__ int wtot[4];
    __shared__ int64_t nb_start[27], nb_off[28];   // neighbour ranges and their prefix counts
    __shared__ int nb_tile[27][3];
    __shared__ double nb_wrap[27][3];
    const int NT = 1 << Lt;
    const int tile = xcd_tile(1 << (3 * Lt));
    if (tile < 0)
        return;
    const uint32_t code = (uint32_t)tile;
    const int tc[3] = {(int)compact3(code >> 2), (int)compact3(code >> 1), (int)compact3(code)};
    const int T0[3] = {tc[0] * B, tc[1] * B, tc[2] * B};
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double hw = 0.5 * w;
    double acc[NO][3];
#pragma unroll
    for (int s = 0; s < NO; ++s)
        acc[s][0] = acc[s][1] = acc[s][2] = 0.0;
    // the 27 neighbouring tiles (periodic images) as one flat candidate list
    if (tid < 27) {
        const int d[3] = {tid / 9 - 1, (tid / 3) % 3 - 1, tid % 3 - 1};
        int nt[3];
        for (int k = 0; k < 3; ++k) {
            int v = tc[k] + d[k];
            double wr = 0.0;
            if (v < 0) {
                v += NT;
                wr = -(double)M;
            } else if (v >= NT) {
                v -= NT;
                wr = (double)M;
            }
            nt[k] = v;
            nb_tile[tid][k] = v;
            nb_wrap[tid][k] = wr;
        }
        const uint32_t ncode = tile_code(nt[0], nt[1], nt[2]);
        nb_start[tid] = tile_start[ncode];
        nb_off[tid] = tile_start[ncode + 1] - tile_start[ncode];
    }
    __syncthreads();
    if (tid == 0) {
        int64_t acc0 = 0;
        for (int v = 0; v < 27; ++v) {
            const int64_t c = nb_off[v];
            nb_off[v] = acc0;
            acc0 += c;
        }
        nb_off[27] = acc0;
    }
    __syncthreads();
    const int64_t total = nb_off[27];
    {
        for (int64_t c0 = 0; c0 < total; c0 += kSpreadChunk) {
            const int64_t q = c0 + tid;
            bool keep = false;
            double X[3] = {0.0, 0.0, 0.0};
            int64_t i = 0;
            if (tid < kSpreadChunk && q < total) {
                int v = 0;
                while (nb_off[v + 1] <= q)
                    ++v;
                i = nb_start[v] + (q - nb_off[v]);
                const double pc[3] = {x[i], y[i], z[i]};
                keep = true;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    X[k] = grid_coord(pc[k], M, B, nb_tile[v][k]) + nb_wrap[v][k];
                    const int n0 = (int)ceil(X[k] - hw);
                    keep = keep && n0 <= T0[k] + B - 1 && n0 + w - 1 >= T0[k];
                }
            }
            const unsigned long long mask = __ballot(keep);
            const int pos = __popcll(mask & ((1ull << lane) - 1ull));
            __syncthreads();  // the previous chunk's accumulation is done with wt / ff
            if (lane == 0)
                wtot[wave] = __popcll(mask);
            __syncthreads();
            int base = 0;
            for (int v = 0; v < wave; ++v)
                base += wtot[v];
            const int kept = wtot[0] + wtot[1] + wtot[2] + wtot[3];
            if (keep) {
                const int slot = base + pos;
                xs[slot][0] = X[0];
                xs[slot][1] = X[1];
                xs[slot][2] = X[2];
                ff[slot][0] = fs[i];
                ff[slot][1] = fs[n + i];
                ff[slot][2] = fs[2 * n + i];
            }
            __syncthreads();
            // the weights of the kept candidates at this tile's grid lines, one per thread
            for (int it = tid; it < kept * 3 * B; it += 256) {
                const int slot = it / (3 * B), k = (it / B) % 3, j = it % B;
                wt[slot][k][j] = gker(g, (xs[slot][k] - (double)(T0[k] + j)) / hw);
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < NO; ++s) {
                const int gp = tid + 256 * s;
                if (gp < B3) {
                    const int ix = gp / (B * B), iy = (gp / B) % B, iz = gp % B;
#pragma unroll 4
                    for (int c = 0; c < kept; ++c) {
                        const double wv = wt[c][0][ix] * wt[c][1][iy] * wt[c][2][iz];
                        acc[s][0] = fma(wv, ff[c][0], acc[s][0]);
                        acc[s][1] = fma(wv, ff[c][1], acc[s][1]);
                        acc[s][2] = fma(wv, ff[c][2], acc[s][2]);
                    }
                }
            }
        }
    }
    const size_t M3 = (size_t)M * M * M;
#pragma unroll
    for (int s = 0; s < NO; ++s) {
        const int gp = tid + 256 * s;
        if (gp < B3) {
            const int ix = gp / (B * B), iy = (gp / B) % B, iz = gp % B;
            const size_t o = ((size_t)(T0[0] + ix) * M + (T0[1] + iy)) * M + (T0[2] + iz);
            grid[o] = acc[s][0];
            grid[M3 + o] = acc[s][1];
            grid[2 * M3 + o] = acc[s][2];
        }
    }
}

__global__ __launch_bounds__(256) void k_ewald_scale(int M, int K, const double* __restrict__ ghat,
                                                     const double* __restrict__ wsym, double2* __restrict__ spec)
{
    const int Mh = M / 2 + 1;
    const int64_t H = (int64_t)M * M * Mh;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= H)
        return;
    const int k3 = (int)(e % Mh);
    const int64_t r = e / Mh;
    const int j = (int)(r % M), i = (int)(r / M);
    const int k1 = i <= M / 2 ? i : i - M;
    const int k2 = j <= M / 2 ? j : j - M;
    const int a1 = abs(k1), a2 = abs(k2);
    const int m2 = k1 * k1 + k2 * k2 + k3 * k3;
    if (a1 > K || a2 > K || k3 > K || m2 == 0) {
        spec[e] = make_double2(0.0, 0.0);
        spec[H + e] = make_double2(0.0, 0.0);
        spec[2 * H + e] = make_double2(0.0, 0.0);
        return;
    }
    const double gg = ghat[a1] * ghat[a2] * ghat[k3];
    const double wv = wsym[m2] / (gg * gg);
    const double2 F0 = spec[e], F1 = spec[H + e], F2 = spec[2 * H + e];
    const double inv = 1.0 / (double)m2;
    const double dr = (k1 * F0.x + k2 * F1.x + k3 * F2.x) * inv;
    const double di = (k1 * F0.y + k2 * F1.y + k3 * F2.y) * inv;
    spec[e] = make_double2(wv * (F0.x - k1 * dr), wv * (F0.y - k1 * di));
    spec[H + e] = make_double2(wv * (F1.x - k2 * dr), wv * (F1.y - k2 * di));
    spec[2 * H + e] = make_double2(wv * (F2.x - k3 * dr), wv * (F2.y - k3 * di));
}

constexpr int kInterpChunk = 64;
constexpr int kMaxW = 12;

// One block per tile, its points in chunks: one thread per (point, axis,
// offset) forms the stencil weights; then, one component at a time, the
// tile's grid region [O, O + B + w)^3 (O = T0 - w/2, periodic) is staged in
// LDS and one wave per point has each lane sum the z-lines of its (x, y)
// stencil columns, the wave adding the lanes by shuffles in a fixed order.
// (One component at a time keeps the block at about 63 KB of LDS, two
// blocks per CU, so region loads of one block overlap the other's work.)
template <int W>
__global__ __launch_bounds__(256) void k_ewald_interp(int M, int B, int Lt, GridPoly g,
                                                      const int64_t* __restrict__ tile_start,
                                                      const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, int64_t n,
                                                      const double* __restrict__ grid, double* __restrict__ u)
{
    constexpr int w = W;
    extern __shared__ double smem[];
    const int R = B + w;
    const int R3 = R * R * R;
    double* reg = smem;                                   // [R][R][R], one component
    double* wts = reg + R3;                               // [CH][3][kMaxW]
    int* a0s = (int*)(wts + kInterpChunk * 3 * kMaxW);    // [CH][3]
    const int tile = xcd_tile(1 << (3 * Lt));
    if (tile < 0)
        return;
    const uint32_t code = (uint32_t)tile;
    const int tc[3] = {(int)compact3(code >> 2), (int)compact3(code >> 1), (int)compact3(code)};
    const int hwi = w / 2;
    const int O[3] = {tc[0] * B - hwi, tc[1] * B - hwi, tc[2] * B - hwi};
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t M3 = (size_t)M * M * M;
    const int64_t ps = tile_start[code], pe = tile_start[code + 1];
    const double hw = 0.5 * w;
    for (int64_t c0 = ps; c0 < pe; c0 += kInterpChunk) {
        const int cnt = (int)min((int64_t)kInterpChunk, pe - c0);
        __syncthreads();  // previous chunk finished with wts / a0s / reg
        // one thread per (point, axis, stencil offset)
        for (int it = tid; it < cnt * 3 * kMaxW; it += 256) {
            const int p = it / (3 * kMaxW), k = (it / kMaxW) % 3, sofs = it % kMaxW;
            const int64_t i = c0 + p;
            const double pc = k == 0 ? x[i] : (k == 1 ? y[i] : z[i]);
            const double X = grid_coord(pc, M, B, tc[k]);
            const int n0 = (int)ceil(X - hw);
            if (sofs == 0)
                a0s[p * 3 + k] = n0 - O[k];
            wts[(p * 3 + k) * kMaxW + sofs] = sofs < w ? gker(g, (X - (double)(n0 + sofs)) / hw) : 0.0;
        }
        for (int c = 0; c < 3; ++c) {
            __syncthreads();  // weights ready / previous component consumed
            const double* gc = grid + c * M3;
#pragma unroll 8
            for (int e = tid; e < R3; e += 256) {
                const int a = e / (R * R), b = (e / R) % R, cz = e % R;
                const int gx = ((O[0] + a) % M + M) % M;
                const int gy = ((O[1] + b) % M + M) % M;
                const int gz = ((O[2] + cz) % M + M) % M;
                reg[e] = gc[((size_t)gx * M + gy) * M + gz];
            }
            __syncthreads();
            for (int p = wave; p < cnt; p += 4) {
                const int ax0 = a0s[p * 3], ay0 = a0s[p * 3 + 1], az0 = a0s[p * 3 + 2];
                const double* wx = wts + (p * 3) * kMaxW;
                const double* wy = wts + (p * 3 + 1) * kMaxW;
                const double* wz = wts + (p * 3 + 2) * kMaxW;
                double s0 = 0.0;
#pragma unroll
                for (int pr0 = 0; pr0 < w * w; pr0 += 64) {
                    const int pr = pr0 + lane;
                    if (pr < w * w) {
                        const int sx = pr / w, sy = pr - sx * w;
                        const int rb = ((ax0 + sx) * R + ay0 + sy) * R + az0;
                        double t0 = 0.0;
#pragma unroll
                        for (int sz = 0; sz < w; ++sz)
                            t0 = fma(wz[sz], reg[rb + sz], t0);
                        s0 = fma(wx[sx] * wy[sy], t0, s0);
                    }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1)
                    s0 += __shfl_xor(s0, off);
                if (lane == 0)
                    u[c * n + c0 + p] = s0;
            }
        }
    }
}

}  // namespace

void launch_ewald_spread(int M, int B, int Lt, int w, const GridPoly& g, const int64_t* tile_start, const double* x,
                         const double* y, const double* z, const double* fs, int64_t n, double* grid, hipStream_t s)
{
    const unsigned ntile = (((1u << (3 * Lt)) + 7u) / 8u) * 8u;
    if (B == 6)
        hipLaunchKernelGGL(k_ewald_spread<6>, dim3(ntile), dim3(256), 0, s, M, Lt, w, g, tile_start, x, y, z, fs, n,
                           grid);
    else
        hipLaunchKernelGGL(k_ewald_spread<8>, dim3(ntile), dim3(256), 0, s, M, Lt, w, g, tile_start, x, y, z, fs, n,
                           grid);
}

void launch_ewald_scale(int M, int K, const double* ghat, const double* wsym, double2* spec, hipStream_t s)
{
    const int64_t H = (int64_t)M * M * (M / 2 + 1);
    hipLaunchKernelGGL(k_ewald_scale, dim3(nblk(H, 256)), dim3(256), 0, s, M, K, ghat, wsym, spec);
}

void launch_ewald_interp(int M, int B, int Lt, int w, const GridPoly& g, const int64_t* tile_start,
                         const double* x, const double* y, const double* z, int64_t n, const double* grid,
                         double* u, hipStream_t s)
{
    const int R = B + w;
    const size_t shm = (size_t)R * R * R * sizeof(double) + (size_t)kInterpChunk * 3 * kMaxW * sizeof(double) +
                       (size_t)kInterpChunk * 3 * sizeof(int);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_ewald_interp<6>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipFuncSetAttribute((const void*)k_ewald_interp<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipFuncSetAttribute((const void*)k_ewald_interp<11>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    const unsigned ntile = (((1u << (3 * Lt)) + 7u) / 8u) * 8u;
#define L_INTERP(W)                                                                                              \
    hipLaunchKernelGGL(k_ewald_interp<W>, dim3(ntile), dim3(256), shm, s, M, B, Lt, g, tile_start, x, y, z, n, \
                       grid, u)
    // the widths the grid parameters produce (6, 8, 11 at 1e-3, 1e-6, 1e-9)
    if (w == 6)
        L_INTERP(6);
    else if (w == 8)
        L_INTERP(8);
    else if (w == 11)
        L_INTERP(11);
#undef L_INTERP
}

}  // namespace dmk
