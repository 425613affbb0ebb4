// Step 1 of the DMK procedure on the device: radix sort of the points'
// Morton keys, the adaptive octree (split while a box holds more than n_s
// points), its 2:1 level restriction over vertex adjacency (through the
// periodic wrap when periodic), and the neighbour lists the passes need
// (Sec. "The DMK method", Step 1; level-restricted trees as in Fig. fig:trees).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "dmk_kernels.hpp"
#include "tree.hpp"

namespace dmk {

namespace {

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---- radix sort ------------------------------------------------------------------
// Least-significant-digit radix sort of (64-bit key, 32-bit value) pairs, 8
// bits per pass, stable.  A pass is a per-tile digit histogram, one exclusive
// scan over [digit][tile], and a stable scatter in which a key's rank among
// the equal digits of its wave comes from eight ballots (one per digit bit).
constexpr int kRsThreads = 256;
constexpr int kRsIpt = 16;
constexpr int kRsTile = kRsThreads * kRsIpt;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                       uint32_t* __restrict__ hist, int ntile)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsIpt; ++r) {
        const int64_t i = base + r * kRsThreads + threadIdx.x;
        if (i < n)
            atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of the 256-thread block's values; *total receives the sum
__device__ inline uint32_t block_scan_256(uint32_t v, uint32_t* wsum, uint32_t* total)
{
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (l >= off)
            x += y;
    }
    if (l == 63)
        wsum[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k)
        before += wsum[k];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return before + x - v;
}

// in-place exclusive scan of m counters by one block, in coalesced chunks
__global__ __launch_bounds__(256) void k_scan_u32(uint32_t* __restrict__ a, int64_t m)
{
    __shared__ uint32_t wsum[4];
    uint32_t carry = 0;
    for (int64_t b = 0; b < m; b += 256) {
        const int64_t i = b + threadIdx.x;
        const uint32_t v = i < m ? a[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_scan_256(v, wsum, &tot);
        if (i < m)
            a[i] = carry + ex;
        carry += tot;
    }
}

// the radix histograms [digit][tile]: block d scans digit d's tiles in place
// and writes the digit's total
__global__ __launch_bounds__(256) void k_rs_scan_digit(uint32_t* __restrict__ hist, int ntile,
                                                      uint32_t* __restrict__ dtot)
{
    __shared__ uint32_t wsum[4];
    uint32_t* h = hist + (size_t)blockIdx.x * ntile;
    uint32_t carry = 0;
    for (int b = 0; b < ntile; b += 256) {
        const int i = b + threadIdx.x;
        const uint32_t v = i < ntile ? h[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_scan_256(v, wsum, &tot);
        if (i < ntile)
            h[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0)
        dtot[blockIdx.x] = carry;
}

// digit totals -> digit offsets (exclusive), one block of 256
__global__ __launch_bounds__(256) void k_rs_scan_totals(uint32_t* __restrict__ dtot)
{
    __shared__ uint32_t wsum[4];
    const uint32_t v = dtot[threadIdx.x];
    uint32_t tot;
    const uint32_t ex = block_scan_256(v, wsum, &tot);
    dtot[threadIdx.x] = ex;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                          const int* __restrict__ vin, int64_t n, int shift,
                                                          const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ doff, int ntile,
                                                          uint64_t* __restrict__ kout, int* __restrict__ vout)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    base[t] = doff[t] + hist[(size_t)t * ntile + blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        wcnt[k][t] = 0;
    __syncthreads();
    const uint64_t below = l == 0 ? 0ull : (~0ull >> (64 - l));
    const int64_t tile = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsIpt; ++r) {
        const int64_t i = tile + r * kRsThreads + t;
        const bool ok = i < n;
        const uint64_t key = ok ? kin[i] : 0ull;
        const int val = ok ? vin[i] : 0;
        const int d = (int)((key >> shift) & 255u);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        const int rank = __popcll(peers & below);
        if (ok && rank == 0)
            wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t pos = base[d] + (uint32_t)rank;
            for (int k = 0; k < w; ++k)
                pos += wcnt[k][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            wcnt[k][t] = 0;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_gather_pid_key(const int* __restrict__ v, const int* __restrict__ pid,
                                                       int64_t n, uint64_t* __restrict__ k, int* __restrict__ idx)
{
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < n) {
        k[i] = (uint64_t)pid[v[i]];
        idx[i] = (int)i;
    }
}

__global__ __launch_bounds__(256) void k_apply_perm(const int* __restrict__ perm, const uint64_t* __restrict__ kin,
                                                   const int* __restrict__ vin, int64_t n,
                                                   uint64_t* __restrict__ kout, int* __restrict__ vout)
{
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < n) {
        const int j = perm[i];
        kout[i] = kin[j];
        vout[i] = vin[j];
    }
}

// Coincident points share a Morton key, so they sit in runs of equal sorted
// keys: every point compares its coordinates with the earlier points of its
// run (at most 64 of them; a longer run sets the flag unchecked).
__global__ __launch_bounds__(256) void k_coincident(const uint64_t* __restrict__ keys, const int* __restrict__ perm,
                                                   const double* __restrict__ pts, int64_t n, int* __restrict__ flag)
{
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i == 0 || i >= n || keys[i] != keys[i - 1])
        return;
    const double* a = pts + 3 * (size_t)perm[i];
    for (int64_t j = i - 1, k = 0; j >= 0 && keys[j] == keys[i]; --j, ++k) {
        if (k == 64) {
            *flag = 1;
            return;
        }
        const double* b = pts + 3 * (size_t)perm[j];
        if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) {
            *flag = 1;
            return;
        }
    }
}

int64_t rs_tiles(int64_t n) { return (n + kRsTile - 1) / kRsTile; }

// Sorts (kin, vin) by the low `bits` bits of the keys into (kout, vout).
// Scratch: two key/value buffers of n and the histogram (rs_temp_bytes).
hipError_t radix_sort(char* temp, const uint64_t* kin, const int* vin, uint64_t* kout, int* vout, int64_t n, int bits,
                      hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const int64_t ntile = rs_tiles(n);
    uint64_t* ka = reinterpret_cast<uint64_t*>(temp);
    uint64_t* kb = ka + n;
    int* va = reinterpret_cast<int*>(kb + n);
    int* vb = va + n;
    uint32_t* hist = reinterpret_cast<uint32_t*>(vb + n + (n & 1));
    uint32_t* doff = hist + (size_t)256 * ntile;
    const int passes = std::max(1, (bits + 7) / 8);
    const uint64_t* ksrc = kin;
    const int* vsrc = vin;
    for (int p = 0; p < passes; ++p) {
        // the last pass writes the output buffers
        uint64_t* kd = p == passes - 1 ? kout : ((p & 1) ? kb : ka);
        int* vd = p == passes - 1 ? vout : ((p & 1) ? vb : va);
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntile), dim3(kRsThreads), 0, s, ksrc, n, 8 * p, hist, (int)ntile);
        hipLaunchKernelGGL(k_rs_scan_digit, dim3(256), dim3(256), 0, s, hist, (int)ntile, doff);
        hipLaunchKernelGGL(k_rs_scan_totals, dim3(1), dim3(256), 0, s, doff);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntile), dim3(kRsThreads), 0, s, ksrc, vsrc, n, 8 * p, hist,
                           doff, (int)ntile, kd, vd);
        ksrc = kd;
        vsrc = vd;
    }
    return hipGetLastError();
}

size_t rs_temp_bytes(int64_t n)
{
    return (size_t)n * 2 * sizeof(uint64_t) + (size_t)(2 * n + 2) * sizeof(int) +
           (size_t)256 * (rs_tiles(std::max<int64_t>(n, 1)) + 1) * sizeof(uint32_t) + 256;
}

// ---- octree ------------------------------------------------------------------------
// The level-restricted tree is the coarsest refinement of the adaptive tree in
// which every cell touching a split cell one level finer is split too.  Its
// split cells S_L at level L are therefore
//     S_L = A_L  united with  { level-L cells touching some cell of S_{L+1} },
// A_L the adaptive tree's split cells (more than n_s points), and the cells
// at level L touching a level-(L+1) cell c are the parents of c's 27-cell
// neighbourhood (at most 2 per axis).  So S is computed bottom-up in one sweep
// over the levels, de-duplicated by a hash set, and the boxes are the roots
// plus the 8 children of every split cell.  A final sort by (level, problem,
// Morton index) gives the box order of a sequential construction.  Every
// level is one short launch over a device-resident count (no host round trip).
constexpr uint64_t kEmpty = ~0ull;
constexpr int kLevels = kMaxLevel + 1;

__device__ inline uint64_t spread3_d(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < kKeyBits; ++b)
        r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}
__device__ inline int64_t compact3_d(uint64_t v)
{
    int64_t r = 0;
    for (int b = 0; b < kKeyBits; ++b)
        r |= (int64_t)((v >> (3 * b)) & 1ull) << b;
    return r;
}
__device__ inline uint64_t cell_of(int64_t ix, int64_t iy, int64_t iz)
{
    return (spread3_d((uint64_t)ix) << 2) | (spread3_d((uint64_t)iy) << 1) | spread3_d((uint64_t)iz);
}
__device__ inline void coords_of(uint64_t cl, int64_t* x)
{
    x[0] = compact3_d(cl >> 2);
    x[1] = compact3_d(cl >> 1);
    x[2] = compact3_d(cl);
}
// level in the top 5 bits, then the problem, then the cell's 3L bits
// (valid while problem bits + 3L <= 59; the host checks)
__device__ inline uint64_t bkey(int L, int p, uint64_t cell)
{
    return ((uint64_t)L << 59) | ((uint64_t)p << (3 * L)) | cell;
}

// first index in [lo, hi) of sorted keys with key >= v
__device__ inline int64_t lower_bound_key(const uint64_t* __restrict__ keys, int64_t lo, int64_t hi, uint64_t v)
{
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// open-addressing hash table of 64-bit keys (multiplicative hashing)
struct Hash {
    uint64_t* keys;
    int* vals;
    int lg;  // log2 of the capacity
};
__device__ inline uint64_t hslot(const Hash& H, uint64_t k)
{
    return (k * 0x9E3779B97F4A7C15ull) >> (64 - H.lg);
}
__device__ inline bool hinsert(const Hash& H, uint64_t k, int v)
{
    const uint64_t mask = (1ull << H.lg) - 1;
    uint64_t h = hslot(H, k);
    for (;;) {
        const uint64_t prev = atomicCAS((unsigned long long*)&H.keys[h], (unsigned long long)kEmpty,
                                        (unsigned long long)k);
        if (prev == kEmpty) {
            if (H.vals)
                H.vals[h] = v;
            return true;
        }
        if (prev == k)
            return false;
        h = (h + 1) & mask;
    }
}
__device__ inline int hfind(const Hash& H, uint64_t k)
{
    const uint64_t mask = (1ull << H.lg) - 1;
    uint64_t h = hslot(H, k);
    for (;;) {
        const uint64_t q = H.keys[h];
        if (q == k)
            return H.vals ? H.vals[h] : 0;
        if (q == kEmpty)
            return -1;
        h = (h + 1) & mask;
    }
}

struct Cell {
    uint64_t cell;
    int pid, level;
    int64_t start, end;
};

struct TreeDev {
    const uint64_t* keys;
    const int64_t* off;
    int np, ns, periodic;
    int capA, capS, capB;
    Cell* A;            // adaptive split cells, level L at A + L capA
    int* cntA;          // kLevels
    Cell* S;            // restricted split cells, appended level by level (finest first)
    int* cntS;          // [0]: total
    int* sbase;         // kLevels + 1: first entry of each level's cells in S
    Hash HS;            // set of split cells
    Hash HB;            // box key -> sorted box index
    uint64_t* bk;       // box keys (unsorted, then sorted)
    int* bidx;          // box indices (identity, then the sorting permutation)
    uint64_t* bk2;
    int* bidx2;
    int64_t* ustart;    // unsorted ranges and flags
    int64_t* uend;
    int* usplit;
    int64_t* start;     // sorted boxes
    int64_t* end;
    int* split;
    int* parent;
    int* child0;
    int* ls;            // level starts, kLevels + 1
    int* status;        // [0] overflow, [1] boxes, [2] deepest level
};

constexpr int kGrid = 1024, kBlk = 256;
#define DMK_GRID_STRIDE(i, count) for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < (count); i += (int64_t)kGrid * kBlk)

// the roots holding more than ns points
__global__ __launch_bounds__(256) void k_roots(TreeDev D)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < D.np && D.off[p + 1] - D.off[p] > D.ns) {
        const int j = atomicAdd(&D.cntA[0], 1);
        D.A[j] = Cell{0ull, p, 0, D.off[p], D.off[p + 1]};
    }
}

// children of the adaptive split cells of level L with more than ns points
__global__ __launch_bounds__(kBlk) void k_adapt(TreeDev D, int L)
{
    const int na = D.cntA[L];
    const int sh3 = 3 * (kKeyBits - (L + 1));
    DMK_GRID_STRIDE(k, 8ll * na)
    {
        const Cell e = D.A[(size_t)L * D.capA + (k >> 3)];
        const uint64_t cc = (e.cell << 3) | (uint64_t)(k & 7);
        const int64_t s = lower_bound_key(D.keys, e.start, e.end, cc << sh3);
        const int64_t t = lower_bound_key(D.keys, s, e.end, (cc + 1) << sh3);
        if (t - s > D.ns && L + 1 < kMaxLevel) {
            const int j = atomicAdd(&D.cntA[L + 1], 1);
            if (j < D.capA)
                D.A[(size_t)(L + 1) * D.capA + j] = Cell{cc, e.pid, L + 1, s, t};
            else
                D.status[0] = 1;
        }
    }
}

__global__ void k_mark(TreeDev D, int L)
{
    D.sbase[L] = D.cntS[0];
}

__device__ inline void add_split(const TreeDev& D, int L, int p, uint64_t cell)
{
    if (D.cntS[0] >= D.capS) {
        D.status[0] = 1;
        return;
    }
    if (hinsert(D.HS, bkey(L, p, cell), 0)) {
        const int j = atomicAdd(&D.cntS[0], 1);
        if (j < D.capS)
            D.S[j] = Cell{cell, p, L, 0, 0};
        else
            D.status[0] = 1;
    }
}

// S_L from A_L and the cells of S_{L+1} (entries [sbase[L+1], sbase[L]))
__global__ __launch_bounds__(kBlk) void k_close(TreeDev D, int L)
{
    const int na = D.cntA[L];
    const int s0 = D.sbase[L + 1], s1 = D.sbase[L];
    const int64_t M = (int64_t)1 << (L + 1);  // cells per axis at level L + 1
    DMK_GRID_STRIDE(k, (int64_t)na + (s1 - s0))
    {
        if (k < na) {
            const Cell e = D.A[(size_t)L * D.capA + k];
            add_split(D, L, e.pid, e.cell);
            continue;
        }
        const Cell e = D.S[s0 + (k - na)];
        int64_t x[3];
        coords_of(e.cell, x);
        int64_t par[3][2];
        int npar[3];
        for (int a = 0; a < 3; ++a) {
            npar[a] = 0;
            for (int o = -1; o <= 1; ++o) {
                int64_t q = x[a] + o;
                if (q < 0 || q >= M) {
                    if (!D.periodic)
                        continue;
                    q = (q + M) % M;
                }
                const int64_t pq = q >> 1;
                bool seen = false;
                for (int u = 0; u < npar[a]; ++u)
                    seen = seen || par[a][u] == pq;
                if (!seen && npar[a] < 2)
                    par[a][npar[a]++] = pq;
            }
        }
        for (int i = 0; i < npar[0]; ++i)
            for (int j = 0; j < npar[1]; ++j)
                for (int m = 0; m < npar[2]; ++m)
                    add_split(D, L, e.pid, cell_of(par[0][i], par[1][j], par[2][m]));
    }
}

// boxes: the roots and the 8 children of every split cell (unsorted)
__global__ __launch_bounds__(kBlk) void k_boxes(TreeDev D)
{
    const int ns_ = D.cntS[0];
    DMK_GRID_STRIDE(i, (int64_t)D.np + 8ll * ns_)
    {
        int L, p;
        uint64_t cc;
        int64_t s, t;
        if (i < D.np) {
            L = 0;
            p = (int)i;
            cc = 0;
            s = D.off[p];
            t = D.off[p + 1];
        } else {
            const Cell e = D.S[(i - D.np) >> 3];
            L = e.level + 1;
            p = e.pid;
            cc = (e.cell << 3) | (uint64_t)((i - D.np) & 7);
            const int sh3 = 3 * (kKeyBits - L);
            s = lower_bound_key(D.keys, D.off[p], D.off[p + 1], cc << sh3);
            t = lower_bound_key(D.keys, s, D.off[p + 1], (cc + 1) << sh3);
        }
        const uint64_t key = bkey(L, p, cc);
        D.bk[i] = key;
        D.bidx[i] = (int)i;
        D.ustart[i] = s;
        D.uend[i] = t;
        D.usplit[i] = hfind(D.HS, key) >= 0 ? 1 : 0;
    }
}

// sorted box arrays, level starts and the key -> index table
__global__ __launch_bounds__(kBlk) void k_sorted(TreeDev D)
{
    const int nb = D.np + 8 * D.cntS[0];
    DMK_GRID_STRIDE(i, nb)
    {
        const int u = D.bidx2[i];
        D.start[i] = D.ustart[u];
        D.end[i] = D.uend[u];
        D.split[i] = D.usplit[u];
        const uint64_t key = D.bk2[i];
        const int L = (int)(key >> 59);
        if (i == 0 || (int)(D.bk2[i - 1] >> 59) != L)
            D.ls[L] = (int)i;
        if (i == nb - 1) {
            D.ls[L + 1] = nb;
            D.status[1] = nb;
            D.status[2] = L;
        }
        hinsert(D.HB, key, (int)i);
    }
}

__device__ inline void key_parts(uint64_t key, int* L, int* p, uint64_t* cell)
{
    *L = (int)(key >> 59);
    const uint64_t rest = key & ((1ull << 59) - 1);
    *p = (int)(rest >> (3 * *L));
    *cell = rest & ((3 * *L) >= 64 ? ~0ull : ((1ull << (3 * *L)) - 1));
}

__global__ __launch_bounds__(kBlk) void k_links(TreeDev D)
{
    const int nb = D.status[1];
    DMK_GRID_STRIDE(i, nb)
    {
        int L, p;
        uint64_t cell;
        key_parts(D.bk2[i], &L, &p, &cell);
        D.parent[i] = L > 0 ? hfind(D.HB, bkey(L - 1, p, cell >> 3)) : -1;
        D.child0[i] = D.split[i] ? hfind(D.HB, bkey(L + 1, p, cell << 3)) : -1;
    }
}

// ---- neighbour lists ------------------------------------------------------------------
struct ListDev {
    int* ncol;          // per box
    FarEntry* col;      // 27 per box
    int* ninc;
    FarEntry* inc;      // 27 per box
    int* nnear;
    NearEntry* near;    // kNearCap per box (leaves only)
    unsigned long long* pairs;
};
constexpr int kNearCap = 96;

// Colleagues (same level, sharing a boundary point, itself included) by
// direct lookup of the 27 neighbour cells.  They are listed in the order of a
// top-down construction (the children of the parent's colleagues, parent
// entry by parent entry, child digit by child digit): offset o at level L
// ranks by the chain (rank of the root offset, d_1, ..., d_L), where going up
// one level o -> floor((o + b) / 2) with b the box's coordinate parities at
// that level and d the child digit of (o + b) mod 2.
__global__ __launch_bounds__(kBlk) void k_colleagues(TreeDev D, ListDev LD)
{
    const int nb = D.status[1];
    DMK_GRID_STRIDE(i, nb)
    {
        int L, p;
        uint64_t cell;
        key_parts(D.bk2[i], &L, &p, &cell);
        int64_t x[3];
        coords_of(cell, x);
        const int64_t M = (int64_t)1 << L;
        uint64_t rank[27];
        FarEntry ent[27];
        int k = 0;
        for (int ox = -1; ox <= 1; ++ox)
            for (int oy = -1; oy <= 1; ++oy)
                for (int oz = -1; oz <= 1; ++oz) {
                    int64_t q[3] = {x[0] + ox, x[1] + oy, x[2] + oz};
                    bool in = true;
                    for (int a = 0; a < 3; ++a)
                        if (q[a] < 0 || q[a] >= M) {
                            if (!D.periodic)
                                in = false;
                            q[a] = (q[a] % M + M) % M;
                        }
                    if (!in)
                        continue;
                    const int j = hfind(D.HB, bkey(L, p, cell_of(q[0], q[1], q[2])));
                    if (j < 0)
                        continue;
                    // order key
                    int o[3] = {ox, oy, oz};
                    uint64_t digits = 0;
                    int64_t xb[3] = {x[0], x[1], x[2]};
                    for (int l = L; l >= 1; --l) {
                        int d = 0;
                        for (int a = 0; a < 3; ++a) {
                            const int v = o[a] + (int)(xb[a] & 1);
                            const int up = v >= 0 ? v / 2 : -1;  // floor of v/2 for v in [-1, 2]
                            d = 2 * d + (v - 2 * up);
                            o[a] = up;
                            xb[a] >>= 1;
                        }
                        digits |= (uint64_t)d << (3 * (L - l));
                    }
                    const uint64_t root = (uint64_t)(9 * (o[0] + 1) + 3 * (o[1] + 1) + (o[2] + 1));
                    rank[k] = (root << (3 * L)) | digits;
                    ent[k] = FarEntry{j, (int8_t)ox, (int8_t)oy, (int8_t)oz};
                    ++k;
                }
        // insertion sort by rank (at most 27 entries)
        for (int a = 1; a < k; ++a) {
            const uint64_t r = rank[a];
            const FarEntry e = ent[a];
            int b = a - 1;
            while (b >= 0 && rank[b] > r) {
                rank[b + 1] = rank[b];
                ent[b + 1] = ent[b];
                --b;
            }
            rank[b + 1] = r;
            ent[b + 1] = e;
        }
        for (int a = 0; a < k; ++a)
            LD.col[(size_t)27 * i + a] = ent[a];
        LD.ncol[i] = k;
    }
}

// Exchange lists (a non-leaf box receives the difference kernel from every
// non-empty colleague, a leaf only from non-leaf ones) and near lists (the
// adjacent non-empty leaves at levels L-1, L, L+1, residual level max of the
// two), one thread per box, in the order a sequential construction lists them.
__global__ __launch_bounds__(kBlk) void k_lists(TreeDev D, ListDev LD)
{
    const int nb = D.status[1];
    DMK_GRID_STRIDE(i, nb)
    {
        int L, p;
        uint64_t cell;
        key_parts(D.bk2[i], &L, &p, &cell);
        const bool leaf = D.split[i] == 0;
        const int64_t cnt = D.end[i] - D.start[i];
        const FarEntry* col = LD.col + (size_t)27 * i;
        const int ncol = LD.ncol[i];
        int ni = 0;
        if (cnt > 0)
            for (int e = 0; e < ncol; ++e) {
                const FarEntry E = col[e];
                if (D.end[E.src] == D.start[E.src])
                    continue;
                if (!leaf || D.split[E.src] != 0)
                    LD.inc[(size_t)27 * i + ni++] = E;
            }
        LD.ninc[i] = ni;
        int nn = 0;
        if (leaf && cnt > 0) {
            NearEntry* out = LD.near + (size_t)kNearCap * i;
            const int64_t M = (int64_t)1 << L;
            int64_t x[3];
            coords_of(cell, x);
            unsigned long long pairs = 0;
            auto add = [&](int S, int px, int py, int pz, int lam) {
                const int64_t sc = D.end[S] - D.start[S];
                if (sc == 0 || nn >= kNearCap)
                    return;
                out[nn++] = NearEntry{S, (int8_t)px, (int8_t)py, (int8_t)pz, (int8_t)lam};
                pairs += (unsigned long long)(cnt * sc);
            };
            for (int e = 0; e < ncol; ++e) {
                const FarEntry E = col[e];
                int pp[3];
                const int o[3] = {E.ox, E.oy, E.oz};
                for (int a = 0; a < 3; ++a) {
                    const int64_t q = x[a] + o[a];
                    pp[a] = q < 0 ? -1 : (q >= M ? 1 : 0);
                }
                if (D.split[E.src] == 0) {
                    add(E.src, pp[0], pp[1], pp[2], L);
                } else {
                    const int base = D.child0[E.src];
                    for (int d = 0; d < 8; ++d) {
                        const int cb[3] = {(d >> 2) & 1, (d >> 1) & 1, d & 1};
                        bool touch = true;
                        for (int a = 0; a < 3; ++a) {
                            if (o[a] == 1 && cb[a] != 0)
                                touch = false;
                            if (o[a] == -1 && cb[a] != 1)
                                touch = false;
                        }
                        if (touch && D.split[base + d] == 0)
                            add(base + d, pp[0], pp[1], pp[2], L + 1);
                    }
                }
            }
            const int P = D.parent[i];
            if (P >= 0) {
                int64_t xp[3];
                for (int a = 0; a < 3; ++a)
                    xp[a] = x[a] >> 1;
                const int64_t MP = (int64_t)1 << (L - 1);
                const int bb[3] = {(int)(x[0] & 1), (int)(x[1] & 1), (int)(x[2] & 1)};
                const FarEntry* pcol = LD.col + (size_t)27 * P;
                const int npc = LD.ncol[P];
                for (int e = 0; e < npc; ++e) {
                    const FarEntry E = pcol[e];
                    if (!E.ox && !E.oy && !E.oz)
                        continue;
                    if (D.split[E.src] != 0)
                        continue;
                    const int o[3] = {E.ox, E.oy, E.oz};
                    bool touch = true;
                    for (int a = 0; a < 3; ++a)
                        if ((o[a] == 1 && bb[a] != 1) || (o[a] == -1 && bb[a] != 0))
                            touch = false;
                    if (!touch)
                        continue;
                    int pp[3];
                    for (int a = 0; a < 3; ++a) {
                        const int64_t q = xp[a] + o[a];
                        pp[a] = q < 0 ? -1 : (q >= MP ? 1 : 0);
                    }
                    add(E.src, pp[0], pp[1], pp[2], L);
                }
            }
            if (pairs)
                atomicAdd(LD.pairs, pairs);
        }
        LD.nnear[i] = nn;
    }
}

// counts -> packed list offsets (scanned afterwards)
__global__ __launch_bounds__(kBlk) void k_list_counts(TreeDev D, ListDev LD, uint32_t* onear, uint32_t* oinc)
{
    const int nb = D.status[1];
    DMK_GRID_STRIDE(i, nb)
    {
        onear[i] = (uint32_t)LD.nnear[i];
        oinc[i] = (uint32_t)LD.ninc[i];
    }
}

// lists packed back to back (offsets from the scans above)
__global__ __launch_bounds__(kBlk) void k_list_pack(TreeDev D, ListDev LD, const uint32_t* onear,
                                                    const uint32_t* oinc, NearEntry* pnear, FarEntry* pinc)
{
    const int nb = D.status[1];
    DMK_GRID_STRIDE(i, nb)
    {
        for (int k = 0; k < LD.nnear[i]; ++k)
            pnear[onear[i] + k] = LD.near[(size_t)kNearCap * i + k];
        for (int k = 0; k < LD.ninc[i]; ++k)
            pinc[oinc[i] + k] = LD.inc[(size_t)27 * i + k];
    }
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* __restrict__ a, int64_t m, uint64_t v)
{
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < m)
        a[i] = v;
}

}  // namespace

size_t sort_temp_bytes(int64_t n)
{
    return rs_temp_bytes(n);
}

void launch_find_coincident(const uint64_t* sorted_keys, const int* perm, const double* pts, int64_t n, int* flag,
                            hipStream_t s)
{
    if (n > 1)
        hipLaunchKernelGGL(k_coincident, dim3(nblocks(n, 256)), dim3(256), 0, s, sorted_keys, perm, pts, n, flag);
}

void launch_sort(void* temp, size_t temp_bytes, const uint64_t* kin, uint64_t* kout, const int* vin, int* vout,
                 int64_t n, int end_bit, hipStream_t s)
{
    (void)temp_bytes;
    (void)radix_sort(static_cast<char*>(temp), kin, vin, kout, vout, n, end_bit, s);
}

size_t seg_sort_temp_bytes(int64_t n, int nseg)
{
    (void)nseg;
    // the key sort's scratch, then key-sorted keys and values, problem keys,
    // positions, the problem-sort output and the permutation
    return rs_temp_bytes(n) + (size_t)n * (3 * sizeof(uint64_t) + 3 * sizeof(int)) + 512;
}

// Points of a problem are contiguous in the input, so a stable sort by the
// Morton key followed by a stable sort by problem sorts every segment by key.
void launch_seg_sort(void* temp, size_t temp_bytes, const uint64_t* kin, uint64_t* kout, const int* vin, int* vout,
                     int64_t n, int nseg, const int* pid, int end_bit, hipStream_t s)
{
    (void)temp_bytes;
    if (n == 0)
        return;
    char* t = static_cast<char*>(temp);
    uint64_t* km = reinterpret_cast<uint64_t*>(t + rs_temp_bytes(n));
    uint64_t* kp = km + n;
    uint64_t* kp2 = kp + n;
    int* vm = reinterpret_cast<int*>(kp2 + n);
    int* idx = vm + n;
    int* perm = idx + n;
    (void)radix_sort(t, kin, vin, km, vm, n, end_bit, s);
    hipLaunchKernelGGL(k_gather_pid_key, dim3(nblocks(n, 256)), dim3(256), 0, s, vm, pid, n, kp, idx);
    int pbits = 1;
    while ((1ll << pbits) < nseg)
        ++pbits;
    // (problem, position) pairs sorted by problem: the positions permute the key-sorted pairs
    (void)radix_sort(t, kp, idx, kp2, perm, n, pbits, s);
    hipLaunchKernelGGL(k_apply_perm, dim3(nblocks(n, 256)), dim3(256), 0, s, perm, km, vm, n, kout, vout);
}

int build_tree_device(const uint64_t* keys, const int64_t* d_off, int np, int64_t n, int ns, bool periodic,
                      DeviceAlloc alloc, void* actx, hipStream_t s, Tree* T, std::string* err)
{
    int pbits = 0;
    while ((1ll << pbits) < np)
        ++pbits;
    const int lmax = std::min(kMaxLevel, (59 - pbits) / 3);  // deepest level the packed box keys hold
    const int64_t base = n / std::max(ns, 1) + 1;
    // split cells of one adaptive level hold more than ns points each
    const int capA = (int)std::min<int64_t>(1 << 26, base + np);
    int capS = (int)std::min<int64_t>(1 << 26, 4 * (base + np) + 1024);
    auto lg2 = [](int64_t v) {
        int g = 1;
        while ((1ll << g) < v)
            ++g;
        return g;
    };
    auto fail_oom = [&]() {
        *err = "device allocation failed (octree)";
        return DMK_TREE_OOM;
    };
    for (int attempt = 0; attempt < 4; ++attempt, capS *= 4) {
        TreeDev D{};
        D.keys = keys;
        D.off = d_off;
        D.np = np;
        D.ns = ns;
        D.periodic = periodic ? 1 : 0;
        D.capA = capA;
        D.capS = capS;
        D.A = (Cell*)alloc(actx, (size_t)kLevels * capA * sizeof(Cell));
        D.cntA = (int*)alloc(actx, (kLevels + 1) * 4);
        D.S = (Cell*)alloc(actx, (size_t)capS * sizeof(Cell));
        D.cntS = (int*)alloc(actx, 16);
        D.sbase = (int*)alloc(actx, (kLevels + 2) * 4);
        D.status = (int*)alloc(actx, 16);
        D.HS.lg = lg2(2 * ((int64_t)capS + (int64_t)kGrid * kBlk));
        D.HS.keys = (uint64_t*)alloc(actx, ((size_t)1 << D.HS.lg) * 8);
        D.HS.vals = nullptr;
        if (!D.A || !D.cntA || !D.S || !D.cntS || !D.sbase || !D.status || !D.HS.keys)
            return fail_oom();
        launch_zero(D.cntA, (kLevels + 1) * 4, s);
        launch_zero(D.cntS, 16, s);
        launch_zero(D.sbase, (kLevels + 2) * 4, s);
        launch_zero(D.status, 16, s);
        hipLaunchKernelGGL(k_fill_u64, dim3(nblocks((int64_t)1 << D.HS.lg, 256)), dim3(256), 0, s, D.HS.keys,
                           (int64_t)1 << D.HS.lg, kEmpty);
        // adaptive refinement, top down (the roots' split cells first)
        hipLaunchKernelGGL(k_roots, dim3(nblocks(np, 256)), dim3(256), 0, s, D);
        for (int L = 0; L + 1 < kMaxLevel; ++L)
            hipLaunchKernelGGL(k_adapt, dim3(kGrid), dim3(kBlk), 0, s, D, L);
        // level restriction, bottom up
        for (int L = kMaxLevel - 1; L >= 0; --L) {
            hipLaunchKernelGGL(k_mark, dim3(1), dim3(1), 0, s, D, L);
            hipLaunchKernelGGL(k_close, dim3(kGrid), dim3(kBlk), 0, s, D, L);
        }
        int st[4] = {0, 0, 0, 0}, nsplit = 0;
        std::vector<int> sb(kLevels + 2);
        hipError_t e = hipMemcpyAsync(st, D.status, sizeof(st), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&nsplit, D.cntS, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sb.data(), D.sbase, sb.size() * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = hipGetLastError();
        if (e != hipSuccess) {
            *err = hipGetErrorString(e);
            return DMK_TREE_HIP;
        }
        if (st[0] || nsplit > capS)
            continue;  // more split cells than the capacity: retry larger
        const int nb = np + 8 * nsplit;
        // the deepest split cell's children must fit the packed keys
        {
            int deep_split = -1;
            // S holds the finest level first: level L occupies [sbase[L], sbase[L-1])
            for (int L = kMaxLevel - 1; L >= 0; --L) {
                const int hi = L > 0 ? sb[L - 1] : nsplit;
                if (hi > sb[L]) {
                    deep_split = L;
                    break;
                }
            }
            if (deep_split + 1 > lmax) {
                *err = "octree too deep for the packed box keys of this many problems";
                return DMK_TREE_UNSUPPORTED;
            }
        }
        D.capB = nb;
        D.bk = (uint64_t*)alloc(actx, (size_t)nb * 8);
        D.bidx = (int*)alloc(actx, (size_t)nb * 4);
        D.bk2 = (uint64_t*)alloc(actx, (size_t)nb * 8);
        D.bidx2 = (int*)alloc(actx, (size_t)nb * 4);
        D.ustart = (int64_t*)alloc(actx, (size_t)nb * 8);
        D.uend = (int64_t*)alloc(actx, (size_t)nb * 8);
        D.usplit = (int*)alloc(actx, (size_t)nb * 4);
        D.start = (int64_t*)alloc(actx, (size_t)nb * 8);
        D.end = (int64_t*)alloc(actx, (size_t)nb * 8);
        D.split = (int*)alloc(actx, (size_t)nb * 4);
        D.parent = (int*)alloc(actx, (size_t)nb * 4);
        D.child0 = (int*)alloc(actx, (size_t)nb * 4);
        D.ls = (int*)alloc(actx, (kLevels + 1) * 4);
        D.HB.lg = lg2(2 * (int64_t)nb);
        D.HB.keys = (uint64_t*)alloc(actx, ((size_t)1 << D.HB.lg) * 8);
        D.HB.vals = (int*)alloc(actx, ((size_t)1 << D.HB.lg) * 4);
        char* stemp = (char*)alloc(actx, rs_temp_bytes(nb));
        if (!D.bk || !D.bidx || !D.bk2 || !D.bidx2 || !D.ustart || !D.uend || !D.usplit || !D.start || !D.end ||
            !D.split || !D.parent || !D.child0 || !D.ls || !D.HB.keys || !D.HB.vals || !stemp)
            return fail_oom();
        hipLaunchKernelGGL(k_fill_u64, dim3(nblocks((int64_t)1 << D.HB.lg, 256)), dim3(256), 0, s, D.HB.keys,
                           (int64_t)1 << D.HB.lg, kEmpty);
        hipLaunchKernelGGL(k_boxes, dim3(kGrid), dim3(kBlk), 0, s, D);
        e = radix_sort(stemp, D.bk, D.bidx, D.bk2, D.bidx2, nb, 64, s);
        if (e != hipSuccess) {
            *err = hipGetErrorString(e);
            return DMK_TREE_HIP;
        }
        hipLaunchKernelGGL(k_sorted, dim3(kGrid), dim3(kBlk), 0, s, D);
        hipLaunchKernelGGL(k_links, dim3(kGrid), dim3(kBlk), 0, s, D);
        ListDev LD;
        LD.ncol = (int*)alloc(actx, (size_t)nb * 4);
        LD.col = (FarEntry*)alloc(actx, (size_t)nb * 27 * sizeof(FarEntry));
        LD.ninc = (int*)alloc(actx, (size_t)nb * 4);
        LD.inc = (FarEntry*)alloc(actx, (size_t)nb * 27 * sizeof(FarEntry));
        LD.nnear = (int*)alloc(actx, (size_t)nb * 4);
        LD.near = (NearEntry*)alloc(actx, (size_t)nb * kNearCap * sizeof(NearEntry));
        LD.pairs = (unsigned long long*)alloc(actx, 8);
        if (!LD.ncol || !LD.col || !LD.ninc || !LD.inc || !LD.nnear || !LD.near || !LD.pairs)
            return fail_oom();
        launch_zero(LD.pairs, 8, s);
        hipLaunchKernelGGL(k_colleagues, dim3(kGrid), dim3(kBlk), 0, s, D, LD);
        hipLaunchKernelGGL(k_lists, dim3(kGrid), dim3(kBlk), 0, s, D, LD);
        uint32_t* onear = (uint32_t*)alloc(actx, (size_t)nb * 4);
        uint32_t* oinc = (uint32_t*)alloc(actx, (size_t)nb * 4);
        NearEntry* pnear = (NearEntry*)alloc(actx, (size_t)nb * kNearCap * sizeof(NearEntry));
        FarEntry* pinc = (FarEntry*)alloc(actx, (size_t)nb * 27 * sizeof(FarEntry));
        if (!onear || !oinc || !pnear || !pinc)
            return fail_oom();
        hipLaunchKernelGGL(k_list_counts, dim3(kGrid), dim3(kBlk), 0, s, D, LD, onear, oinc);
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(256), 0, s, onear, (int64_t)nb);
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(256), 0, s, oinc, (int64_t)nb);
        hipLaunchKernelGGL(k_list_pack, dim3(kGrid), dim3(kBlk), 0, s, D, LD, onear, oinc, pnear, pinc);
        // download
        std::vector<uint64_t> key(nb);
        std::vector<int> split(nb), parent(nb), child0(nb), ninc(nb), nnear(nb), ls(kLevels + 1), st2(4);
        std::vector<int64_t> bs(nb), be(nb);
        unsigned long long pairs = 0;
        auto cp = [&](void* dst, const void* src, size_t bytes) {
            if (e == hipSuccess && bytes)
                e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
        };
        cp(key.data(), D.bk2, (size_t)nb * 8);
        cp(split.data(), D.split, (size_t)nb * 4);
        cp(parent.data(), D.parent, (size_t)nb * 4);
        cp(child0.data(), D.child0, (size_t)nb * 4);
        cp(bs.data(), D.start, (size_t)nb * 8);
        cp(be.data(), D.end, (size_t)nb * 8);
        cp(ls.data(), D.ls, (kLevels + 1) * 4);
        cp(st2.data(), D.status, 16);
        cp(ninc.data(), LD.ninc, (size_t)nb * 4);
        cp(nnear.data(), LD.nnear, (size_t)nb * 4);
        cp(&pairs, LD.pairs, 8);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            *err = hipGetErrorString(e);
            return DMK_TREE_HIP;
        }
        const int deep = st2[2];
        size_t tinc = 0, tnear = 0;
        int maxnear = 0;
        for (int i = 0; i < nb; ++i) {
            tinc += ninc[i];
            tnear += nnear[i];
            maxnear = std::max(maxnear, nnear[i]);
        }
        if (maxnear >= kNearCap) {
            *err = "near list capacity exceeded";
            return DMK_TREE_HIP;
        }
        std::vector<FarEntry> inc(std::max<size_t>(tinc, 1));
        std::vector<NearEntry> nr(std::max<size_t>(tnear, 1));
        cp(inc.data(), pinc, tinc * sizeof(FarEntry));
        cp(nr.data(), pnear, tnear * sizeof(NearEntry));
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            *err = hipGetErrorString(e);
            return DMK_TREE_HIP;
        }
        // host mirror (boxes level-major, problem and Morton order within a level)
        std::vector<int> pid(nb);
        T->periodic = periodic;
        T->n = n;
        T->max_level = deep;
        T->level_start.assign(ls.begin(), ls.begin() + deep + 2);
        T->boxes.resize(nb);
        for (int i = 0; i < nb; ++i) {
            Box& B = T->boxes[i];
            const int L = (int)(key[i] >> 59);
            const uint64_t rest = key[i] & ((1ull << 59) - 1);
            pid[i] = (int)(rest >> (3 * L));
            const uint64_t v = L == 0 ? 0ull : (rest & ((1ull << (3 * L)) - 1));
            int64_t xyz[3] = {0, 0, 0};
            for (int b = 0; b < kKeyBits; ++b) {
                xyz[0] |= (int64_t)((v >> (3 * b + 2)) & 1) << b;
                xyz[1] |= (int64_t)((v >> (3 * b + 1)) & 1) << b;
                xyz[2] |= (int64_t)((v >> (3 * b)) & 1) << b;
            }
            B.level = L;
            B.ix = xyz[0];
            B.iy = xyz[1];
            B.iz = xyz[2];
            B.parent = parent[i];
            B.start = bs[i];
            B.end = be[i];
            B.leaf = split[i] == 0;
            for (int d = 0; d < 8; ++d)
                B.child[d] = B.leaf ? -1 : child0[i] + d;
        }
        T->colleagues.clear();
        T->incoming.assign(nb, {});
        std::vector<size_t> onr(nb);
        {
            size_t oi = 0, on = 0;
            for (int i = 0; i < nb; ++i) {
                T->incoming[i].assign(inc.begin() + oi, inc.begin() + oi + ninc[i]);
                oi += ninc[i];
                onr[i] = on;
                on += nnear[i];
            }
        }
        // non-empty leaves, problem by problem (box order within a problem)
        T->leaves.clear();
        for (int i = 0; i < nb; ++i)
            if (split[i] == 0 && be[i] > bs[i])
                T->leaves.push_back(i);
        std::stable_sort(T->leaves.begin(), T->leaves.end(), [&](int a, int b) { return pid[a] < pid[b]; });
        T->near.assign(T->leaves.size(), {});
        for (size_t li = 0; li < T->leaves.size(); ++li) {
            const int i = T->leaves[li];
            T->near[li].assign(nr.begin() + onr[i], nr.begin() + onr[i] + nnear[i]);
        }
        T->n_near_pairs = (int64_t)pairs;
        return 0;
    }
    *err = "octree capacity exceeded";
    return DMK_TREE_OOM;
}

}  // namespace dmk
