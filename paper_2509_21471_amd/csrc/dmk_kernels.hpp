// Device kernels of the DMK Stokeslet path and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace dmk {

struct cplx {
    double re, im;
};

// ---- tree construction -----------------------------------------------------
// per-block partial bounding box / finiteness of (n,3) row-major points
void launch_bbox(const double* pts, int64_t n, double* partial /*nblk*8*/, int nblk, hipStream_t s);
// per problem b (points [off[b], off[b+1])): partial[8b..8b+6] = lo, hi, non-finite count
void launch_bbox_seg(const double* pts, const int64_t* off, int nprob, double* partial, hipStream_t s);
void launch_fill_pid(const int64_t* off, int nprob, int64_t n, int* pid, hipStream_t s);
// unit-box coordinates, Morton keys (19 bits per dimension), identity index
// geo: per problem (cx, cy, cz, 1/len); pid: problem of each point (NULL: one problem)
void launch_morton(const double* pts, int64_t n, const int* pid, const double* geo, uint64_t* keys, int* idx,
                   hipStream_t s);
// sorted SoA unit coordinates
void launch_gather_points(const double* pts, int64_t n, const int* perm, const int* pid, const double* geo,
                          double* x, double* y, double* z, hipStream_t s);
// Reorder of the points inside leaves so that runs of 8, 16, 32 and 64 points
// (the near field's target groups and source chunks) are spatially compact:
// recursive balanced bisection across the longest side of each segment's
// bounding box, cutting after whole 64-point chunks, then whole 8-point groups.
// A segment starts where a leaf's sources (or targets) start and holds at
// most kKdCap points.  src[i] = sorted position whose point moves to i
// (identity outside the segments); perm_out[i] = perm[src[i]].
constexpr int kKdCap = 2048;
struct KdSeg {
    int64_t start;
    int len;          // 9 .. kKdCap
    int pad;
};
void launch_leaf_order(const KdSeg* segs, int nseg, const int* perm, const double* x, const double* y,
                       const double* z, int64_t n, int* src, int* perm_out, hipStream_t s);
// radix sort of (key, index) pairs by the low end_bit key bits (stable, 8-bit
// digits); temp storage is allocated by the caller
size_t sort_temp_bytes(int64_t n);
void launch_sort(void* temp, size_t temp_bytes, const uint64_t* kin, uint64_t* kout, const int* vin, int* vout,
                 int64_t n, int end_bit, hipStream_t s);
// the same within each problem: points of problem b are contiguous in the
// input and pid[v] is the problem of value v (the input positions)
size_t seg_sort_temp_bytes(int64_t n, int nseg);
void launch_seg_sort(void* temp, size_t temp_bytes, const uint64_t* kin, uint64_t* kout, const int* vin, int* vout,
                     int64_t n, int nseg, const int* pid, int end_bit, hipStream_t s);
// Level-restricted octree (a forest over np problems) of the sorted Morton
// keys, built on the device, and its exchange and near lists (Step 1); the
// result is mirrored into *T (boxes level-major, problem and Morton order
// within a level, as build_tree / merge_forest order them; colleague lists are
// not mirrored).  d_off: device offsets of the problems (np + 1).  alloc
// returns device scratch that stays valid until the call returns.  Returns 0,
// or DMK_TREE_OOM / DMK_TREE_HIP / DMK_TREE_UNSUPPORTED with *err set.
// Synchronises s.
struct Tree;
using DeviceAlloc = void* (*)(void* ctx, size_t bytes);
constexpr int DMK_TREE_OOM = 1;
constexpr int DMK_TREE_HIP = 2;
constexpr int DMK_TREE_UNSUPPORTED = 3;  // too deep for the packed keys: use the host construction
int build_tree_device(const uint64_t* keys, const int64_t* d_off, int np, int64_t n, int ns, bool periodic,
                      DeviceAlloc alloc, void* actx, hipStream_t s, Tree* T, std::string* err);
// per 64-point chunk bounding boxes (chunk list given as starts/ends)
void launch_chunk_bbox(const double* x, const double* y, const double* z, const int64_t* cstart,
                       const int* clen, int nchunk, double* bbox /*nchunk*6*/, hipStream_t s);

// ---- per evaluation --------------------------------------------------------
// forces (n,3) original order -> sorted SoA fs[3][n]
// points with input index < nsrc carry forces, the others (targets only) zero
void launch_gather_forces(const double* f, int64_t n, int64_t nsrc, const int* perm, double* fs, hipStream_t s);
// stresslet: rho[6][n] symmetric densities of f n^T (off-diagonal pairs summed), fn[6][n] = (f, n)
void launch_gather_stresslet(const double* f, const double* nv, int64_t n, int64_t nsrc, const int* perm, double* rho,
                             double* fn, hipStream_t s);

struct LeafDesc {
    int fid;          // far-field slot of the leaf
    int level;
    int64_t start, end;
    double cx, cy, cz;
};

// Lagrange values of each sorted point on its leaf's proxy grid:
// Ltab[i][d][0..lagrange_pad(p)) for d = x, y, z (zero padded); float when
// f32 (plans whose far field is stored in FP32), else double
int lagrange_pad(int p);
// Chebyshev orders p the point kernels are compiled for
bool p_supported(int p);
void launch_lagrange_table(int p, const LeafDesc* leaves, int nleaf, const double* x, const double* y,
                           const double* z, const double* cheb_t, const double* cheb_w, void* Ltab, bool f32,
                           hipStream_t s);
// proxy charges of leaves (Step 2a): Q[fid][j][a][b][c] = sum_pt L_a L_b L_c f_j
// nc = 3 (Stokeslet forces) or 6 (stresslet densities); Q[fid][nc][a][b][c].
// f32: FP32 Ltab and Q, contraction on FP32 MFMA with FP64 blocked sums
void launch_anterp(int p, int nc, const LeafDesc* leaves, int nleaf, const void* Ltab, const double* fs, int64_t n,
                   void* Q, bool f32, hipStream_t s);
// far-field value at the points (final interpolation), V z-major V[fid][j][c][b][a]:
// u[j][i] += sum V L L L, over chunks of at most eval_chunk_points(p) points of
// one leaf (one block of 4 threads per point)
// points per block: `request` (128 or 256) where the kernel takes it, else the largest that fits
int eval_chunk_points(int p, int request = 0);
struct EvalChunk {
    int fid;
    int64_t start, end;
};
// f32: FP32 Ltab and V, contraction over a on FP32 MFMA, the rest FP64
void launch_leaf_eval(int p, int pts, const EvalChunk* chunks, int nchunk, const void* Ltab, const void* V,
                      int64_t n, double* u, bool f32, hipStream_t s);

// ---- separable tensor stages ------------------------------------------------
// Every far-field tensor stage contracts the leading axis of a per-(slot,
// component) tensor X[k][r] and appends the new axis last: Y[r][n].  The 1D
// operators are centro-symmetric (symmetric Chebyshev nodes, +-m modes), so
// each stage folds the input pair (k, Nin-1-k) into even/odd parts, applies
// two half-size real matrices Me, Mo (interleaved per entry in `mat`,
// Nh x Kh) and unfolds the output pair (n, Nout-1-n).
enum StageMode {
    ST_SYM_REAL = 0,      // real -> real, y = U + W / U - W (interpolation)
    ST_OUT_HALF = 1,      // real nodes -> complex half modes, y = U - iW
    ST_OUT_FULL = 2,      // complex nodes -> complex +-m modes, y(+m) = U - iW, y(-m) = U + iW
    ST_IN_FULL = 3,       // complex +-m modes -> complex nodes, y = U + iW / U - iW
    ST_IN_HALF_REAL = 4   // complex half modes -> real nodes (accumulated), y = U - W / U + W
};
enum StageIO { IO_PLAIN = 0, IO_GATHER8 = 1, IO_SCATTER8 = 2 };
struct StageArgs {
    const void* X;
    long xstride;        // elements per (slot, component)
    const int* xmap;     // slot -> X slot (nullptr: identity)
    void* Y;
    long ystride;
    const int* ymap;
    int accumulate;      // add into Y instead of storing (real outputs)
    const double* mat;   // Nh x Kh pairs (Me, Mo)
    int Nin, Nout, in_off, out_off;
    int Kh, Nh;          // folded input / output half lengths
    int R;               // rows
    int nslots;
    int p;               // proxy order (gather / scatter addressing)
    const int* child_fid;// 8 per slot (gather / scatter)
    int f32;             // X and Y hold float (else double); arithmetic is FP64
    int ncomp = 3;       // components per slot (3; 6 for stresslet densities)
    int slot0 = 0;       // first slot of the launch (slots [slot0, nslots))
    int xbase = 0;       // X (without xmap) holds slots [xbase, ...): row slot - xbase
    int ybase = 0;       // the same for Y
    int rt_request = 0;  // requested rows per tile (16, 32, 64; 0 = by LDS footprint)
};
void launch_stage(int mode, int io, const StageArgs& a, hipStream_t s);

// plane-wave translation with the difference-kernel symbol (Step 3b)
struct RecvDesc {
    int slot;         // receiver slot in Psi
    int level;
    int ebeg, eend;   // entries in the entry arrays
};
// Phi / Psi hold complex float (f32) or complex double
// plain: the symbol was applied on the sending side (phases only here)
// e_pk: one int per entry, 32 * (sender slot) + 9 (o_x + 1) + 3 (o_y + 1) + (o_z + 1)
// with the sender's offset o from the receiver in box widths, each in {-1, 0, 1}
void launch_translate(int q, int n1, const RecvDesc* recv, int nrecv, const int* e_pk, const void* Phi,
                      const double* wdiff, void* Psi, bool f32, bool plain, hipStream_t s);
// stresslet difference symbol per sender: Phi6[slot][6][H] -> Phi3[slot][3][H] (x-major half spectrum)
void launch_stress_symbol(int q, int n1, int nsend, const int* send_level, const void* Phi6, const double* wdiff_t,
                          void* Phi3, bool f32, hipStream_t s);
// root symbol multiply: Psi[j][mz][my][mx] = w(|m|^2) (I - m m^T/|m|^2) Phi[j][mx][my][mz]
// one root per problem: Phi / Psi hold nroot consecutive [3][H] grids
void launch_root_symbol(int mh, int mf, int nroot, const void* Phi, const double* w, void* Psi, bool f32,
                        hipStream_t s);
// stresslet root symbol: Phi[nroot][6][H] x-major -> Psi[nroot][3][H] z-major, k = kscale m
void launch_root_symbol_t(int mh, int mf, int nroot, const void* Phi, const double* w, double kscale, void* Psi,
                          bool f32, hipStream_t s);

// near field (Step 4); the self term comes out of the r = 0 pair
struct NearLeaf {
    int64_t tstart, tend;
    int ebeg, eend;
    int level;
    int cbase;        // first 64-point chunk of the leaf
};
struct NearEntryDev {
    int64_t sstart, send;
    int cbase;        // first chunk of the source leaf
    int8_t sx, sy, sz, lambda;
};
struct NearWork {
    int leaf;         // -1: an empty item (padding)
    int chunk;        // target group index within the leaf (groups of 64/sg points)
};
// P and Q as monomials in t = 2s - 1, both padded with zero leading
// coefficients to nd terms (nd <= 24)
struct RadialPoly {
    int nd;
    double P[24], Q[24];
    double p_self;  // P at t = -1 (s = 0): the self pair's -S_M(0) f = -(2 / r_l) P(-1) f / (8 pi)
};
// sg: source lanes per target (1, 2, 4, 8); a wave holds 64/sg targets
// kernel 0 (Stokeslet): forces and outputs [nr][3][n]; nr in {1, 2, 4, 8}
// kernel 1 (stresslet): fs = (f, n) as [6][n], output [3][n], nr = 1;
// poly holds the stresslet's radial functions A (P) and D (Q)
// refine = false (Stokeslet, tol >= 1e-6 only): the hardware reciprocal square
// root without the Newton step (relative error below 6e-8)
// no_coincident (Stokeslet): no two distinct points coincide, so pairs at
// r = 0 are skipped and, with self_term (sources = targets), the self pair's
// term is added per target instead
void launch_near(int kernel, int sg, int nr, bool refine, bool no_coincident, bool self_term, const NearWork* work,
                 int nwork, const NearLeaf* leaves, const NearEntryDev* entries, const double* cbbox, const double* x,
                 const double* y, const double* z, const double* fs, int64_t n, const RadialPoly& poly, double* u,
                 hipStream_t s);
// flag = 1 if two of the points coincide (exact equality), else unchanged:
// points with equal Morton keys are compared within runs of the sorted keys
// (a run longer than 64 keys sets the flag without comparing)
void launch_find_coincident(const uint64_t* sorted_keys, const int* perm, const double* pts, int64_t n, int* flag,
                            hipStream_t s);

// pair counts of the near field: out[0] += evaluated pairs, out[1] += pairs in support
void launch_near_count(int sg, const NearWork* work, int nwork, const NearLeaf* leaves, const NearEntryDev* entries,
                       const double* cbbox, const double* x, const double* y, const double* z,
                       unsigned long long* out, hipStream_t s);

// brute-force residual sum over all source points (stage entry point), with
// the near field's pair routine; refine: Newton step on 1/r as in launch_near
void launch_residual_direct(const double* tx, const double* ty, const double* tz, int64_t m, const double* sx,
                            const double* sy, const double* sz, const double* sf, int64_t ns, double r_lambda,
                            bool refine, const RadialPoly& poly, double* u, hipStream_t s);
// the same for the residual stresslet, sf = (f, n) as [6][ns]
void launch_residual_direct_t(const double* tx, const double* ty, const double* tz, int64_t m, const double* sx,
                              const double* sy, const double* sz, const double* sf, int64_t ns, double r_lambda,
                              const RadialPoly& poly, double* u, hipStream_t s);

// out[j] = coef * sum of the root proxy charges (equals coef * net force)
// out[3r + j] = coef * sum_k Q[root_fid[r]][j][k]
void launch_sum_root(const void* Q, const int* root_fid, int nroot, int p3, double coef, double* out, bool f32,
                     hipStream_t s);
// periodic stresslet, per root r: out[4r] = sum f.n, out[4r+1+d] = sum x_d f.n
// (unit-box coordinates), from the root's 6-component proxy densities
void launch_stress_moment(const void* Q, const int* root_fid, int nroot, int p, const double* cheb_t, double* out,
                          bool f32, hipStream_t s);
// per point of problem b with input index o >= tofs (the points with an output):
// vel[o - tofs] = scale[b]^(sq ? 2 : 1) * (u + cst[3b..] + lin[4b+1..] - x lin[4b])
// (cst and lin may be NULL; x, y, z: sorted unit-box coordinates, read when lin is set)
void launch_finalize(const double* u, int64_t n, const int* perm, int64_t tofs, const int* pid, const double* scale,
                     int sq, const double* cst, const double* lin, const double* x, const double* y, const double* z,
                     double* vel, hipStream_t s);
// zero `bytes` (a multiple of 4) at p
void launch_zero(void* p, size_t bytes, hipStream_t s);

// Fixed device workspace (no allocation): its size in doubles, and its device
// address on the current GPU (looked up once per device).
size_t scratch_doubles();
hipError_t scratch_address(double** out);

}  // namespace dmk
