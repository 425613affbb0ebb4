// C ABI: plan construction (tree, lists, buffers) and the evaluation pass.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dmk_stokes.h"
#include "dmk_kernels.hpp"
#include "ewald_kernels.hpp"
#include "kernel_math.hpp"
#include "tree.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(DMK_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr double kPi = 3.14159265358979323846;

bool is_device_ptr(const void* p)
{
    if (!p)
        return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Newton step on the Stokeslet near field's reciprocal square root: the
// unrefined hardware estimate (relative error below 6e-8) is used where the
// row's tolerance is 1e-6 or looser (and the fits are the shortest compiled
// length); the stresslet (1/r^5) always refines.
bool stokes_near_refine(double row_tol)
{
    return !(row_tol >= 1e-6 * (1 - 1e-9));
}

// Process-wide cache of device buffers: destroyed plans hand their buffers
// back and later plans reuse any cached block of at least the requested size
// (and at most twice it).  Sizes are rounded to 2 MiB above 1 MiB.
struct Pool {
    std::mutex mu;
    std::multimap<size_t, std::pair<int, void*>> free_blocks;  // size -> (device, ptr)
    static size_t round(size_t b)
    {
        const size_t g = (size_t)2 << 20;
        return b > ((size_t)1 << 20) ? (b + g - 1) / g * g : (b + 255) / 256 * 256;
    }
    void* get(size_t bytes, size_t* got)
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        const size_t want = round(bytes);
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = free_blocks.lower_bound(want); it != free_blocks.end() && it->first <= 2 * want; ++it) {
                if (it->second.first != dev)
                    continue;
                void* p = it->second.second;
                *got = it->first;
                free_blocks.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            release_all();
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        *got = want;
        return p;
    }
    void put(void* p, size_t bytes)
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lk(mu);
        free_blocks.emplace(bytes, std::make_pair(dev, p));
    }
    void release_all()
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : free_blocks)
            (void)hipFree(kv.second.second);
        free_blocks.clear();
    }
};
Pool& pool()
{
    static Pool* P = new Pool();
    return *P;
}

// device allocation registry with an optional cap
struct DevMem {
    std::vector<std::pair<void*, size_t>> ptrs;
    size_t total = 0, cap = 0;
    bool oom = false;
    template <class T>
    T* alloc(size_t count)
    {
        if (count == 0)
            count = 1;
        const size_t bytes = count * sizeof(T);
        if (cap && total + bytes > cap) {
            oom = true;
            return nullptr;
        }
        size_t got = 0;
        void* p = pool().get(bytes, &got);
        if (!p) {
            oom = true;
            return nullptr;
        }
        ptrs.emplace_back(p, got);
        total += bytes;
        return (T*)p;
    }
    ~DevMem()
    {
        for (auto& pr : ptrs)
            pool().put(pr.first, pr.second);
    }
};

// Stream-ordered host -> device copy; the caller keeps `src` alive until the
// stream is synchronised (build_plan synchronises before returning).
template <class T>
hipError_t upload(T* dst, const std::vector<T>& src, hipStream_t st)
{
    if (src.empty())
        return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// Idle FFT plan pairs of destroyed spectral Ewald plans, by (device, grid
// size): creating a 3D FFT plan costs tens of milliseconds, so a new plan of
// the same grid reuses one.  A pair belongs to one live plan at a time.
struct FftPair {
    hipfftHandle fwd, inv;
};
std::mutex g_fft_mu;
std::multimap<std::pair<int, int>, FftPair>& fft_pool()
{
    static auto* m = new std::multimap<std::pair<int, int>, FftPair>();
    return *m;
}

// The library's own stream for plans built with DMK_FLAG_CONCURRENT_PLAN
// (non-blocking: it does not wait for work on the null stream; default
// priority).  One per device, created on first use.
hipStream_t plan_stream()
{
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it != streams.end())
        return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return nullptr;
    streams[dev] = s;
    return s;
}

}  // namespace

struct dmk_plan_s {
    dmk::Params prm;
    const dmk::Tables* tab = nullptr;
    hipStream_t stream = nullptr;
    int precision = 0;
    int64_t n = 0;
    bool periodic = false;
    double center[3] = {0, 0, 0}, box_len = 1.0;
    dmk::Tree tree;
    DevMem mem;
    double plan_ms = 0;
    double plan_phase[6] = {0, 0, 0, 0, 0, 0};

    // points
    int* perm = nullptr;       // sorted position -> caller index
    double *x = nullptr, *y = nullptr, *z = nullptr;
    // tables on device
    double *cheb_t = nullptr, *cheb_w = nullptr;
    double *merge_mat = nullptr, *interp_mat = nullptr;
    double *pw_out = nullptr, *pw_in_full = nullptr, *pw_in_half = nullptr;
    double *r_out = nullptr, *r_in_full = nullptr, *r_in_half = nullptr;
    double *wdiff = nullptr, *wroot = nullptr;
    int root_mh = 0, root_mf = 0;
    dmk::RadialPoly poly;
    // far-field structure
    int nf = 0;                       // non-empty boxes (far-field slots)
    // separate targets: input indices < nsrc are sources, indices >= tofs have
    // an output (a plan with targets = sources: nsrc = n, tofs = 0)
    int64_t nsrc = 0, tofs = 0, nout = 0;
    int64_t near_listed = 0;          // sum over near entries of |targets| * |sources|
    dmk::LeafDesc* leaves_src = nullptr;  // leaves over their source points (anterpolation)
    // independent problems of a batched plan (one problem for dmk_stokes_plan)
    int nprob = 1;
    std::vector<int64_t> offsets;     // point ranges of the problems, caller's order
    int64_t* d_off = nullptr;
    int* pid = nullptr;               // problem of each point (NULL for one problem)
    double* geo = nullptr;            // per problem: centre (3), 1 / cube side
    double* scale = nullptr;          // per problem: 1 / cube side (velocity scaling)
    std::vector<double> h_center, h_len;
    std::vector<int> root_fid;        // far-field slot of each problem's root
    int* d_root_fid = nullptr;
    std::vector<int> box_fid;         // box id -> fid or -1
    dmk::LeafDesc* leaves = nullptr;  // non-empty leaves
    int nleaf = 0;
    void* Ltab = nullptr;             // Lagrange values of the points on their leaf grids (float when f32)
    dmk::EvalChunk* echunks = nullptr;
    int n_echunk = 0;
    struct LevelLists {
        int nparent = 0;
        int* child_fid = nullptr;     // 8 per parent
        int* parent_fid = nullptr;
    };
    std::vector<LevelLists> lev;
    int nsend = 0, nrecv = 0;
    int* send_fid = nullptr;          // sender slot -> fid
    int* recv_fid = nullptr;          // receiver slot -> fid
    dmk::RecvDesc* recv = nullptr;
    int* e_pk = nullptr;  // translation entries: 32 * sender slot + offset code
    // near field
    dmk::NearLeaf* nleaves = nullptr;
    dmk::NearEntryDev* nentries = nullptr;
    dmk::NearWork* nwork = nullptr;
    int n_nwork = 0;
    int near_sg = 4;                  // source lanes per target in the near field
    double* cbbox = nullptr;
    // work buffers
    double* fs = nullptr;             // sorted forces [3][n]
    double* u = nullptr;              // sorted velocities [3][n]
    // far-field buffers hold double (FP64 plans) or float (mixed precision)
    bool f32 = false;
    size_t es = 8;                    // bytes per real element of Q, V, Phi, Psi, s1, s2
    void *Q = nullptr, *V = nullptr;
    void *Phi = nullptr, *Psi = nullptr;
    void *s1 = nullptr, *s2 = nullptr;
    void *phi_root = nullptr, *psi_root = nullptr;
    // stresslet plans: 6 density components in (Q, Phi, root Phi), the
    // sending-side symbol writes 3 velocity components to Phi3
    int kern = DMK_KERNEL_STOKESLET;
    int nc_in = 3;
    void* Phi3 = nullptr;
    int* send_level = nullptr;        // sender slot -> level
    // stage pipelines run over slot chunks so that the scratch buffers s1, s2
    // hold one chunk: ck_slots merge / interpolation slots, ck_pw plane-wave
    // slots or ck_roots roots at a time
    int ck_slots = 1, ck_pw = 1, ck_roots = 1;
    bool ck_on = false;
    int ck0 = 0, ck1 = 0;
    // single-level spectral Ewald plans (DMK_METHOD_EWALD)
    int method = DMK_METHOD_DMK;
    dmk::EwaldGrid eg;
    dmk::GridPoly gpoly;
    int64_t* tile_start = nullptr;    // 8^Lt + 1 point ranges of the spreading tiles
    double* egrid = nullptr;          // [3][M^3] real grid
    double2* espec = nullptr;         // [3][M][M][M/2+1] half spectrum
    double *eghat = nullptr, *ewsym = nullptr;
    hipfftHandle fft_fwd = 0, fft_inv = 0;
    bool fft_made = false;
    int64_t n_cells_nonempty = 0;
    double* cst = nullptr;
    size_t H = 0, Hroot = 0;
    std::vector<int> leaf_box;        // leaf index (all leaves) -> box id
    // phase timing
    bool timing = false;
    // ev[0..8]: far-field phase boundaries (first vector of a batch); ev[11]
    // to ev[9]: the near field (with the force gather); ev[12] to ev[10]:
    // finalize.  The near field runs first, so an evaluation ends with many
    // short far-field launches, between which the work of a plan being built
    // concurrently on another stream gets onto the device.
    hipEvent_t ev[DMK_NUM_PHASES + 3] = {};
    int rhs_batch = 8;                // force vectors per near-field pass
    bool concurrent = false;          // build on the library's plan stream
    // DMK_FLAG_GRAPH: evaluation captured once per (forces, n_rhs, velocities)
    bool use_graph = false;
    bool leaf_order = true;           // compact groups inside leaves (near-field pruning)
    bool host_tree = false;           // octree and lists built on the host (reference construction)
    bool near_refine = true;          // Newton step on the near field's reciprocal square root
    int stage_rows = 0;               // requested rows per stage tile (0 = by LDS footprint)
    int eval_pts = 0;                 // points per leaf-evaluation block
    bool no_coincident = false;       // no two distinct points coincide (near field skips r = 0 pairs)
    int h_coincident = 1;             // host copy of the plan-time coincidence flag
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double* g_forces = nullptr;
    double* g_vel = nullptr;
    int g_nrhs = 0;
    hipEvent_t done = nullptr;        // end of the most recent eval on `stream`
    bool done_recorded = false;
    bool ev_recorded = false;
    ~dmk_plan_s()
    {
        for (auto& e : ev)
            if (e)
                (void)hipEventDestroy(e);
        if (done)
            (void)hipEventDestroy(done);
        if (gexec)
            (void)hipGraphExecDestroy(gexec);
        if (graph)
            (void)hipGraphDestroy(graph);
        if (cap_stream)
            (void)hipStreamDestroy(cap_stream);
        if (fft_made) {
            int dev = 0;
            (void)hipGetDevice(&dev);
            std::lock_guard<std::mutex> lk(g_fft_mu);
            fft_pool().emplace(std::make_pair(dev, eg.M), FftPair{fft_fwd, fft_inv});
        }
    }
};

namespace {

int validate_common(int dim, double tol, const dmk_opts* opts)
{
    if (dim != 3)
        return fail(DMK_ERR_UNSUPPORTED, "only dim = 3 is supported");
    if (!(tol >= 1e-12 * (1 - 1e-9) && tol <= 1e-3 * (1 + 1e-9)))
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    if (opts) {
        if (opts->precision != DMK_PREC_FP64 && opts->precision != DMK_PREC_MIXED)
            return fail(DMK_ERR_ARG, "unknown precision");
        // FP32 storage of the far field leaves relative errors near 1.2e-7
        if (opts->precision == DMK_PREC_MIXED && tol < 1e-6 * (1 - 1e-9))
            return fail(DMK_ERR_TOL, "mixed precision needs tol >= 1e-6");
        if (opts->leaf_size < 0)
            return fail(DMK_ERR_ARG, "leaf_size must be >= 0");
        if (opts->near_lanes != 0 && opts->near_lanes != 1 && opts->near_lanes != 2 && opts->near_lanes != 4 &&
            opts->near_lanes != 8)
            return fail(DMK_ERR_ARG, "near_lanes must be 0, 1, 2, 4 or 8");
        if (opts->q != 0 && (opts->q < 4 || opts->q > 40))
            return fail(DMK_ERR_ARG, "q must be 0 or in [4, 40]");
        if (opts->rhs_batch != 0 && opts->rhs_batch != 1 && opts->rhs_batch != 2 && opts->rhs_batch != 4 &&
            opts->rhs_batch != 8)
            return fail(DMK_ERR_ARG, "rhs_batch must be 0, 1, 2, 4 or 8");
        if (opts->p != 0 && !dmk::p_supported(opts->p))
            return fail(DMK_ERR_ARG, "p must be 0 or one of 11, 12, 14, 16, 20, 22, 23, 26, 28, 30, 33, 36, 40, 43, 44, 48");
        if (opts->stage_rows != 0 && opts->stage_rows != 16 && opts->stage_rows != 32 && opts->stage_rows != 64)
            return fail(DMK_ERR_ARG, "stage_rows must be 0, 16, 32 or 64");
        if (opts->eval_points != 0 && opts->eval_points != 128 && opts->eval_points != 256)
            return fail(DMK_ERR_ARG, "eval_points must be 0, 128 or 256");
        if (opts->window != DMK_WINDOW_PROLATE && opts->window != DMK_WINDOW_GAUSSIAN)
            return fail(DMK_ERR_ARG, "unknown window");
        if (opts->window == DMK_WINDOW_GAUSSIAN && tol < 1e-6 * (1 - 1e-9))
            return fail(DMK_ERR_TOL, "the Gaussian window is offered for tol >= 1e-6");
        if (opts->kernel != DMK_KERNEL_STOKESLET && opts->kernel != DMK_KERNEL_STRESSLET)
            return fail(DMK_ERR_ARG, "unknown kernel");
        if (opts->method != DMK_METHOD_DMK && opts->method != DMK_METHOD_EWALD)
            return fail(DMK_ERR_ARG, "unknown method");
        if (opts->method == DMK_METHOD_EWALD) {
            if (opts->kernel != DMK_KERNEL_STOKESLET || opts->window != DMK_WINDOW_PROLATE ||
                opts->precision != DMK_PREC_FP64)
                return fail(DMK_ERR_UNSUPPORTED, "the spectral Ewald method takes the FP64 prolate Stokeslet only");
            if (opts->flags & DMK_FLAG_GRAPH)
                return fail(DMK_ERR_UNSUPPORTED, "DMK_FLAG_GRAPH is not available for the spectral Ewald method");
            if (tol < 1e-9 * (1 - 1e-9))
                return fail(DMK_ERR_TOL, "the spectral Ewald method is offered for tol >= 1e-9");
        }
        if (opts->kernel == DMK_KERNEL_STRESSLET) {
            if (opts->window != DMK_WINDOW_PROLATE)
                return fail(DMK_ERR_UNSUPPORTED, "the stresslet is offered with the prolate window only");
            if (opts->flags & DMK_FLAG_GRAPH)
                return fail(DMK_ERR_UNSUPPORTED, "DMK_FLAG_GRAPH is not available for the stresslet");
        }
    }
    return DMK_OK;
}

// One separable stage over `nslots` (slot, component) tensors.
void stage(dmk_plan_t P, int mode, int io, const void* X, long xs, const int* xmap, void* Y, long ys,
           const int* ymap, int accumulate, const double* mat, int Nin, int Nout, int in_off, int out_off, int Kh,
           int Nh, int R, int nslots, const int* child_fid = nullptr, int nc = 3)
{
    dmk::StageArgs a;
    a.X = X;
    a.xstride = xs;
    a.xmap = xmap;
    a.Y = Y;
    a.ystride = ys;
    a.ymap = ymap;
    a.accumulate = accumulate;
    a.mat = mat;
    a.Nin = Nin;
    a.Nout = Nout;
    a.in_off = in_off;
    a.out_off = out_off;
    a.Kh = Kh;
    a.Nh = Nh;
    a.R = R;
    a.nslots = nslots;
    a.p = P->prm.p;
    a.child_fid = child_fid;
    a.f32 = P->f32 ? 1 : 0;
    a.ncomp = nc;
    a.rt_request = P->stage_rows;
    if (P->ck_on) {
        // one chunk of a pipeline: slots [ck0, ck1); the scratch buffers hold
        // only this chunk's rows
        a.slot0 = P->ck0;
        a.nslots = P->ck1;
        a.xbase = (X == P->s1 || X == P->s2) ? P->ck0 : 0;
        a.ybase = (Y == P->s1 || Y == P->s2) ? P->ck0 : 0;
    }
    dmk::launch_stage(mode, io, a, P->stream);
}

// Plane-wave matrices of one grid on the device.
struct PWDev {
    int M = 0;
    double *out = nullptr, *in_full = nullptr, *in_half = nullptr;
};

// Chebyshev series in t -> monomial coefficients in t (long double), both
// padded to a kernel instantiation length
bool make_poly(const dmk::Tables& TB, dmk::RadialPoly* poly)
{
    const int nmax = (int)std::max(TB.fits.P.a.size(), TB.fits.Q.a.size());
    const int nd = nmax <= 14 ? 14 : nmax <= 18 ? 18 : nmax <= 21 ? 21 : 24;
    if (nmax > 24)
        return false;
    auto conv = [&](const std::vector<double>& a, double* out) {
        const int n = (int)a.size();
        std::vector<long double> tkm1(nd, 0.0L), tk(nd, 0.0L), acc(nd, 0.0L);
        tkm1[0] = 1.0L;  // T_0
        if (nd > 1)
            tk[1] = 1.0L;  // T_1
        for (int k = 0; k < n; ++k) {
            const std::vector<long double>& T = (k == 0) ? tkm1 : tk;
            for (int j = 0; j < nd; ++j)
                acc[j] += (long double)a[k] * T[j];
            if (k >= 1) {  // advance: T_{k+1} = 2 t T_k - T_{k-1}
                std::vector<long double> nx(nd, 0.0L);
                for (int j = 0; j + 1 < nd; ++j)
                    nx[j + 1] += 2.0L * tk[j];
                for (int j = 0; j < nd; ++j)
                    nx[j] -= tkm1[j];
                tkm1 = tk;
                tk = nx;
            }
        }
        for (int j = 0; j < nd; ++j)
            out[j] = (double)acc[j];
    };
    poly->nd = nd;
    conv(TB.fits.P.a, poly->P);
    conv(TB.fits.Q.a, poly->Q);
    // P at t = -1: T_k(-1) = (-1)^k
    long double ps = 0.0L;
    for (size_t k = 0; k < TB.fits.P.a.size(); ++k)
        ps += (k % 2 ? -1.0L : 1.0L) * (long double)TB.fits.P.a[k];
    poly->p_self = (double)ps;
    return true;
}

// Near-field work items in launch order.  Workgroups go to the 8 XCDs of the
// device in turn (workgroup g to XCD g % 8), and each XCD has its own L2.  The
// leaves, in Morton order, are cut into 8 * kPieces runs of about equal cost
// (listed pairs); run r goes to XCD r % 8, so all target groups of a leaf and
// most of its neighbours' sources meet in one L2, and the XCDs get equal work.
// Each XCD's items sit at positions x, x + 8, x + 16, ...; the shorter lists
// are padded with empty items (leaf -1).
std::vector<dmk::NearWork> xcd_work_order(const std::vector<dmk::NearWork>& items, const std::vector<double>& cost)
{
    constexpr int kXcd = 8, kPieces = 16;
    const size_t nl = cost.size();
    if (items.empty() || nl == 0)
        return items;
    double total = 0;
    for (double c : cost)
        total += c;
    std::vector<int> xcd_of(nl);
    double run = 0;
    for (size_t l = 0; l < nl; ++l) {
        // run index of the leaf's cost midpoint
        const double mid = run + 0.5 * cost[l];
        const int r = total > 0 ? std::min(kXcd * kPieces - 1, (int)(mid / total * kXcd * kPieces)) : (int)(l % kXcd);
        xcd_of[l] = r % kXcd;
        run += cost[l];
    }
    std::vector<std::vector<dmk::NearWork>> lists(kXcd);
    for (const dmk::NearWork& w : items)
        lists[xcd_of[w.leaf]].push_back(w);
    size_t len = 0;
    for (const auto& v : lists)
        len = std::max(len, v.size());
    std::vector<dmk::NearWork> out(kXcd * len, dmk::NearWork{-1, 0});
    for (int x = 0; x < kXcd; ++x)
        for (size_t k = 0; k < lists[x].size(); ++k)
            out[kXcd * k + x] = lists[x][k];
    return out;
}

// Morton code at a level <-> integer cell coordinates (digit 4 bx + 2 by + bz)
uint64_t cell_code(int64_t ix, int64_t iy, int64_t iz, int level)
{
    uint64_t c = 0;
    for (int b = level - 1; b >= 0; --b)
        c = (c << 3) | (uint64_t)((((ix >> b) & 1) << 2) | (((iy >> b) & 1) << 1) | ((iz >> b) & 1));
    return c;
}

// The rest of a spectral Ewald plan once the points are sorted: split level,
// grid and gridding kernel, tile and cell ranges from the sorted keys, the
// near lists between cells of the split level (27 neighbours through the
// periodic wrap, residual at that level), buffers and FFT plans.
int build_ewald(dmk_plan_t P, const std::vector<uint64_t>& keys, hipStream_t st)
{
    using namespace dmk;
    const int64_t n = P->n;
    int L = 1;
    while (L < 8 && (double)n / (double)(1ll << (3 * L)) > (double)P->prm.ns)
        ++L;
    if (!ewald_grid(P->prm, L, &P->eg))
        return fail(DMK_ERR_UNSUPPORTED, "no spectral Ewald grid for this tolerance and size");
    const EwaldGrid& E = P->eg;
    if (E.M > 768)
        return fail(DMK_ERR_UNSUPPORTED, "spectral Ewald grid above 768^3 (use the DMK method)");
    if ((int)E.g_cheb.size() > kGridTerms)
        return fail(DMK_ERR_UNSUPPORTED, "gridding kernel series too long");
    P->gpoly.nc = (int)E.g_cheb.size();
    for (int k = 0; k < kGridTerms; ++k)
        P->gpoly.a[k] = k < P->gpoly.nc ? E.g_cheb[k] : 0.0;
    auto ranges = [&](int level) {
        const int64_t nc = 1ll << (3 * level);
        std::vector<int64_t> r(nc + 1);
        const int sh = 3 * (kKeyBits - level);
        for (int64_t c = 0; c <= nc; ++c)
            r[c] = std::lower_bound(keys.begin(), keys.end(), (uint64_t)c << sh) - keys.begin();
        return r;
    };
    const std::vector<int64_t> ts = ranges(E.Lt);
    const std::vector<int64_t> cs = ranges(L);
    // near field: cells of side 2^-L, residual at level L
    const int NC = 1 << L;
    std::vector<int> cbase((size_t)1 << (3 * L), -1);
    std::vector<int64_t> cstart;
    std::vector<int> clen;
    for (size_t c = 0; c + 1 < cs.size(); ++c) {
        if (cs[c + 1] == cs[c])
            continue;
        cbase[c] = (int)cstart.size();
        for (int64_t a = cs[c]; a < cs[c + 1]; a += 64) {
            cstart.push_back(a);
            clen.push_back((int)std::min<int64_t>(64, cs[c + 1] - a));
        }
    }
    std::vector<NearLeaf> nlv;
    std::vector<NearEntryDev> nent;
    std::vector<NearWork> nwk;
    std::vector<double> cell_cost;
    P->near_listed = 0;
    P->n_cells_nonempty = 0;
    for (int64_t ix = 0; ix < NC; ++ix)
        for (int64_t iy = 0; iy < NC; ++iy)
            for (int64_t iz = 0; iz < NC; ++iz) {
                const uint64_t c = cell_code(ix, iy, iz, L);
                if (cs[c + 1] == cs[c])
                    continue;
                ++P->n_cells_nonempty;
                const int64_t listed0 = P->near_listed;
                NearLeaf T;
                T.tstart = cs[c];
                T.tend = cs[c + 1];
                T.level = L;
                T.cbase = cbase[c];
                T.ebeg = (int)nent.size();
                for (int d = 0; d < 27; ++d) {
                    const int64_t o[3] = {d / 9 - 1, (d / 3) % 3 - 1, d % 3 - 1};
                    const int64_t v[3] = {ix + o[0], iy + o[1], iz + o[2]};
                    int64_t w[3];
                    int8_t sh[3];
                    for (int k = 0; k < 3; ++k) {
                        w[k] = v[k];
                        sh[k] = 0;
                        if (w[k] < 0) {
                            w[k] += NC;
                            sh[k] = -1;
                        } else if (w[k] >= NC) {
                            w[k] -= NC;
                            sh[k] = 1;
                        }
                    }
                    const uint64_t sc = cell_code(w[0], w[1], w[2], L);
                    if (cs[sc + 1] == cs[sc])
                        continue;
                    NearEntryDev e;
                    e.sstart = cs[sc];
                    e.send = cs[sc + 1];
                    e.cbase = cbase[sc];
                    e.sx = sh[0];
                    e.sy = sh[1];
                    e.sz = sh[2];
                    e.lambda = (int8_t)L;
                    nent.push_back(e);
                    P->near_listed += (T.tend - T.tstart) * (e.send - e.sstart);
                }
                T.eend = (int)nent.size();
                const int li = (int)nlv.size();
                const int tg = 64 / P->near_sg;
                const int nch = (int)((T.tend - T.tstart + tg - 1) / tg);
                for (int k = 0; k < nch; ++k)
                    nwk.push_back(NearWork{li, k});
                nlv.push_back(T);
                cell_cost.push_back((double)(P->near_listed - listed0));
            }
    nwk = xcd_work_order(nwk, cell_cost);
    P->n_nwork = (int)nwk.size();
    P->nleaves = P->mem.alloc<NearLeaf>(nlv.size());
    P->nentries = P->mem.alloc<NearEntryDev>(nent.size());
    P->nwork = P->mem.alloc<NearWork>(nwk.size());
    P->cbbox = P->mem.alloc<double>(cstart.size() * 6);
    int64_t* d_cstart = P->mem.alloc<int64_t>(cstart.size());
    int* d_clen = P->mem.alloc<int>(clen.size());
    P->tile_start = P->mem.alloc<int64_t>(ts.size());
    const size_t M = E.M, M3 = M * M * M, H = M * M * (M / 2 + 1);
    P->egrid = P->mem.alloc<double>(3 * M3);
    P->espec = P->mem.alloc<double2>(3 * H);
    P->eghat = P->mem.alloc<double>(E.ghat.size());
    P->ewsym = P->mem.alloc<double>(E.wsym.size());
    P->fs = P->mem.alloc<double>(3 * (size_t)n);
    P->u = P->mem.alloc<double>(3 * (size_t)n);
    if (P->mem.oom)
        return fail(DMK_ERR_OOM, "device allocation failed (or above mem_cap_bytes)");
    HIPCHK(upload(P->nleaves, nlv, st));
    HIPCHK(upload(P->nentries, nent, st));
    HIPCHK(upload(P->nwork, nwk, st));
    HIPCHK(upload(d_cstart, cstart, st));
    HIPCHK(upload(d_clen, clen, st));
    HIPCHK(upload(P->tile_start, ts, st));
    HIPCHK(upload(P->eghat, E.ghat, st));
    HIPCHK(upload(P->ewsym, E.wsym, st));
    launch_chunk_bbox(P->x, P->y, P->z, d_cstart, d_clen, (int)cstart.size(), P->cbbox, st);
    if (!make_poly(*P->tab, &P->poly))
        return fail(DMK_ERR_UNSUPPORTED, "radial fit degree too high");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_fft_mu);
        auto it = fft_pool().find(std::make_pair(dev, E.M));
        if (it != fft_pool().end()) {
            P->fft_fwd = it->second.fwd;
            P->fft_inv = it->second.inv;
            fft_pool().erase(it);
            P->fft_made = true;
        }
    }
    if (!P->fft_made) {
        int dims[3] = {(int)M, (int)M, (int)M};
        if (hipfftPlanMany(&P->fft_fwd, 3, dims, nullptr, 1, (int)M3, nullptr, 1, (int)H, HIPFFT_D2Z, 3) !=
            HIPFFT_SUCCESS)
            return fail(DMK_ERR_HIP, "hipfftPlanMany (forward) failed");
        if (hipfftPlanMany(&P->fft_inv, 3, dims, nullptr, 1, (int)H, nullptr, 1, (int)M3, HIPFFT_Z2D, 3) !=
            HIPFFT_SUCCESS) {
            (void)hipfftDestroy(P->fft_fwd);
            return fail(DMK_ERR_HIP, "hipfftPlanMany (inverse) failed");
        }
        P->fft_made = true;
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    return DMK_OK;
}

int build_plan(dmk_plan_t P, const double* points)
{
    using namespace dmk;
    hipStream_t st = P->stream;
    if (P->concurrent) {
        st = plan_stream();
        if (!st)
            return fail(DMK_ERR_HIP, "could not create the plan stream");
    }
    auto tlast = std::chrono::steady_clock::now();
    auto lap = [&](int k) {
        const auto now = std::chrono::steady_clock::now();
        P->plan_phase[k] += std::chrono::duration<double, std::milli>(now - tlast).count();
        tlast = now;
    };
    const int64_t n = P->n;
    const int np = P->nprob;
    // ---- bounding boxes and finiteness (per problem) ----
    std::vector<double> hp;
    if (np == 1) {
        const int nblk = (int)std::min<int64_t>(1024, (n + 255) / 256);
        double* part = P->mem.alloc<double>((size_t)nblk * 8);
        if (!part)
            return fail(DMK_ERR_OOM, "device allocation failed");
        launch_bbox(points, n, part, nblk, st);
        std::vector<double> hb((size_t)nblk * 8);
        HIPCHK(hipMemcpyAsync(hb.data(), part, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        hp.assign(8, 0.0);
        for (int d = 0; d < 3; ++d) {
            hp[d] = 1e300;
            hp[3 + d] = -1e300;
        }
        for (int b = 0; b < nblk; ++b) {
            for (int d = 0; d < 3; ++d) {
                hp[d] = std::min(hp[d], hb[8 * b + d]);
                hp[3 + d] = std::max(hp[3 + d], hb[8 * b + 3 + d]);
            }
            hp[6] += hb[8 * b + 6];
        }
    } else {
        P->d_off = P->mem.alloc<int64_t>(np + 1);
        double* part = P->mem.alloc<double>((size_t)np * 8);
        P->pid = P->mem.alloc<int>(n);
        if (P->mem.oom)
            return fail(DMK_ERR_OOM, "device allocation failed");
        HIPCHK(upload(P->d_off, P->offsets, st));
        launch_bbox_seg(points, P->d_off, np, part, st);
        launch_fill_pid(P->d_off, np, n, P->pid, st);
        hp.resize((size_t)np * 8);
        HIPCHK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    P->h_center.assign(3 * (size_t)np, 0.5);
    P->h_len.assign(np, 1.0);
    std::vector<double> geo(4 * (size_t)np), scl(np);
    for (int b = 0; b < np; ++b) {
        const double* lo = &hp[8 * b];
        const double* hi = &hp[8 * b + 3];
        if (hp[8 * b + 6] > 0)
            return fail(DMK_ERR_NONFINITE, "points contain NaN or Inf");
        if (P->periodic) {
            for (int d = 0; d < 3; ++d)
                if (lo[d] < 0.0 || hi[d] >= 1.0)
                    return fail(DMK_ERR_DOMAIN, "periodic points must lie in [0,1)^3");
        } else {
            double ext = 0;
            for (int d = 0; d < 3; ++d) {
                P->h_center[3 * b + d] = 0.5 * (lo[d] + hi[d]);
                ext = std::max(ext, hi[d] - lo[d]);
            }
            if (ext <= 0)
                ext = 1.0;
            // slightly larger cube so that all unit coordinates lie in [-1/2, 1/2)
            P->h_len[b] = ext * (1.0 + 1e-9);
        }
        for (int d = 0; d < 3; ++d)
            geo[4 * b + d] = P->h_center[3 * b + d];
        geo[4 * b + 3] = 1.0 / P->h_len[b];
        scl[b] = 1.0 / P->h_len[b];
    }
    for (int d = 0; d < 3; ++d)
        P->center[d] = P->h_center[d];
    P->box_len = P->h_len[0];
    P->geo = P->mem.alloc<double>(geo.size());
    P->scale = P->mem.alloc<double>(scl.size());
    if (P->mem.oom)
        return fail(DMK_ERR_OOM, "device allocation failed");
    HIPCHK(upload(P->geo, geo, st));
    HIPCHK(upload(P->scale, scl, st));
    lap(0);
    // ---- Morton keys and sort (within each problem) ----
    uint64_t* k0 = P->mem.alloc<uint64_t>(n);
    uint64_t* k1 = P->mem.alloc<uint64_t>(n);
    int* i0 = P->mem.alloc<int>(n);
    P->perm = P->mem.alloc<int>(n);
    const size_t tb = np == 1 ? sort_temp_bytes(n) : seg_sort_temp_bytes(n, np);
    void* tmp = P->mem.alloc<char>(tb);
    if (P->mem.oom)
        return fail(DMK_ERR_OOM, "device allocation failed");
    launch_morton(points, n, P->pid, P->geo, k0, i0, st);
    if (np == 1)
        launch_sort(tmp, tb, k0, k1, i0, P->perm, n, 3 * kKeyBits, st);
    else
        launch_seg_sort(tmp, tb, k0, k1, i0, P->perm, n, np, P->pid, 3 * kKeyBits, st);
    HIPCHK(hipGetLastError());
    // coincident points: the flag reaches the host with the tree (the build synchronises st)
    int* d_coinc = P->mem.alloc<int>(1);
    if (!d_coinc)
        return fail(DMK_ERR_OOM, "device allocation failed");
    launch_zero(d_coinc, sizeof(int), st);
    launch_find_coincident(k1, P->perm, points, n, d_coinc, st);
    HIPCHK(hipMemcpyAsync(&P->h_coincident, d_coinc, sizeof(int), hipMemcpyDeviceToHost, st));
    std::vector<uint64_t> keys;
    if (P->method == DMK_METHOD_EWALD || P->host_tree) {
        keys.resize(n);
        HIPCHK(hipMemcpyAsync(keys.data(), k1, n * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    lap(1);
    if (P->method == DMK_METHOD_EWALD) {
        P->x = P->mem.alloc<double>(n);
        P->y = P->mem.alloc<double>(n);
        P->z = P->mem.alloc<double>(n);
        if (P->mem.oom)
            return fail(DMK_ERR_OOM, "device allocation failed");
        launch_gather_points(points, n, P->perm, P->pid, P->geo, P->x, P->y, P->z, st);
        const int rc = build_ewald(P, keys, st);
        lap(2);
        return rc;
    }
    // ---- tree (a forest of one octree per problem), built on the device ----
    const int ns = P->prm.ns;
    std::vector<int> roots(np);
    for (int b = 0; b < np; ++b)
        roots[b] = b;  // level 0 holds the roots in problem order
    bool host = P->host_tree;
    if (!host) {
        const int64_t* d_off = P->d_off;
        if (np == 1) {
            int64_t* o = P->mem.alloc<int64_t>(2);
            if (!o)
                return fail(DMK_ERR_OOM, "device allocation failed");
            const std::vector<int64_t> h_off = {0, n};
            HIPCHK(upload(o, h_off, st));  // h_off outlives the build, which synchronises st
            d_off = o;
        }
        DevMem scratch;
        auto alloc = [](void* ctx, size_t bytes) -> void* { return static_cast<DevMem*>(ctx)->alloc<char>(bytes); };
        std::string err;
        const int rc = build_tree_device(k1, d_off, np, n, ns, P->periodic, alloc, &scratch, st, &P->tree, &err);
        if (rc == DMK_TREE_UNSUPPORTED)
            host = true;  // a forest too deep for the device construction's packed keys
        else if (rc != 0)
            return fail(rc == DMK_TREE_OOM ? DMK_ERR_OOM : DMK_ERR_HIP, "octree: " + err);
    }
    if (host) {
        // the sequential construction from the same sorted keys
        if (keys.empty()) {
            keys.resize(n);
            HIPCHK(hipMemcpyAsync(keys.data(), k1, n * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        if (np == 1) {
            build_tree(keys.data(), n, ns, P->periodic, &P->tree);
        } else {
            std::vector<Tree> parts(np);
#pragma omp parallel for schedule(dynamic)
            for (int b = 0; b < np; ++b)
                build_tree(keys.data() + P->offsets[b], P->offsets[b + 1] - P->offsets[b], ns, P->periodic,
                           &parts[b]);
            merge_forest(parts, P->offsets, &P->tree, &roots);
        }
    }
    HIPCHK(hipStreamSynchronize(st));  // (already reached by the tree build)
    P->no_coincident = P->h_coincident == 0;
    lap(2);
    const Tree& T = P->tree;
    // ---- separate targets: sources first within every leaf ----
    std::vector<int64_t> box_nsrc(T.boxes.size(), 0);
    if (P->nsrc < n) {
        std::vector<int> hperm(n);
        HIPCHK(hipMemcpyAsync(hperm.data(), P->perm, n * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (size_t i = 0; i < T.boxes.size(); ++i) {
            const Box& B = T.boxes[i];
            if (!B.leaf)
                continue;
            auto first = hperm.begin() + B.start, last = hperm.begin() + B.end;
            const int64_t ns = P->nsrc;
            auto mid = std::stable_partition(first, last, [ns](int o) { return o < ns; });
            box_nsrc[i] = mid - first;
        }
        HIPCHK(upload(P->perm, hperm, st));
        HIPCHK(hipStreamSynchronize(st));
    } else {
        for (size_t i = 0; i < T.boxes.size(); ++i)
            box_nsrc[i] = T.boxes[i].end - T.boxes[i].start;
    }
    // ---- sorted points ----
    P->x = P->mem.alloc<double>(n);
    P->y = P->mem.alloc<double>(n);
    P->z = P->mem.alloc<double>(n);
    if (P->mem.oom)
        return fail(DMK_ERR_OOM, "device allocation failed");
    launch_gather_points(points, n, P->perm, P->pid, P->geo, P->x, P->y, P->z, st);
    // ---- compact groups inside leaves (sources and targets separately) ----
    std::vector<KdSeg> kseg;
    if (P->leaf_order) {
        auto add = [&](int64_t a, int64_t b) {
            const int64_t len = b - a;
            if (len <= 8)
                return;
            // pieces of at most kKdCap points, cut at 64-point chunk boundaries
            const int64_t pieces = (len + kKdCap - 1) / kKdCap, chunks = (len + 63) / 64;
            for (int64_t k = 0; k < pieces; ++k) {
                const int64_t s = a + 64 * (chunks * k / pieces);
                const int64_t e = std::min(b, a + 64 * (chunks * (k + 1) / pieces));
                if (e - s > 8)
                    kseg.push_back(KdSeg{s, (int)(e - s), 0});
            }
        };
        for (size_t i = 0; i < T.boxes.size(); ++i) {
            const Box& B = T.boxes[i];
            if (!B.leaf || B.end == B.start)
                continue;
            add(B.start, B.start + box_nsrc[i]);
            if (box_nsrc[i] < B.end - B.start)
                add(B.start + box_nsrc[i], B.end);
        }
        KdSeg* d_seg = P->mem.alloc<KdSeg>(std::max<size_t>(kseg.size(), 1));
        if (P->mem.oom)
            return fail(DMK_ERR_OOM, "device allocation failed");
        HIPCHK(upload(d_seg, kseg, st));
        int* perm2 = reinterpret_cast<int*>(k0);  // the sort's key buffers are free now
        launch_leaf_order(d_seg, (int)kseg.size(), P->perm, P->x, P->y, P->z, n, i0, perm2, st);
        HIPCHK(hipMemcpyAsync(P->perm, perm2, n * sizeof(int), hipMemcpyDeviceToDevice, st));
        launch_gather_points(points, n, P->perm, P->pid, P->geo, P->x, P->y, P->z, st);
    }
    // ---- far-field slots ----
    const int nb = (int)T.boxes.size();
    P->box_fid.assign(nb, -1);
    P->nf = 0;
    for (int i = 0; i < nb; ++i)
        if (T.boxes[i].end > T.boxes[i].start)
            P->box_fid[i] = P->nf++;
    P->root_fid.clear();
    for (int r : roots)
        P->root_fid.push_back(P->box_fid[r]);
    auto center = [&](const Box& B, double* c) {
        const double h = 1.0 / (double)(1ll << B.level);
        c[0] = -0.5 + (B.ix + 0.5) * h;
        c[1] = -0.5 + (B.iy + 0.5) * h;
        c[2] = -0.5 + (B.iz + 0.5) * h;
    };
    std::vector<LeafDesc> hl, hl_src;
    P->leaf_box.clear();
    for (int i = 0; i < nb; ++i) {
        const Box& B = T.boxes[i];
        if (!B.leaf)
            continue;
        P->leaf_box.push_back(i);
        if (B.end == B.start)
            continue;
        LeafDesc d;
        d.fid = P->box_fid[i];
        d.level = B.level;
        d.start = B.start;
        d.end = B.end;
        double c[3];
        center(B, c);
        d.cx = c[0];
        d.cy = c[1];
        d.cz = c[2];
        hl.push_back(d);
        d.end = d.start + box_nsrc[i];
        hl_src.push_back(d);
    }
    P->nleaf = (int)hl.size();
    P->leaves = P->mem.alloc<LeafDesc>(hl.size());
    P->leaves_src = P->nsrc < n ? P->mem.alloc<LeafDesc>(hl_src.size()) : P->leaves;
    // far field at the target points of each leaf (after its sources)
    std::vector<EvalChunk> ech;
    for (size_t k = 0; k < hl.size(); ++k) {
        const LeafDesc& d = hl[k];
        const int64_t t0 = P->nsrc < n ? hl_src[k].end : d.start;
        for (int64_t s0 = t0; s0 < d.end; s0 += P->eval_pts)
            ech.push_back(EvalChunk{d.fid, s0, std::min<int64_t>(s0 + P->eval_pts, d.end)});
    }
    P->n_echunk = (int)ech.size();
    P->echunks = P->mem.alloc<EvalChunk>(ech.size());
    if (P->f32)
        P->Ltab = P->mem.alloc<float>((size_t)n * 3 * lagrange_pad(P->prm.p));
    else
        P->Ltab = P->mem.alloc<double>((size_t)n * 3 * lagrange_pad(P->prm.p));
    // per-level parent lists (non-empty, non-leaf)
    P->lev.assign(T.max_level + 1, {});
    // host sources of the stream-ordered uploads stay alive until the final sync
    std::vector<std::vector<int>> lev_hold(2 * (size_t)std::max(T.max_level, 1));
    for (int l = 0; l < T.max_level; ++l) {
        std::vector<int>& cf = lev_hold[2 * l];
        std::vector<int>& pf = lev_hold[2 * l + 1];
        for (int i = T.level_start[l]; i < T.level_start[l + 1]; ++i) {
            const Box& B = T.boxes[i];
            if (B.leaf || B.end == B.start)
                continue;
            pf.push_back(P->box_fid[i]);
            for (int d = 0; d < 8; ++d)
                cf.push_back(B.child[d] >= 0 ? P->box_fid[B.child[d]] : -1);
        }
        P->lev[l].nparent = (int)pf.size();
        P->lev[l].child_fid = P->mem.alloc<int>(cf.size());
        P->lev[l].parent_fid = P->mem.alloc<int>(pf.size());
        if (P->mem.oom)
            return fail(DMK_ERR_OOM, "device allocation failed");
        HIPCHK(upload(P->lev[l].child_fid, cf, st));
        HIPCHK(upload(P->lev[l].parent_fid, pf, st));
    }
    // senders / receivers (difference-kernel exchange lists)
    std::vector<int> send_slot(nb, -1), sfid, slev, rfid, epk;
    std::vector<RecvDesc> rd;
    for (int i = 0; i < nb; ++i)
        for (const FarEntry& e : T.incoming[i])
            if (send_slot[e.src] < 0) {
                send_slot[e.src] = (int)sfid.size();
                sfid.push_back(P->box_fid[e.src]);
                slev.push_back(T.boxes[e.src].level);
            }
    for (int i = 0; i < nb; ++i) {
        if (T.incoming[i].empty())
            continue;
        RecvDesc r;
        r.slot = (int)rfid.size();
        r.level = T.boxes[i].level;
        r.ebeg = (int)epk.size();
        for (const FarEntry& e : T.incoming[i]) {
            // colleagues only: offsets within one box width, slots below 2^26
            if (std::abs(e.ox) > 1 || std::abs(e.oy) > 1 || std::abs(e.oz) > 1 || send_slot[e.src] >= (1 << 26))
                return fail(DMK_ERR_UNSUPPORTED, "translation entry out of range (more than 2^26 senders)");
            epk.push_back(32 * send_slot[e.src] + 9 * (e.ox + 1) + 3 * (e.oy + 1) + (e.oz + 1));
        }
        r.eend = (int)epk.size();
        rfid.push_back(P->box_fid[i]);
        rd.push_back(r);
    }
    P->nsend = (int)sfid.size();
    P->nrecv = (int)rfid.size();
    P->send_fid = P->mem.alloc<int>(sfid.size());
    if (P->kern == DMK_KERNEL_STRESSLET)
        P->send_level = P->mem.alloc<int>(slev.size());
    P->recv_fid = P->mem.alloc<int>(rfid.size());
    P->recv = P->mem.alloc<RecvDesc>(rd.size());
    P->e_pk = P->mem.alloc<int>(epk.size());
    // near field: chunks of 64 sorted points per non-empty leaf
    std::vector<int> leaf_cbase(nb, -1);
    std::vector<int64_t> cstart;
    std::vector<int> clen;
    const bool split = P->nsrc < n;
    for (int li = 0; li < (int)T.leaves.size(); ++li) {
        const Box& B = T.boxes[T.leaves[li]];
        const int64_t se = B.start + box_nsrc[T.leaves[li]];
        leaf_cbase[T.leaves[li]] = (int)cstart.size();
        for (int64_t s = B.start; s < se; s += 64) {
            cstart.push_back(s);
            clen.push_back((int)std::min<int64_t>(64, se - s));
        }
    }
    std::vector<NearLeaf> nlv;
    std::vector<NearEntryDev> nent;
    std::vector<NearWork> nwk;
    std::vector<double> leaf_cost;
    for (int li = 0; li < (int)T.leaves.size(); ++li) {
        const Box& B = T.boxes[T.leaves[li]];
        const int64_t listed0 = P->near_listed;
        NearLeaf L;
        L.tstart = split ? B.start + box_nsrc[T.leaves[li]] : B.start;
        L.tend = B.end;
        L.level = B.level;
        L.cbase = leaf_cbase[T.leaves[li]];
        L.ebeg = (int)nent.size();
        for (const NearEntry& e : T.near[li]) {
            const Box& S = T.boxes[e.src];
            NearEntryDev d;
            d.sstart = S.start;
            d.send = S.start + box_nsrc[e.src];
            d.cbase = leaf_cbase[e.src];
            d.sx = e.sx;
            d.sy = e.sy;
            d.sz = e.sz;
            d.lambda = e.lambda;
            nent.push_back(d);
            P->near_listed += (L.tend - L.tstart) * (d.send - d.sstart);
        }
        L.eend = (int)nent.size();
        const int tg = 64 / P->near_sg;
        const int nch = (int)((L.tend - L.tstart + tg - 1) / tg);
        for (int c = 0; c < nch; ++c)
            nwk.push_back(NearWork{li, c});
        nlv.push_back(L);
        leaf_cost.push_back((double)(P->near_listed - listed0));
    }
    nwk = xcd_work_order(nwk, leaf_cost);
    P->n_nwork = (int)nwk.size();
    lap(3);
    P->nleaves = P->mem.alloc<NearLeaf>(nlv.size());
    P->nentries = P->mem.alloc<NearEntryDev>(nent.size());
    P->nwork = P->mem.alloc<NearWork>(nwk.size());
    P->cbbox = P->mem.alloc<double>(cstart.size() * 6);
    int64_t* d_cstart = P->mem.alloc<int64_t>(cstart.size());
    int* d_clen = P->mem.alloc<int>(clen.size());
    // tables
    const Tables& TB = *P->tab;
    const int p = P->prm.p, q = P->prm.q, n1 = P->prm.n1;
    std::vector<double> ct(p), cw(p);
    for (int a = 0; a < p; ++a) {
        ct[a] = TB.cheb_t[a];
        cw[a] = ((a & 1) ? -1.0 : 1.0) * std::sin((2.0 * a + 1) * kPi / (2.0 * p));
    }
    P->cheb_t = P->mem.alloc<double>(p);
    P->cheb_w = P->mem.alloc<double>(p);
    auto dup = [&](const std::vector<double>& v) {
        double* d = P->mem.alloc<double>(v.size());
        if (d)
            (void)hipMemcpyAsync(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st);
        return d;
    };
    P->merge_mat = dup(TB.merge_mat);
    P->interp_mat = dup(TB.interp_mat);
    P->pw_out = dup(TB.pw.out);
    P->pw_in_full = dup(TB.pw.in_full);
    P->pw_in_half = dup(TB.pw.in_half);
    const Tables::PW& rw = P->periodic ? TB.pw_per : TB.pw_root;
    P->r_out = dup(rw.out);
    P->r_in_full = dup(rw.in_full);
    P->r_in_half = dup(rw.in_half);
    P->root_mh = rw.M + 1;
    P->root_mf = 2 * rw.M + 1;
    const bool stress = P->kern == DMK_KERNEL_STRESSLET;
    const std::vector<double>& wr =
        P->periodic ? (stress ? TB.wper_t : TB.wper) : (stress ? TB.wroot_t : TB.wroot);
    const std::vector<double>& wd = stress ? TB.wdiff_t : TB.wdiff;
    P->wdiff = P->mem.alloc<double>(wd.size());
    P->wroot = P->mem.alloc<double>(wr.size());
    // work buffers
    P->H = (size_t)q * n1 * n1;
    P->Hroot = (size_t)P->root_mh * P->root_mf * P->root_mf;
    const size_t p3 = (size_t)p * p * p;
    // forces [rhs_batch][3][n]; stresslet: densities [6][n], then (f, n) [6][n]
    const int nc = P->nc_in;
    P->fs = P->mem.alloc<double>(n * std::max<size_t>(3 * (size_t)P->rhs_batch, stress ? 12 : 0));
    P->u = P->mem.alloc<double>(3 * n * (size_t)P->rhs_batch);
    const size_t es = P->es, cs = 2 * P->es;  // real / complex element bytes
    P->Q = P->mem.alloc<char>((size_t)P->nf * nc * p3 * es);
    P->V = P->mem.alloc<char>((size_t)P->nf * 3 * p3 * es);
    P->Phi = P->mem.alloc<char>((size_t)P->nsend * nc * P->H * cs);
    if (stress)
        P->Phi3 = P->mem.alloc<char>((size_t)P->nsend * 3 * P->H * cs);
    P->Psi = P->mem.alloc<char>((size_t)P->nrecv * 3 * P->H * cs);
    // scratch: largest intermediate of the plane-wave and of the merge /
    // interpolation stages, per (slot, component)
    size_t per_pw = 0;
    per_pw = std::max(per_pw, (size_t)p * p * q * cs);           // outgoing stage 1
    per_pw = std::max(per_pw, (size_t)p * q * n1 * cs);          // outgoing stage 2
    per_pw = std::max(per_pw, (size_t)n1 * n1 * p * cs);         // incoming stage 1
    per_pw = std::max(per_pw, (size_t)n1 * p * p * cs);          // incoming stage 2
    const size_t per_mg = (size_t)8 * p3 * es;                   // merge/interp stages
    const int pwslots = std::max({P->nsend, P->nrecv, 1});
    int mgslots = 1;
    for (auto& L : P->lev)
        mgslots = std::max(mgslots, L.nparent);
    size_t per_root = 0;
    {
        const size_t mh = P->root_mh, mf = P->root_mf;
        per_root = std::max({(size_t)p * p * mh, (size_t)p * mh * mf, mf * mf * (size_t)p, mf * (size_t)p * p}) * cs;
    }
    // scratch for one chunk of slots: at most about 4 GiB per buffer (fewer,
    // larger stage launches; a sixteenth of this GPU's 288 GB for both), or an
    // eighth of the caller's memory cap
    size_t budget = (size_t)4 << 30;
    if (P->mem.cap)
        budget = std::min(budget, std::max<size_t>((size_t)64 << 20, P->mem.cap / 8));
    P->ck_slots = (int)std::max<size_t>(1, std::min<size_t>((size_t)mgslots, budget / (per_mg * nc)));
    P->ck_pw = (int)std::max<size_t>(1, std::min<size_t>((size_t)pwslots, budget / (per_pw * nc)));
    P->ck_roots = (int)std::max<size_t>(1, std::min<size_t>((size_t)np, budget / (per_root * nc)));
    const size_t sbytes = std::max({per_mg * nc * (size_t)P->ck_slots, per_pw * nc * (size_t)P->ck_pw,
                                    per_root * nc * (size_t)P->ck_roots});
    P->s1 = P->mem.alloc<char>(sbytes);
    P->s2 = P->mem.alloc<char>(sbytes);
    P->phi_root = P->mem.alloc<char>(nc * P->Hroot * cs * np);
    P->psi_root = P->mem.alloc<char>(3 * P->Hroot * cs * np);
    P->cst = P->mem.alloc<double>(std::max<size_t>(3 * (size_t)P->rhs_batch, 4) * np);
    P->d_root_fid = P->mem.alloc<int>(np);
    if (P->mem.oom)
        return fail(DMK_ERR_OOM, "device allocation failed (or above mem_cap_bytes)");
    lap(4);
    HIPCHK(upload(P->d_root_fid, P->root_fid, st));
    HIPCHK(upload(P->leaves, hl, st));
    if (P->leaves_src != P->leaves)
        HIPCHK(upload(P->leaves_src, hl_src, st));
    HIPCHK(upload(P->echunks, ech, st));
    HIPCHK(upload(P->send_fid, sfid, st));
    if (stress)
        HIPCHK(upload(P->send_level, slev, st));
    HIPCHK(upload(P->recv_fid, rfid, st));
    HIPCHK(upload(P->recv, rd, st));
    HIPCHK(upload(P->e_pk, epk, st));
    HIPCHK(upload(P->nleaves, nlv, st));
    HIPCHK(upload(P->nentries, nent, st));
    HIPCHK(upload(P->nwork, nwk, st));
    HIPCHK(upload(d_cstart, cstart, st));
    HIPCHK(upload(d_clen, clen, st));
    HIPCHK(upload(P->cheb_t, ct, st));
    HIPCHK(upload(P->cheb_w, cw, st));
    HIPCHK(upload(P->wdiff, wd, st));
    HIPCHK(upload(P->wroot, wr, st));
    launch_chunk_bbox(P->x, P->y, P->z, d_cstart, d_clen, (int)cstart.size(), P->cbbox, st);
    launch_lagrange_table(P->prm.p, P->leaves, P->nleaf, P->x, P->y, P->z, P->cheb_t, P->cheb_w, P->Ltab, P->f32,
                          st);
    // radial polynomials
    if (!make_poly(TB, &P->poly))
        return fail(DMK_ERR_UNSUPPORTED, "radial fit degree too high");
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    lap(5);
    return DMK_OK;
}

// Far field of force vector r of the current batch (sorted forces at
// fs + 3nr): every pass from the proxy charges to the potential at the points
// (added to u + 3nr).  The work buffers are shared, so the passes of the
// batch's vectors run one vector after the other.
void far_field(dmk_plan_t P, int r, bool record)
{
    using namespace dmk;
    hipStream_t st = P->stream;
    auto mark = [&](int k) {
        if (record)
            (void)hipEventRecord(P->ev[k], st);
    };
    const int64_t n = P->n;
    const double* fs = P->fs + (size_t)r * 3 * n;
    double* u = P->u + (size_t)r * 3 * n;
    double* cst = P->cst + (size_t)3 * P->nprob * r;
    const int p = P->prm.p, q = P->prm.q, n1 = P->prm.n1;
    const long p3 = (long)p * p * p, p2 = (long)p * p;
    const Tree& T = P->tree;
    // Step 2a: proxy charges of the leaves
    const int nc = P->nc_in;
    const bool stress = P->kern == DMK_KERNEL_STRESSLET;
    launch_anterp(p, nc, P->leaves_src, P->nleaf, P->Ltab, fs, n, P->Q, P->f32, st);
    mark(1);
    const int h = (p + 1) / 2, M = q - 1;
    // a pipeline of stages over slots [0, ns) in chunks of ck (scratch holds one chunk)
    auto chunks = [&](int ns, int ck, const auto& body) {
        for (int c0 = 0; c0 < ns; c0 += ck) {
            P->ck_on = true;
            P->ck0 = c0;
            P->ck1 = std::min(ns, c0 + ck);
            body();
        }
        P->ck_on = false;
    };
    // Step 2b: merge children into parents, finest level first (Q is x-major [a][b][c])
    for (int l = T.max_level - 1; l >= 0; --l) {
        const auto& L = P->lev[l];
        if (!L.nparent)
            continue;
        chunks(L.nparent, P->ck_slots, [&] {
        stage(P, ST_SYM_REAL, IO_GATHER8, P->Q, 0, nullptr, P->s1, 4 * p3, nullptr, 0, P->merge_mat, 2 * p, p, 0, 0,
              p, h, 4 * p * p, L.nparent, L.child_fid, nc);
        stage(P, ST_SYM_REAL, IO_PLAIN, P->s1, 4 * p3, nullptr, P->s2, 2 * p3, nullptr, 0, P->merge_mat, 2 * p, p, 0,
              0, p, h, 2 * p * p, L.nparent, nullptr, nc);
        stage(P, ST_SYM_REAL, IO_PLAIN, P->s2, 2 * p3, nullptr, P->Q, p3, L.parent_fid, 0, P->merge_mat, 2 * p, p, 0,
              0, p, h, p * p, L.nparent, nullptr, nc);
        });
    }
    mark(2);
    // outgoing plane waves of the senders: Phi[mx][my][mz], mx >= 0
    const long H = (long)P->H;
    chunks(P->nsend, P->ck_pw, [&] {
    stage(P, ST_OUT_HALF, IO_PLAIN, P->Q, p3, P->send_fid, P->s1, p2 * q, nullptr, 0, P->pw_out, p, q, 0, 0, h, M + 1,
          p * p, P->nsend, nullptr, nc);
    stage(P, ST_OUT_FULL, IO_PLAIN, P->s1, p2 * q, nullptr, P->s2, (long)p * q * n1, nullptr, 0, P->pw_out, p, n1, 0,
          M, h, M + 1, p * q, P->nsend, nullptr, nc);
    stage(P, ST_OUT_FULL, IO_PLAIN, P->s2, (long)p * q * n1, nullptr, P->Phi, H, nullptr, 0, P->pw_out, p, n1, 0, M,
          h, M + 1, q * n1, P->nsend, nullptr, nc);
    });
    // stresslet: the difference symbol (6 -> 3 components) on the sending side
    if (stress)
        launch_stress_symbol(q, n1, P->nsend, P->send_level, P->Phi, P->wdiff, P->Phi3, P->f32, st);
    mark(3);
    // Step 3b: translation with the difference-kernel symbol -> Psi[mz][my][mx]
    launch_translate(q, n1, P->recv, P->nrecv, P->e_pk, stress ? P->Phi3 : P->Phi, P->wdiff, P->Psi,
                     P->f32, stress, st);
    mark(4);
    // incoming plane waves -> proxy potentials, z-major V[c][b][a]
    launch_zero(P->V, (size_t)P->nf * 3 * p3 * P->es, st);
    chunks(P->nrecv, P->ck_pw, [&] {
    stage(P, ST_IN_FULL, IO_PLAIN, P->Psi, H, nullptr, P->s1, (long)n1 * q * p, nullptr, 0, P->pw_in_full, n1, p, M,
          0, M + 1, h, n1 * q, P->nrecv);
    stage(P, ST_IN_FULL, IO_PLAIN, P->s1, (long)n1 * q * p, nullptr, P->s2, (long)q * p * p, nullptr, 0,
          P->pw_in_full, n1, p, M, 0, M + 1, h, q * p, P->nrecv);
    stage(P, ST_IN_HALF_REAL, IO_PLAIN, P->s2, (long)q * p * p, nullptr, P->V, p3, P->recv_fid, 1, P->pw_in_half, q,
          p, 0, 0, q, h, p * p, P->nrecv);
    });
    mark(5);
    // Step 3a: root convolution with the (truncated or periodic) mollified kernel
    {
        const int mh = P->root_mh, mf = P->root_mf, RM = mh - 1;
        const long Hr = (long)P->Hroot;
        const int nr = P->nprob;  // one root per problem; stage slots map to their far-field slots
        chunks(nr, P->ck_roots, [&] {
        stage(P, ST_OUT_HALF, IO_PLAIN, P->Q, p3, P->d_root_fid, P->s1, p2 * mh, nullptr, 0, P->r_out, p, mh, 0, 0, h,
              mh, p * p, nr, nullptr, nc);
        stage(P, ST_OUT_FULL, IO_PLAIN, P->s1, p2 * mh, nullptr, P->s2, (long)p * mh * mf, nullptr, 0, P->r_out, p, mf,
              0, RM, h, mh, p * mh, nr, nullptr, nc);
        stage(P, ST_OUT_FULL, IO_PLAIN, P->s2, (long)p * mh * mf, nullptr, P->phi_root, Hr, nullptr, 0, P->r_out, p,
              mf, 0, RM, h, mh, mh * mf, nr, nullptr, nc);
        });
        if (stress)
            launch_root_symbol_t(mh, mf, nr, P->phi_root, P->wroot,
                                 P->periodic ? 2.0 * kPi : 2.0 * kPi / P->tab->root_period, P->psi_root, P->f32, st);
        else
            launch_root_symbol(mh, mf, nr, P->phi_root, P->wroot, P->psi_root, P->f32, st);
        chunks(nr, P->ck_roots, [&] {
        stage(P, ST_IN_FULL, IO_PLAIN, P->psi_root, Hr, nullptr, P->s1, (long)mf * mh * p, nullptr, 0, P->r_in_full,
              mf, p, RM, 0, mh, h, mf * mh, nr);
        stage(P, ST_IN_FULL, IO_PLAIN, P->s1, (long)mf * mh * p, nullptr, P->s2, (long)mh * p * p, nullptr, 0,
              P->r_in_full, mf, p, RM, 0, mh, h, mh * p, nr);
        stage(P, ST_IN_HALF_REAL, IO_PLAIN, P->s2, (long)mh * p * p, nullptr, P->V, p3, P->d_root_fid, 1, P->r_in_half,
              mh, p, 0, 0, mh, h, p * p, nr);
        });
        if (P->periodic && stress)
            launch_stress_moment(P->Q, P->d_root_fid, nr, p, P->cheb_t, cst, P->f32, st);
        if (!P->periodic && !stress)
            launch_sum_root(P->Q, P->d_root_fid, nr, (int)p3, 1.0 / (4.0 * kPi * (1.0 + std::sqrt(3.0))), cst, P->f32,
                            st);
    }
    mark(6);
    // downward interpolation, coarsest level first (V is z-major, all axes alike)
    for (int l = 0; l < T.max_level; ++l) {
        const auto& L = P->lev[l];
        if (!L.nparent)
            continue;
        chunks(L.nparent, P->ck_slots, [&] {
        stage(P, ST_SYM_REAL, IO_PLAIN, P->V, p3, L.parent_fid, P->s1, 2 * p3, nullptr, 0, P->interp_mat, p, 2 * p, 0,
              0, h, p, p * p, L.nparent);
        stage(P, ST_SYM_REAL, IO_PLAIN, P->s1, 2 * p3, nullptr, P->s2, 4 * p3, nullptr, 0, P->interp_mat, p, 2 * p, 0,
              0, h, p, 2 * p * p, L.nparent);
        stage(P, ST_SYM_REAL, IO_SCATTER8, P->s2, 4 * p3, nullptr, P->V, 0, nullptr, 1, P->interp_mat, p, 2 * p, 0, 0,
              h, p, 4 * p * p, L.nparent, L.child_fid);
        });
    }
    mark(7);
    // far field at the points
    launch_leaf_eval(p, P->eval_pts, P->echunks, P->n_echunk, P->Ltab, P->V, n, u, P->f32, st);
    mark(8);
}

// Evaluates nb (1, 2, 4 or 8) force vectors: gather, one near-field pass for
// the whole batch (Step 4, self term included), the far field per vector
// (added), then the constant, scaling and unpermutation per vector.  Phase
// events cover the batch's near field, the first vector's far field and the
// finish.
int eval_batch(dmk_plan_t P, const double* f, int nb, double* vel, bool record)
{
    using namespace dmk;
    hipStream_t st = P->stream;
    const int64_t n = P->n;
    if (record)
        (void)hipEventRecord(P->ev[DMK_NUM_PHASES + 1], st);
    for (int r = 0; r < nb; ++r)
        launch_gather_forces(f + (size_t)r * 3 * P->nsrc, n, P->nsrc, P->perm, P->fs + (size_t)r * 3 * n, st);
    launch_zero(P->u, (size_t)nb * 3 * n * sizeof(double), st);
    launch_near(DMK_KERNEL_STOKESLET, P->near_sg, nb, P->near_refine, P->no_coincident, P->nsrc == n, P->nwork,
                P->n_nwork, P->nleaves, P->nentries,
                P->cbbox, P->x, P->y, P->z, P->fs, n, P->poly, P->u, st);
    if (record) {
        (void)hipEventRecord(P->ev[9], st);
        (void)hipEventRecord(P->ev[0], st);
    }
    for (int r = 0; r < nb; ++r)
        far_field(P, r, record && r == 0);
    if (record)
        (void)hipEventRecord(P->ev[DMK_NUM_PHASES + 2], st);
    for (int r = 0; r < nb; ++r)
        launch_finalize(P->u + (size_t)r * 3 * n, n, P->perm, P->tofs, P->pid, P->scale, 0,
                        P->periodic ? nullptr : P->cst + (size_t)3 * P->nprob * r, nullptr, nullptr, nullptr, nullptr,
                        vel + (size_t)r * 3 * P->nout, st);
    if (record) {
        (void)hipEventRecord(P->ev[10], st);
        P->ev_recorded = true;
    }
    return DMK_OK;
}

// One stresslet vector: densities and (f, n) in sorted order, the far field
// of the 6 density components, the residual stresslet near field, and the
// scaling by 1/L^2 (the stresslet is homogeneous of degree -2).  There is no
// self term (the mollified kernel at 0 and every residual term are odd in the
// separation) and no free-space constant; a periodic plan adds the k = 0 term
// the paper fixes for the stresslet (after eq. ewald_far).
int eval_stresslet(dmk_plan_t P, const double* f, const double* nv, double* vel, bool record)
{
    using namespace dmk;
    hipStream_t st = P->stream;
    const int64_t n = P->n;
    if (record)
        (void)hipEventRecord(P->ev[DMK_NUM_PHASES + 1], st);
    launch_gather_stresslet(f, nv, n, P->nsrc, P->perm, P->fs, P->fs + 6 * (size_t)n, st);
    launch_zero(P->u, 3 * (size_t)n * sizeof(double), st);
    launch_near(DMK_KERNEL_STRESSLET, P->near_sg, 1, true, false, false, P->nwork, P->n_nwork, P->nleaves, P->nentries, P->cbbox, P->x,
                P->y, P->z, P->fs + 6 * (size_t)n, n, P->poly, P->u, st);
    if (record) {
        (void)hipEventRecord(P->ev[9], st);
        (void)hipEventRecord(P->ev[0], st);
    }
    far_field(P, 0, record);
    if (record)
        (void)hipEventRecord(P->ev[DMK_NUM_PHASES + 2], st);
    // periodic: the k = 0 term -sum_s (x_t - x_s)(f_s . n_s) from the root moments in cst
    launch_finalize(P->u, n, P->perm, P->tofs, P->pid, P->scale, 1, nullptr, P->periodic ? P->cst : nullptr, P->x,
                    P->y, P->z, vel, st);
    if (record) {
        (void)hipEventRecord(P->ev[10], st);
        P->ev_recorded = true;
    }
    return DMK_OK;
}

// One force vector by the single-level spectral Ewald method: sorted forces,
// spreading to the grid, forward FFT, scaling by the mollified kernel and the
// gridding deconvolution, inverse FFT, interpolation at the points, the
// residual between neighbouring cells (self term from the r = 0 pair), and
// unpermute.  Phase events: spreading in the anterpolation slot, the FFTs
// and scaling in the root slot, interpolation in the leaf-evaluation slot.
int eval_ewald(dmk_plan_t P, const double* f, double* vel, bool record)
{
    using namespace dmk;
    hipStream_t st = P->stream;
    const int64_t n = P->n;
    const EwaldGrid& E = P->eg;
    auto mark = [&](int k) {
        if (record)
            (void)hipEventRecord(P->ev[k], st);
    };
    mark(0);
    launch_gather_forces(f, n, P->nsrc, P->perm, P->fs, st);
    launch_ewald_spread(E.M, E.B, E.Lt, E.w, P->gpoly, P->tile_start, P->x, P->y, P->z, P->fs, n, P->egrid, st);
    for (int k = 1; k <= 5; ++k)
        mark(k);
    if (hipfftSetStream(P->fft_fwd, st) != HIPFFT_SUCCESS || hipfftSetStream(P->fft_inv, st) != HIPFFT_SUCCESS)
        return fail(DMK_ERR_HIP, "hipfftSetStream failed");
    if (hipfftExecD2Z(P->fft_fwd, (hipfftDoubleReal*)P->egrid, (hipfftDoubleComplex*)P->espec) != HIPFFT_SUCCESS)
        return fail(DMK_ERR_HIP, "forward FFT failed");
    launch_ewald_scale(E.M, E.K, P->eghat, P->ewsym, P->espec, st);
    if (hipfftExecZ2D(P->fft_inv, (hipfftDoubleComplex*)P->espec, (hipfftDoubleReal*)P->egrid) != HIPFFT_SUCCESS)
        return fail(DMK_ERR_HIP, "inverse FFT failed");
    mark(6);
    mark(7);
    launch_ewald_interp(E.M, E.B, E.Lt, E.w, P->gpoly, P->tile_start, P->x, P->y, P->z, n, P->egrid, P->u, st);
    mark(8);
    mark(DMK_NUM_PHASES + 1);
    launch_near(DMK_KERNEL_STOKESLET, P->near_sg, 1, P->near_refine, P->no_coincident, P->nsrc == n, P->nwork,
                P->n_nwork, P->nleaves, P->nentries, P->cbbox, P->x,
                P->y, P->z, P->fs, n, P->poly, P->u, st);
    mark(9);
    mark(DMK_NUM_PHASES + 2);
    launch_finalize(P->u, n, P->perm, P->tofs, P->pid, P->scale, 0, nullptr, nullptr, nullptr, nullptr, nullptr, vel,
                    st);
    if (record) {
        (void)hipEventRecord(P->ev[10], st);
        P->ev_recorded = true;
    }
    return DMK_OK;
}

}  // namespace

extern "C" {

const char* dmk_last_error(void) { return g_err.c_str(); }

int dmk_stokes_params(double tol, dmk_plan_info* info) { return dmk_stokes_params_ex(tol, DMK_WINDOW_PROLATE, info); }

int dmk_stokes_params_ex(double tol, int window, dmk_plan_info* info)
{
    return dmk_stokes_params_kernel(tol, window, DMK_KERNEL_STOKESLET, info);
}

int dmk_stokes_params_kernel(double tol, int window, int kernel, dmk_plan_info* info)
{
    if (!info)
        return fail(DMK_ERR_ARG, "info is NULL");
    std::memset(info, 0, sizeof(*info));
    if (window != DMK_WINDOW_PROLATE && window != DMK_WINDOW_GAUSSIAN)
        return fail(DMK_ERR_ARG, "unknown window");
    if (kernel != DMK_KERNEL_STOKESLET && kernel != DMK_KERNEL_STRESSLET)
        return fail(DMK_ERR_ARG, "unknown kernel");
    dmk::Params prm;
    if (!dmk::select_params(tol, &prm, window, kernel))
        return fail(DMK_ERR_TOL, "tol outside the window's range (or no such kernel/window pair)");
    const dmk::Tables* T = dmk::get_tables(prm);
    info->tol = prm.tol;
    info->c = prm.c;
    info->q = prm.q;
    info->p = prm.p;
    info->n1 = prm.n1;
    info->nper = prm.nper;
    info->leaf_size = prm.ns;
    info->deg_P = (int)T->fits.P.a.size() - 1;
    info->deg_Q = (int)T->fits.Q.a.size() - 1;
    info->window = prm.window;
    info->sigma = prm.sigma;
    info->kernel = prm.kernel;
    return DMK_OK;
}

int dmk_stokes_radial(double tol, const double* rho, int64_t n, double* out)
{
    if (!rho || !out || n < 0)
        return fail(DMK_ERR_ARG, "bad arguments");
    const dmk::Tables* T = dmk::get_tables(tol);
    if (!T)
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    dmk::Prolate w(T->prm.c);
    for (int64_t i = 0; i < n; ++i) {
        const double r = rho[i];
        out[4 * i] = w.phi(r);
        out[4 * i + 1] = w.Phi(r);
        const double s = r * r;
        out[4 * i + 2] = s < 1.0 ? T->fits.P.eval(s) : 0.0;
        out[4 * i + 3] = s < 1.0 ? T->fits.Q.eval(s) : 0.0;
    }
    return DMK_OK;
}

int dmk_stokes_ewald_params(double tol, int64_t n, int leaf_size, dmk_plan_info* info)
{
    if (!info || n < 1 || leaf_size < 0)
        return fail(DMK_ERR_ARG, "bad arguments");
    std::memset(info, 0, sizeof(*info));
    dmk::Params prm;
    if (!dmk::select_params(tol, &prm) || tol < 1e-9 * (1 - 1e-9))
        return fail(DMK_ERR_TOL, "the spectral Ewald method is offered for tol in [1e-9, 1e-3]");
    if (leaf_size > 0)
        prm.ns = leaf_size;
    int L = 1;
    while (L < 8 && (double)n / (double)(1ll << (3 * L)) > (double)prm.ns)
        ++L;
    dmk::EwaldGrid E;
    if (!dmk::ewald_grid(prm, L, &E))
        return fail(DMK_ERR_UNSUPPORTED, "no spectral Ewald grid for this tolerance and size");
    info->tol = prm.tol;
    info->c = prm.c;
    info->q = prm.q;
    info->leaf_size = prm.ns;
    info->periodic = 1;
    info->n_points = n;
    info->levels = L + 1;
    info->method = DMK_METHOD_EWALD;
    info->ewald_grid = E.M;
    info->ewald_modes = E.K;
    info->ewald_width = E.w;
    return DMK_OK;
}

int dmk_stokes_radial_stresslet(double tol, const double* rho, int64_t n, double* out)
{
    if (!rho || !out || n < 0)
        return fail(DMK_ERR_ARG, "bad arguments");
    dmk::Params prm;
    if (!dmk::select_params(tol, &prm, DMK_WINDOW_PROLATE, DMK_KERNEL_STRESSLET))
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    const dmk::Tables* T = dmk::get_tables(prm);
    for (int64_t i = 0; i < n; ++i) {
        const double s = rho[i] * rho[i];
        out[2 * i] = s < 1.0 ? T->fits.P.eval(s) : 0.0;
        out[2 * i + 1] = s < 1.0 ? T->fits.Q.eval(s) : 0.0;
    }
    return DMK_OK;
}

int dmk_stokes_mollifier(double tol, const double* k, int64_t n, double* out)
{
    if (!k || !out || n < 0)
        return fail(DMK_ERR_ARG, "bad arguments");
    dmk::Params prm;
    if (!dmk::select_params(tol, &prm))
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    dmk::Prolate w(prm.c);
    for (int64_t i = 0; i < n; ++i) {
        out[2 * i] = w.phihat(k[i]);
        out[2 * i + 1] = w.gammahat(k[i]);
    }
    return DMK_OK;
}

namespace {

// Common plan construction for one problem (offsets {0, n}) or a batch.
int create_plan(const double* points, const std::vector<int64_t>& offsets, int dim, int periodic, double tol,
                const dmk_opts* opts, dmk_plan_t* out, int64_t nsrc = -1)
{
    const int64_t n = offsets.back();

    int rc = validate_common(dim, tol, opts);
    if (rc != DMK_OK)
        return rc;
    if (periodic != 0 && periodic != 1)
        return fail(DMK_ERR_ARG, "periodic must be 0 or 1");
    if (!is_device_ptr(points))
        return fail(DMK_ERR_ARG, "points must be a device pointer");
    const auto t0 = std::chrono::steady_clock::now();
    dmk_plan_t P = new (std::nothrow) dmk_plan_s();
    if (!P)
        return fail(DMK_ERR_OOM, "host allocation failed");
    const int kern = opts ? opts->kernel : DMK_KERNEL_STOKESLET;
    if (!dmk::select_params(tol, &P->prm, opts ? opts->window : 0, kern)) {
        delete P;
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    }
    P->kern = kern;
    P->nc_in = kern == DMK_KERNEL_STRESSLET ? 6 : 3;
    P->method = opts ? opts->method : DMK_METHOD_DMK;
    if (P->method == DMK_METHOD_EWALD && (!periodic || offsets.size() != 2 || nsrc >= 0)) {
        delete P;
        return fail(DMK_ERR_UNSUPPORTED, "the spectral Ewald method takes one periodic problem without separate targets");
    }
    if (opts)
        dmk::override_params(&P->prm, opts->q, opts->p);
    P->tab = dmk::get_tables(P->prm);
    P->near_refine = P->prm.kernel != DMK_KERNEL_STOKESLET || stokes_near_refine(P->prm.tol);
    if (opts) {
        P->stream = (hipStream_t)opts->stream;
        P->precision = opts->precision;
        P->f32 = opts->precision == DMK_PREC_MIXED;
        P->es = P->f32 ? 4 : 8;
        if (opts->leaf_size > 0)
            P->prm.ns = opts->leaf_size;
        P->mem.cap = opts->mem_cap_bytes;
        P->timing = (opts->flags & DMK_FLAG_PHASE_TIMING) != 0;
        if (opts->near_lanes > 0)
            P->near_sg = opts->near_lanes;
        if (opts->rhs_batch > 0)
            P->rhs_batch = opts->rhs_batch;
        P->concurrent = (opts->flags & DMK_FLAG_CONCURRENT_PLAN) != 0;
        P->use_graph = (opts->flags & DMK_FLAG_GRAPH) != 0;
        P->leaf_order = (opts->flags & DMK_FLAG_MORTON_ORDER) == 0;
        P->host_tree = (opts->flags & DMK_FLAG_HOST_TREE) != 0;
        P->stage_rows = opts->stage_rows;
    }
    P->eval_pts = dmk::eval_chunk_points(P->prm.p, opts ? opts->eval_points : 0);
    if (hipEventCreateWithFlags(&P->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete P;
        return fail(DMK_ERR_HIP, "hipEventCreate failed");
    }
    if (P->timing)
        for (auto& e : P->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                delete P;
                return fail(DMK_ERR_HIP, "hipEventCreate failed");
            }
    P->n = n;
    P->periodic = periodic != 0;
    P->nprob = (int)offsets.size() - 1;
    P->offsets = offsets;
    P->nsrc = nsrc < 0 ? n : nsrc;
    P->tofs = nsrc < 0 ? 0 : nsrc;
    P->nout = n - P->tofs;
    rc = build_plan(P, points);
    if (rc != DMK_OK) {
        (void)hipStreamSynchronize(P->concurrent ? plan_stream() : P->stream);
        delete P;
        return rc;
    }
    P->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = P;
    return DMK_OK;
}


}  // namespace

int dmk_stokes_plan_ex(const double* points, int64_t n, int dim, int periodic, double tol, const dmk_opts* opts,
                       dmk_plan_t* out)
{
    if (!out)
        return fail(DMK_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!points)
        return fail(DMK_ERR_ARG, "points is NULL");
    if (n < 1)
        return fail(DMK_ERR_ARG, "n must be >= 1");
    if (n > (int64_t)2000000000)
        return fail(DMK_ERR_ARG, "n too large");
    return create_plan(points, {0, n}, dim, periodic, tol, opts, out);
}

int dmk_stokes_plan_targets(const double* sources, int64_t n_sources, const double* targets, int64_t n_targets,
                            int dim, int periodic, double tol, const dmk_opts* opts, dmk_plan_t* out)
{
    if (!out)
        return fail(DMK_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!sources || !targets)
        return fail(DMK_ERR_ARG, "sources or targets is NULL");
    if (n_sources < 1 || n_targets < 1)
        return fail(DMK_ERR_ARG, "n_sources and n_targets must be >= 1");
    if (n_sources + n_targets > (int64_t)2000000000)
        return fail(DMK_ERR_ARG, "n too large");
    if (!is_device_ptr(sources) || !is_device_ptr(targets))
        return fail(DMK_ERR_ARG, "sources and targets must be device pointers");
    if (opts && (opts->flags & DMK_FLAG_CONCURRENT_PLAN))
        return fail(DMK_ERR_ARG, "DMK_FLAG_CONCURRENT_PLAN is not available for separate targets");
    int rc = validate_common(dim, tol, opts);
    if (rc != DMK_OK)
        return rc;
    // one point set: sources then targets, in order on the caller's stream
    const int64_t n = n_sources + n_targets;
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    double* pts = nullptr;
    HIPCHK(hipMalloc((void**)&pts, (size_t)n * 3 * sizeof(double)));
    hipError_t e = hipMemcpyAsync(pts, sources, (size_t)n_sources * 3 * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pts + 3 * n_sources, targets, (size_t)n_targets * 3 * sizeof(double),
                           hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        (void)hipFree(pts);
        return fail(DMK_ERR_HIP, std::string("copy of the points failed: ") + hipGetErrorString(e));
    }
    rc = create_plan(pts, {0, n}, dim, periodic, tol, opts, out, n_sources);
    (void)hipStreamSynchronize(st);
    (void)hipFree(pts);
    return rc;
}

int dmk_stokes_plan_batch(const double* points, const int64_t* offsets, int n_problems, int dim, int periodic,
                          double tol, const dmk_opts* opts, dmk_plan_t* out)
{
    if (!out)
        return fail(DMK_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!points || !offsets)
        return fail(DMK_ERR_ARG, "points or offsets is NULL");
    if (n_problems < 1 || n_problems > (1 << 20))
        return fail(DMK_ERR_ARG, "n_problems must be in [1, 2^20]");
    if (offsets[0] != 0)
        return fail(DMK_ERR_ARG, "offsets[0] must be 0");
    for (int b = 0; b < n_problems; ++b)
        if (offsets[b + 1] <= offsets[b])
            return fail(DMK_ERR_ARG, "every problem needs at least one point (offsets strictly increasing)");
    if (offsets[n_problems] > (int64_t)2000000000)
        return fail(DMK_ERR_ARG, "n too large");
    return create_plan(points, std::vector<int64_t>(offsets, offsets + n_problems + 1), dim, periodic, tol, opts,
                       out);
}

int dmk_stokes_plan(const double* points, int64_t n, int dim, int periodic, double tol, dmk_plan_t* out)
{
    return dmk_stokes_plan_ex(points, n, dim, periodic, tol, nullptr, out);
}

int dmk_stokes_eval(dmk_plan_t plan, const double* forces, int n_rhs, double* velocities)
{
    if (!plan)
        return fail(DMK_ERR_ARG, "plan is NULL");
    if (plan->kern != DMK_KERNEL_STOKESLET)
        return fail(DMK_ERR_ARG, "a stresslet plan is evaluated with dmk_stokes_eval_stresslet");
    if (plan->method == DMK_METHOD_EWALD) {
        if (n_rhs < 1)
            return fail(DMK_ERR_ARG, "n_rhs must be >= 1");
        if (!is_device_ptr(forces) || !is_device_ptr(velocities))
            return fail(DMK_ERR_ARG, "forces and velocities must be device pointers");
        for (int r = 0; r < n_rhs; ++r) {
            const int rc = eval_ewald(plan, forces + (size_t)r * 3 * plan->n, velocities + (size_t)r * 3 * plan->n,
                                      plan->timing && r == 0);
            if (rc != DMK_OK)
                return rc;
        }
        HIPCHK(hipEventRecord(plan->done, plan->stream));
        plan->done_recorded = true;
        HIPCHK(hipGetLastError());
        return DMK_OK;
    }
    if (n_rhs < 1)
        return fail(DMK_ERR_ARG, "n_rhs must be >= 1");
    if (!is_device_ptr(forces) || !is_device_ptr(velocities))
        return fail(DMK_ERR_ARG, "forces and velocities must be device pointers");
    auto run = [&](bool timing) {
        for (int r = 0; r < n_rhs;) {
            // largest supported batch that fits the remaining vectors
            int nb = plan->rhs_batch;
            while (nb > n_rhs - r)
                nb >>= 1;
            const int rc = eval_batch(plan, forces + (size_t)r * 3 * plan->nsrc, nb,
                                      velocities + (size_t)r * 3 * plan->nout, timing && r == 0);
            if (rc != DMK_OK)
                return rc;
            r += nb;
        }
        return (int)DMK_OK;
    };
    if (!plan->use_graph) {
        const int rc = run(plan->timing);
        if (rc != DMK_OK)
            return rc;
    } else {
        if (!(plan->gexec && plan->g_forces == forces && plan->g_vel == velocities && plan->g_nrhs == n_rhs)) {
            if (plan->gexec) {
                (void)hipGraphExecDestroy(plan->gexec);
                (void)hipGraphDestroy(plan->graph);
                plan->gexec = nullptr;
                plan->graph = nullptr;
            }
            if (!plan->cap_stream)
                HIPCHK(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
            hipStream_t user = plan->stream;
            plan->stream = plan->cap_stream;
            HIPCHK(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
            const int rc = run(false);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(plan->cap_stream, &g);
            plan->stream = user;
            if (rc != DMK_OK) {
                if (g)
                    (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess)
                return fail(DMK_ERR_HIP, std::string("stream capture failed: ") + hipGetErrorString(e));
            const hipError_t ei = hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                (void)hipGraphDestroy(g);
                plan->gexec = nullptr;
                return fail(DMK_ERR_HIP, std::string("graph instantiation failed: ") + hipGetErrorString(ei));
            }
            plan->graph = g;
            plan->g_forces = forces;
            plan->g_vel = velocities;
            plan->g_nrhs = n_rhs;
        }
        HIPCHK(hipGraphLaunch(plan->gexec, plan->stream));
    }
    HIPCHK(hipEventRecord(plan->done, plan->stream));
    plan->done_recorded = true;
    HIPCHK(hipGetLastError());
    return DMK_OK;
}

int dmk_stokes_eval_stresslet(dmk_plan_t plan, const double* forces, const double* normals, int n_rhs,
                              double* velocities)
{
    if (!plan)
        return fail(DMK_ERR_ARG, "plan is NULL");
    if (plan->kern != DMK_KERNEL_STRESSLET)
        return fail(DMK_ERR_ARG, "the plan was not built for the stresslet (dmk_opts.kernel)");
    if (n_rhs < 1)
        return fail(DMK_ERR_ARG, "n_rhs must be >= 1");
    if (!is_device_ptr(forces) || !is_device_ptr(normals) || !is_device_ptr(velocities))
        return fail(DMK_ERR_ARG, "forces, normals and velocities must be device pointers");
    for (int r = 0; r < n_rhs; ++r) {
        const size_t so = (size_t)r * 3 * plan->nsrc;
        const int rc = eval_stresslet(plan, forces + so, normals + so, velocities + (size_t)r * 3 * plan->nout,
                                      plan->timing && r == 0);
        if (rc != DMK_OK)
            return rc;
    }
    HIPCHK(hipEventRecord(plan->done, plan->stream));
    plan->done_recorded = true;
    HIPCHK(hipGetLastError());
    return DMK_OK;
}

int dmk_stokes_autotune(const double* points, int64_t n, const int64_t* offsets, int n_problems, int dim,
                        int periodic, double tol, const dmk_opts* opts, int n_rhs, dmk_opts* tuned, double* best_ms)
{
    if (!tuned)
        return fail(DMK_ERR_ARG, "tuned is NULL");
    if (!points || n < 1 || n_rhs < 1 || n_rhs > 64)
        return fail(DMK_ERR_ARG, "bad points, n or n_rhs");
    if (offsets && (n_problems < 1 || offsets[0] != 0 || offsets[n_problems] != n))
        return fail(DMK_ERR_ARG, "offsets must run from 0 to n");
    int rc = validate_common(dim, tol, opts);
    if (rc != DMK_OK)
        return rc;
    if (opts && opts->kernel != DMK_KERNEL_STOKESLET)
        return fail(DMK_ERR_UNSUPPORTED, "the autotuner times the Stokeslet evaluation only");
    dmk_opts base{};
    if (opts)
        base = *opts;
    base.flags &= ~(DMK_FLAG_PHASE_TIMING | DMK_FLAG_GRAPH);
    dmk::Params prm;
    if (!dmk::select_params(tol, &prm))
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    // cached per workload class: size (powers of 2), problem count, periodicity, tolerance, precision
    const int nb = offsets ? n_problems : 1;
    const auto key = std::make_tuple((int)std::lround(std::log2((double)n)), (int)std::lround(std::log2((double)nb)),
                                     periodic, tol, base.precision, n_rhs, base.q, base.p,
                                     base.window * 4 + base.method);
    static std::mutex mu;
    static std::map<decltype(key), std::pair<dmk_opts, double>> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *tuned = base;
            tuned->leaf_size = it->second.first.leaf_size;
            tuned->near_lanes = it->second.first.near_lanes;
            tuned->stage_rows = it->second.first.stage_rows;
            tuned->eval_points = it->second.first.eval_points;
            if (best_ms)
                *best_ms = it->second.second;
            return DMK_OK;
        }
    }
    double* f = nullptr;
    double* v = nullptr;
    const size_t bytes = (size_t)n * 3 * n_rhs * sizeof(double);
    HIPCHK(hipMalloc((void**)&f, bytes));
    if (hipMalloc((void**)&v, bytes) != hipSuccess) {
        (void)hipFree(f);
        return fail(DMK_ERR_OOM, "autotune buffers");
    }
    (void)hipMemset(f, 0, bytes);
    hipStream_t st = (hipStream_t)base.stream;
    // one trial: plan + evaluation, wall time (the plan part includes its host work)
    const int p_used = base.p > 0 ? base.p : prm.p;
    int best_rows = base.stage_rows, best_pts = dmk::eval_chunk_points(p_used, base.eval_points);
    auto trial = [&](int leaf, int lanes, double* ms) {
        dmk_opts o = base;
        o.leaf_size = leaf;
        o.near_lanes = lanes;
        o.stage_rows = best_rows;
        o.eval_points = best_pts;
        double best = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipStreamSynchronize(st);
            const auto t0 = std::chrono::steady_clock::now();
            dmk_plan_t P = nullptr;
            const int r = offsets ? dmk_stokes_plan_batch(points, offsets, n_problems, dim, periodic, tol, &o, &P)
                                  : dmk_stokes_plan_ex(points, n, dim, periodic, tol, &o, &P);
            if (r != DMK_OK)
                return r;
            const int r2 = dmk_stokes_eval(P, f, n_rhs, v);
            (void)hipStreamSynchronize(st);
            const auto t1 = std::chrono::steady_clock::now();
            dmk_stokes_destroy(P);
            if (r2 != DMK_OK)
                return r2;
            best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        *ms = best;
        return (int)DMK_OK;
    };
    const int ns0 = opts && opts->leaf_size > 0 ? opts->leaf_size : prm.ns;
    int best_leaf = ns0, best_lanes = opts && opts->near_lanes > 0 ? opts->near_lanes : 4;
    double best = 1e300;
    for (double fac : {0.5, 0.75, 1.0, 1.35, 1.8, 2.4}) {
        const int leaf = std::max(32, (int)std::lround(ns0 * fac));
        double ms = 0;
        rc = trial(leaf, best_lanes, &ms);
        if (rc != DMK_OK)
            break;
        if (ms < best) {
            best = ms;
            best_leaf = leaf;
        }
    }
    for (int lanes : {2, 8}) {
        if (rc != DMK_OK)
            break;
        double ms = 0;
        rc = trial(best_leaf, lanes, &ms);
        if (rc == DMK_OK && ms < best) {
            best = ms;
            best_lanes = lanes;
        }
    }
    // tile shapes of the far-field kernels at the chosen leaf size and split
    for (int rows : {16, 32, 64}) {
        if (rc != DMK_OK)
            break;
        if (rows == best_rows)
            continue;
        const int keep = best_rows;
        best_rows = rows;
        double ms = 0;
        rc = trial(best_leaf, best_lanes, &ms);
        if (rc == DMK_OK && ms < best)
            best = ms;
        else
            best_rows = keep;
    }
    for (int pts : {128, 256}) {
        if (rc != DMK_OK)
            break;
        if (pts == best_pts || dmk::eval_chunk_points(p_used, pts) != pts)
            continue;
        const int keep = best_pts;
        best_pts = pts;
        double ms = 0;
        rc = trial(best_leaf, best_lanes, &ms);
        if (rc == DMK_OK && ms < best)
            best = ms;
        else
            best_pts = keep;
    }
    (void)hipFree(f);
    (void)hipFree(v);
    if (rc != DMK_OK)
        return rc;
    *tuned = base;
    tuned->leaf_size = best_leaf;
    tuned->near_lanes = best_lanes;
    tuned->stage_rows = best_rows;
    tuned->eval_points = best_pts;
    if (opts)
        tuned->flags = opts->flags;
    if (best_ms)
        *best_ms = best;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = {*tuned, best};
    return DMK_OK;
}

int dmk_stokes_plan_info(dmk_plan_t plan, dmk_plan_info* info)
{
    if (!plan || !info)
        return fail(DMK_ERR_ARG, "plan or info is NULL");
    std::memset(info, 0, sizeof(*info));
    const dmk_plan_s& P = *plan;
    info->tol = P.prm.tol;
    info->c = P.prm.c;
    info->q = P.prm.q;
    info->p = P.prm.p;
    info->n1 = P.prm.n1;
    info->nper = P.prm.nper;
    info->leaf_size = P.prm.ns;
    info->deg_P = (int)P.tab->fits.P.a.size() - 1;
    info->deg_Q = (int)P.tab->fits.Q.a.size() - 1;
    info->levels = P.tree.max_level + 1;
    info->periodic = P.periodic;
    info->n_points = P.n;
    info->n_boxes = (int64_t)P.tree.boxes.size();
    info->n_leaves = (int64_t)P.leaf_box.size();
    info->n_nonempty_boxes = P.nf;
    info->n_nonempty_leaves = P.nleaf;
    info->no_coincident = P.no_coincident ? 1 : 0;
    info->near_pairs = P.near_listed;
    info->n_senders = P.nsend;
    info->n_receivers = P.nrecv;
    for (int d = 0; d < 3; ++d)
        info->center[d] = P.center[d];
    info->box_len = P.box_len;
    info->device_bytes = P.mem.total;
    info->plan_ms = P.plan_ms;
    for (int k = 0; k < 6; ++k)
        info->plan_phase_ms[k] = P.plan_phase[k];
    info->near_lanes = P.near_sg;
    info->precision = P.precision;
    info->window = P.prm.window;
    info->sigma = P.prm.sigma;
    info->kernel = P.kern;
    info->method = P.method;
    if (P.method == DMK_METHOD_EWALD) {
        info->levels = P.eg.L + 1;
        info->n_leaves = (int64_t)1 << (3 * P.eg.L);
        info->n_boxes = info->n_leaves;
        info->n_nonempty_leaves = P.n_cells_nonempty;
        info->n_nonempty_boxes = P.n_cells_nonempty;
        info->ewald_grid = P.eg.M;
        info->ewald_modes = P.eg.K;
        info->ewald_width = P.eg.w;
    }
    return DMK_OK;
}

int dmk_stokes_tree_leaves(dmk_plan_t plan, int32_t* leaf_level, int64_t* leaf_coord, int64_t* leaf_count,
                           int64_t* point_leaf)
{
    if (!plan)
        return fail(DMK_ERR_ARG, "plan is NULL");
    if (plan->method != DMK_METHOD_DMK)
        return fail(DMK_ERR_ARG, "a spectral Ewald plan has no octree");
    const dmk_plan_s& P = *plan;
    const auto& B = P.tree.boxes;
    for (size_t li = 0; li < P.leaf_box.size(); ++li) {
        const dmk::Box& b = B[P.leaf_box[li]];
        if (leaf_level)
            leaf_level[li] = b.level;
        if (leaf_coord) {
            leaf_coord[3 * li] = b.ix;
            leaf_coord[3 * li + 1] = b.iy;
            leaf_coord[3 * li + 2] = b.iz;
        }
        if (leaf_count)
            leaf_count[li] = b.end - b.start;
    }
    if (point_leaf) {
        std::vector<int> perm(P.n);
        HIPCHK(hipMemcpyAsync(perm.data(), P.perm, P.n * sizeof(int), hipMemcpyDeviceToHost, P.stream));
        HIPCHK(hipStreamSynchronize(P.stream));
        for (size_t li = 0; li < P.leaf_box.size(); ++li) {
            const dmk::Box& b = B[P.leaf_box[li]];
            for (int64_t i = b.start; i < b.end; ++i)
                point_leaf[perm[i]] = (int64_t)li;
        }
    }
    return DMK_OK;
}

int dmk_stokes_phase_ms(dmk_plan_t plan, double* out)
{
    if (!plan || !out)
        return fail(DMK_ERR_ARG, "plan or out is NULL");
    if (!plan->timing || !plan->ev_recorded)
        return fail(DMK_ERR_ARG, "no timed evaluation recorded (DMK_FLAG_PHASE_TIMING)");
    HIPCHK(hipEventSynchronize(plan->ev[DMK_NUM_PHASES]));
    for (int k = 0; k < DMK_NUM_PHASES; ++k) {
        float ms = 0;
        if (k == DMK_PHASE_NEAR)
            HIPCHK(hipEventElapsedTime(&ms, plan->ev[DMK_NUM_PHASES + 1], plan->ev[k + 1]));
        else if (k == DMK_PHASE_FINALIZE)
            HIPCHK(hipEventElapsedTime(&ms, plan->ev[DMK_NUM_PHASES + 2], plan->ev[k + 1]));
        else
            HIPCHK(hipEventElapsedTime(&ms, plan->ev[k], plan->ev[k + 1]));
        out[k] = ms;
    }
    return DMK_OK;
}

int dmk_stokes_near_stats(dmk_plan_t plan, int64_t* listed, int64_t* evaluated, int64_t* in_support)
{
    if (!plan)
        return fail(DMK_ERR_ARG, "plan is NULL");
    if (listed)
        *listed = plan->near_listed;
    DevMem mem;
    unsigned long long* d = mem.alloc<unsigned long long>(2);
    if (!d)
        return fail(DMK_ERR_OOM, "device allocation failed");
    HIPCHK(hipMemsetAsync(d, 0, 2 * sizeof(unsigned long long), plan->stream));
    dmk::launch_near_count(plan->near_sg, plan->nwork, plan->n_nwork, plan->nleaves, plan->nentries, plan->cbbox, plan->x,
                           plan->y, plan->z, d, plan->stream);
    unsigned long long h[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, plan->stream));
    HIPCHK(hipStreamSynchronize(plan->stream));
    if (evaluated)
        *evaluated = (int64_t)h[0];
    if (in_support)
        *in_support = (int64_t)h[1];
    return DMK_OK;
}

void dmk_stokes_release_cached_memory(void)
{
    pool().release_all();
    std::lock_guard<std::mutex> lk(g_fft_mu);
    for (auto& e : fft_pool()) {
        (void)hipfftDestroy(e.second.fwd);
        (void)hipfftDestroy(e.second.inv);
    }
    fft_pool().clear();
}

void dmk_stokes_destroy(dmk_plan_t plan)
{
    if (!plan)
        return;
    // the buffers go back to the cache only once the plan's last evaluation
    // has finished reading them
    if (plan->done_recorded)
        (void)hipEventSynchronize(plan->done);
    delete plan;
}

int dmk_stokes_host_tree(const double* points, int64_t n, int leaf_size, int periodic, int64_t cap,
                         int32_t* leaf_level, int64_t* leaf_coord, int64_t* leaf_count, int64_t* n_leaves,
                         int64_t* n_near_pairs)
{
    if (!points || n < 1 || leaf_size < 1 || !n_leaves || (periodic != 0 && periodic != 1))
        return fail(DMK_ERR_ARG, "bad arguments");
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = points[3 * i + d];
            if (!std::isfinite(v))
                return fail(DMK_ERR_NONFINITE, "points contain NaN or Inf");
            lo[d] = std::min(lo[d], v);
            hi[d] = std::max(hi[d], v);
        }
    double c[3], len = 1.0;
    if (periodic) {
        for (int d = 0; d < 3; ++d)
            if (lo[d] < 0.0 || hi[d] >= 1.0)
                return fail(DMK_ERR_DOMAIN, "periodic points must lie in [0,1)^3");
        c[0] = c[1] = c[2] = 0.5;
    } else {
        double ext = 0;
        for (int d = 0; d < 3; ++d) {
            c[d] = 0.5 * (lo[d] + hi[d]);
            ext = std::max(ext, hi[d] - lo[d]);
        }
        len = (ext > 0 ? ext : 1.0) * (1.0 + 1e-9);
    }
    std::vector<uint64_t> keys(n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t q[3];
        for (int d = 0; d < 3; ++d) {
            double g = std::floor(((points[3 * i + d] - c[d]) / len + 0.5) * 524288.0);
            g = std::min(std::max(g, 0.0), 524287.0);
            q[d] = (uint64_t)g;
        }
        uint64_t k = 0;
        for (int bt = 18; bt >= 0; --bt)
            k = (k << 3) | (((q[0] >> bt) & 1) << 2) | (((q[1] >> bt) & 1) << 1) | ((q[2] >> bt) & 1);
        keys[i] = k;
    }
    std::sort(keys.begin(), keys.end());
    dmk::Tree T;
    dmk::build_tree(keys.data(), n, leaf_size, periodic != 0, &T);
    int64_t L = 0;
    for (const dmk::Box& B : T.boxes)
        L += B.leaf ? 1 : 0;
    *n_leaves = L;
    if (n_near_pairs)
        *n_near_pairs = T.n_near_pairs;
    if (L > cap)
        return fail(DMK_ERR_ARG, "cap smaller than the number of leaves");
    int64_t li = 0;
    for (const dmk::Box& B : T.boxes) {
        if (!B.leaf)
            continue;
        if (leaf_level)
            leaf_level[li] = B.level;
        if (leaf_coord) {
            leaf_coord[3 * li] = B.ix;
            leaf_coord[3 * li + 1] = B.iy;
            leaf_coord[3 * li + 2] = B.iz;
        }
        if (leaf_count)
            leaf_count[li] = B.end - B.start;
        ++li;
    }
    return DMK_OK;
}

}  // extern "C"

namespace {

// Argument checks shared by the residual-sum entry points; *T receives the
// tolerance's tables.
int residual_sum_check(const double* targets, int64_t m, const double* sources, const double* forces, int64_t ns,
                       double r_lambda, double tol, const double* out, const dmk::Tables** T)
{
    if (m < 0 || ns < 0 || !(r_lambda > 0))
        return fail(DMK_ERR_ARG, "bad sizes or r_lambda");
    if (m == 0)
        return DMK_OK;
    if (!is_device_ptr(targets) || !is_device_ptr(out) || (ns > 0 && (!is_device_ptr(sources) || !is_device_ptr(forces))))
        return fail(DMK_ERR_ARG, "arrays must be device pointers");
    *T = dmk::get_tables(tol);
    if (!*T)
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    return DMK_OK;
}

// Copies targets, sources and forces to SoA staging (tx: 3m, sx, sf: 3ns
// doubles each) and launches the brute-force residual kernel, all on st.
int residual_sum_enqueue(const double* targets, int64_t m, const double* sources, const double* forces, int64_t ns,
                         double r_lambda, const dmk::Tables& T, hipStream_t st, double* tx, double* sx, double* sf,
                         double* out)
{
    // (k,3) row-major -> SoA by strided 2D copies
    for (int d = 0; d < 3; ++d)
        HIPCHK(hipMemcpy2DAsync(tx + d * m, sizeof(double), targets + d, 3 * sizeof(double), sizeof(double), m,
                                hipMemcpyDeviceToDevice, st));
    for (int d = 0; d < 3 && ns > 0; ++d) {
        HIPCHK(hipMemcpy2DAsync(sx + d * ns, sizeof(double), sources + d, 3 * sizeof(double), sizeof(double), ns,
                                hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpy2DAsync(sf + d * ns, sizeof(double), forces + d, 3 * sizeof(double), sizeof(double), ns,
                                hipMemcpyDeviceToDevice, st));
    }
    dmk::RadialPoly poly;
    if (!make_poly(T, &poly))
        return fail(DMK_ERR_UNSUPPORTED, "radial fit degree too high");
    dmk::launch_residual_direct(tx, tx + m, tx + 2 * m, m, sx, sx + ns, sx + 2 * ns, sf, ns, r_lambda,
                                stokes_near_refine(T.prm.tol), poly, out, st);
    HIPCHK(hipGetLastError());
    return DMK_OK;
}

}  // namespace

extern "C" {

int dmk_stokes_residual_sum(const double* targets, int64_t m, const double* sources, const double* forces,
                            int64_t ns, double r_lambda, double tol, void* stream, double* out)
{
    const dmk::Tables* T = nullptr;
    const int chk = residual_sum_check(targets, m, sources, forces, ns, r_lambda, tol, out, &T);
    if (chk != DMK_OK || m == 0)
        return chk;
    hipStream_t st = (hipStream_t)stream;
    DevMem mem;
    double* tx = mem.alloc<double>(3 * m);
    double* sx = mem.alloc<double>(3 * std::max<int64_t>(ns, 1));
    double* sf = mem.alloc<double>(3 * std::max<int64_t>(ns, 1));
    if (mem.oom)
        return fail(DMK_ERR_OOM, "device allocation failed");
    const int rc = residual_sum_enqueue(targets, m, sources, forces, ns, r_lambda, *T, st, tx, sx, sf, out);
    if (rc != DMK_OK)
        return rc;
    HIPCHK(hipStreamSynchronize(st));  // temporaries are freed on return
    return DMK_OK;
}

int dmk_stokes_residual_sum_noalloc(const double* targets, int64_t m, const double* sources, const double* forces,
                                    int64_t ns, double r_lambda, double tol, void* stream, double* out)
{
    const dmk::Tables* T = nullptr;
    const int chk = residual_sum_check(targets, m, sources, forces, ns, r_lambda, tol, out, &T);
    if (chk != DMK_OK || m == 0)
        return chk;
    const size_t cap = dmk::scratch_doubles();
    if ((size_t)m > cap / 3 || (size_t)ns > cap / 6 || 3 * (size_t)m + 6 * (size_t)ns > cap)
        return fail(DMK_ERR_ARG, "3 m + 6 ns exceeds the fixed workspace of " + std::to_string(cap) +
                                     " doubles (dmk_stokes_residual_sum has no such limit)");
    double* base = nullptr;
    HIPCHK(dmk::scratch_address(&base));
    double* tx = base;
    double* sx = base + 3 * m;
    double* sf = sx + 3 * ns;
    return residual_sum_enqueue(targets, m, sources, forces, ns, r_lambda, *T, (hipStream_t)stream, tx, sx, sf, out);
}

int dmk_stokes_residual_sum_stresslet(const double* targets, int64_t m, const double* sources, const double* forces,
                                      const double* normals, int64_t ns, double r_lambda, double tol, void* stream,
                                      double* out)
{
    if (m < 0 || ns < 0 || !(r_lambda > 0))
        return fail(DMK_ERR_ARG, "bad sizes or r_lambda");
    if (m == 0)
        return DMK_OK;
    if (!is_device_ptr(targets) || !is_device_ptr(out) ||
        (ns > 0 && (!is_device_ptr(sources) || !is_device_ptr(forces) || !is_device_ptr(normals))))
        return fail(DMK_ERR_ARG, "arrays must be device pointers");
    dmk::Params prm;
    if (!dmk::select_params(tol, &prm, DMK_WINDOW_PROLATE, DMK_KERNEL_STRESSLET))
        return fail(DMK_ERR_TOL, "tol must lie in [1e-12, 1e-3]");
    const dmk::Tables* T = dmk::get_tables(prm);
    hipStream_t st = (hipStream_t)stream;
    DevMem mem;
    double* tx = mem.alloc<double>(3 * m);
    double* sx = mem.alloc<double>(3 * std::max<int64_t>(ns, 1));
    double* sf = mem.alloc<double>(6 * std::max<int64_t>(ns, 1));
    if (mem.oom)
        return fail(DMK_ERR_OOM, "device allocation failed");
    for (int d = 0; d < 3; ++d)
        HIPCHK(hipMemcpy2DAsync(tx + d * m, sizeof(double), targets + d, 3 * sizeof(double), sizeof(double), m,
                                hipMemcpyDeviceToDevice, st));
    for (int d = 0; d < 3 && ns > 0; ++d) {
        HIPCHK(hipMemcpy2DAsync(sx + d * ns, sizeof(double), sources + d, 3 * sizeof(double), sizeof(double), ns,
                                hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpy2DAsync(sf + d * ns, sizeof(double), forces + d, 3 * sizeof(double), sizeof(double), ns,
                                hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpy2DAsync(sf + (3 + d) * ns, sizeof(double), normals + d, 3 * sizeof(double), sizeof(double),
                                ns, hipMemcpyDeviceToDevice, st));
    }
    dmk::RadialPoly poly;
    if (!make_poly(*T, &poly))
        return fail(DMK_ERR_UNSUPPORTED, "radial fit degree too high");
    dmk::launch_residual_direct_t(tx, tx + m, tx + 2 * m, m, sx, sx + ns, sx + 2 * ns, sf, ns, r_lambda, poly, out,
                                  st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));  // temporaries are freed on return
    return DMK_OK;
}

}  // extern "C"
