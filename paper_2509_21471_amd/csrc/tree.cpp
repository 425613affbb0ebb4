// Adaptive octree construction, 2:1 level restriction and neighbour lists.
#include "tree.hpp"

#include <algorithm>

namespace dmk {

namespace {

// bit b of a byte -> bit 3b
struct Spread {
    uint32_t t[256];
    Spread()
    {
        for (int v = 0; v < 256; ++v) {
            uint32_t r = 0;
            for (int b = 0; b < 8; ++b)
                r |= (uint32_t)((v >> b) & 1) << (3 * b);
            t[v] = r;
        }
    }
};
const Spread kSpread;

inline uint64_t spread3(uint64_t v)
{
    return (uint64_t)kSpread.t[v & 255] | ((uint64_t)kSpread.t[(v >> 8) & 255] << 24) |
           ((uint64_t)kSpread.t[(v >> 16) & 255] << 48);
}

// level in the top bits, Morton index of the box below (digit per level = 4 bx + 2 by + bz)
inline uint64_t box_key(int level, int64_t ix, int64_t iy, int64_t iz)
{
    const uint64_t m = (spread3((uint64_t)ix) << 2) | (spread3((uint64_t)iy) << 1) | spread3((uint64_t)iz);
    return ((uint64_t)level << 58) | m;
}

// open-addressing hash map uint64 -> int (keys never equal ~0)
struct FlatMap {
    std::vector<uint64_t> k;
    std::vector<int> v;
    size_t mask = 0, count = 0;
    FlatMap() { rehash(1 << 12); }
    static inline size_t mix(uint64_t x)
    {
        x ^= x >> 33;
        x *= 0xff51afd7ed558ccdull;
        x ^= x >> 33;
        x *= 0xc4ceb9fe1a85ec53ull;
        x ^= x >> 33;
        return (size_t)x;
    }
    void rehash(size_t cap)
    {
        std::vector<uint64_t> ok;
        std::vector<int> ov;
        ok.swap(k);
        ov.swap(v);
        k.assign(cap, ~0ull);
        v.assign(cap, -1);
        mask = cap - 1;
        count = 0;
        for (size_t i = 0; i < ok.size(); ++i)
            if (ok[i] != ~0ull)
                set(ok[i], ov[i]);
    }
    void set(uint64_t key, int val)
    {
        if (2 * (count + 1) > k.size())
            rehash(2 * k.size());
        size_t i = mix(key) & mask;
        while (k[i] != ~0ull && k[i] != key)
            i = (i + 1) & mask;
        if (k[i] == ~0ull)
            ++count;
        k[i] = key;
        v[i] = val;
    }
    int get(uint64_t key) const
    {
        size_t i = mix(key) & mask;
        while (k[i] != ~0ull) {
            if (k[i] == key)
                return v[i];
            i = (i + 1) & mask;
        }
        return -1;
    }
    void clear() { rehash(1 << 12); }
};

struct Builder {
    const uint64_t* keys;
    int64_t n;
    bool periodic;
    std::vector<Box> boxes;
    FlatMap lookup;

    int64_t lower_bound(int64_t lo, int64_t hi, uint64_t v) const
    {
        return std::lower_bound(keys + lo, keys + hi, v) - keys;
    }

    int add(int level, int64_t ix, int64_t iy, int64_t iz, int parent, int64_t s, int64_t e)
    {
        Box b;
        b.level = level;
        b.ix = ix;
        b.iy = iy;
        b.iz = iz;
        b.parent = parent;
        for (int c = 0; c < 8; ++c)
            b.child[c] = -1;
        b.start = s;
        b.end = e;
        b.leaf = true;
        boxes.push_back(b);
        const int id = (int)boxes.size() - 1;
        lookup.set(box_key(level, ix, iy, iz), id);
        return id;
    }

    void split(int id)
    {
        const Box B = boxes[id];
        const int L = B.level + 1;
        const int sh = 3 * (kKeyBits - L);
        const uint64_t base = box_key(B.level, B.ix, B.iy, B.iz) & ((1ull << 58) - 1);
        int64_t s = B.start;
        int ch[8];
        for (int d = 0; d < 8; ++d) {
            const uint64_t hi_key = ((base << 3) | (uint64_t)d) + 1;
            const int64_t e = (d == 7) ? B.end : lower_bound(s, B.end, hi_key << sh);
            const int bx = (d >> 2) & 1, by = (d >> 1) & 1, bz = d & 1;
            ch[d] = add(L, 2 * B.ix + bx, 2 * B.iy + by, 2 * B.iz + bz, id, s, e);
            s = e;
        }
        Box& Bm = boxes[id];
        Bm.leaf = false;
        for (int d = 0; d < 8; ++d)
            Bm.child[d] = ch[d];
    }

    // neighbour at offset o of box (L, c); returns false outside the domain
    bool neighbour(int L, int64_t ix, int64_t iy, int64_t iz, int ox, int oy, int oz, int64_t* nx,
                   int64_t* ny, int64_t* nz, int* px, int* py, int* pz) const
    {
        const int64_t M = (int64_t)1 << L;
        int64_t c[3] = {ix + ox, iy + oy, iz + oz};
        int p[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) {
            if (c[k] < 0 || c[k] >= M) {
                if (!periodic)
                    return false;
                p[k] = c[k] < 0 ? -1 : 1;
                c[k] -= p[k] * M;
            }
        }
        *nx = c[0];
        *ny = c[1];
        *nz = c[2];
        *px = p[0];
        *py = p[1];
        *pz = p[2];
        return true;
    }

    int find(int L, int64_t ix, int64_t iy, int64_t iz) const { return lookup.get(box_key(L, ix, iy, iz)); }

    // Makes sure the box at (L, ix, iy, iz) exists, splitting the leaf that
    // currently covers that cell (and its descendants on the way) as needed.
    int ensure(int L, int64_t ix, int64_t iy, int64_t iz)
    {
        int id = find(L, ix, iy, iz);
        if (id >= 0)
            return id;
        int l = L - 1;
        int anc = -1;
        while (l >= 0 && (anc = find(l, ix >> (L - l), iy >> (L - l), iz >> (L - l))) < 0)
            --l;
        while (l < L) {  // anc is a leaf at level l covering the cell
            split(anc);
            ++l;
            const int sh = L - l;
            const int d = (int)((((ix >> sh) & 1) << 2) | (((iy >> sh) & 1) << 1) | ((iz >> sh) & 1));
            anc = boxes[anc].child[d];
        }
        return anc;
    }

    // true if a child (bits cx,cy,cz) of the neighbour at offset o touches the
    // box itself (closed boxes sharing at least a point)
    static bool child_touches(int ox, int oy, int oz, int d)
    {
        const int c[3] = {(d >> 2) & 1, (d >> 1) & 1, d & 1};
        const int o[3] = {ox, oy, oz};
        for (int k = 0; k < 3; ++k) {
            if (o[k] == 1 && c[k] != 0)
                return false;
            if (o[k] == -1 && c[k] != 1)
                return false;
        }
        return true;
    }

};

}  // namespace

void build_tree(const uint64_t* sorted_keys, int64_t n, int ns, bool periodic, Tree* T)
{
    Builder b;
    b.keys = sorted_keys;
    b.n = n;
    b.periodic = periodic;
    b.boxes.reserve(1024);
    b.add(0, 0, 0, 0, -1, 0, n);
    // adaptive refinement: split while a box holds more than ns points
    for (size_t i = 0; i < b.boxes.size(); ++i) {
        const Box& B = b.boxes[i];
        if (B.end - B.start > ns && B.level < kMaxLevel)
            b.split((int)i);
    }
    // 2:1 level restriction over vertex adjacency (empty leaves included).
    // A leaf at level L must be split when a box at level L+1 touching it has
    // children, i.e. every box at level L touching a non-leaf box at level L+1
    // must exist and be split.  Processing non-leaf boxes from the deepest
    // level upwards settles each level once: splits only create non-leaf boxes
    // at coarser levels, which are visited later.
    {
        int maxl = 0;
        for (const Box& B : b.boxes)
            maxl = std::max(maxl, B.level);
        for (int l = maxl; l >= 1; --l) {
            // non-leaf boxes at level l (including ones created by splits below)
            std::vector<int> nl;
            for (size_t i = 0; i < b.boxes.size(); ++i)
                if (b.boxes[i].level == l && !b.boxes[i].leaf)
                    nl.push_back((int)i);
            for (int id : nl) {
                const Box C = b.boxes[id];
                // boxes at level l-1 touching C: the parents' cells of C's
                // neighbour cells at level l
                for (int ox = -1; ox <= 1; ++ox)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int oz = -1; oz <= 1; ++oz) {
                            if (!ox && !oy && !oz)
                                continue;
                            int64_t nx, ny, nz;
                            int px, py, pz;
                            if (!b.neighbour(l, C.ix, C.iy, C.iz, ox, oy, oz, &nx, &ny, &nz, &px, &py, &pz))
                                continue;
                            const int Lc = l - 1;
                            const int tgt = b.ensure(Lc, nx >> 1, ny >> 1, nz >> 1);
                            if (b.boxes[tgt].leaf && b.boxes[tgt].level < kMaxLevel)
                                b.split(tgt);
                        }
            }
        }
    }
    // order by level, Morton order within a level
    std::vector<int> order(b.boxes.size());
    for (size_t i = 0; i < order.size(); ++i)
        order[i] = (int)i;
    std::vector<uint64_t> kk(b.boxes.size());
    for (size_t i = 0; i < kk.size(); ++i)
        kk[i] = box_key(b.boxes[i].level, b.boxes[i].ix, b.boxes[i].iy, b.boxes[i].iz);
    std::sort(order.begin(), order.end(), [&](int a, int c) { return kk[a] < kk[c]; });
    std::vector<int> newid(order.size());
    for (size_t i = 0; i < order.size(); ++i)
        newid[order[i]] = (int)i;
    T->boxes.resize(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
        Box B = b.boxes[order[i]];
        if (B.parent >= 0)
            B.parent = newid[B.parent];
        for (int d = 0; d < 8; ++d)
            if (B.child[d] >= 0)
                B.child[d] = newid[B.child[d]];
        T->boxes[i] = B;
    }
    T->periodic = periodic;
    T->n = n;
    T->max_level = 0;
    for (const Box& B : T->boxes)
        T->max_level = std::max(T->max_level, B.level);
    T->level_start.assign(T->max_level + 2, 0);
    for (const Box& B : T->boxes)
        T->level_start[B.level + 1]++;
    for (int l = 0; l <= T->max_level; ++l)
        T->level_start[l + 1] += T->level_start[l];

    const int nb = (int)T->boxes.size();
    // colleagues (same level, sharing a boundary point, incl. itself), top
    // down: the colleagues of a box are the children of its parent's
    // colleagues that touch it (offsets in box lengths of its own level)
    T->colleagues.assign(nb, {});
    T->colleagues[0].reserve(27);
    if (periodic) {
        for (int ox = -1; ox <= 1; ++ox)
            for (int oy = -1; oy <= 1; ++oy)
                for (int oz = -1; oz <= 1; ++oz)
                    T->colleagues[0].push_back(FarEntry{0, (int8_t)ox, (int8_t)oy, (int8_t)oz});
    } else {
        T->colleagues[0].push_back(FarEntry{0, 0, 0, 0});
    }
    for (int l = 1; l <= T->max_level; ++l) {
#pragma omp parallel for schedule(static, 64)
      for (int i = T->level_start[l]; i < T->level_start[l + 1]; ++i) {
        const Box& B = T->boxes[i];
        const int bb[3] = {(int)(B.ix & 1), (int)(B.iy & 1), (int)(B.iz & 1)};
        auto& out = T->colleagues[i];
        out.reserve(27);
        for (const FarEntry& e : T->colleagues[B.parent]) {
            const Box& C = T->boxes[e.src];
            if (C.leaf)
                continue;
            const int oP[3] = {e.ox, e.oy, e.oz};
            for (int d = 0; d < 8; ++d) {
                const int cb[3] = {(d >> 2) & 1, (d >> 1) & 1, d & 1};
                int o[3];
                bool ok = true;
                for (int k = 0; k < 3; ++k) {
                    o[k] = 2 * oP[k] + cb[k] - bb[k];
                    ok = ok && o[k] >= -1 && o[k] <= 1;
                }
                if (ok && C.child[d] >= 0)
                    out.push_back(FarEntry{C.child[d], (int8_t)o[0], (int8_t)o[1], (int8_t)o[2]});
            }
        }
      }
    }
    // periodic image shift of the colleague at offset o of box B
    auto image = [&](const Box& B, const FarEntry& e, int* px, int* py, int* pz) {
        const int64_t M = (int64_t)1 << B.level;
        const int64_t c[3] = {B.ix + e.ox, B.iy + e.oy, B.iz + e.oz};
        int pp[3];
        for (int k = 0; k < 3; ++k)
            pp[k] = c[k] < 0 ? -1 : (c[k] >= M ? 1 : 0);
        *px = pp[0];
        *py = pp[1];
        *pz = pp[2];
    };
    // difference-kernel exchange (leaf/non-leaf rule): a non-leaf box receives
    // D_l from every non-empty colleague; a leaf receives D_l only from
    // non-leaf colleagues.  Adjacent leaves then exchange the residual at the
    // finer of their two levels directly, and every pair of points telescopes
    // M_0 + sum D_l + R_lambda = K (or the omitted terms vanish by support).
    T->incoming.assign(nb, {});
    for (int i = 0; i < nb; ++i) {
        const Box& B = T->boxes[i];
        if (B.end == B.start)
            continue;
        for (const FarEntry& e : T->colleagues[i]) {
            const Box& C = T->boxes[e.src];
            if (C.end == C.start)
                continue;
            if (!B.leaf || !C.leaf)
                T->incoming[i].push_back(e);
        }
    }
    // near lists: adjacent non-empty leaves at levels L-1, L, L+1
    T->leaves.clear();
    for (int i = 0; i < nb; ++i)
        if (T->boxes[i].leaf && T->boxes[i].end > T->boxes[i].start)
            T->leaves.push_back(i);
    const int nl = (int)T->leaves.size();
    T->near.assign(nl, {});
    int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : pairs)
    for (int li = 0; li < nl; ++li) {
        const int i = T->leaves[li];
        const Box& B = T->boxes[i];
        std::vector<NearEntry>& list = T->near[li];
        list.reserve(64);
        auto add_entry = [&](int S, int px, int py, int pz, int lam) {
            const Box& Sb = T->boxes[S];
            if (Sb.end == Sb.start)
                return;
            list.push_back(NearEntry{S, (int8_t)px, (int8_t)py, (int8_t)pz, (int8_t)lam});
            pairs += (B.end - B.start) * (Sb.end - Sb.start);
        };
        for (const FarEntry& e : T->colleagues[i]) {
            int px, py, pz;
            image(B, e, &px, &py, &pz);
            const int C = e.src;
            if (T->boxes[C].leaf) {
                add_entry(C, px, py, pz, B.level);  // colleague leaf
            } else {
                for (int d = 0; d < 8; ++d) {  // fine neighbours
                    const int ch = T->boxes[C].child[d];
                    if (ch >= 0 && T->boxes[ch].leaf && Builder::child_touches(e.ox, e.oy, e.oz, d))
                        add_entry(ch, px, py, pz, B.level + 1);
                }
            }
        }
        if (B.parent >= 0) {  // coarse neighbours: leaf colleagues of the parent touching B
            const Box& P = T->boxes[B.parent];
            const int bx = (int)(B.ix & 1), by = (int)(B.iy & 1), bz = (int)(B.iz & 1);
            for (const FarEntry& e : T->colleagues[B.parent]) {
                if (!e.ox && !e.oy && !e.oz)
                    continue;
                const Box& C = T->boxes[e.src];
                if (!C.leaf)
                    continue;
                const int o[3] = {e.ox, e.oy, e.oz};
                const int bb[3] = {bx, by, bz};
                bool touch = true;
                for (int k = 0; k < 3; ++k)
                    if ((o[k] == 1 && bb[k] != 1) || (o[k] == -1 && bb[k] != 0))
                        touch = false;
                if (!touch)
                    continue;
                // periodic image shift of the parent's colleague
                int px, py, pz;
                image(P, e, &px, &py, &pz);
                add_entry(e.src, px, py, pz, B.level);
            }
        }
    }
    T->n_near_pairs = pairs;
}

void merge_forest(std::vector<Tree>& parts, const std::vector<int64_t>& offsets, Tree* out, std::vector<int>* roots)
{
    const int np = (int)parts.size();
    Tree& F = *out;
    F = Tree();
    F.periodic = np > 0 && parts[0].periodic;
    int maxl = 0;
    for (const Tree& t : parts)
        maxl = std::max(maxl, t.max_level);
    F.max_level = maxl;
    // new index of box i of tree t: level-major, problem order within a level
    std::vector<std::vector<int>> remap(np);
    std::vector<int> count(maxl + 1, 0);
    for (const Tree& t : parts)
        for (int l = 0; l <= t.max_level; ++l)
            count[l] += t.level_start[l + 1] - t.level_start[l];
    F.level_start.assign(maxl + 2, 0);
    for (int l = 0; l <= maxl; ++l)
        F.level_start[l + 1] = F.level_start[l] + count[l];
    std::vector<int> fill(F.level_start.begin(), F.level_start.end() - 1);
    for (int t = 0; t < np; ++t) {
        const Tree& T = parts[t];
        remap[t].assign(T.boxes.size(), -1);
        for (int l = 0; l <= T.max_level; ++l)
            for (int i = T.level_start[l]; i < T.level_start[l + 1]; ++i)
                remap[t][i] = fill[l]++;
    }
    const int nb = F.level_start[maxl + 1];
    F.boxes.resize(nb);
    F.colleagues.resize(nb);
    F.incoming.resize(nb);
    roots->assign(np, -1);
    for (int t = 0; t < np; ++t) {
        const Tree& T = parts[t];
        const std::vector<int>& R = remap[t];
        auto m = [&](int i) { return i < 0 ? -1 : R[i]; };
        const int64_t off = offsets[t];
        for (int i = 0; i < (int)T.boxes.size(); ++i) {
            Box b = T.boxes[i];
            b.parent = m(b.parent);
            for (int c = 0; c < 8; ++c)
                b.child[c] = m(b.child[c]);
            b.start += off;
            b.end += off;
            F.boxes[R[i]] = b;
            std::vector<FarEntry> col = T.colleagues[i];
            for (FarEntry& e : col)
                e.src = R[e.src];
            F.colleagues[R[i]] = std::move(col);
            std::vector<FarEntry> inc = T.incoming[i];
            for (FarEntry& e : inc)
                e.src = R[e.src];
            F.incoming[R[i]] = std::move(inc);
        }
        for (int li = 0; li < (int)T.leaves.size(); ++li) {
            F.leaves.push_back(R[T.leaves[li]]);
            std::vector<NearEntry> nl = T.near[li];
            for (NearEntry& e : nl)
                e.src = R[e.src];
            F.near.push_back(std::move(nl));
        }
        (*roots)[t] = R[0];
        F.n += T.n;
        F.n_near_pairs += T.n_near_pairs;
    }
}

}  // namespace dmk
