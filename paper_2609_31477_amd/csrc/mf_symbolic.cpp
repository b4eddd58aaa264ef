// Host symbolic analysis: the specified nested-dissection front tree.
//
// The paper computes one fill-reducing analysis per sparsity pattern and reuses
// it for every later factorization (Sec. 6, "Scaling").  Its orderings (ParMetis
// in 2D, Scotch in 3D) are not reproducible bit for bit; this analysis is
// fully specified so that an independent implementation reproduces it exactly:
//   * G = pattern(A) U pattern(A^T) without self loops, root set R removed;
//   * components in order of their minimum vertex;
//   * ND(K): leaves of at most leaf_max vertices; otherwise a George-Liu
//     pseudo-peripheral root (start at min(K); from the last BFS level take the
//     vertex of least degree within K, lowest index on ties; move there while
//     the eccentricity grows); e < 2 makes K a leaf; split level j = first
//     level whose cumulative size reaches |K|/2, clamped to [1, e-1]; the
//     separator is the part of L_j adjacent to L_{j+1}; recurse on the
//     components of K \ S in min-index order, then emit S;
//   * R last, as the root front (pivots in the given order);
//   * fronts numbered in completion order; rows(f) = pivots, then ascending new
//     index of the children's non-pivot rows and of the neighbours of the pivots
//     numbered after the last pivot; var_etree = Liu's elimination tree.
// Every set above is a set, so BFS visiting order never matters; only the
// explicit tie-breaks do.
#include <algorithm>
#include <numeric>
#include <stdexcept>

#include "mf_internal.h"

namespace mf {
namespace {

struct Graph {
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
};

Graph symmetric_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind) {
    Graph g;
    g.n = n;
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t r = 0; r < n; r++)
        for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) {
            int64_t c = colind[t];
            if (c == r) continue;
            deg[r]++;
            deg[c]++;
        }
    std::vector<int64_t> ptr(n + 1, 0);
    for (int64_t i = 0; i < n; i++) ptr[i + 1] = ptr[i] + deg[i];
    std::vector<int32_t> adj(ptr[n]);
    std::vector<int64_t> nxt(ptr.begin(), ptr.end() - 1);
    for (int64_t r = 0; r < n; r++)
        for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) {
            int64_t c = colind[t];
            if (c == r) continue;
            adj[nxt[r]++] = (int32_t)c;
            adj[nxt[c]++] = (int32_t)r;
        }
    // sort + unique each row, compact
    g.ptr.assign(n + 1, 0);
    int64_t w = 0;
    for (int64_t r = 0; r < n; r++) {
        auto b = adj.begin() + ptr[r], e = adj.begin() + ptr[r + 1];
        std::sort(b, e);
        auto u = std::unique(b, e);
        int64_t cnt = u - b;
        std::copy(b, u, adj.begin() + w);  // w <= ptr[r]: safe left shift
        w += cnt;
        g.ptr[r + 1] = w;
    }
    adj.resize(w);
    adj.shrink_to_fit();
    g.adj = std::move(adj);
    return g;
}

class ND {
   public:
    ND(const Graph& g, int32_t leaf_max) : g_(g), leaf_max_(leaf_max), mask_(g.n, 0), lev_(g.n, -1) {}

    // Fronts as emitted: pivot lists and child lists.
    std::vector<std::vector<int32_t>> piv;
    std::vector<std::vector<int32_t>> children;

    int32_t emit(std::vector<int32_t> p, std::vector<int32_t> ch) {
        piv.push_back(std::move(p));
        children.push_back(std::move(ch));
        return (int32_t)piv.size() - 1;
    }

    // Components of the sorted vertex set K, ordered by minimum vertex.
    std::vector<std::vector<int32_t>> components(const std::vector<int32_t>& K) {
        for (int32_t v : K) mask_[v] = 1;
        std::vector<std::vector<int32_t>> comps;
        for (int32_t v : K) {
            if (lev_[v] >= 0) continue;
            std::vector<int32_t> comp;
            lev_[v] = 0;
            comp.push_back(v);
            for (size_t h = 0; h < comp.size(); h++) {
                int32_t u = comp[h];
                for (int64_t t = g_.ptr[u]; t < g_.ptr[u + 1]; t++) {
                    int32_t w = g_.adj[t];
                    if (mask_[w] && lev_[w] < 0) {
                        lev_[w] = 0;
                        comp.push_back(w);
                    }
                }
            }
            std::sort(comp.begin(), comp.end());
            comps.push_back(std::move(comp));
        }
        for (int32_t v : K) {
            mask_[v] = 0;
            lev_[v] = -1;
        }
        return comps;
    }

    int32_t run(const std::vector<int32_t>& K0) {
        struct Frame {
            std::vector<int32_t> K;
            std::vector<int32_t> S;
            std::vector<std::vector<int32_t>> comps;
            size_t next = 0;
            std::vector<int32_t> tops;
            bool split = false;
        };
        std::vector<Frame> stack;
        stack.push_back(Frame{K0, {}, {}, 0, {}, false});
        int32_t ret = -1;
        while (!stack.empty()) {
            Frame& fr = stack.back();
            if (!fr.split) {
                std::vector<int32_t> S;
                if ((int64_t)fr.K.size() <= leaf_max_ || !separator(fr.K, S)) {
                    ret = emit(fr.K, {});
                    stack.pop_back();
                    if (!stack.empty()) stack.back().tops.push_back(ret);
                    continue;
                }
                std::vector<int32_t> rest;
                rest.reserve(fr.K.size() - S.size());
                std::set_difference(fr.K.begin(), fr.K.end(), S.begin(), S.end(), std::back_inserter(rest));
                fr.S = std::move(S);
                fr.comps = components(rest);
                fr.split = true;
                fr.next = 0;
            }
            if (fr.next < fr.comps.size()) {
                std::vector<int32_t> C = std::move(fr.comps[fr.next]);
                fr.next++;
                stack.push_back(Frame{std::move(C), {}, {}, 0, {}, false});
                continue;
            }
            ret = emit(fr.S, fr.tops);
            stack.pop_back();
            if (!stack.empty()) stack.back().tops.push_back(ret);
        }
        return ret;
    }

   private:
    // BFS level structure from r inside the mask; order[] holds vertices level by level.
    void bfs(int32_t r, std::vector<int32_t>& order, std::vector<int64_t>& lptr) {
        order.clear();
        lptr.clear();
        order.push_back(r);
        lev_[r] = 0;
        lptr.push_back(0);
        int64_t head = 0;
        int32_t d = 0;
        while (true) {
            int64_t end = (int64_t)order.size();
            lptr.push_back(end);
            for (int64_t h = head; h < end; h++) {
                int32_t u = order[h];
                for (int64_t t = g_.ptr[u]; t < g_.ptr[u + 1]; t++) {
                    int32_t w = g_.adj[t];
                    if (mask_[w] && lev_[w] < 0) {
                        lev_[w] = d + 1;
                        order.push_back(w);
                    }
                }
            }
            if ((int64_t)order.size() == end) break;
            head = end;
            d++;
        }
    }
    void clear(const std::vector<int32_t>& order) {
        for (int32_t v : order) lev_[v] = -1;
    }

    bool separator(const std::vector<int32_t>& K, std::vector<int32_t>& S) {
        for (int32_t v : K) mask_[v] = 1;
        std::vector<int32_t> order, ox;
        std::vector<int64_t> lptr, lx;
        int32_t r = K[0];
        bfs(r, order, lptr);
        int32_t e = (int32_t)lptr.size() - 2;
        while (true) {
            int32_t x = -1;
            int64_t best = -1;
            for (int64_t h = lptr[e]; h < lptr[e + 1]; h++) {
                int32_t v = order[h];
                int64_t dg = 0;
                for (int64_t t = g_.ptr[v]; t < g_.ptr[v + 1]; t++) dg += mask_[g_.adj[t]];
                if (best < 0 || dg < best || (dg == best && v < x)) {
                    best = dg;
                    x = v;
                }
            }
            clear(order);
            bfs(x, ox, lx);
            int32_t ex = (int32_t)lx.size() - 2;
            if (ex > e) {
                order.swap(ox);
                lptr.swap(lx);
                e = ex;
                r = x;
                continue;
            }
            clear(ox);
            bfs(r, order, lptr);
            break;
        }
        bool ok = e >= 2;
        if (ok) {
            int64_t Ksz = (int64_t)K.size();
            int32_t j = -1;
            for (int32_t l = 0; l <= e; l++)
                if (2 * lptr[l + 1] >= Ksz) {
                    j = l;
                    break;
                }
            j = std::min(std::max(j, 1), e - 1);
            S.clear();
            for (int64_t h = lptr[j]; h < lptr[j + 1]; h++) {
                int32_t v = order[h];
                for (int64_t t = g_.ptr[v]; t < g_.ptr[v + 1]; t++) {
                    int32_t w = g_.adj[t];
                    if (mask_[w] && lev_[w] == j + 1) {
                        S.push_back(v);
                        break;
                    }
                }
            }
            std::sort(S.begin(), S.end());
        }
        clear(order);
        for (int32_t v : K) mask_[v] = 0;
        return ok;
    }

    const Graph& g_;
    int32_t leaf_max_;
    std::vector<char> mask_;
    std::vector<int32_t> lev_;
};

}  // namespace

void analyze_pattern(Symbolic& S, int64_t n, const int64_t* rowptr, const int32_t* colind,
                     int32_t nroot, const int32_t* root_idx, int32_t leaf_max) {
    if (n < 0 || n > INT32_MAX - 1) throw std::invalid_argument("n out of range");
    if (leaf_max < 1) throw std::invalid_argument("leaf_max must be >= 1");
    if (nroot < 0 || nroot > n) throw std::invalid_argument("nroot out of range");
    if ((n > 0 || nroot > 0) && (!rowptr || (nroot > 0 && !root_idx))) throw std::invalid_argument("null pointer");
    if (rowptr && rowptr[0] != 0) throw std::invalid_argument("rowptr[0] != 0");
    for (int64_t i = 0; i < n; i++)
        if (rowptr[i + 1] < rowptr[i]) throw std::invalid_argument("rowptr not monotone");
    int64_t nnz = n > 0 ? rowptr[n] : 0;
    if (nnz > 0 && !colind) throw std::invalid_argument("null colind");
    if (nnz > INT32_MAX) throw std::invalid_argument("nnz above 2^31-1 is not supported");
    for (int64_t t = 0; t < nnz; t++)
        if (colind[t] < 0 || colind[t] >= n) throw std::invalid_argument("column index out of range");
    std::vector<char> inroot(n, 0);
    for (int32_t i = 0; i < nroot; i++) {
        int32_t v = root_idx[i];
        if (v < 0 || v >= n || inroot[v]) throw std::invalid_argument("bad root index");
        inroot[v] = 1;
    }
    S.n = n;
    S.nnz = nnz;
    S.leaf_max = leaf_max;
    S.seg_row0 = {0};
    S.seg_n = {n};
    S.seg_nnz0 = {0};
    S.rowptr.assign(rowptr, rowptr + n + 1);
    S.colind.assign(colind, colind + nnz);
    S.root.assign(root_idx, root_idx + nroot);

    Graph g = symmetric_pattern(n, rowptr, colind);
    ND nd(g, leaf_max);
    std::vector<int32_t> active;
    active.reserve(n);
    for (int64_t v = 0; v < n; v++)
        if (!inroot[v]) active.push_back((int32_t)v);
    std::vector<int32_t> tops;
    for (auto& K : nd.components(active)) tops.push_back(nd.run(K));
    if (nroot > 0) nd.emit(S.root, tops);

    const int32_t nf = (int32_t)nd.piv.size();
    S.nf = nf;
    S.front_parent.assign(nf, -1);
    for (int32_t f = 0; f < nf; f++)
        for (int32_t c : nd.children[f]) S.front_parent[c] = f;
    S.front_ptr.assign(nf + 1, 0);
    S.perm.clear();
    S.perm.reserve(n);
    for (int32_t f = 0; f < nf; f++) {
        S.perm.insert(S.perm.end(), nd.piv[f].begin(), nd.piv[f].end());
        S.front_ptr[f + 1] = (int32_t)S.perm.size();
    }
    std::vector<int32_t> newidx(n);
    for (int64_t i = 0; i < n; i++) newidx[S.perm[i]] = (int32_t)i;

    // front rows: pivots, then ascending new index of the union of the children's
    // non-pivot rows and the pivots' neighbours numbered after the last pivot
    std::vector<std::vector<int32_t>> cb(nf);  // non-pivot rows, as new indices
    std::vector<char> seen(n, 0);
    S.rows_ptr.assign(nf + 1, 0);
    S.rows.clear();
    for (int32_t f = 0; f < nf; f++) {
        int32_t lo = S.front_ptr[f], hi = S.front_ptr[f + 1];
        std::vector<int32_t> cand;
        for (int32_t k = lo; k < hi; k++) {
            int32_t v = S.perm[k];
            for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; t++) {
                int32_t u = newidx[g.adj[t]];
                if (u >= hi && !seen[u]) {
                    seen[u] = 1;
                    cand.push_back(u);
                }
            }
        }
        for (int32_t c : nd.children[f]) {
            for (int32_t u : cb[c])
                if (u >= hi && !seen[u]) {
                    seen[u] = 1;
                    cand.push_back(u);
                }
            std::vector<int32_t>().swap(cb[c]);
        }
        std::sort(cand.begin(), cand.end());
        for (int32_t u : cand) seen[u] = 0;
        for (int32_t k = lo; k < hi; k++) S.rows.push_back(S.perm[k]);
        for (int32_t u : cand) S.rows.push_back(S.perm[u]);
        S.rows_ptr[f + 1] = (int64_t)S.rows.size();
        cb[f] = std::move(cand);
    }

    // Liu's elimination tree with path compression
    S.var_etree.assign(n, -1);
    {
        std::vector<int32_t> anc(n, -1);
        for (int64_t j = 0; j < n; j++) {
            int32_t v = S.perm[j];
            for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; t++) {
                int32_t r = newidx[g.adj[t]];
                if (r >= j) continue;
                while (true) {
                    int32_t a = anc[r];
                    if (a == j) break;
                    anc[r] = (int32_t)j;
                    if (a == -1) {
                        S.var_etree[r] = (int32_t)j;
                        break;
                    }
                    r = a;
                }
            }
        }
    }

    // ---------------- derived data for the numeric phase
    S.npiv.resize(nf);
    S.mnom.resize(nf);
    S.nominal_flops = 0.0;
    S.nominal_nnz_lu = 0.0;
    for (int32_t f = 0; f < nf; f++) {
        S.npiv[f] = S.front_ptr[f + 1] - S.front_ptr[f];
        S.mnom[f] = (int32_t)(S.rows_ptr[f + 1] - S.rows_ptr[f]);
        double m = S.mnom[f], p = S.npiv[f];
        for (int64_t i = (int64_t)(m - p); i < (int64_t)m; i++) S.nominal_flops += (double)i + 2.0 * (double)i * (double)i;
        S.nominal_nnz_lu += 2.0 * m * p - p * p;
    }
    S.child_ptr.assign(nf + 1, 0);
    for (int32_t f = 0; f < nf; f++)
        if (S.front_parent[f] >= 0) S.child_ptr[S.front_parent[f] + 1]++;
    for (int32_t f = 0; f < nf; f++) S.child_ptr[f + 1] += S.child_ptr[f];
    S.child_idx.assign(S.child_ptr[nf], 0);
    {
        std::vector<int32_t> nx(S.child_ptr.begin(), S.child_ptr.end() - 1);
        for (int32_t f = 0; f < nf; f++)
            if (S.front_parent[f] >= 0) S.child_idx[nx[S.front_parent[f]]++] = f;
    }
    S.level.assign(nf, 0);
    S.nlevels = 0;
    for (int32_t f = 0; f < nf; f++) {  // children precede parents
        int32_t l = 0;
        for (int32_t t = S.child_ptr[f]; t < S.child_ptr[f + 1]; t++) l = std::max(l, S.level[S.child_idx[t]] + 1);
        S.level[f] = l;
        S.nlevels = std::max(S.nlevels, l + 1);
    }
    S.level_ptr.assign(S.nlevels + 1, 0);
    for (int32_t f = 0; f < nf; f++) S.level_ptr[S.level[f] + 1]++;
    for (int32_t l = 0; l < S.nlevels; l++) S.level_ptr[l + 1] += S.level_ptr[l];
    S.level_fronts.assign(nf, 0);
    {
        std::vector<int32_t> nx(S.level_ptr.begin(), S.level_ptr.end() - 1);
        for (int32_t f = 0; f < nf; f++) S.level_fronts[nx[S.level[f]]++] = f;
    }

    // inverse nominal maps child -> parent
    S.imap_off.assign(nf + 1, 0);
    for (int32_t f = 0; f < nf; f++) {
        int32_t p = S.front_parent[f];
        S.imap_off[f + 1] = S.imap_off[f] + (p >= 0 ? S.mnom[p] : 0);
    }
    S.imap.assign(S.imap_off[nf], -1);
    {
        std::vector<int32_t> pos(n, -1);
        for (int32_t c = 0; c < nf; c++) {
            int32_t p = S.front_parent[c];
            if (p < 0) continue;
            const int32_t* rc = S.rows.data() + S.rows_ptr[c];
            for (int32_t t = S.npiv[c]; t < S.mnom[c]; t++) pos[rc[t]] = t - S.npiv[c];
            const int32_t* rp = S.rows.data() + S.rows_ptr[p];
            int32_t* im = S.imap.data() + S.imap_off[c];
            int32_t found = 0;
            for (int32_t i = 0; i < S.mnom[p]; i++) {
                im[i] = pos[rp[i]];
                found += im[i] >= 0;
            }
            for (int32_t t = S.npiv[c]; t < S.mnom[c]; t++) pos[rc[t]] = -1;
            if (found != S.mnom[c] - S.npiv[c]) throw std::runtime_error("internal: child rows not in parent");
        }
    }

    // original entries -> (front, nominal row position, nominal col position)
    {
        std::vector<int32_t> front_of_new(n);
        for (int32_t f = 0; f < nf; f++)
            for (int32_t k = S.front_ptr[f]; k < S.front_ptr[f + 1]; k++) front_of_new[k] = f;
        std::vector<int32_t> efront(nnz);
        std::vector<int64_t> cnt(nf + 1, 0);
        for (int64_t r = 0; r < n; r++)
            for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) {
                int32_t a = newidx[r], b = newidx[colind[t]];
                efront[t] = front_of_new[std::min(a, b)];
                cnt[efront[t] + 1]++;
            }
        // front order = level order
        std::vector<int32_t> order_pos(nf);
        for (int32_t i = 0; i < nf; i++) order_pos[S.level_fronts[i]] = i;
        std::vector<int64_t> start(nf + 1, 0);
        for (int32_t i = 0; i < nf; i++) start[i + 1] = start[i] + cnt[S.level_fronts[i] + 1];
        std::vector<int64_t> nx(start.begin(), start.end() - 1);
        std::vector<int64_t> byfront(nnz);
        std::vector<int32_t> erow(nnz);
        for (int64_t r = 0; r < n; r++)
            for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) {
                byfront[nx[order_pos[efront[t]]]++] = t;
                erow[t] = (int32_t)r;
            }
        std::vector<int32_t> pos(n, -1);
        S.ue_front.clear();
        S.ue_row.clear();
        S.ue_col.clear();
        S.ue_src_ptr.assign(1, 0);
        S.ue_src.clear();
        S.level_ue_ptr.assign(S.nlevels + 1, 0);
        std::vector<std::pair<int64_t, int64_t>> key;  // (col*m + row, csr pos)
        for (int32_t i = 0; i < nf; i++) {
            int32_t f = S.level_fronts[i];
            const int32_t* rf = S.rows.data() + S.rows_ptr[f];
            int32_t m = S.mnom[f];
            for (int32_t t = 0; t < m; t++) pos[rf[t]] = t;
            key.clear();
            for (int64_t q = start[i]; q < start[i + 1]; q++) {
                int64_t t = byfront[q];
                int32_t rp = pos[erow[t]], cp = pos[colind[t]];
                if (rp < 0 || cp < 0) throw std::runtime_error("internal: entry outside its front");
                key.emplace_back((int64_t)cp * m + rp, t);
            }
            std::sort(key.begin(), key.end());
            for (size_t q = 0; q < key.size(); q++) {
                if (q == 0 || key[q].first != key[q - 1].first) {
                    if (q > 0) S.ue_src_ptr.push_back((int64_t)S.ue_src.size());
                    S.ue_front.push_back(f);
                    S.ue_row.push_back((int32_t)(key[q].first % m));
                    S.ue_col.push_back((int32_t)(key[q].first / m));
                }
                S.ue_src.push_back((int32_t)key[q].second);
            }
            if (!key.empty()) S.ue_src_ptr.push_back((int64_t)S.ue_src.size());
            for (int32_t t = 0; t < m; t++) pos[rf[t]] = -1;
            S.level_ue_ptr[S.level[f] + 1] = (int64_t)S.ue_front.size();
        }
        for (int32_t l = 0; l < S.nlevels; l++)
            S.level_ue_ptr[l + 1] = std::max(S.level_ue_ptr[l + 1], S.level_ue_ptr[l]);
    }
}

void merge_symbolic(Symbolic& M, const std::vector<const Symbolic*>& parts, bool light) {
    M = Symbolic();
    M.seg_row0.clear();
    M.seg_n.clear();
    M.seg_nnz0.clear();
    // sizes first, then bulk fills with offsets (no per-element growth)
    int64_t N = 0, NNZ = 0, NROWS = 0, NIMAP = 0, NUE = 0, NSRC = 0, NROOT = 0;
    int32_t NF = 0;
    for (const Symbolic* P : parts) {
        N += P->n;
        NNZ += P->nnz;
        NF += P->nf;
        NROWS += (int64_t)P->rows.size();
        NIMAP += (int64_t)P->imap.size();
        NUE += (int64_t)P->ue_front.size();
        NSRC += (int64_t)P->ue_src.size();
        NROOT += (int64_t)P->root.size();
    }
    if (NNZ > INT32_MAX) throw std::invalid_argument("batch nnz above 2^31-1 is not supported");
    M.n = N;
    M.nnz = NNZ;
    M.nf = NF;
    M.leaf_max = parts.empty() ? 64 : parts[0]->leaf_max;
    M.light = light;
    M.n_ue = NUE;
    M.n_src = NSRC;
    if (!light) {
        M.rowptr.resize(N + 1);
        M.colind.resize(NNZ);
    }
    M.root.reserve(NROOT);
    M.perm.resize(N);
    M.var_etree.resize(N);
    M.front_ptr.resize(NF + 1);
    M.front_parent.resize(NF);
    M.rows_ptr.resize(NF + 1);
    M.rows.resize(NROWS);
    M.npiv.resize(NF);
    M.mnom.resize(NF);
    M.level.resize(NF);
    M.imap.resize(NIMAP);
    M.imap_off.resize(NF + 1);
    if (!light) M.rowptr[0] = 0;
    M.front_ptr[0] = 0;
    M.rows_ptr[0] = 0;
    M.imap_off[0] = 0;
    int64_t voff = 0, eoff = 0, roff = 0, ioff = 0;
    int32_t foff = 0;
    for (size_t q = 0; q < parts.size(); q++) {
        const Symbolic& P = *parts[q];
        M.seg_row0.push_back(voff);
        M.seg_n.push_back(P.n);
        M.seg_nnz0.push_back(eoff);
        const int32_t v32 = (int32_t)voff;
        if (!light) {
            for (int64_t r = 0; r < P.n; r++) M.rowptr[voff + r + 1] = P.rowptr[r + 1] + eoff;
            for (int64_t t = 0; t < P.nnz; t++) M.colind[eoff + t] = P.colind[t] + v32;
        }
        for (int32_t v : P.root) M.root.push_back(v + v32);
        for (int64_t i = 0; i < P.n; i++) {
            M.perm[voff + i] = P.perm[i] + v32;
            M.var_etree[voff + i] = P.var_etree[i] < 0 ? -1 : P.var_etree[i] + v32;
        }
        for (size_t t = 0; t < P.rows.size(); t++) M.rows[roff + (int64_t)t] = P.rows[t] + v32;
        std::copy(P.imap.begin(), P.imap.end(), M.imap.begin() + ioff);
        for (int32_t f = 0; f < P.nf; f++) {
            M.front_ptr[foff + f + 1] = P.front_ptr[f + 1] + v32;
            M.front_parent[foff + f] = P.front_parent[f] < 0 ? -1 : P.front_parent[f] + foff;
            M.rows_ptr[foff + f + 1] = P.rows_ptr[f + 1] + roff;
            M.imap_off[foff + f + 1] = P.imap_off[f + 1] + ioff;
            M.npiv[foff + f] = P.npiv[f];
            M.mnom[foff + f] = P.mnom[f];
            M.level[foff + f] = P.level[f];
        }
        M.nominal_flops += P.nominal_flops;
        M.nominal_nnz_lu += P.nominal_nnz_lu;
        M.nlevels = std::max(M.nlevels, P.nlevels);
        voff += P.n;
        eoff += P.nnz;
        foff += P.nf;
        roff += (int64_t)P.rows.size();
        ioff += (int64_t)P.imap.size();
    }
    const int32_t nf = M.nf;
    M.child_ptr.assign(nf + 1, 0);
    for (int32_t f = 0; f < nf; f++)
        if (M.front_parent[f] >= 0) M.child_ptr[M.front_parent[f] + 1]++;
    for (int32_t f = 0; f < nf; f++) M.child_ptr[f + 1] += M.child_ptr[f];
    M.child_idx.assign(M.child_ptr[nf], 0);
    {
        std::vector<int32_t> nx(M.child_ptr.begin(), M.child_ptr.end() - 1);
        for (int32_t f = 0; f < nf; f++)
            if (M.front_parent[f] >= 0) M.child_idx[nx[M.front_parent[f]]++] = f;
    }
    M.level_ptr.assign(M.nlevels + 1, 0);
    for (int32_t f = 0; f < nf; f++) M.level_ptr[M.level[f] + 1]++;
    for (int32_t l = 0; l < M.nlevels; l++) M.level_ptr[l + 1] += M.level_ptr[l];
    M.level_fronts.assign(nf, 0);
    {
        std::vector<int32_t> nx(M.level_ptr.begin(), M.level_ptr.end() - 1);
        for (int32_t f = 0; f < nf; f++) M.level_fronts[nx[M.level[f]]++] = f;
    }
    // unique entries in level order, system by system within a level
    M.level_ue_ptr.assign(M.nlevels + 1, 0);
    std::vector<int32_t> foffs(parts.size() + 1, 0);
    for (size_t q = 0; q < parts.size(); q++) foffs[q + 1] = foffs[q] + parts[q]->nf;
    if (light) {
        // per (level, system): where the system's own maps go in the batch; a
        // system's level-l fronts follow those of the systems before it, so
        // batch slot = level start + fronts of earlier systems at l + own index
        int64_t uo = 0, so = 0;
        for (int32_t l = 0; l < M.nlevels; l++) {
            int32_t before = 0;
            for (size_t q = 0; q < parts.size(); q++) {
                const Symbolic& P = *parts[q];
                if (l >= P.nlevels) continue;
                const int64_t u0 = P.level_ue_ptr[l], u1 = P.level_ue_ptr[l + 1];
                const int32_t own = P.level_ptr[l + 1] - P.level_ptr[l];
                Symbolic::UeBlock b;
                b.part = (int32_t)q;
                b.slot_delta = M.level_ptr[l] + before - P.level_ptr[l];
                b.u0 = u0;
                b.cnt = u1 - u0;
                b.dst_u = uo;
                b.s0 = P.ue_src_ptr[u0];
                b.scnt = P.ue_src_ptr[u1] - P.ue_src_ptr[u0];
                b.dst_s = so;
                if (b.cnt) M.ue_blocks.push_back(b);
                uo += b.cnt;
                so += b.scnt;
                before += own;
            }
            M.level_ue_ptr[l + 1] = uo;
        }
        if (M.nnz > INT32_MAX) throw std::invalid_argument("batch nnz above 2^31-1 is not supported");
        return;
    }
    M.ue_front.resize(NUE);
    M.ue_row.resize(NUE);
    M.ue_col.resize(NUE);
    M.ue_src_ptr.resize(NUE + 1);
    M.ue_src.resize(NSRC);
    M.ue_src_ptr[0] = 0;
    int64_t uo = 0, so = 0;
    for (int32_t l = 0; l < M.nlevels; l++) {
        for (size_t q = 0; q < parts.size(); q++) {
            const Symbolic& P = *parts[q];
            if (l >= P.nlevels) continue;
            const int32_t e32 = (int32_t)M.seg_nnz0[q];
            const int64_t u0 = P.level_ue_ptr[l], u1 = P.level_ue_ptr[l + 1];
            for (int64_t u = u0; u < u1; u++, uo++) {
                M.ue_front[uo] = P.ue_front[u] + foffs[q];
                M.ue_row[uo] = P.ue_row[u];
                M.ue_col[uo] = P.ue_col[u];
                for (int64_t t = P.ue_src_ptr[u]; t < P.ue_src_ptr[u + 1]; t++) M.ue_src[so++] = P.ue_src[t] + e32;
                M.ue_src_ptr[uo + 1] = so;
            }
        }
        M.level_ue_ptr[l + 1] = uo;
    }
    if (M.nnz > INT32_MAX) throw std::invalid_argument("batch nnz above 2^31-1 is not supported");
}

}  // namespace mf
