// CPU emulation of the persistent sweeps' work-list protocol on random front
// forests: work-groups take bundles by ticket from one counter and, inside a
// task, wait on the same per-front counts the kernels wait on (children
// finished / parent finished, fully summed blocks finished) and post the same
// updates.  Random interleavings of 1..64 work-groups must never deadlock, must
// run every task exactly once, and every task must run only after the tasks
// whose data it reads (checked against the tree itself, not the counters).
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2609_31477_amd/csrc/mf_tasks.h"

using namespace mf;

struct Forest {
    int ns = 0, nlevels = 0, first = 0;  // first: lowest listed level (the rest ran before / runs after)
    std::vector<int32_t> level_ptr, parent, m, k, level;
    std::vector<std::vector<int>> kids;
    bool listed(int s) const { return level[s] >= first; }
};

static Forest random_forest(std::mt19937& rng) {
    Forest F;
    F.nlevels = 1 + (int)(rng() % 7);
    F.level_ptr.push_back(0);
    std::vector<int> level_of;
    for (int L = 0; L < F.nlevels; L++) {
        const int cnt = 1 + (int)(rng() % (L + 1 == F.nlevels ? 3 : 12));
        for (int i = 0; i < cnt; i++) level_of.push_back(L);
        F.level_ptr.push_back((int32_t)level_of.size());
    }
    F.ns = (int)level_of.size();
    F.level.assign(level_of.begin(), level_of.end());
    F.parent.assign(F.ns, -1);
    F.kids.assign(F.ns, {});
    for (int s = 0; s < F.ns; s++) {
        const int L = level_of[s];
        if (L + 1 < F.nlevels && rng() % 8) {
            const int lo = F.level_ptr[L + 1 + (int)(rng() % (F.nlevels - L - 1))];
            const int hi = F.level_ptr[F.nlevels];
            F.parent[s] = lo + (int)(rng() % (hi - lo));
            F.kids[F.parent[s]].push_back(s);
        }
        const int shape = (int)(rng() % 4);
        const int mm = shape == 0 ? 1 + (int)(rng() % 256) : 1 + (int)(rng() % 1400);
        F.m.push_back(mm);
        F.k.push_back(shape == 1 ? 0 : (int)(rng() % (mm + 1)));
    }
    return F;
}

struct WG {
    int bundle = -1, q = 0, wait = 0;  // wait: index of the next wait of the current task
    bool exited = false;
};

// Waits of task (s, code) in direction dir, in kernel order; returns the wait
// count and fills (counter kind, target): kind 0 = dep[s], 1 = blk[s].
static int waits_of(const Forest& F, int dir, int s, int code, int* wk, int* wt) {
    int n = 0;
    wk[n] = 0;
    int listed_kids = 0;
    for (int c : F.kids[s]) listed_kids += F.listed(c) ? 1 : 0;
    wt[n++] = dir == 0 ? listed_kids : (F.parent[s] >= 0 ? 1 : 0);
    const int kind = sweep_kind(code), j = sweep_blk(code);
    const int nfs = (F.k[s] + 63) / 64;
    if (kind == kSwKindWhole) return n;
    if (dir == 0) {
        const int nb = kind == kSwKindFs ? j : nfs;
        for (int jj = 0; jj < nb; jj++) {
            wk[n] = 1;
            wt[n++] = jj + 1;
        }
    } else if (j * 64 < F.k[s]) {
        for (int jj = nfs - 1; jj > j; jj--) {
            wk[n] = 1;
            wt[n++] = nfs - jj;
        }
    }
    return n;
}

static bool run(const Forest& F, int dir, const std::vector<int32_t>& tk, const std::vector<int32_t>& bp,
                const std::vector<int32_t>& nt, int G, std::mt19937& rng, long& steps) {
    const int nb = (int)bp.size() - 1, ntasks = (int)tk.size() / 2;
    std::vector<int> dep(F.ns, 0), blk(F.ns, 0), done(F.ns, 0), ran(ntasks, 0);
    std::vector<std::vector<char>> blk_ran(F.ns);
    for (int s = 0; s < F.ns; s++) blk_ran[s].assign(256, 0);
    int head = 0;
    std::vector<WG> wg(G);
    int wk[300], wt[300];
    for (;;) {
        std::vector<int> ready;
        bool all_exited = true;
        for (int g = 0; g < G; g++) {
            WG& w = wg[g];
            if (w.exited) continue;
            all_exited = false;
            if (w.bundle < 0) {
                ready.push_back(g);
                continue;
            }
            const int t = bp[w.bundle] + w.q, s = tk[2 * t], code = tk[2 * t + 1];
            const int nw = waits_of(F, dir, s, code, wk, wt);
            if (w.wait >= nw || (wk[w.wait] == 0 ? dep[s] : blk[s]) >= wt[w.wait]) ready.push_back(g);
        }
        if (all_exited) break;
        if (ready.empty()) {
            std::printf("FAIL deadlock (dir %d, %d work-groups)\n", dir, G);
            return false;
        }
        WG& w = wg[ready[rng() % ready.size()]];
        steps++;
        if (w.bundle < 0) {
            const int ticket = head++;
            if (ticket >= nb) w.exited = true;
            else {
                w.bundle = ticket;
                w.q = 0;
                w.wait = 0;
            }
            continue;
        }
        const int t = bp[w.bundle] + w.q, s = tk[2 * t], code = tk[2 * t + 1];
        const int nw = waits_of(F, dir, s, code, wk, wt);
        if (w.wait < nw) {
            w.wait++;
            continue;
        }
        // the task runs: check what it reads against the tree
        const int kind = sweep_kind(code), j = sweep_blk(code), nfs = (F.k[s] + 63) / 64;
        if (dir == 0) {
            for (int c : F.kids[s])
                if (F.listed(c) && done[c] != nt[c]) {
                    std::printf("FAIL forward task before child %d\n", c);
                    return false;
                }
            if (kind == kSwKindFs)
                for (int jj = 0; jj < j; jj++)
                    if (!blk_ran[s][jj]) { std::printf("FAIL block order\n"); return false; }
            if (kind == kSwKindCb)
                for (int jj = 0; jj < nfs; jj++)
                    if (!blk_ran[s][jj]) { std::printf("FAIL contribution tile before block\n"); return false; }
        } else {
            if (F.parent[s] >= 0 && done[F.parent[s]] != nt[F.parent[s]]) {
                std::printf("FAIL backward task before parent\n");
                return false;
            }
            if (kind == kSwKindFs)
                for (int jj = j + 1; jj < nfs; jj++)
                    if (!blk_ran[s][jj]) { std::printf("FAIL backward block order\n"); return false; }
        }
        ran[t]++;
        if (kind == kSwKindFs && (dir == 0 || j * 64 < F.k[s])) {
            blk_ran[s][j] = 1;
            blk[s]++;
        }
        if (++done[s] == nt[s]) {
            if (dir == 0) {
                if (F.parent[s] >= 0) dep[F.parent[s]]++;
            } else {
                for (int c : F.kids[s]) dep[c] = 1;
            }
        }
        w.q++;
        w.wait = 0;
        if (bp[w.bundle] + w.q >= bp[w.bundle + 1]) w.bundle = -1;
    }
    for (int t = 0; t < ntasks; t++)
        if (ran[t] != 1) { std::printf("FAIL task %d ran %d times\n", t, ran[t]); return false; }
    for (int s = 0; s < F.ns; s++)
        if (done[s] != nt[s] || (F.listed(s) != (nt[s] >= 1))) {
            std::printf("FAIL front %d incomplete or wrongly listed\n", s);
            return false;
        }
    return true;
}

int main() {
    std::mt19937 rng(2024);
    long steps = 0, tasks = 0;
    for (int trial = 0; trial < 400; trial++) {
        Forest F = random_forest(rng);
        F.first = (trial % 3 == 0) ? 0 : (int)(rng() % (F.nlevels + 1));
        if (trial % 5 == 0) F.first = sweep_first_level(F.nlevels, F.level_ptr.data(), 4);
        std::vector<int32_t> tk[2], bp[2], nt[2];
        std::vector<uint8_t> listed(F.ns);
        for (int s = 0; s < F.ns; s++) listed[s] = F.listed(s) ? 1 : 0;
        if (!sweep_lists(F.nlevels, F.level_ptr.data(), F.m.data(), F.k.data(), F.ns, tk, bp, nt, listed.data())) {
            std::printf("FAIL list build\n");
            return 1;
        }
        for (int dir = 0; dir < 2; dir++) {
            for (int rep = 0; rep < 3; rep++) {
                const int G = 1 + (int)(rng() % 64);
                if (!run(F, dir, tk[dir], bp[dir], nt[dir], G, rng, steps)) {
                    std::printf("  trial %d dir %d G %d\n", trial, dir, G);
                    return 1;
                }
            }
            tasks += (long)tk[dir].size() / 2;
        }
    }
    std::printf("OK %ld tasks, %ld steps\n", tasks, steps);
    return 0;
}
