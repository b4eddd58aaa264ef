// Per-level tile work lists of the factorization kernels (host side): counted
// exactly first, then written straight into a caller buffer.  Shared by the
// numeric driver and a CPU unit test that checks count == fill.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "mf_device.h"

namespace mf {

// Swap tile width: few (large) fronts get narrow tiles so that more blocks share
// the latency-bound work.
inline int swap_tile_cols(int count, int sw_force) { return sw_force ? sw_force : (count < 32 ? 16 : 64); }

// Fronts with many children are gathered in row chunks as well as column tiles.
inline bool gather_split(const FrontNum& f, const int32_t* nkid, int i) {
    return nkid && nkid[i] > kGatherChunkKids && f.m > kGatherChunkRows;
}

// Entry counts of one level's lists: swap tiles, eager GEMM tiles, Schur GEMM
// tiles, extend-add tasks (pointers left null; place them with the device copy).
// nkid (optional): children per front of the level, for the extend-add row chunks.
inline LevelTasks level_task_count(const FrontNum* hf, int count, int sw_force, const int32_t* nkid) {
    const int sw = swap_tile_cols(count, sw_force);
    size_t nswap = 0, ng0 = 0, ng1 = 0, ngather = 0;
    for (int i = 0; i < count; i++) {
        const int m = hf[i].m, P = hf[i].P, T = (m + 63) / 64;
        nswap += (size_t)((m + sw - 1) / sw);
        const int tcb = std::max(0, T - (P + 63) / 64);  // tiles at or beyond P
        ng0 += (size_t)T * T - (size_t)tcb * tcb;
        const int T1 = (m - P + 63) / 64;
        ng1 += (size_t)T1 * T1;
        const int lg = gather_lg(m), TG = (m + kGatherTileCols - 1) / kGatherTileCols;
        const size_t nt = (size_t)((TG + (1 << lg) - 1) >> lg);
        ngather += gather_split(hf[i], nkid, i) ? nt * (size_t)((m + kGatherChunkRows - 1) / kGatherChunkRows) : nt;
    }
    LevelTasks tk{};
    tk.nswap = (int32_t)nswap;
    tk.swap_cols = sw;
    tk.ng0 = (int32_t)ng0;
    tk.ng1 = (int32_t)ng1;
    tk.ngather = (int32_t)ngather;
    return tk;
}

inline size_t level_task_total(const LevelTasks& tk) { return (size_t)tk.nswap + tk.ng0 + tk.ng1 + tk.ngather; }

// Write the lists of level_task_count's shape to o (room for cap entries).
// Returns the number of entries written, or SIZE_MAX (with nothing written
// beyond o + cap) if they would not fit.
inline size_t fill_level_tasks(const FrontNum* hf, int count, const LevelTasks& tk, const int32_t* nkid, int32_t* o,
                               size_t cap) {
    int32_t* const o0 = o;
    int32_t* const end = o + cap;
    bool over = false;
    auto put = [&](int32_t v) {
        if (o == end) {
            over = true;
            return;
        }
        *o++ = v;
    };
    const int sw = tk.swap_cols;
    for (int i = 0; i < count && !over; i++) {
        const int T = (hf[i].m + sw - 1) / sw;
        for (int a = 0; a < T; a++) put(task_code(i, a >> 6, a & 63));
    }
    for (int i = 0; i < count && !over; i++) {
        const int m = hf[i].m, P = hf[i].P, T = (m + 63) / 64;
        for (int a = 0; a < T; a++)
            for (int b = 0; b < T; b++)
                if (!(a * 64 >= P && b * 64 >= P)) put(task_code(i, a, b));
    }
    for (int i = 0; i < count && !over; i++) {
        const int T = (hf[i].m - hf[i].P + 63) / 64;
        for (int a = 0; a < T; a++)
            for (int b = 0; b < T; b++) put(task_code(i, a, b));
    }
    // extend-add: 16-column tiles, 4 (order <= 64) or 2 (<= 128) of them per block;
    // fronts with many children split their rows into chunks as well
    for (int i = 0; i < count && !over; i++) {
        const int m = hf[i].m, lg = gather_lg(m), T = (m + kGatherTileCols - 1) / kGatherTileCols;
        const int nch = gather_split(hf[i], nkid, i) ? (m + kGatherChunkRows - 1) / kGatherChunkRows : 0;
        for (int a = 0; a < T; a += 1 << lg) {
            if (nch)
                for (int c = 0; c < nch; c++) put(gather_task(i, lg, a, c));
            else
                put(gather_task(i, lg, a));
        }
    }
    return over ? SIZE_MAX : (size_t)(o - o0);
}

// First level of the persistent part of the sweeps: the lowest level from which
// every level has at most max_fronts fronts (the upper tree, where few large
// fronts leave most of the GPU idle in a launch per level); nlevels if none.
inline int sweep_first_level(int nlevels, const int32_t* level_ptr, int max_fronts) {
    int T = nlevels;
    while (T > 0 && level_ptr[T] - level_ptr[T - 1] <= max_fronts) T--;
    return T;
}

// Task lists of the persistent sweeps (direction 0 forward, 1 backward), from
// the slots' actual orders m and eliminated counts k and the level ranges
// level_ptr[0..nlevels].  Per direction: tk = (slot, code) pairs in ticket
// order, bp = bundle pointers into the pairs, nt = tasks per slot.  The forward
// list goes up the tree level by level, the backward list down; a front of
// order <= kSwWhole is one task (runs of them share a bundle, kSwBundle at most),
// a larger one is its fully summed 64-row blocks (forward: in order, then its
// contribution tiles; backward: last block first).  A front with nothing to
// eliminate still gets one task, which releases its dependants.  Returns false
// if a front needs more than 255 blocks of either kind.
// Only slots with listed[slot] != 0 are listed (nullptr: all); the others run
// as one launch per level and direction, before the forward list and after the
// backward list, so a listed front's unlisted children are finished before the
// forward list starts and its unlisted descendants wait for the backward list.
inline bool sweep_lists(int nlevels, const int32_t* level_ptr, const int32_t* m_of, const int32_t* k_of, int ns,
                        std::vector<int32_t> tk[2], std::vector<int32_t> bp[2], std::vector<int32_t> nt[2],
                        const uint8_t* listed = nullptr) {
    for (int dir = 0; dir < 2; dir++) {
        tk[dir].clear();
        bp[dir].assign(1, 0);
        nt[dir].assign(std::max(ns, 1), 0);
        int open = 0;  // whole-front tasks in the open bundle
        auto close = [&]() {
            if (open) bp[dir].push_back((int32_t)(tk[dir].size() / 2));
            open = 0;
        };
        auto single = [&](int sl, int kind, int blk) {
            close();
            tk[dir].push_back(sl);
            tk[dir].push_back(sweep_code(kind, blk));
            bp[dir].push_back((int32_t)(tk[dir].size() / 2));
            nt[dir][sl]++;
        };
        for (int q = 0; q < nlevels; q++) {
            const int L = dir == 0 ? q : nlevels - 1 - q;
            for (int sl = level_ptr[L]; sl < level_ptr[L + 1]; sl++) {
                if (listed && !listed[sl]) continue;
                const int m = m_of[sl], k = k_of[sl];
                if (m <= kSwWhole) {
                    if (open == kSwBundle) close();
                    tk[dir].push_back(sl);
                    tk[dir].push_back(sweep_code(kSwKindWhole, 0));
                    open++;
                    nt[dir][sl]++;
                    continue;
                }
                const int nfs = (k + 63) / 64, ncb = (m - k + 63) / 64;
                if (nfs > 255 || ncb > 255) return false;
                if (dir == 0) {
                    for (int i = 0; i < nfs; i++) single(sl, kSwKindFs, i);
                    for (int r = 0; r < ncb; r++) single(sl, kSwKindCb, r);
                } else {
                    for (int i = nfs - 1; i >= 0; i--) single(sl, kSwKindFs, i);
                    if (nfs == 0) single(sl, kSwKindFs, 0);
                }
            }
        }
        close();
    }
    return true;
}

}  // namespace mf
