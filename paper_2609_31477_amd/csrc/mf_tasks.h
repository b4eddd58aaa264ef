// Per-level tile work lists of the factorization kernels (host side): counted
// exactly first, then written straight into a caller buffer.  Shared by the
// numeric driver and a CPU unit test that checks count == fill.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>

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

}  // namespace mf
