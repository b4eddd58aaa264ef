// CPU unit test of the per-level tile work lists: the exact count equals what the
// fill writes, over random front orders, pivot counts, child counts and swap
// widths (including the row-chunked extend-add of fronts with many children), and
// a buffer one entry short is detected without a write past its end.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2609_31477_amd/csrc/mf_tasks.h"

using namespace mf;

int main() {
    std::mt19937 rng(12345);
    long checked = 0;
    for (int trial = 0; trial < 3000; trial++) {
        const int count = 1 + (int)(rng() % 40);
        std::vector<FrontNum> hf(count);
        std::vector<int32_t> nkid(count);
        for (int i = 0; i < count; i++) {
            const int m = 1 + (int)(rng() % (trial % 3 == 0 ? 4096 : 700));
            hf[i] = FrontNum{};
            hf[i].m = m;
            hf[i].P = 1 + (int)(rng() % m);
            nkid[i] = (int)(rng() % 64);
        }
        const int sw_force = (int)(rng() % 3) == 0 ? 0 : ((rng() & 1) ? 16 : 64);
        const int32_t* kids = (trial & 1) ? nkid.data() : nullptr;
        const LevelTasks tk = level_task_count(hf.data(), count, sw_force, kids);
        const size_t total = level_task_total(tk);
        std::vector<int32_t> buf(total + 1, -7);
        const size_t wrote = fill_level_tasks(hf.data(), count, tk, kids, buf.data(), total);
        if (wrote != total || buf[total] != -7) {
            std::printf("FAIL count %zu fill %zu (trial %d)\n", total, wrote, trial);
            return 1;
        }
        // swap and GEMM tile codes name a front of the level and tiles inside it
        for (size_t q = 0; q < (size_t)tk.nswap + tk.ng0 + tk.ng1; q++) {
            const int rel = buf[q] >> 12, a = (buf[q] >> 6) & 63, b = buf[q] & 63;
            if (rel < 0 || rel >= count || (q >= (size_t)tk.nswap && (a * 64 >= hf[rel].m || b * 64 >= hf[rel].m))) {
                std::printf("FAIL bad tile code at %zu (trial %d)\n", q, trial);
                return 1;
            }
        }
        for (size_t q = total - tk.ngather; q < total; q++) {
            const int rel = gather_task_rel(buf[q]);
            if (rel < 0 || rel >= count || gather_task_tile(buf[q]) * kGatherTileCols >= hf[rel].m) {
                std::printf("FAIL bad gather code at %zu (trial %d)\n", q, trial);
                return 1;
            }
        }
        if (total > 0) {
            std::vector<int32_t> shortbuf(total, -7);
            shortbuf.push_back(-9);  // guard one past the short capacity
            if (fill_level_tasks(hf.data(), count, tk, kids, shortbuf.data(), total - 1) != SIZE_MAX ||
                shortbuf[total - 1] != -7 || shortbuf[total] != -9) {
                std::printf("FAIL short buffer not detected (trial %d)\n", trial);
                return 1;
            }
        }
        checked += (long)total;
    }
    std::printf("OK %ld task entries\n", checked);
    return 0;
}
