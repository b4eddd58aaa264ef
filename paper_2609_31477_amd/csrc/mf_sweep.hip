// Persistent forward and backward sweeps of the multifrontal solve.
//
// The level-by-level sweeps launch two kernels per tree level and direction and
// give each front of the upper levels to a single work-group, which then streams
// the front's triangular factor through one CU.  Here one launch per direction
// runs the whole tree from a device work list:
//
//   * tasks are listed in an order where every task's inputs come from tasks
//     listed before it (children before parents in the forward sweep, parents
//     before children in the backward sweep, and the blocks of one front in
//     dependency order);
//   * work-groups take tickets from one atomic counter, a bundle of consecutive
//     small-front tasks per ticket, so a task is only ever taken by a running
//     work-group and every task it waits for was taken earlier by a running one:
//     the waits cannot deadlock, whatever the number of resident work-groups;
//   * readiness is counted per front: children finished (forward), parent
//     finished (backward), fully summed blocks finished, tasks finished.  Every
//     wait is bounded: past its limit it sets an error word that the host
//     reports, and the kernel still ends;
//   * a large front's fully summed part is split into 64-row blocks solved by
//     different work-groups: block i subtracts the finished blocks' products as
//     they appear (in block order, so its sums do not depend on timing) and then
//     solves its diagonal block; its contribution rows are 64-row tiles that
//     follow the same blocks.  The factor is read by many CUs at once.
//
// Arithmetic per front depends only on the front (its order decides whole-front
// or blocked processing), so a system's solution is bitwise the same alone and
// in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mf_device.h"
#include "mf_kutil.h"

namespace mf {

namespace {

constexpr int kSwT = 256;  // threads per work-group (4 waves)
constexpr int kSwB = 64;   // rows per block, one lane per row

struct SweepArgs {
    DevSym S;
    const FrontNum* fn;
    const int32_t* tasks;   // 2 ints per task: slot, code
    const int32_t* bptr;    // bundle b holds tasks [bptr[b], bptr[b + 1])
    int32_t nbund;
    const int32_t* ntask;   // per slot: tasks of the front in this direction
    const int32_t* need;    // per slot (forward): children in the list, whose completion the front awaits
    int32_t* ctr;           // [0] ticket counter, [1] error word
    int32_t* dep;           // per slot: children finished (forward) / parent finished (backward)
    int32_t* blk;           // per slot: fully summed blocks finished
    int32_t* done;          // per slot: tasks finished
    const double* b;        // forward: right-hand sides (ldb)
    int64_t ldb;
    double* x;              // backward: solution (ldx)
    int64_t ldx;
    double* vec;            // per-front vector blocks
    int32_t nrhs, c0, nrc;
    int32_t cap;            // wait limit (polls)
};

// Cross-work-group data.  The L2 caches of the XCDs are not coherent with one
// another; an agent-scope release (write back the whole L2) or acquire
// (invalidate it) per event costs far more than the data it orders.  Instead,
// every vector value that one work-group of a sweep writes and another reads
// goes through device-coherent accesses (relaxed agent-scope atomic loads and
// stores, i.e. the "sc1" loads and write-through stores of this ISA), and the
// order of such a store before the count that publishes it is the store's
// completion (s_waitcnt) ahead of the block barrier and the count update.  The
// factors, the right-hand side and the front records were written by earlier
// launches and are read through the caches.
__device__ __forceinline__ double ld_dev(const double* p) {
    return __longlong_as_double(__hip_atomic_load((const long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_dev(double* p, double v) {
    __hip_atomic_store((long long*)p, __double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *p >= target, bounded by cap polls (device-coherent
// loads, a short sleep between them); the barrier then holds the block's loads
// behind it.  On timeout the error word is set and the wait ends (as do all
// later waits).
__device__ __forceinline__ void wait_geq(const SweepArgs& A, int32_t* p, int target) {
    if (threadIdx.x == 0) {
        int it = 0;
        while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++it > A.cap || __hip_atomic_load(A.ctr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(A.ctr + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Every wave's device-coherent stores have completed before the barrier, so a
// count that thread 0 updates after it publishes them.
__device__ __forceinline__ void post_stores() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// End of a task: count it; the front's last task releases its dependants.
__device__ __forceinline__ void finish_task(const SweepArgs& A, int s, bool forward) {
    post_stores();
    if (threadIdx.x == 0) {
        const int old = __hip_atomic_fetch_add(A.done + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == A.ntask[s]) {
            // the front's other tasks completed their stores before their counts
            if (forward) {
                const int p = A.S.parent[s];
                if (p >= 0) __hip_atomic_fetch_add(A.dep + p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                for (int t = A.S.child_ptr[s]; t < A.S.child_ptr[s + 1]; t++)
                    __hip_atomic_store(A.dep + A.S.child_slot[t], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __syncthreads();
}

// Right-hand side of front row i: the original entries of the front's own
// pivot rows plus the children's contribution entries, in child order.
// Written to z[(i - zoff) + c * ldz].
template <int NR>
__device__ __forceinline__ void gather_row(const SweepArgs& A, int s, const FrontNum& d, int i, double* z,
                                           int zoff, int ldz) {
    const int m = d.m, P = d.P;
    const int src = i < P ? as_global(iv_rowperm(d.iv, P, m))[i] : i;
    const int32_t* rows = A.S.rows + A.S.rows_ptr[s];
    // (columns c >= nrc repeat column nrc - 1, so no load waits on a per-column
    // branch; they are not stored)
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; c++)
        acc[c] = src < d.npiv ? A.b[rows[src] + (int64_t)(A.c0 + min(c, A.nrc - 1)) * A.ldb] : 0.0;
    int dseg = 0;
    for (int tt = A.S.child_ptr[s]; tt < A.S.child_ptr[s + 1]; tt++) {
        const int cs = A.S.child_slot[tt];
        const FrontNum* dc = A.fn + cs;
        const int ck = dc->k, dout = dc->P - ck;
        const int ci = child_pos(src, d.npiv, d.din, dseg, dout, A.S.imap + A.S.imap_off[cs]);
        if (ci >= 0) {
            const double* vc = A.vec + dc->voff * A.nrhs;
            const int cm = dc->m;
#pragma unroll
            for (int c = 0; c < NR; c++) acc[c] += ld_dev(vc + ck + ci + (int64_t)(A.c0 + min(c, A.nrc - 1)) * cm);
        }
        dseg += dout;
    }
#pragma unroll
    for (int c = 0; c < NR; c++)
        if (c < A.nrc) z[(i - zoff) + c * ldz] = acc[c];
}

// Stage the bs x bs diagonal block at (j0, j0) into LDS (column a at a * 64),
// by the whole block.
template <typename T>
__device__ __forceinline__ void stage_diag(gptr<const T> F, int64_t m, int j0, int bs, T* dblk) {
    // every thread loads its 16 entries (clamped into the block) before storing
    // any, so all loads are in flight together
    constexpr int kQ = kSwB * kSwB / kSwT;
    T tmp[kQ];
#pragma unroll
    for (int q = 0; q < kQ; q++) {
        const int e = threadIdx.x + q * kSwT, a = e / kSwB, r = e % kSwB;
        tmp[q] = F[(j0 + min(r, bs - 1)) + (int64_t)(j0 + min(a, bs - 1)) * m];
    }
#pragma unroll
    for (int q = 0; q < kQ; q++) {
        const int e = threadIdx.x + q * kSwT, a = e / kSwB, r = e % kSwB;
        dblk[e] = (a < bs && r < bs) ? tmp[q] : T(0);
    }
}

// The same staging in two halves, for a block task whose diagonal block does not
// depend on what it waits for: the loads are issued before the waits (so they
// are in flight meanwhile) and the block goes to LDS after the last update.
template <typename T>
struct DiagPre {
    static constexpr int kQ = kSwB * kSwB / kSwT;
    T tmp[kQ];
    __device__ __forceinline__ void load(gptr<const T> F, int64_t m, int j0, int bs) {
#pragma unroll
        for (int q = 0; q < kQ; q++) {
            const int e = threadIdx.x + q * kSwT, a = e / kSwB, r = e % kSwB;
            tmp[q] = F[(j0 + min(r, bs - 1)) + (int64_t)(j0 + min(a, bs - 1)) * m];
        }
    }
    __device__ __forceinline__ void store(int bs, T* dblk) const {
#pragma unroll
        for (int q = 0; q < kQ; q++) {
            const int e = threadIdx.x + q * kSwT, a = e / kSwB, r = e % kSwB;
            dblk[e] = (a < bs && r < bs) ? tmp[q] : T(0);
        }
    }
};

// acc[c] += sum_{a < n} F[r, col0 + a] y[a + c * ldy] for one row r (n <= 256),
// in order of a, with the row's entries loaded 16 at a time ahead of their use.
// NR: right-hand sides handled per pass (1, or kSwRhs with nrc of them live).
template <typename T, int NR>
__device__ __forceinline__ void row_dot(gptr<const T> F, int64_t m, int r, int col0, int n, const double* y, int ldy,
                                        int nrc, double* acc) {
    constexpr int kC = 16;
    // every column accumulated without a per-column branch (columns c >= nrc
    // repeat column nrc - 1; their sums are not used), so the products of a
    // batch of entries issue as one block
    const double* yc[NR];
#pragma unroll
    for (int c = 0; c < NR; c++) yc[c] = y + min(c, nrc - 1) * ldy;
    for (int a0 = 0; a0 < n; a0 += kC) {
        T f[kC];
#pragma unroll
        for (int q = 0; q < kC; q++) f[q] = F[r + (int64_t)(col0 + min(a0 + q, n - 1)) * m];
#pragma unroll
        for (int q = 0; q < kC; q++) {
            if (a0 + q < n) {
#pragma unroll
                for (int c = 0; c < NR; c++) acc[c] += (double)f[q] * yc[c][a0 + q];
            }
        }
    }
}

// Forward substitution with the unit lower diagonal block in LDS on rows
// [j0, j0 + bs) of z (columns c at c * ldz), called by the whole work-group.
// One right-hand side: wave 0.  Several: column c goes to wave c mod 4, and a
// wave's chains advance together, one step at a time (each step reads the
// block's column once), so their latencies overlap.  Each column's operations
// are those of a chain run alone.  Columns c >= nrc repeat column nrc - 1 and
// are not stored.
template <int NR>
struct ChainSplit {
    static constexpr int kW = NR == 1 ? 1 : (NR < kSwT / 64 ? NR : kSwT / 64);  // waves with chains
    static constexpr int kN = NR / kW;                                           // chains per wave
};
template <typename T, int NR>
__device__ __forceinline__ void solve_lower(const T* dblk, int j0, int bs, double* z, int ldz, int nrc) {
    using C = ChainSplit<NR>;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= C::kW || w >= nrc) return;
    double x[C::kN];
#pragma unroll
    for (int q = 0; q < C::kN; q++) x[q] = lane < bs ? z[j0 + lane + min(w + C::kW * q, nrc - 1) * ldz] : 0.0;
    // a fixed 63 steps (entries beyond the block are staged as zeros), so the
    // loop unrolls and the LDS reads run ahead of the dependent chains
#pragma unroll 8
    for (int a = 0; a < kSwB - 1; a++) {
        const double l = (double)dblk[a * kSwB + lane];
#pragma unroll
        for (int q = 0; q < C::kN; q++) {
            const double xa = readlane_d(x[q], a);
            if (lane > a) x[q] -= l * xa;
        }
    }
#pragma unroll
    for (int q = 0; q < C::kN; q++)
        if (w + C::kW * q < nrc && lane < bs) z[j0 + lane + (w + C::kW * q) * ldz] = x[q];
}

// Back substitution with the upper diagonal block in LDS on rows [j0, j0 + bs)
// of t (columns c at c * ldt), by the whole work-group, the chains split over
// the waves as in solve_lower.
template <typename T, int NR>
__device__ __forceinline__ void solve_upper(const T* dblk, int j0, int bs, double* t, int ldt, int nrc) {
    using C = ChainSplit<NR>;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= C::kW || w >= nrc) return;
    const int ld = min(lane, bs - 1);
    const double rd = 1.0 / (double)dblk[ld * kSwB + ld];
    double xl[C::kN];
#pragma unroll
    for (int q = 0; q < C::kN; q++) xl[q] = lane < bs ? t[j0 + lane + min(w + C::kW * q, nrc - 1) * ldt] : 0.0;
#pragma unroll 8
    for (int a = kSwB - 1; a >= 0; a--) {
        const double u = (double)dblk[a * kSwB + lane];
        const double ra = readlane_d(rd, a);
#pragma unroll
        for (int q = 0; q < C::kN; q++) {
            const double xa = readlane_d(xl[q], a) * ra;
            if (lane == a) xl[q] = xa;
            if (lane < a) xl[q] -= u * xa;
        }
    }
#pragma unroll
    for (int q = 0; q < C::kN; q++)
        if (w + C::kW * q < nrc && lane < bs) t[j0 + lane + (w + C::kW * q) * ldt] = xl[q];
}

// acc[c] (rows r0 + lane) -= sum over a tile's columns of F[r, col0 + a] y[a, c],
// in two halves: the tile's entries are loaded first (before the task waits for
// the vector block they multiply, or while the previous tile is multiplied: they
// do not depend on it), and the product is formed afterwards.  The 64 columns are
// split over the 4 waves (a = wave + 4 q), and the partial sums are combined in
// wave order by wave 0, which returns them in sub.
template <typename T, int NR>
struct GemvPre {
    static constexpr int kQ = kSwB / 4;
    T f[kQ];
    __device__ __forceinline__ void load(gptr<const T> F, int64_t m, int r0, int nr, int col0, int ncol) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int r = r0 + min(lane, nr - 1);
#pragma unroll
        for (int q = 0; q < kQ; q++) f[q] = F[r + (int64_t)(col0 + min(w + 4 * q, ncol - 1)) * m];
    }
    __device__ __forceinline__ void gemv(int ncol, const double* y, int ldy, int nrc, double* part,
                                         double* sub) const {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        // no per-column branches (as in row_dot): columns c >= nrc repeat column
        // nrc - 1 and their sums are not used
        const double* yc[NR];
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; c++) {
            yc[c] = y + min(c, nrc - 1) * ldy;
            acc[c] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < kQ; q++) {
            const int a = w + 4 * q;
            if (a < ncol) {
#pragma unroll
                for (int c = 0; c < NR; c++) acc[c] += (double)f[q] * yc[c][a];
            }
        }
#pragma unroll
        for (int c = 0; c < NR; c++) part[(w * kSwRhs + c) * 64 + lane] = acc[c];
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int c = 0; c < NR; c++)
                sub[c] = (part[(0 * kSwRhs + c) * 64 + lane] + part[(1 * kSwRhs + c) * 64 + lane]) +
                         (part[(2 * kSwRhs + c) * 64 + lane] + part[(3 * kSwRhs + c) * 64 + lane]);
        }
        __syncthreads();
    }
};

struct SweepLds {
    double z[kSwWhole * kSwRhs];  // whole front: its rows; blocks: own rows [0, 64 nrc) and a vector block after
    union {                       // never live at the same time
        double part[4 * kSwRhs * 64];  // GemvPre partial sums
        double dblk[kSwB * kSwB];      // staged diagonal block (as double or float)
    } u;
};

// ---------------------------------------------------------------- forward
// Whole front (order <= kSwWhole): gather, then for each 64-column block of the
// eliminated part, wave 0 solves its diagonal block and every thread updates its
// row below it.  Result [y; c] to the front's vector block.
template <typename T, int NR>
__device__ void fwd_whole(const SweepArgs& A, int s, const FrontNum& d, SweepLds& L) {
    const int m = d.m, k = d.k, nrc = A.nrc, tid = threadIdx.x;
    const gptr<const T> F = as_global((const T*)d.F);
    double* z = L.z;
    T* dblk = (T*)L.u.dblk;
    if (tid < m) gather_row<NR>(A, s, d, tid, z, 0, m);
    for (int j0 = 0; j0 < k; j0 += kSwB) {
        const int bs = min(kSwB, k - j0);
        stage_diag<T>(F, m, j0, bs, dblk);
        __syncthreads();
        solve_lower<T, NR>(dblk, j0, bs, z, m, nrc);
        __syncthreads();
        if (tid >= j0 + bs && tid < m) {
            double acc[NR];
#pragma unroll
            for (int c = 0; c < NR; c++) acc[c] = 0.0;
            row_dot<T, NR>(F, m, tid, j0, bs, z + j0, m, nrc, acc);
#pragma unroll
            for (int c = 0; c < NR; c++)
                if (c < nrc) z[tid + c * m] -= acc[c];
        }
        __syncthreads();
    }
    double* v = A.vec + d.voff * A.nrhs;
    if (tid < m)
        for (int c = 0; c < nrc; c++) st_dev(v + tid + (int64_t)(A.c0 + c) * m, z[tid + c * m]);
}

// Rows [r0, r0 + nr) of a large front (a fully summed block when fs, else a
// contribution tile): gather, subtract the finished blocks' products in block
// order (block j waits until the front has finished j + 1 blocks), then, for a
// fully summed block, solve its diagonal block.
template <typename T, int NR>
__device__ void fwd_block(const SweepArgs& A, int s, const FrontNum& d, int r0, int nr, bool fs, SweepLds& L) {
    const int m = d.m, k = d.k, nrc = A.nrc, tid = threadIdx.x, lane = tid & 63;
    const gptr<const T> F = as_global((const T*)d.F);
    double* zr = L.z;              // own rows, column c at c * 64
    double* yb = L.z + 64 * kSwRhs;  // one finished block of y
    double* v = A.vec + d.voff * A.nrhs;
    DiagPre<T> pre;
    if (fs) pre.load(F, m, r0, nr);
    if (tid < nr) gather_row<NR>(A, s, d, r0 + tid, zr, r0, 64);
    const int nblk = fs ? (r0 / kSwB) : (k + kSwB - 1) / kSwB;
    for (int j = 0; j < nblk; j++) {
        const int j0 = j * kSwB, bs = min(kSwB, k - j0);
        GemvPre<T, NR> g;
        g.load(F, m, r0, nr, j0, bs);  // in flight during the wait
        wait_geq(A, A.blk + s, j + 1);
        for (int e = tid; e < bs * nrc; e += kSwT) {
            const int a = e % bs, c = e / bs;
            yb[a + c * 64] = ld_dev(v + j0 + a + (int64_t)(A.c0 + c) * m);
        }
        __syncthreads();
        double sub[NR];
        g.gemv(bs, yb, 64, nrc, L.u.part, sub);
        if (tid < 64 && lane < nr) {
#pragma unroll
            for (int c = 0; c < NR; c++)
                if (c < nrc) zr[lane + c * 64] -= sub[c];
        }
        __syncthreads();
    }
    if (fs) {
        T* dblk = (T*)L.u.dblk;
        pre.store(nr, dblk);
        __syncthreads();
        solve_lower<T, NR>(dblk, 0, nr, zr, 64, nrc);
        __syncthreads();
    }
    if (tid < nr)
        for (int c = 0; c < nrc; c++) st_dev(v + r0 + tid + (int64_t)(A.c0 + c) * m, zr[tid + c * 64]);
    if (fs) {
        post_stores();
        if (tid == 0) __hip_atomic_fetch_add(A.blk + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T, int NR>
__device__ void fwd_task(const SweepArgs& A, int s, int32_t code, SweepLds& L) {
    const FrontNum d = A.fn[s];
    wait_geq(A, A.dep + s, A.need[s]);
    const int kind = sweep_kind(code), j = sweep_blk(code);
    if (kind == kSwKindWhole) {
        fwd_whole<T, NR>(A, s, d, L);
    } else if (kind == kSwKindFs) {
        const int r0 = j * kSwB;
        fwd_block<T, NR>(A, s, d, r0, min(kSwB, d.k - r0), true, L);
    } else {
        const int r0 = d.k + j * kSwB;
        fwd_block<T, NR>(A, s, d, r0, min(kSwB, d.m - r0), false, L);
    }
    finish_task(A, s, true);
}

// ---------------------------------------------------------------- backward
// Whole front: t = y - U12 x[colvar[k:m]], then back substitution block by block
// from the last one, each thread updating its row above the block; x to colvar.
template <typename T, int NR>
__device__ void bwd_whole(const SweepArgs& A, int s, const FrontNum& d, SweepLds& L) {
    const int m = d.m, P = d.P, k = d.k, nrc = A.nrc, tid = threadIdx.x;
    const gptr<const T> F = as_global((const T*)d.F);
    const gptr<const int32_t> colvar = as_global(iv_colvar(d.iv, P, m));
    const double* v = A.vec + d.voff * A.nrhs;
    double* t = L.z;            // rows [0, k), column c at c * k
    double* xs = L.z + k * nrc;  // solution values of columns [k, m), column c at c * (m - k)
    const int nc = m - k;
    for (int e = tid; e < nc * nrc; e += kSwT) {
        const int j = e % nc, c = e / nc;
        const int var = colvar[k + j];
        xs[j + c * nc] = var >= 0 ? ld_dev(A.x + var + (int64_t)(A.c0 + c) * A.ldx) : 0.0;
    }
    __syncthreads();
    if (tid < k) {
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; c++) acc[c] = (c < nrc) ? v[tid + (int64_t)(A.c0 + c) * m] : 0.0;
        double dot[NR];
#pragma unroll
        for (int c = 0; c < NR; c++) dot[c] = 0.0;
        if (nc > 0) row_dot<T, NR>(F, m, tid, k, nc, xs, nc, nrc, dot);
#pragma unroll
        for (int c = 0; c < NR; c++)
            if (c < nrc) t[tid + c * k] = acc[c] - dot[c];
    }
    T* dblk = (T*)L.u.dblk;
    for (int j1 = k; j1 > 0; j1 -= kSwB) {
        const int j0 = max(0, j1 - kSwB), bs = j1 - j0;
        __syncthreads();
        stage_diag<T>(F, m, j0, bs, dblk);
        __syncthreads();
        solve_upper<T, NR>(dblk, j0, bs, t, k, nrc);
        __syncthreads();
        if (tid < j0) {
            double acc[NR];
#pragma unroll
            for (int c = 0; c < NR; c++) acc[c] = 0.0;
            row_dot<T, NR>(F, m, tid, j0, bs, t + j0, k, nrc, acc);
#pragma unroll
            for (int c = 0; c < NR; c++)
                if (c < nrc) t[tid + c * k] -= acc[c];
        }
    }
    __syncthreads();
    if (tid < k) {
        const int var = colvar[tid];
        if (var >= 0)
            for (int c = 0; c < nrc; c++) st_dev(A.x + var + (int64_t)(A.c0 + c) * A.ldx, t[tid + c * k]);
    }
}

// Fully summed block [r0, r0 + nr) of a large front: t = y - U12 x over the
// contribution columns (64 at a time), then the products of the finished blocks
// after it (from the last one down, each waited for), then its diagonal block.
// Its x goes to the front's vector block (for the blocks above) and to colvar.
template <typename T, int NR>
__device__ void bwd_block(const SweepArgs& A, int s, const FrontNum& d, int r0, int nr, SweepLds& L) {
    const int m = d.m, P = d.P, k = d.k, nrc = A.nrc, tid = threadIdx.x, lane = tid & 63;
    const gptr<const T> F = as_global((const T*)d.F);
    const gptr<const int32_t> colvar = as_global(iv_colvar(d.iv, P, m));
    double* v = A.vec + d.voff * A.nrhs;
    double* tr = L.z;
    double* xb = L.z + 64 * kSwRhs;
    DiagPre<T> pre;
    pre.load(F, m, r0, nr);
    if (tid < nr)
        for (int c = 0; c < nrc; c++) tr[tid + c * 64] = v[r0 + tid + (int64_t)(A.c0 + c) * m];
    // the contribution columns 64 at a time, the next tile's entries loaded while
    // the current one is multiplied
    GemvPre<T, NR> g;
    if (k < m) g.load(F, m, r0, nr, k, min(kSwB, m - k));
    for (int j0 = k; j0 < m; j0 += kSwB) {
        const int bs = min(kSwB, m - j0);
        for (int e = tid; e < bs * nrc; e += kSwT) {
            const int a = e % bs, c = e / bs;
            const int var = colvar[j0 + a];
            xb[a + c * 64] = var >= 0 ? ld_dev(A.x + var + (int64_t)(A.c0 + c) * A.ldx) : 0.0;
        }
        __syncthreads();
        const bool more = j0 + kSwB < m;
        GemvPre<T, NR> gn;
        if (more) gn.load(F, m, r0, nr, j0 + kSwB, min(kSwB, m - j0 - kSwB));
        double sub[NR];
        g.gemv(bs, xb, 64, nrc, L.u.part, sub);
        if (tid < 64 && lane < nr) {
#pragma unroll
            for (int c = 0; c < NR; c++)
                if (c < nrc) tr[lane + c * 64] -= sub[c];
        }
        __syncthreads();
        if (more) g = gn;
    }
    const int nfs = (k + kSwB - 1) / kSwB, me = r0 / kSwB;
    for (int j = nfs - 1; j > me; j--) {
        const int j0 = j * kSwB, bs = min(kSwB, k - j0);
        GemvPre<T, NR> g;
        g.load(F, m, r0, nr, j0, bs);  // in flight during the wait
        wait_geq(A, A.blk + s, nfs - j);
        for (int e = tid; e < bs * nrc; e += kSwT) {
            const int a = e % bs, c = e / bs;
            xb[a + c * 64] = ld_dev(v + j0 + a + (int64_t)(A.c0 + c) * m);
        }
        __syncthreads();
        double sub[NR];
        g.gemv(bs, xb, 64, nrc, L.u.part, sub);
        if (tid < 64 && lane < nr) {
#pragma unroll
            for (int c = 0; c < NR; c++)
                if (c < nrc) tr[lane + c * 64] -= sub[c];
        }
        __syncthreads();
    }
    T* dblk = (T*)L.u.dblk;
    pre.store(nr, dblk);
    __syncthreads();
    solve_upper<T, NR>(dblk, 0, nr, tr, 64, nrc);
    __syncthreads();
    if (tid < nr) {
        const int var = colvar[r0 + tid];
        for (int c = 0; c < nrc; c++) {
            const double xv = tr[tid + c * 64];
            st_dev(v + r0 + tid + (int64_t)(A.c0 + c) * m, xv);
            if (var >= 0) st_dev(A.x + var + (int64_t)(A.c0 + c) * A.ldx, xv);
        }
    }
    post_stores();
    if (tid == 0) __hip_atomic_fetch_add(A.blk + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int NR>
__device__ void bwd_task(const SweepArgs& A, int s, int32_t code, SweepLds& L) {
    const FrontNum d = A.fn[s];
    wait_geq(A, A.dep + s, A.S.parent[s] >= 0 ? 1 : 0);
    const int kind = sweep_kind(code), j = sweep_blk(code);
    if (kind == kSwKindWhole) {
        bwd_whole<T, NR>(A, s, d, L);
    } else {
        const int r0 = j * kSwB;
        if (r0 < d.k) bwd_block<T, NR>(A, s, d, r0, min(kSwB, d.k - r0), L);
    }
    finish_task(A, s, false);
}

// One kernel per direction: work-groups take bundles of tasks by ticket until
// the list is exhausted.
template <bool FWD, int NR>
__global__ __launch_bounds__(kSwT, NR == 1 ? 3 : 1) void k_sweep_persist(SweepArgs A) {
    __shared__ SweepLds L;
    __shared__ int ticket;
    for (;;) {
        if (threadIdx.x == 0) ticket = __hip_atomic_fetch_add(A.ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int bnd = ticket;
        __syncthreads();
        if (bnd >= A.nbund) return;
        for (int q = A.bptr[bnd]; q < A.bptr[bnd + 1]; q++) {
            const int s = A.tasks[2 * q], code = A.tasks[2 * q + 1];
            if (A.fn[s].prec) {
                if constexpr (FWD) fwd_task<float, NR>(A, s, code, L);
                else bwd_task<float, NR>(A, s, code, L);
            } else {
                if constexpr (FWD) fwd_task<double, NR>(A, s, code, L);
                else bwd_task<double, NR>(A, s, code, L);
            }
        }
    }
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

// Counters: ctr = [ticket, error, dep[ns], blk[ns], done[ns]] (3 ns + 2 ints).
// tasks/bptr/ntask: the direction's list.  Resets the counters and launches.
hipError_t launch_sweep_persist(bool forward, const DevSym& S, const FrontNum* fn, const int32_t* tasks,
                                const int32_t* bptr, int nbund, const int32_t* ntask, const int32_t* need,
                                int32_t* ctr,
                                const double* b, int64_t ldb, double* x, int64_t ldx, double* vec, int nrhs, int c0,
                                int nrc, int grid, int cap, hipStream_t st) {
    const int ns = S.nslots;
    // the ticket and the per-slot counts (the error word at ctr[1] is kept)
    const int64_t nctr = 2 + 3 * (int64_t)ns;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, ctr, (int64_t)1);
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)std::min<int64_t>((nctr - 2 + 255) / 256, 1024)), dim3(256), 0, st,
                       ctr + 2, nctr - 2);
    if (nbund <= 0) return hipGetLastError();
    SweepArgs A;
    A.S = S;
    A.fn = fn;
    A.tasks = tasks;
    A.bptr = bptr;
    A.nbund = nbund;
    A.ntask = ntask;
    A.need = need;
    A.ctr = ctr;
    A.dep = ctr + 2;
    A.blk = ctr + 2 + ns;
    A.done = ctr + 2 + 2 * (int64_t)ns;
    A.b = b;
    A.ldb = ldb;
    A.x = x;
    A.ldx = ldx;
    A.vec = vec;
    A.nrhs = nrhs;
    A.c0 = c0;
    A.nrc = nrc;
    A.cap = cap;
    const unsigned g = (unsigned)std::max(1, std::min(grid, nbund));
    // one right-hand side has its own instantiation (fewer registers)
    if (forward) {
        if (nrc == 1) hipLaunchKernelGGL((k_sweep_persist<true, 1>), dim3(g), dim3(kSwT), 0, st, A);
        else hipLaunchKernelGGL((k_sweep_persist<true, kSwRhs>), dim3(g), dim3(kSwT), 0, st, A);
    } else {
        if (nrc == 1) hipLaunchKernelGGL((k_sweep_persist<false, 1>), dim3(g), dim3(kSwT), 0, st, A);
        else hipLaunchKernelGGL((k_sweep_persist<false, kSwRhs>), dim3(g), dim3(kSwT), 0, st, A);
    }
    return hipGetLastError();
}

}  // namespace mf
