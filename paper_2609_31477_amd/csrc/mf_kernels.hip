// gfx950 kernels of the multifrontal factorization and solve.
//
// One tree level of fronts is processed per launch; fronts of a level are
// contiguous "slots".  Every kernel re-reads the front's FrontNum and returns
// early when the front has no work for the launch, so grids are sized from the
// level's largest front.
//
// Front layout (column-major, ld = m), rows and columns in the same order:
//   [0, npiv)            nominal pivots of the front
//   [npiv, npiv+din)     variables delayed in from the children (child order)
//   [npiv+din, m)        nominal contribution-block rows
// After the partial factorization the first k positions hold L11\U11, L21 and
// U12; F[k:m, k:m] is the contribution block (CB) passed to the parent, whose
// leading P-k rows/columns are the delayed (uneliminated) fully summed ones.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "mf_device.h"
#include "mf_kutil.h"

namespace mf {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kGatherCols = kGatherTileCols;  // columns per gather tile
static_assert(kGatherCols == 16, "gather column decoding assumes 16-column tiles");
constexpr int kTile = 64;         // GEMM tile (rows and columns)
constexpr int kKC = 32;           // GEMM K chunk staged through LDS
constexpr int kLdsPad = kTile + 1;

__device__ __forceinline__ double load_front(const FrontNum& d, int64_t idx) {
    return d.prec ? (double)((const float*)d.F)[idx] : ((const double*)d.F)[idx];
}

// ------------------------------------------------------------------ assembly
// Owner-computes extend-add: every entry of the front is written exactly once,
// as the sum over children (in child order) of the matching CB entries.  One
// block per task (front, first column tile); the block covers G = 1, 2 or 4
// consecutive tiles of kGatherCols columns, one per group of 256/G threads (the
// host picks G = 4 for fronts of order <= 64 and 2 up to 128, so that small
// fronts keep every lane busy).  Also resets the front's pivot bookkeeping.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(DevSym S, FrontNum* fn, int slot0, int want_prec,
                                                     const int32_t* tasks) {
    const int32_t code = tasks[blockIdx.x];
    const int s = slot0 + gather_task_rel(code);
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m;
    const int lg = gather_task_lg(code);
    const int jb = gather_task_tile(code) * kGatherCols;  // first column of the block
    const int ch = gather_task_chunk(code);
    const int i_lo = ch < 0 ? 0 : ch * kGatherChunkRows;  // rows [i_lo, i_hi) of this block
    const int i_hi = ch < 0 ? m : min(m, i_lo + kGatherChunkRows);
    if (jb >= m || i_lo >= m) return;
    const int rstep = kThreads >> lg;                 // rows per pass of a group
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> (8 - lg));  // (uniform per wave)
    const int r = threadIdx.x & (rstep - 1);
    const int bc = kGatherCols << lg;                 // columns of the block
    const int j0 = jb + g * kGatherCols;              // first column of this group
    T* F = (T*)d.F;
    if (jb == 0 && i_lo == 0) {
        int32_t* colperm = iv_colperm(d.iv, d.P, m);
        int32_t* rowperm = iv_rowperm(d.iv, d.P, m);
        for (int i = threadIdx.x; i < d.P; i += kThreads) {
            colperm[i] = i;
            rowperm[i] = i;
        }
    }
    const int cb = S.child_ptr[s], ce = S.child_ptr[s + 1];
    // per child: its FrontNum fields and the child column of each of this block's
    // columns, computed once per block into LDS (then every row's loads of a child
    // are independent)
    constexpr int kMaxKids = 64;
    constexpr int kFewKids = 8;
    constexpr int kMaxCols = 4 * kGatherCols;
    __shared__ int cj_s[kMaxKids][kMaxCols];
    __shared__ int kid_dout[kMaxKids], kid_dseg[kMaxKids], kid_k[kMaxKids], kid_m[kMaxKids], kid_prec[kMaxKids];
    __shared__ int64_t kid_im[kMaxKids];
    __shared__ const void* kid_F[kMaxKids];
    __shared__ int act_s[kMaxKids];
    __shared__ int nact_s;
    const int nk = ce - cb;
    const bool staged = nk <= kMaxKids;
    if (staged) {
        // one thread per child reads its fields (no chain of dependent loads),
        // then one thread forms the delayed-segment offsets in child order
        if (threadIdx.x < nk) {
            const int t = threadIdx.x;
            const int cs = S.child_slot[cb + t];
            const FrontNum dc = fn[cs];
            kid_dout[t] = dc.P - dc.k;
            kid_k[t] = dc.k;
            kid_m[t] = dc.m;
            kid_prec[t] = dc.prec;
            kid_im[t] = S.imap_off[cs];
            kid_F[t] = dc.F;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int dseg = 0;
            for (int t = 0; t < nk; t++) {
                kid_dseg[t] = dseg;
                dseg += kid_dout[t];
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nk * bc; q += kThreads) {
            const int t = q >> (4 + lg), c = q & (bc - 1), j = jb + c;
            cj_s[t][c] = j < m ? child_pos(j, d.npiv, d.din, kid_dseg[t], kid_dout[t], S.imap + kid_im[t]) : -1;
        }
        __syncthreads();
        // children that reach none of this block's columns (or have an empty
        // contribution block) add only zeros: the first wave lists the others,
        // in child order, with one ballot
        if (threadIdx.x < kMaxKids) {
            const int t = threadIdx.x;
            bool act = false;
            if (t < nk && kid_m[t] != kid_k[t])
                for (int c = 0; c < bc; c++) act |= cj_s[t][c] >= 0;
            const uint64_t mask = __ballot(act);
            if (act) act_s[__popcll(mask & ((1ull << t) - 1))] = t;
            if (t == 0) nact_s = __popcll(mask);
        }
        __syncthreads();
        if (j0 >= m) return;  // (no barrier follows)
        const int gc = g * kGatherCols;
        const int nact = nact_s;
        // Many children (a front whose columns every child reaches, such as the
        // ones tied to all multipliers): row positions are looked up for kCiBatch
        // children at once, and a child none of whose rows meets the wave's rows
        // is skipped (wave-uniform test).
        if (nact > kFewKids) {
            constexpr int kCiBatch = 4;
            for (int i = i_lo + r; i < i_hi; i += rstep) {
                double acc[kGatherCols];
#pragma unroll
                for (int jj = 0; jj < kGatherCols; jj++) acc[jj] = 0.0;
                for (int a0 = 0; a0 < nact; a0 += kCiBatch) {
                    int ci[kCiBatch];
#pragma unroll
                    for (int b = 0; b < kCiBatch; b++) {
                        const int t = act_s[min(a0 + b, nact - 1)];
                        ci[b] = child_pos(i, d.npiv, d.din, kid_dseg[t], kid_dout[t], S.imap + kid_im[t]);
                    }
#pragma unroll
                    for (int b = 0; b < kCiBatch; b++) {
                        if (a0 + b >= nact) break;
                        if (!__any(ci[b] >= 0)) continue;
                        const int t = act_s[a0 + b];
                        const int ck = kid_k[t], cm = kid_m[t];
                        const int64_t rbase = ck + (ci[b] >= 0 ? ci[b] : 0);
                        double val[kGatherCols];
                        if (kid_prec[t]) {
                            const gptr<const float> Fc = as_global((const float*)kid_F[t]);
                            float raw[kGatherCols];
#pragma unroll
                            for (int jj = 0; jj < kGatherCols; jj++)
                                raw[jj] = Fc[rbase + (int64_t)(ck + max(cj_s[t][gc + jj], 0)) * cm];
#pragma unroll
                            for (int jj = 0; jj < kGatherCols; jj++) val[jj] = (double)raw[jj];
                        } else {
                            const gptr<const double> Fc = as_global((const double*)kid_F[t]);
#pragma unroll
                            for (int jj = 0; jj < kGatherCols; jj++)
                                val[jj] = Fc[rbase + (int64_t)(ck + max(cj_s[t][gc + jj], 0)) * cm];
                        }
#pragma unroll
                        for (int jj = 0; jj < kGatherCols; jj++)
                            acc[jj] += ((ci[b] >= 0) & (cj_s[t][gc + jj] >= 0)) ? val[jj] : 0.0;
                    }
                }
#pragma unroll
                for (int jj = 0; jj < kGatherCols; jj++) {
                    const int j = j0 + jj;
                    if (j < m) F[i + (int64_t)j * m] = (T)acc[jj];
                }
            }
            return;
        }
        // Each child's 16 values of a row are loaded at once, at clamped in-range
        // positions (its first contribution-block row or column where the parent
        // row or column has no counterpart) and masked after: one memory round trip
        // per child instead of one per value; the next child's row position is
        // looked up while these loads are in flight.  Misses add +0.0, which leaves
        // the sums exactly as skipping them would (they never hold -0.0).
        for (int i = i_lo + r; i < i_hi; i += rstep) {
            double acc[kGatherCols];
#pragma unroll
            for (int jj = 0; jj < kGatherCols; jj++) acc[jj] = 0.0;
            int ci_next = 0;
            if (nact > 0) {
                const int t = act_s[0];
                ci_next = child_pos(i, d.npiv, d.din, kid_dseg[t], kid_dout[t], S.imap + kid_im[t]);
            }
            for (int a = 0; a < nact; a++) {
                const int t = act_s[a];
                const int ck = kid_k[t], cm = kid_m[t];
                const int ci = ci_next;
                const int64_t rbase = ck + (ci >= 0 ? ci : 0);
                double val[kGatherCols];
                if (kid_prec[t]) {
                    const gptr<const float> Fc = as_global((const float*)kid_F[t]);
                    float raw[kGatherCols];
#pragma unroll
                    for (int jj = 0; jj < kGatherCols; jj++)
                        raw[jj] = Fc[rbase + (int64_t)(ck + max(cj_s[t][gc + jj], 0)) * cm];
#pragma unroll
                    for (int jj = 0; jj < kGatherCols; jj++) val[jj] = (double)raw[jj];
                } else {
                    const gptr<const double> Fc = as_global((const double*)kid_F[t]);
#pragma unroll
                    for (int jj = 0; jj < kGatherCols; jj++)
                        val[jj] = Fc[rbase + (int64_t)(ck + max(cj_s[t][gc + jj], 0)) * cm];
                }
                if (a + 1 < nact) {
                    const int tn = act_s[a + 1];
                    ci_next = child_pos(i, d.npiv, d.din, kid_dseg[tn], kid_dout[tn], S.imap + kid_im[tn]);
                }
#pragma unroll
                for (int jj = 0; jj < kGatherCols; jj++)
                    acc[jj] += ((ci >= 0) & (cj_s[t][gc + jj] >= 0)) ? val[jj] : 0.0;
            }
#pragma unroll
            for (int jj = 0; jj < kGatherCols; jj++) {
                const int j = j0 + jj;
                if (j < m) F[i + (int64_t)j * m] = (T)acc[jj];
            }
        }
        return;
    }
    if (j0 >= m) return;
    for (int i = i_lo + r; i < i_hi; i += rstep) {
        double acc[kGatherCols];
#pragma unroll
        for (int jj = 0; jj < kGatherCols; jj++) acc[jj] = 0.0;
        int dseg = 0;
        for (int t = cb; t < ce; t++) {
            const int cs = S.child_slot[t];
            const FrontNum dc = fn[cs];
            const int dout = dc.P - dc.k;
            const int32_t* im = S.imap + S.imap_off[cs];
            const int ci = child_pos(i, d.npiv, d.din, dseg, dout, im);
            if (ci >= 0) {  // (more children than the staging holds: maps looked up per value)
                const int64_t rbase = (int64_t)(dc.k + ci);
#pragma unroll
                for (int jj = 0; jj < kGatherCols; jj++) {
                    const int j = j0 + jj;
                    if (j < m) {
                        const int cj = child_pos(j, d.npiv, d.din, dseg, dout, im);
                        if (cj >= 0) acc[jj] += load_front(dc, rbase + (int64_t)(dc.k + cj) * dc.m);
                    }
                }
            }
            dseg += dout;
        }
#pragma unroll
        for (int jj = 0; jj < kGatherCols; jj++) {
            const int j = j0 + jj;
            if (j < m) F[i + (int64_t)j * m] = (T)acc[jj];
        }
    }
}

// Original matrix entries of the level's fronts (each unique entry owns one
// front position; duplicates in the CSR are summed here).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter(DevSym S, FrontNum* fn, const double* vals, int64_t u0,
                                                      int64_t u1, int want_prec) {
    const int64_t u = u0 + (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (u >= u1) return;
    const int s = S.ue_slot[u];
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    int r = S.ue_row[u], c = S.ue_col[u];
    if (r >= d.npiv) r += d.din;
    if (c >= d.npiv) c += d.din;
    double v = 0.0;
    for (int64_t q = S.ue_src_ptr[u]; q < S.ue_src_ptr[u + 1]; q++) v += vals[S.ue_src[q]];
    const gptr<T> F = as_global((T*)d.F);
    const int64_t idx = r + (int64_t)c * d.m;
    F[idx] = (T)((double)F[idx] + v);
}

// ------------------------------------------------------------------ panel
// Column bookkeeping of a front during its partial factorization:
//   [0, k)        eliminated pivots
//   [k, pcur)     fully summed columns not tried yet
//   [pcur, P)     delayed columns (no acceptable pivot when tried)
//   [P, m)        contribution-block columns
// One panel tries the window [k, k + w), w = min(NB, pcur - k).  Column c is
// accepted when its largest entry among the remaining fully summed rows is at
// least u times its largest entry among all remaining rows (threshold partial
// pivoting); otherwise it is delayed and keeps receiving the panel's updates.
// Rows [k, m) of the window live in registers (RS rows per thread, TH threads:
// 512, or 256 on levels whose fronts are all small), so a column step costs two
// barriers, a DPP wave reduction and no global traffic.  At the
// end, accepted columns go to [k, k + nb), delayed ones to the tail of the
// untried range, and the untried columns they displace move into the freed
// window slots; rows are permuted by the LAPACK-style swap sequence, which is
// also published as (destination, source) pairs for the columns outside the
// window.  Columns [x0, x1) (the ones just delayed) are already up to date.
constexpr int kPanelThreads = 512;

// (panel shape classes: front_class / class_nb in mf_device.h)

// Work-group barrier that orders LDS only: global stores issued before it stay in
// flight (the panel streams its multipliers to scratch while it factors).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Candidate of a column step: largest magnitude over all remaining rows (aall),
// largest over the remaining fully summed rows (afs) and its row (ifs, lowest
// row among equal magnitudes).
struct PivCand {
    double aall, afs;
    int ifs;
};
template <int CTRL, int RM>
__device__ __forceinline__ int dpp_i(int x) {
    // all rows enabled (quad permutations, row rotations): every lane has a valid
    // source, so no old value needs to be kept and the move needs no copy first
    if constexpr (RM == 0xF) return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
    else return __builtin_amdgcn_update_dpp(x, x, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i<CTRL, RM>((int)b), hi = dpp_i<CTRL, RM>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Two-phase wave reduction of a candidate (short dependency chains): first the
// maxima of aall and afs (independent DPP chains of plain max), then the lowest row
// among the lanes whose afs equals that maximum (a DPP chain of integer min).  Each
// chain runs within each quad (quad permutations), across the quads of a 16-lane
// row (row rotations by 4 and 8), then across rows (row 0 into row 1 and row 2 into
// row 3 by the row-15 broadcast, then row 1 into rows 2 and 3 by the lane-31
// broadcast), so lane 63 holds the result and is read out uniformly.  Lanes
// outside a step's row mask keep their own value.  The result is the same as
// merging the candidates one by one in any order.
template <int CTRL, int RM>
__device__ __forceinline__ void dmax_step(double& x) {
    x = fmax(x, dpp_d<CTRL, RM>(x));
}
template <int CTRL, int RM>
__device__ __forceinline__ void imin_step(int& x) {
    x = min(x, dpp_i<CTRL, RM>(x));
}
__device__ __forceinline__ PivCand cand_wave2(PivCand a) {
    double ma = a.aall, mf = a.afs;
    dmax_step<0xB1, 0xF>(ma); dmax_step<0xB1, 0xF>(mf);
    dmax_step<0x4E, 0xF>(ma); dmax_step<0x4E, 0xF>(mf);
    dmax_step<0x124, 0xF>(ma); dmax_step<0x124, 0xF>(mf);
    dmax_step<0x128, 0xF>(ma); dmax_step<0x128, 0xF>(mf);
    dmax_step<0x142, 0xA>(ma); dmax_step<0x142, 0xA>(mf);
    dmax_step<0x143, 0xC>(ma); dmax_step<0x143, 0xC>(mf);
    PivCand r;
    r.aall = readlane_d(ma, 63);
    r.afs = readlane_d(mf, 63);
    int ri = (a.afs == r.afs) ? a.ifs : INT_MAX;
    imin_step<0xB1, 0xF>(ri);
    imin_step<0x4E, 0xF>(ri);
    imin_step<0x124, 0xF>(ri);
    imin_step<0x128, 0xF>(ri);
    imin_step<0x142, 0xA>(ri);
    imin_step<0x143, 0xC>(ri);
    r.ifs = __builtin_amdgcn_readlane(ri, 63);
    return r;
}

// Reciprocal of an accepted pivot (finite, nonzero): the hardware estimate
// refined by Newton steps e = 1 - x r, r += r e (two for double, whose estimate
// is good to about half the bits; one for float), a shorter dependent chain than
// the correctly rounded quotient 1 / x and within an ulp of it.
__device__ __forceinline__ double pivot_recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float pivot_recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <typename T, int NB, int RS, int TH>
__device__ __forceinline__ void panel_front(FrontNum* fn, int s, double u, int* dyn) {
    constexpr int kWaves = TH / 64;
    // per wave: its candidate (magnitudes, row) and that row's window values;
    // double-buffered by step parity so that one barrier per column suffices
    __shared__ T urow_w[2][kWaves][NB];
    __shared__ double red_a[2][kWaves], red_f[2][kWaves];
    __shared__ int red_i[2][kWaves];
    __shared__ int acc_col[NB], piv_row[NB], col_dst[NB], old_tag[NB];
    __shared__ int mv_src[NB], mv_dst[NB], mv_tag[NB];
    __shared__ int npairs_s;
    const FrontNum d = fn[s];
    const int m = d.m, P = d.P;
    const int kd0 = d.k, pc = d.pcur;
    if (kd0 >= pc) {
        // nothing left to try: mark an empty round so the trailing updates skip it
        if (threadIdx.x == 0) fn[s].k0 = kd0;
        return;
    }
    const int w = min(NB, pc - kd0);
    const gptr<T> F = as_global((T*)d.F);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int* lmap = dyn;
    int* dstm = dyn + (P - kd0);

    T v[RS][NB];
    int pstep[RS];
#pragma unroll
    for (int r = 0; r < RS; r++) pstep[r] = kd0 + tid + TH * r < m ? -1 : -2;
    // issued column by column, so the first column steps wait only for the first
    // columns while the rest of the window is still arriving
#pragma unroll
    for (int c = 0; c < NB; c++)
#pragma unroll
        for (int r = 0; r < RS; r++) {
            const int row = kd0 + tid + TH * r;
            v[r][c] = (row < m && c < w) ? F[row + (int64_t)(kd0 + c) * m] : T(0);
        }
    uint64_t elim = 0;
    int nb = 0;
    // The window rotates through the registers G columns at a time: in the group
    // of steps starting at column c0, slot j of every row holds window column
    // (c0 + j) mod NB, so the columns being factored are slots 0 .. G-1, every
    // register index is a compile-time constant and the step loop stays rolled (a
    // fully unrolled loop would not fit the instruction cache).  After NB / G
    // groups each column is back in its own slot.
    // (more where the window's registers leave room for the extra temporaries;
    // G = NB needs no rotation at all)
    constexpr int G = (NB == 8 || (NB % 8 == 0 && NB * RS * sizeof(T) <= 32 * sizeof(double))) ? 8
                      : (NB % 4 == 0 && NB * RS * sizeof(T) <= 64 * sizeof(double))           ? 4
                                                                                               : 2;
    static_assert(NB % 2 == 0, "window width must be even");
    // Eliminated columns keep their multipliers in place.  The published pivot row
    // carries zeros in the eliminated slots (written by the lanes of those slots after
    // the owner's row), so the rank-1 updates leave the multipliers exactly unchanged
    // without any per-column mask in the update.
    auto step = [&](int c0, auto Uc) {
        constexpr int U = decltype(Uc)::value;
        const int c = c0 + U;
        if (c >= w) return;
        PivCand cd{0.0, -1.0, INT_MAX};
#pragma unroll
        for (int r = 0; r < RS; r++) {
            if (pstep[r] == -1) {
                const double a = fabs((double)v[r][U]);
                if (!(a <= cd.aall)) cd.aall = (a != a) ? INFINITY : a;
                const int row = kd0 + tid + TH * r;
                if (row < P && a > cd.afs) {
                    cd.afs = a;
                    cd.ifs = row;
                }
            }
        }
        cd = cand_wave2(cd);
        const int par = c & 1;
        // the lane holding the wave's candidate row publishes it with the candidate;
        // LDS writes of one wave land in order, so the zeros follow the row
        if (cd.ifs != INT_MAX && ((cd.ifs - kd0) % TH) == tid) {
            const int rs = (cd.ifs - kd0) / TH;
#pragma unroll
            for (int r = 0; r < RS; r++)
                if (r == rs) {
#pragma unroll
                    for (int j = 0; j < NB; j++) urow_w[par][wid][j] = v[r][j];
                }
        }
        {
            const uint64_t er = (c0 == 0) ? elim : ((elim >> c0) | (elim << (NB - c0)));  // slot order
            if (lane < NB && ((er >> lane) & 1ull)) urow_w[par][wid][lane] = T(0);
        }
        if (lane == 0) {
            red_a[par][wid] = cd.aall;
            red_f[par][wid] = cd.afs;
            red_i[par][wid] = cd.ifs;
        }
        lds_barrier();
        // the wave candidates are merged lane-parallel: lane l holds candidate
        // l mod kWaves, so after the quad (and, for 8 waves, the row-rotation) DPP
        // steps every lane of row 0 holds the merge of all of them
        double ma, mf;
        int ci;
        {
            const int q = lane & (kWaves - 1);
            ma = red_a[par][q];
            mf = red_f[par][q];
            ci = red_i[par][q];
        }
        static_assert(kWaves == 4 || kWaves == 8, "panel blocks of 4 or 8 waves");
        const double cf = mf;
        dmax_step<0xB1, 0xF>(ma); dmax_step<0xB1, 0xF>(mf);
        dmax_step<0x4E, 0xF>(ma); dmax_step<0x4E, 0xF>(mf);
        if constexpr (kWaves > 4) { dmax_step<0x124, 0xF>(ma); dmax_step<0x124, 0xF>(mf); }
        const double aall = readlane_d(ma, 0), afs = readlane_d(mf, 0);
        ci = (cf == afs) ? ci : INT_MAX;
        imin_step<0xB1, 0xF>(ci);
        imin_step<0x4E, 0xF>(ci);
        if constexpr (kWaves > 4) imin_step<0x124, 0xF>(ci);
        const int ifs = __builtin_amdgcn_readlane(ci, 0);
        const bool accept = (afs > 0.0) && (afs <= DBL_MAX) && (afs >= u * aall);
        if (accept) {
            const int qwin = ((ifs - kd0) % TH) >> 6;  // the wave holding the pivot row
            const T* ur = urow_w[par][qwin];
            const int rel = ifs - kd0;
            if ((rel % TH) == tid) {
                const int rs = rel / TH;
#pragma unroll
                for (int r = 0; r < RS; r++)
                    if (r == rs) pstep[r] = nb;
            }
            if (tid == 0) {
                acc_col[nb] = c;
                piv_row[nb] = ifs;
            }
            // one reciprocal of the (uniform) pivot, then a multiply per row: shorter
            // dependency chain than a full division per row, within 1.5 ulp of it
            const T rpiv = pivot_recip(ur[U]);
            // multipliers (zero for rows that are not updated, so their entries stay
            // exactly unchanged)
            T lr[RS];
#pragma unroll
            for (int r = 0; r < RS; r++) {
                const bool act = pstep[r] == -1;
                const T l = v[r][U] * rpiv;
                lr[r] = act ? l : T(0);
                if (act) v[r][U] = l;
            }
#pragma unroll
            for (int j = 0; j < NB; j++) {
                if (j == U) continue;
                const T uj = ur[j];
#pragma unroll
                for (int r = 0; r < RS; r++) v[r][j] -= lr[r] * uj;
            }
            elim |= 1ull << c;
            nb++;
        }
        // one barrier per column: the buffers written in the next step are the
        // other parity, and this parity is rewritten only after every wave has
        // passed the next step's barrier (so all of this step's reads are done)
    };
    // A wave whose rows all lie beyond the front (its first row is >= m) has no
    // candidate, no update and no row to publish: it posts "no candidate" once for
    // both parities and only keeps the block's barrier count, one per column.
    // Its registers are never stored, and nb reaches it through LDS below.
    __shared__ int nb_s;
    if (kd0 + (__builtin_amdgcn_readfirstlane(wid) << 6) >= m) {
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 2; q++) {
                red_a[q][wid] = 0.0;
                red_f[q][wid] = -1.0;
                red_i[q][wid] = INT_MAX;
            }
        }
        for (int c = 0; c < w; c++) lds_barrier();
    } else {
#pragma unroll 1
        for (int c0 = 0; c0 < NB; c0 += G) {
            step(c0, std::integral_constant<int, 0>());
            step(c0, std::integral_constant<int, 1>());
            if constexpr (G >= 4) {
                step(c0, std::integral_constant<int, 2>());
                step(c0, std::integral_constant<int, 3>());
            }
            if constexpr (G == 8) {
                step(c0, std::integral_constant<int, 4>());
                step(c0, std::integral_constant<int, 5>());
                step(c0, std::integral_constant<int, 6>());
                step(c0, std::integral_constant<int, 7>());
            }
#pragma unroll
            for (int r = 0; r < RS; r++) {
                T t[G];
#pragma unroll
                for (int g = 0; g < G; g++) t[g] = v[r][g];
#pragma unroll
                for (int j = 0; j + G < NB; j++) v[r][j] = v[r][j + G];
#pragma unroll
                for (int g = 0; g < G; g++) v[r][NB - G + g] = t[g];
            }
        }
    }
    if (tid == 0) nb_s = nb;
    __syncthreads();
    nb = nb_s;

    // ---- final column and row positions
    const int nrej = w - nb;
    const int pc_new = pc - nrej;
    // accepted columns go to [k0, k0 + nb) in step order, delayed ones to
    // [pc_new, pc) in window order (their rank among the delayed)
    if (tid < w && !((elim >> tid) & 1ull)) col_dst[tid] = pc_new + __popcll(~elim & ((1ull << tid) - 1ull));
    if (tid < nb) col_dst[acc_col[tid]] = kd0 + tid;
    if (tid == 0) {
        // untried columns displaced by the delayed block move into freed window slots
        int nm = 0;
        int fslot = kd0 + nb;
        for (int q = max(pc_new, kd0 + w); q < pc; q++) {
            while (fslot >= pc_new && fslot < pc) fslot++;  // never reached: freed slots precede pc_new
            mv_src[nm] = q;
            mv_dst[nm] = fslot++;
            nm++;
        }
        npairs_s = nm;  // reused below as the move count
    }
    for (int i = kd0 + tid; i < P; i += TH) {
        lmap[i - kd0] = i;   // position -> original row now there
        dstm[i - kd0] = i;   // original row -> its current position
    }
    __syncthreads();
    const int nmove = npairs_s;
    // row permutation: the pivot row of step t goes to position k0 + t; the rows
    // displaced from [k0, k0 + nb) take, in increasing order, the positions the
    // pivot rows vacated beyond k0 + nb (one wave, ballots for the ranks)
    // (LDS written and read back by lanes of the one wave: its LDS accesses are
    // carried out in program order)
    __shared__ int ispiv_s[NB], vac_s[NB];
    if (wid == 0) {
        const bool has = lane < nb;
        const int pr = has ? piv_row[lane] : 0;
        if (has) {
            lmap[lane] = pr;             // position k0 + lane receives pivot row pr
            dstm[pr - kd0] = kd0 + lane;
        }
        // is position k0 + lane itself a pivot row?  (pivot rows are never above k0)
        if (lane < NB) ispiv_s[lane] = 0;
        if (has && pr < kd0 + nb) ispiv_s[pr - kd0] = 1;
        const bool slot_is_piv = has && ispiv_s[lane] != 0;
        const bool displaced = has && !slot_is_piv;           // row k0 + lane must move away
        const bool vacancy = has && (pr >= kd0 + nb);          // position pr frees up
        const uint64_t bd = __ballot(displaced), bv = __ballot(vacancy);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        // the i-th displaced row (in lane order) takes the i-th vacancy (in lane order)
        if (vacancy) vac_s[__popcll(bv & below)] = pr;
        if (displaced) {
            const int p = vac_s[__popcll(bd & below)];
            lmap[p - kd0] = kd0 + lane;
            dstm[lane] = p;
        }
    }
    __syncthreads();
    // column tags (before any column moves)
    const gptr<int32_t> colperm = as_global(iv_colperm(d.iv, P, m));
    const gptr<int32_t> rowperm = as_global(iv_rowperm(d.iv, P, m));
    if (tid < w) old_tag[tid] = colperm[kd0 + tid];
    if (tid < nmove) mv_tag[tid] = colperm[mv_src[tid]];
    int rtag[RS];  // rows [k0, P) lie within the TH * RS register rows
#pragma unroll
    for (int q = 0; q < RS; q++) {
        const int i = kd0 + tid + TH * q;
        rtag[q] = (i < P) ? rowperm[lmap[i - kd0]] : 0;
    }
    __syncthreads();
    // commit the column permutation on every row, inside this block:
    //   scratch = [ old rows [0, k0) of the w window columns | whole displaced columns ]
    // then window columns go to col_dst (rows < k0 from scratch, rows >= k0 from
    // registers in final row order) and displaced columns to mv_dst
    // (with no rejected column every window column stays in place and nothing moves)
    if (nrej > 0) {
        const gptr<T> Wp = as_global((T*)d.W);
        const gptr<T> Wm = Wp + (int64_t)kd0 * w;
        for (int64_t q = tid; q < (int64_t)kd0 * w; q += TH) {
            const int c = (int)(q / kd0), i = (int)(q % kd0);
            Wp[q] = F[i + (int64_t)(kd0 + c) * m];
        }
        for (int64_t q = tid; q < (int64_t)m * nmove; q += TH) {
            const int t = (int)(q / m), i = (int)(q % m);
            Wm[q] = F[i + (int64_t)mv_src[t] * m];
        }
        __syncthreads();
        for (int64_t q = tid; q < (int64_t)kd0 * w; q += TH) {
            const int c = (int)(q / kd0), i = (int)(q % kd0);
            F[i + (int64_t)col_dst[c] * m] = Wp[q];
        }
        for (int64_t q = tid; q < (int64_t)m * nmove; q += TH) {
            const int t = (int)(q / m), i = (int)(q % m);
            F[i + (int64_t)mv_dst[t] * m] = Wm[q];
        }
    }
#pragma unroll
    for (int r = 0; r < RS; r++) {
        const int row = kd0 + tid + TH * r;
        if (row >= m) continue;
        const int drow = row < P ? dstm[row - kd0] : row;
#pragma unroll
        for (int c = 0; c < NB; c++)
            if (c < w) F[drow + (int64_t)col_dst[c] * m] = v[r][c];
    }
    if (tid < w) colperm[col_dst[tid]] = old_tag[tid];
    if (tid < nmove) colperm[mv_dst[tid]] = mv_tag[tid];
#pragma unroll
    for (int q = 0; q < RS; q++) {
        const int i = kd0 + tid + TH * q;
        if (i < P) rowperm[i] = rtag[q];
    }
    // (destination, source) row pairs for the columns outside the window
    if (tid == 0) npairs_s = 0;
    __syncthreads();
    const gptr<int32_t> pairs = as_global(iv_pairs(d.iv, P, m));
    for (int i = kd0 + tid; i < P; i += TH) {
        const int src = lmap[i - kd0];
        if (src != i) {
            const int slot = atomicAdd(&npairs_s, 1);
            pairs[1 + 2 * slot] = i;
            pairs[2 + 2 * slot] = src;
        }
    }
    __syncthreads();
    if (tid == 0) {
        pairs[0] = npairs_s;
        fn[s].k = kd0 + nb;
        fn[s].k0 = kd0;
        fn[s].pcur = pc_new;
        fn[s].x0 = pc_new;
        fn[s].x1 = pc;
    }
}

// One launch per panel round for all fronts of a level: each block runs the
// register panel specialised for its front's class.
template <typename T>
__global__ __launch_bounds__(kPanelThreads) void k_panel(FrontNum* fn, int slot0, double u, int want_prec) {
    extern __shared__ int dyn[];  // lmap[P] | dst[P] (row positions relative to k)
    const int s = slot0 + blockIdx.x;
    const int prec = fn[s].prec;
    if (prec != want_prec) return;
    // The window width follows the front's class (its order); the rows per thread
    // follow the rows still to factor, [k, m), which shrink round by round (the
    // arithmetic does not depend on how rows are spread over threads).
    const int m = fn[s].m, rem = m - fn[s].k;
    switch (front_class(m)) {
        case 0: panel_front<T, 32, 1, kPanelThreads>(fn, s, u, dyn); break;
        case 1:
            if (rem <= kPanelThreads) panel_front<T, 32, 1, kPanelThreads>(fn, s, u, dyn);
            else panel_front<T, 32, 2, kPanelThreads>(fn, s, u, dyn);
            break;
        case 2:
            if constexpr (sizeof(T) == 8) {
                if (rem <= kPanelThreads) panel_front<T, 26, 1, kPanelThreads>(fn, s, u, dyn);
                else if (rem <= 2 * kPanelThreads) panel_front<T, 26, 2, kPanelThreads>(fn, s, u, dyn);
                else panel_front<T, 26, 3, kPanelThreads>(fn, s, u, dyn);
            } else {
                if (rem <= kPanelThreads) panel_front<T, 32, 1, kPanelThreads>(fn, s, u, dyn);
                else if (rem <= 2 * kPanelThreads) panel_front<T, 32, 2, kPanelThreads>(fn, s, u, dyn);
                else panel_front<T, 32, 3, kPanelThreads>(fn, s, u, dyn);
            }
            break;
        case 3:
            if constexpr (sizeof(T) == 8) panel_front<T, 20, 4, kPanelThreads>(fn, s, u, dyn);
            else {
                if (rem <= kPanelThreads) panel_front<T, 32, 1, kPanelThreads>(fn, s, u, dyn);
                else if (rem <= 2 * kPanelThreads) panel_front<T, 32, 2, kPanelThreads>(fn, s, u, dyn);
                else if (rem <= 3 * kPanelThreads) panel_front<T, 32, 3, kPanelThreads>(fn, s, u, dyn);
                else panel_front<T, 32, 4, kPanelThreads>(fn, s, u, dyn);
            }
            break;
        default:
            if constexpr (sizeof(T) == 8) panel_front<T, 8, 8, kPanelThreads>(fn, s, u, dyn);
            else panel_front<T, 16, 8, kPanelThreads>(fn, s, u, dyn);
            break;
    }
}

// Levels whose fronts all have order <= 512 (class 0): the class-0 panel (same
// window, same arithmetic) on 256 threads with RS = 1 or 2 rows per thread.
constexpr int kPanelSmallThreads = 256;
template <typename T, int RS>
__global__ __launch_bounds__(kPanelSmallThreads, (RS == 1 ? (sizeof(T) == 8 ? 4 : 5) : 1)) void k_panel_small(FrontNum* fn, int slot0, double u, int want_prec) {
    extern __shared__ int dyn[];
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    // two rows per thread only where the front's remaining rows need them (the
    // arithmetic of the two variants is the same)
    if (RS == 1 || d.m - d.k <= kPanelSmallThreads) panel_front<T, 32, 1, kPanelSmallThreads>(fn, s, u, dyn);
    else panel_front<T, 32, RS, kPanelSmallThreads>(fn, s, u, dyn);
}

// Forward substitution x <- L11^-1 x for the columns [c0, cend) of the tile that
// lie ahead of the panel (>= kd1) and outside the just-delayed block [x0, x1),
// one column per lane of the calling wave (so cend - c0 <= 64), on rows
// [kd0, kd0 + nb).  L11 is unit lower, column-major with leading dimension
// kNBMax, in LDS.  Each row is updated in step order with one fused multiply-add
// per step, in double precision, and rounded to T once at the end.
template <typename T, int N>
__device__ __forceinline__ void trsm_lane_cols(const gptr<T> F, const T* L11, int m, int kd0, int kd1, int x0,
                                               int x1, int nb, int c0, int cend) {
    const int lane = threadIdx.x & 63;
    const int j = c0 + lane;
    const bool live = j < cend && j >= kd1 && !(j >= x0 && j < x1);
    if (!__any(live)) return;
    const gptr<T> colp = F + (int64_t)(live ? j : c0) * m + kd0;
    double x[N];
#pragma unroll
    for (int r = 0; r < N; r++) x[r] = (double)colp[min(r, nb - 1)];
#pragma unroll
    for (int a = 0; a < N - 1; a++) {
        const double xa = x[a];
        // a zero the compiler cannot see through, computed from x[a]: step a's L11
        // reads wait for x[a] instead of all being hoisted to the start, which
        // would hold every entry of L11 in registers at once
        int z;
        asm("v_mov_b32 %0, 0" : "=v"(z) : "v"((int)(__double_as_longlong(xa) >> 32)));
        const T* Lc = L11 + a * kNBMax + z;
#pragma unroll
        for (int r = a + 1; r < N; r++) x[r] -= (double)Lc[r] * xa;
    }
    if (live) {
#pragma unroll
        for (int r = 0; r < N; r++)
            if (r < nb) colp[r] = (T)x[r];
    }
}

// Columns outside the last panel's window: apply its row swaps; for columns
// ahead of it (>= k, outside the just-delayed block) also form the new U rows
// with the unit-lower L11 of the panel.  One block per (front, tile of sw <= 64
// columns): 64-column tiles on levels of many fronts, 16-column tiles on levels of
// few large fronts (more blocks in flight, fewer sequential passes per block).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_swap_trsm(FrontNum* fn, int slot0, int want_prec, const int32_t* tasks,
                                                        int sw) {
    __shared__ T L11[kNBMax * kNBMax];
    __shared__ int pd[2 * kNBMax], ps[2 * kNBMax];
    const int task = tasks[blockIdx.x];
    const int s = slot0 + (task >> 12);
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P;
    const int kd0 = d.k0, kd1 = d.k, nb = kd1 - kd0;
    if (nb <= 0) return;
    const int c0 = (task & 4095) * sw, cend = min(c0 + sw, m);
    if (c0 >= m) return;
    const gptr<T> F = as_global((T*)d.F);
    const gptr<const int32_t> pairs = as_global(iv_pairs(d.iv, P, m));
    const int np = pairs[0];
    const int tid = threadIdx.x;
    {
        // L11 and the pair list: every global load issued before the first LDS
        // store (a store could alias a later load and would serialize them)
        constexpr int kL = kNBMax * kNBMax / kThreads;
        T l11[kL];
#pragma unroll
        for (int q = 0; q < kL; q++) {
            const int idx = tid + q * kThreads;
            const int a = idx % nb, b = idx / nb;
            l11[q] = idx < nb * nb ? F[(kd0 + a) + (int64_t)(kd0 + b) * m] : T(0);
        }
        // (the list's slots exist up to 2 kNBMax pairs: loaded without waiting for np)
        const int pdv = tid < 2 * kNBMax ? pairs[1 + 2 * tid] : 0, psv = tid < 2 * kNBMax ? pairs[2 + 2 * tid] : 0;
#pragma unroll
        for (int q = 0; q < kL; q++) {
            const int idx = tid + q * kThreads;
            if (idx < nb * nb) L11[idx % nb + (idx / nb) * kNBMax] = l11[q];
        }
        if (tid < np) {
            pd[tid] = pdv;
            ps[tid] = psv;
        }
    }
    __syncthreads();
    // row swaps of the panel through registers: every source of a column is read
    // (all loads of a thread issued together) before any destination is written
    {
        constexpr int kQ = 2 * kNBMax / (kThreads / 64);
        const int jl = c0 + (tid & 63);
        const bool live = jl < cend && !(jl >= kd0 && jl < kd1) && !(jl >= d.x0 && jl < d.x1);
        const gptr<T> cp = F + (int64_t)jl * m;
        T tmp[kQ];
#pragma unroll
        for (int i = 0; i < kQ; i++) {
            const int q = (tid >> 6) + i * (kThreads / 64);
            tmp[i] = (live && q < np) ? cp[ps[q]] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kQ; i++) {
            const int q = (tid >> 6) + i * (kThreads / 64);
            if (live && q < np) cp[pd[q]] = tmp[i];
        }
        __syncthreads();
    }
    // new U rows: unit-lower solve with L11, one lane per column with the column's
    // rows in registers and L11's entries read as wave-uniform LDS broadcasts, so
    // a step needs no cross-lane traffic.  N >= nb is a compile-time row count:
    // rows [nb, N) and steps [nb - 1, N - 1) only touch rows that are not stored.
    if (tid < 64) {
        if (nb <= 8) trsm_lane_cols<T, 8>(F, L11, m, kd0, kd1, d.x0, d.x1, nb, c0, cend);
        else if (nb <= 16) trsm_lane_cols<T, 16>(F, L11, m, kd0, kd1, d.x0, d.x1, nb, c0, cend);
        else if (nb <= 20) trsm_lane_cols<T, 20>(F, L11, m, kd0, kd1, d.x0, d.x1, nb, c0, cend);
        else if (nb <= 26) trsm_lane_cols<T, 26>(F, L11, m, kd0, kd1, d.x0, d.x1, nb, c0, cend);
        else trsm_lane_cols<T, kNBMax>(F, L11, m, kd0, kd1, d.x0, d.x1, nb, c0, cend);
    }
}

// ------------------------------------------------------------------ GEMM
template <typename T>
struct Mfma;
// Operand layouts of both 16x16x4 MFMAs: lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Result register r of lane l is D[row(l, r)][l%16], where the
// row mapping differs between the FP64 and FP32 instructions (measured on gfx950).
template <>
struct Mfma<double> {
    typedef dbl4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef flt4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// C -= A * B on a 64x64 tile of one front, with A = F[rows, ka:kb], B = F[ka:kb, cols].
// mode 0 (eager, after a panel): rows [k, m) x cols [k, m) except the columns the
//        panel just delayed [x0, x1) and the deferred block rows >= P and cols >= P;
//        K = the panel's pivots [k0, k).
// mode 1 (Schur): rows [P, m) x cols [P, m); K = all pivots [0, k).
// Block (x: column tile, y: row tile, z: front).  4 waves, each a 32x32 quarter
// made of 2x2 MFMA 16x16 blocks; K staged through LDS in chunks of 32.
template <typename T>
__global__ __launch_bounds__(kThreads, 4) void k_gemm(FrontNum* fn, int slot0, int mode, int want_prec,
                                                   const int32_t* tasks) {
    // A and B chunks, then (aliased) the C tile for the transposed epilogue
    __shared__ T smem_ab[2 * kKC * kLdsPad];
    static_assert(2 * kKC * kLdsPad >= kTile * kLdsPad, "C tile must fit in the A/B buffer");
    T* As = smem_ab;
    T* Bs = smem_ab + kKC * kLdsPad;
    T* Cs = smem_ab;
    const int task = tasks[blockIdx.x];
    const int s = slot0 + (task >> 12);
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P;
    int rlo, clo, ka, kb;
    if (mode == 0) {
        rlo = d.k;
        clo = 0;
        ka = d.k0;
        kb = d.k;
    } else {
        rlo = P;
        clo = P;
        ka = 0;
        kb = d.k;
    }
    if (kb <= ka) return;
    const int col0 = clo + (task & 63) * kTile;
    const int row0 = (mode == 0 ? 0 : P) + ((task >> 6) & 63) * kTile;
    if (col0 >= m || row0 >= m || row0 + kTile <= rlo || col0 + kTile <= rlo) return;
    if (mode == 0 && row0 >= P && col0 >= P) return;
    if (mode == 0 && col0 >= d.x0 && col0 + kTile <= d.x1) return;
    const gptr<const T> F = as_global((const T*)d.F);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wi = wid & 1, wj = wid >> 1;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = acc_t{0, 0, 0, 0};
    constexpr int kPer = kKC * kTile / kThreads;  // staged elements per thread and operand
    // K chunks pass through registers: all global loads of a chunk are issued
    // together (a load after an LDS store could not be hoisted above it, which
    // would serialize the latencies), and the next chunk's loads are in flight
    // while the MFMAs of the current one run
    T ra[kPer], rb[kPer];
    auto load_chunk = [&](int k0) {
        const int kc = min(kKC, kb - k0);
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const int idx = tid + q * kThreads;
            const int r = idx % kTile, a = idx / kTile;
            const int row = row0 + r;
            ra[q] = (a < kc && row < m) ? F[row + (int64_t)(k0 + a) * m] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const int idx = tid + q * kThreads;
            const int a = idx % kKC, c = idx / kKC;
            const int col = col0 + c;
            rb[q] = (a < kc && col < m) ? F[(k0 + a) + (int64_t)col * m] : T(0);
        }
    };
    load_chunk(ka);
    for (int k0 = ka; k0 < kb; k0 += kKC) {
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const int idx = tid + q * kThreads;
            As[(idx / kTile) * kLdsPad + idx % kTile] = ra[q];
            Bs[(idx % kKC) * kLdsPad + idx / kKC] = rb[q];
        }
        __syncthreads();
        if (k0 + kKC < kb) load_chunk(k0 + kKC);
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 4) {
            T av[2], bv[2];
#pragma unroll
            for (int bi = 0; bi < 2; bi++) av[bi] = As[(kk + lane / 16) * kLdsPad + wi * 32 + bi * 16 + (lane & 15)];
#pragma unroll
            for (int bj = 0; bj < 2; bj++) bv[bj] = Bs[(kk + lane / 16) * kLdsPad + wj * 32 + bj * 16 + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 2; bi++)
#pragma unroll
                for (int bj = 0; bj < 2; bj++) acc[bi][bj] = Mfma<T>::mma(av[bi], bv[bj], acc[bi][bj]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = wi * 32 + bi * 16 + Mfma<T>::row(lane, r);
                const int j = wj * 32 + bj * 16 + (lane & 15);
                Cs[j * kLdsPad + i] = acc[bi][bj][r];
            }
    __syncthreads();
    const gptr<T> Fw = as_global((T*)d.F);
    // read every C entry of this thread before the first store, then update
    constexpr int kOut = kTile * kTile / kThreads;
    T cold[kOut];
    bool live[kOut];
#pragma unroll
    for (int q = 0; q < kOut; q++) {
        const int idx = tid + q * kThreads;
        const int i = idx % kTile, j = idx / kTile;
        const int row = row0 + i, col = col0 + j;
        bool ok = !(row < rlo || row >= m || col >= m || col < rlo);
        if (mode == 0 && ((row >= P && col >= P) || (col >= d.x0 && col < d.x1))) ok = false;
        live[q] = ok;
        cold[q] = ok ? Fw[row + (int64_t)col * m] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kOut; q++) {
        const int idx = tid + q * kThreads;
        const int i = idx % kTile, j = idx / kTile;
        if (live[q]) Fw[(row0 + i) + (int64_t)(col0 + j) * m] = cold[q] - Cs[j * kLdsPad + i];
    }
}

// BF16 variant of the deferred Schur update (mode 1) for FP32 fronts:
// C[P:m, P:m] -= bf16(L21) * bf16(U12), FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  Operand layout (measured on gfx950): lane l holds
// A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) .. +7][l%16]; result register r of
// lane l is D[4(l/16) + r][l%16].  LDS keeps A as [row][k] and B as [col][k] so a
// lane's 8 operands are one 16-byte read.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kKB = 32;          // K per MFMA
constexpr int kKBPad = kKB + 8;  // row pitch in LDS (bf16 elements)

__global__ __launch_bounds__(kThreads) void k_gemm_bf16(FrontNum* fn, int slot0, const int32_t* tasks) {
    __shared__ __attribute__((aligned(16))) __bf16 As[kTile * kKBPad];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kTile * kKBPad];
    __shared__ float Cs[kTile * kLdsPad];
    const int task = tasks[blockIdx.x];
    const int s = slot0 + (task >> 12);
    const FrontNum d = fn[s];
    if (d.prec != 1) return;
    const int m = d.m, P = d.P, kb = d.k;
    if (kb <= 0) return;
    const int col0 = P + (task & 63) * kTile;
    const int row0 = P + ((task >> 6) & 63) * kTile;
    if (col0 >= m || row0 >= m) return;
    const gptr<const float> F = as_global((const float*)d.F);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wi = wid & 1, wj = wid >> 1;
    flt4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = flt4{0, 0, 0, 0};
    constexpr int kPerB = kKB * kTile / kThreads;
    // K chunks through registers, the next chunk's loads in flight during the
    // current chunk's MFMAs (as in k_gemm)
    float ra[kPerB], rb[kPerB];
    auto load_chunk = [&](int k0) {
        const int kc = min(kKB, kb - k0);
#pragma unroll
        for (int q = 0; q < kPerB; q++) {
            const int idx = tid + q * kThreads;
            const int r = idx % kTile, a = idx / kTile;
            const int row = row0 + r;
            ra[q] = (a < kc && row < m) ? F[row + (int64_t)(k0 + a) * m] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kPerB; q++) {
            const int idx = tid + q * kThreads;
            const int a = idx % kKB, c = idx / kKB;
            const int col = col0 + c;
            rb[q] = (a < kc && col < m) ? F[(k0 + a) + (int64_t)col * m] : 0.0f;
        }
    };
    if (kb > 0) load_chunk(0);
    for (int k0 = 0; k0 < kb; k0 += kKB) {
#pragma unroll
        for (int q = 0; q < kPerB; q++) {
            const int idx = tid + q * kThreads;
            As[(idx % kTile) * kKBPad + idx / kTile] = (__bf16)ra[q];
            Bs[(idx / kKB) * kKBPad + idx % kKB] = (__bf16)rb[q];
        }
        __syncthreads();
        if (k0 + kKB < kb) load_chunk(k0 + kKB);
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int bi = 0; bi < 2; bi++)
            av[bi] = *(const bf16x8*)&As[(wi * 32 + bi * 16 + (lane & 15)) * kKBPad + 8 * (lane >> 4)];
#pragma unroll
        for (int bj = 0; bj < 2; bj++)
            bv[bj] = *(const bf16x8*)&Bs[(wj * 32 + bj * 16 + (lane & 15)) * kKBPad + 8 * (lane >> 4)];
#pragma unroll
        for (int bi = 0; bi < 2; bi++)
#pragma unroll
            for (int bj = 0; bj < 2; bj++)
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[bi], bv[bj], acc[bi][bj], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = wi * 32 + bi * 16 + 4 * (lane >> 4) + r;
                const int j = wj * 32 + bj * 16 + (lane & 15);
                Cs[j * kLdsPad + i] = acc[bi][bj][r];
            }
    __syncthreads();
    const gptr<float> Fw = as_global((float*)d.F);
    constexpr int kOutB = kTile * kTile / kThreads;
    float cold[kOutB];
#pragma unroll
    for (int q = 0; q < kOutB; q++) {
        const int idx = tid + q * kThreads;
        const int row = row0 + idx % kTile, col = col0 + idx / kTile;
        cold[q] = (row < m && col < m) ? Fw[row + (int64_t)col * m] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kOutB; q++) {
        const int idx = tid + q * kThreads;
        const int i = idx % kTile, j = idx / kTile;
        const int row = row0 + i, col = col0 + j;
        if (row < m && col < m) Fw[row + (int64_t)col * m] = cold[q] - Cs[j * kLdsPad + i];
    }
}

// Start of a tree level in the planned schedule: each front's delayed-in count is
// the sum of its children's delayed-out counts (P - k), read from the children's
// finished bookkeeping, and the front's order and fully summed count follow from
// it.  Everything else (storage, scratch, vector offset) comes from the template,
// whose din field holds the capacity the storage was sized for.  A front that
// would outgrow it lowers *overflow (INT_MAX when none) to its level and is
// clamped to the capacity, which keeps every access inside its allocations.
// From then on fronts are given a precision no kernel takes (kSkipPrec), so
// the rest of the schedule only pays its launches; the caller redoes the levels
// from the first overflowing one with per-level synchronization.  One thread
// per front.
__global__ __launch_bounds__(kThreads) void k_level_setup(DevSym S, FrontNum* fn, const FrontNum* tmpl, int slot0,
                                                          int count, int level, int32_t* overflow) {
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q >= count) return;
    const int s = slot0 + q;
    FrontNum d = tmpl[s];
    int din = 0;
    for (int t = S.child_ptr[s]; t < S.child_ptr[s + 1]; t++) {
        const int cs = S.child_slot[t];
        din += fn[cs].P - fn[cs].k;
    }
    bool skip = *overflow != INT_MAX;  // an earlier level overflowed
    if (din > d.din) {
        atomicMin(overflow, level);
        din = d.din;
        skip = true;
    }
    d.din = din;
    d.m = d.mnom + din;
    d.P = d.npiv + din;
    d.k = 0;
    d.k0 = 0;
    d.pcur = d.P;
    d.x0 = 0;
    d.x1 = 0;
    if (skip) d.prec = kSkipPrec;
    fn[s] = d;
}

__global__ __launch_bounds__(64) void k_fill_i32(int32_t* y, int32_t v) {
    if (threadIdx.x == 0) *y = v;
}

// Post-factorization bookkeeping: column variables in final order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_finalize(DevSym S, FrontNum* fn, int slot0, int want_prec) {
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P;
    const int32_t* rows = S.rows + S.rows_ptr[s];
    const gptr<const int32_t> colperm = as_global(iv_colperm(d.iv, P, m));
    const gptr<int32_t> colvar = as_global(iv_colvar(d.iv, P, m));
    const int cb = S.child_ptr[s], ce = S.child_ptr[s + 1];
    for (int i = threadIdx.x; i < m; i += kThreads) {
        const int src = i < P ? colperm[i] : i;
        int v;
        if (src < d.npiv) {
            v = rows[src];
        } else if (src < d.npiv + d.din) {
            int off = src - d.npiv;
            v = -1;
            for (int tt = cb; tt < ce; tt++) {
                const FrontNum dc = fn[S.child_slot[tt]];
                const int dout = dc.P - dc.k;
                if (off < dout) {
                    v = as_global(iv_colvar(dc.iv, dc.P, dc.m))[dc.k + off];
                    break;
                }
                off -= dout;
            }
        } else {
            v = rows[src - d.din];
        }
        colvar[i] = v;
    }
}

// ------------------------------------------------------------------ solve
// Each front owns a block of `vec` (m x nrhs, column-major, ld m).  Forward
// sweep (leaves to root), per front:
//   z = rows of (b + the children's contribution vectors) in final row order
//   y = L11^{-1} z[0:k]            (k_fwd_tri: one block; 16x16 diagonal blocks
//                                    are solved by one wave from registers)
//   c = z[k:m] - L21 y             (k_fwd_gemv: many blocks per large front)
// and the block of `vec` holds [y; c].  Backward sweep (root to leaves):
//   t = y - U12 x[colvar[k:m]]     (k_bwd_gemv)
//   x[colvar[0:k]] = U11^{-1} t    (k_bwd_tri)
constexpr int kBS = 64;       // diagonal block of the triangular sweeps (one lane per row)
constexpr int kTriThreads = 512;
constexpr int kTriSmallOrder = 256;  // levels whose fronts are all at most this order sweep with one wave per front
constexpr int kGemvRows = 64;    // rows per block of the solve GEMVs

// Dot product of one row of a diagonal block's column strip (bs <= kBS columns,
// stride m) with a vector in LDS.  A full strip is unrolled with 8 accumulators,
// so all 64 loads of the row are in flight together.
template <typename T>
__device__ __forceinline__ double block_dot(gptr<const T> Fi, int64_t m, const double* z, int bs) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (bs == kBS) {
        // the strip is loaded in the storage type before any use, a whole strip
        // (FP32) or half of one (FP64, register budget) at a time
        constexpr int kChunk = sizeof(T) == 4 ? kBS : kBS / 2;
#pragma unroll
        for (int c0 = 0; c0 < kBS; c0 += kChunk) {
            T raw[kChunk];
#pragma unroll
            for (int a = 0; a < kChunk; a++) raw[a] = Fi[(int64_t)(c0 + a) * m];
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the first use
#pragma unroll
            for (int a = 0; a < kChunk; a++) acc[a & 7] += (double)raw[a] * z[c0 + a];
        }
    } else {
        for (int a = 0; a < bs; a++) acc[a & 7] += (double)Fi[(int64_t)a * m] * z[a];
    }
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// tile_dot's dot product of one row computed by a single lane, with exactly its
// arithmetic (the four column groups of the block's waves, four accumulators each,
// combined in the same order), so that the fused small-front sweeps give results
// bitwise equal to the two-kernel path used on levels of larger fronts.
template <typename T>
__device__ __forceinline__ double row_dot_tiled(gptr<const T> Fcol0, int64_t m, const double* xv, int ncols) {
    double p[4];
#pragma unroll
    for (int g = 0; g < 4; g++) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int j = g;
        for (; j + 12 < ncols; j += 16) {
            a0 += (double)Fcol0[(int64_t)j * m] * xv[j];
            a1 += (double)Fcol0[(int64_t)(j + 4) * m] * xv[j + 4];
            a2 += (double)Fcol0[(int64_t)(j + 8) * m] * xv[j + 8];
            a3 += (double)Fcol0[(int64_t)(j + 12) * m] * xv[j + 12];
        }
        for (; j < ncols; j += 4) a0 += (double)Fcol0[(int64_t)j * m] * xv[j];
        p[g] = (a0 + a1) + (a2 + a3);
    }
    return (p[0] + p[1]) + (p[2] + p[3]);
}

// Several right-hand sides at once (NR of them, nrc live; column c of a vector
// at c * ld): every factor entry is loaded once and used for all columns, and
// each column's sum is formed with exactly the operations, in the order, of the
// one-column function, so a column's result does not depend on how many are
// solved together.  Columns c >= nrc repeat column nrc - 1; their results are
// not used.
template <typename T, int NR>
__device__ __forceinline__ void block_dot_n(gptr<const T> Fi, int64_t m, const double* z, int ldz, int bs, int nrc,
                                            double* out) {
    if constexpr (NR == 1) {
        out[0] = block_dot<T>(Fi, m, z, bs);
    } else {
        const double* zc[NR];
        double acc[NR][8];
#pragma unroll
        for (int c = 0; c < NR; c++) {
            zc[c] = z + min(c, nrc - 1) * ldz;
#pragma unroll
            for (int q = 0; q < 8; q++) acc[c][q] = 0.0;
        }
        if (bs == kBS) {
            // fewer entries ahead than block_dot: the accumulators need the registers
            constexpr int kChunk = sizeof(T) == 4 ? kBS / 2 : kBS / 4;
#pragma unroll
            for (int c0 = 0; c0 < kBS; c0 += kChunk) {
                T raw[kChunk];
#pragma unroll
                for (int a = 0; a < kChunk; a++) raw[a] = Fi[(int64_t)(c0 + a) * m];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int a = 0; a < kChunk; a++) {
                    const double f = (double)raw[a];
#pragma unroll
                    for (int c = 0; c < NR; c++) acc[c][a & 7] += f * zc[c][c0 + a];
                }
            }
        } else {
            for (int a = 0; a < bs; a++) {
                const double f = (double)Fi[(int64_t)a * m];
#pragma unroll
                for (int c = 0; c < NR; c++) acc[c][a & 7] += f * zc[c][a];
            }
        }
#pragma unroll
        for (int c = 0; c < NR; c++)
            out[c] = ((acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3])) +
                     ((acc[c][4] + acc[c][5]) + (acc[c][6] + acc[c][7]));
    }
}

template <typename T, int NR>
__device__ __forceinline__ void row_dot_tiled_n(gptr<const T> Fcol0, int64_t m, const double* xv, int ldx, int ncols,
                                                int nrc, double* out) {
    if constexpr (NR == 1) {
        out[0] = row_dot_tiled<T>(Fcol0, m, xv, ncols);
    } else {
        const double* xc[NR];
#pragma unroll
        for (int c = 0; c < NR; c++) xc[c] = xv + min(c, nrc - 1) * ldx;
        double p[NR][4];
#pragma unroll
        for (int g = 0; g < 4; g++) {
            double a0[NR], a1[NR], a2[NR], a3[NR];
#pragma unroll
            for (int c = 0; c < NR; c++) a0[c] = a1[c] = a2[c] = a3[c] = 0.0;
            int j = g;
            for (; j + 12 < ncols; j += 16) {
                const double f0 = (double)Fcol0[(int64_t)j * m], f1 = (double)Fcol0[(int64_t)(j + 4) * m];
                const double f2 = (double)Fcol0[(int64_t)(j + 8) * m], f3 = (double)Fcol0[(int64_t)(j + 12) * m];
#pragma unroll
                for (int c = 0; c < NR; c++) {
                    a0[c] += f0 * xc[c][j];
                    a1[c] += f1 * xc[c][j + 4];
                    a2[c] += f2 * xc[c][j + 8];
                    a3[c] += f3 * xc[c][j + 12];
                }
            }
            for (; j < ncols; j += 4) {
                const double f0 = (double)Fcol0[(int64_t)j * m];
#pragma unroll
                for (int c = 0; c < NR; c++) a0[c] += f0 * xc[c][j];
            }
#pragma unroll
            for (int c = 0; c < NR; c++) p[c][g] = (a0[c] + a1[c]) + (a2[c] + a3[c]);
        }
#pragma unroll
        for (int c = 0; c < NR; c++) out[c] = (p[c][0] + p[c][1]) + (p[c][2] + p[c][3]);
    }
}

// Diagonal blocks of the sweeps staged through LDS (blocks of more than one
// wave): while the block's threads form the dot products of one diagonal block,
// waves 1.. load the next block into registers and store it to LDS after their
// dot products, so the wave that solves the next block reads LDS instead of
// waiting for global memory.  Column a, row r of the block at a * kBS + r, with
// rows and columns clamped into the block exactly as the direct loads are.
template <typename T, int TT>
struct DiagStage {
    static constexpr int kN = (kBS * kBS + TT - 64 - 1) / (TT - 64);  // entries per thread of waves 1..
    T pre[kN];
    __device__ __forceinline__ void load(const gptr<const T> F, int64_t m, int jb0, int jbs) {
        const int t = (int)threadIdx.x - 64;
#pragma unroll
        for (int q = 0; q < kN; q++) {
            const int e = min(t + q * (TT - 64), kBS * kBS - 1);
            const int a = e / kBS, r = e % kBS;
            pre[q] = F[(jb0 + min(r, jbs - 1)) + (int64_t)(jb0 + min(a, jbs - 1)) * m];
        }
    }
    __device__ __forceinline__ void store(T* blk) const {
        const int t = (int)threadIdx.x - 64;
#pragma unroll
        for (int q = 0; q < kN; q++) {
            const int e = t + q * (TT - 64);
            if (e < kBS * kBS) blk[e] = pre[q];
        }
    }
};

// The nrc columns of one row of a vector block, loaded into registers before
// any is stored (a loop that loads and stores to LDS in each iteration would wait
// for every load in turn): W = 1, or kSwRhs for passes of several columns
// (nrc <= kSwRhs; columns beyond nrc load column nrc - 1 and are not used).
template <int W, typename Src>
__device__ __forceinline__ void load_cols(double (&r)[W], int nrc, Src src) {
#pragma unroll
    for (int c = 0; c < W; c++) r[c] = src(min(c, nrc - 1));
}

// FUSE (one-wave blocks of small-front levels): the same block also forms
// c = z[k:m] - L21 y, which k_fwd_gemv does otherwise.
template <typename T, int TT, bool FUSE, int NR>
__global__ __launch_bounds__(TT, TT == 64 && NR > 1 ? 3 : 1) void k_fwd_tri(DevSym S, const FrontNum* fn, int slot0,
                                                                   int want_prec, const double* b, int64_t ldb,
                                                                   double* vec, int nrhs, int c0, int nrc,
                                                                   const uint8_t* skip) {
    extern __shared__ double zs[];
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec || (skip && skip[s])) return;
    const int m = d.m, P = d.P, k = d.k;
    const gptr<const T> F = as_global((const T*)d.F);
    const gptr<const int32_t> rowperm = as_global(iv_rowperm(d.iv, P, m));
    const int32_t* rows = S.rows + S.rows_ptr[s];
    double* v = vec + d.voff * nrhs;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int cb = S.child_ptr[s], ce = S.child_ptr[s + 1];
    constexpr bool kStage = TT > 64;
    __shared__ T dblk[kStage ? kBS * kBS : 1];
    if constexpr (kStage) {
        if (wid > 0 && k > 0) {
            DiagStage<T, TT> st0;
            st0.load(F, m, 0, min(kBS, k));
            st0.store(dblk);
        }
    }
    constexpr int kCL = NR == 1 ? 1 : kSwRhs;  // columns a row's loads cover
    for (int i = tid; i < m; i += TT) {
        const int src = i < P ? rowperm[i] : i;
        double zr[kCL];
        if (src < d.npiv) {
            const double* br = b + rows[src];
            load_cols<kCL>(zr, nrc, [&](int c) { return br[(int64_t)(c0 + c) * ldb]; });
        } else {
#pragma unroll
            for (int c = 0; c < kCL; c++) zr[c] = 0.0;
        }
        int dseg = 0;
        for (int tt = cb; tt < ce; tt++) {
            const int cs = S.child_slot[tt];
            const FrontNum dc = fn[cs];
            const int dout = dc.P - dc.k;
            const int ci = child_pos(src, d.npiv, d.din, dseg, dout, S.imap + S.imap_off[cs]);
            if (ci >= 0) {
                const double* vc = vec + dc.voff * nrhs + dc.k + ci;
                double t[kCL];
                load_cols<kCL>(t, nrc, [&](int c) { return vc[(int64_t)(c0 + c) * dc.m]; });
#pragma unroll
                for (int c = 0; c < kCL; c++) zr[c] += t[c];
            }
            dseg += dout;
        }
#pragma unroll
        for (int c = 0; c < kCL; c++)
            if (c < nrc) zs[i + c * m] = zr[c];
    }
    __syncthreads();
    // the columns in groups of NR (one group unless a one-wave block serves more
    // columns than NR; a staged block, TT > 64, is always called with nrc <= NR)
    for (int cg = 0; cg < nrc; cg += NR) {
        double* const zg = zs + (int64_t)cg * m;
        const int ng = min(NR, nrc - cg);
        // the diagonal blocks' chains: one right-hand side on wave 0; several, one
        // per wave of a multi-wave block (or all on the one wave of a small-front block)
        constexpr int kCW = (NR > 1 && TT > 64) ? (NR < TT / 64 ? NR : TT / 64) : 1;  // waves with chains
        constexpr int kCN = NR / kCW;                                               // chains per wave
        for (int j0 = 0; j0 < k; j0 += kBS) {
            const int bs = min(kBS, k - j0);
            if (wid < kCW && wid < ng) {
                // every lane loads an in-range entry (row and column clamped into the
                // block) and masks it afterwards: the 64 loads are unconditional and all
                // in flight together instead of one branch (and wait) per column
                T raw[kBS];
                const int lr = j0 + min(lane, bs - 1);
                if constexpr (kStage) {
#pragma unroll
                    for (int a = 0; a < kBS; a++) raw[a] = dblk[a * kBS + lane];
                } else {
#pragma unroll
                    for (int a = 0; a < kBS; a++) raw[a] = F[lr + (int64_t)(j0 + min(a, bs - 1)) * m];
                }
                if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
                double Lr[kBS];
#pragma unroll
                for (int a = 0; a < kBS; a++) Lr[a] = ((lane < bs) & (a < lane)) ? (double)raw[a] : 0.0;
                // a wave's chains (columns wid + kCW q) step together: independent, so
                // their latencies overlap; each is the one-column chain.  Columns
                // >= ng repeat column ng - 1 and are not stored.
                double x[kCN];
#pragma unroll
                for (int q = 0; q < kCN; q++) x[q] = lane < bs ? zg[j0 + lane + min(wid + kCW * q, ng - 1) * m] : 0.0;
#pragma unroll
                for (int a = 0; a < kBS - 1; a++) {
                    // the steps after the block's last row would only subtract zeros
                    // (Lr vanishes there): a small front stops after bs - 1 steps
                    if (a + 1 >= bs) break;
#pragma unroll
                    for (int q = 0; q < kCN; q++) {
                        const double xa = readlane_d(x[q], a);  // uniform broadcast, no LDS round trip
                        x[q] -= Lr[a] * xa;
                    }
                }
#pragma unroll
                for (int q = 0; q < kCN; q++)
                    if (wid + kCW * q < ng && lane < bs) zg[j0 + lane + (wid + kCW * q) * m] = x[q];
            }
            __syncthreads();
            if constexpr (kStage) {
                const bool nxt = wid > 0 && j0 + kBS < k;
                DiagStage<T, TT> st1;
                if (nxt) st1.load(F, m, j0 + kBS, min(kBS, k - j0 - kBS));
                for (int i = j0 + bs + tid; i < k; i += TT) {
                    const gptr<const T> Fi = F + i + (int64_t)j0 * m;
                    double o[NR];
                    block_dot_n<T, NR>(Fi, m, zg + j0, m, bs, ng, o);
#pragma unroll
                    for (int c = 0; c < NR; c++)
                        if (c < ng) zg[i + c * m] -= o[c];
                }
                if (nxt) st1.store(dblk);
            } else {
                for (int i = j0 + bs + tid; i < k; i += TT) {
                    const gptr<const T> Fi = F + i + (int64_t)j0 * m;
                    double o[NR];
                    block_dot_n<T, NR>(Fi, m, zg + j0, m, bs, ng, o);
#pragma unroll
                    for (int c = 0; c < NR; c++)
                        if (c < ng) zg[i + c * m] -= o[c];
                }
            }
            __syncthreads();
        }
        if constexpr (FUSE) {
            if (k > 0) {
                for (int i = k + tid; i < m; i += TT) {
                    double o[NR];
                    row_dot_tiled_n<T, NR>(F + i, m, zg, m, k, ng, o);
#pragma unroll
                    for (int c = 0; c < NR; c++)
                        if (c < ng) zg[i + c * m] -= o[c];
                }
                __syncthreads();
            }
        }
    }
    for (int i = tid; i < m; i += TT)
        for (int c = 0; c < nrc; c++) v[i + (int64_t)(c0 + c) * m] = zs[i + c * m];
}

// Row tile of a front times a vector staged in LDS: 64 rows per block (one lane
// per row, coalesced column reads), the columns split over the block's 4 waves
// (column j to wave j mod 4, four independent accumulators per lane), and the 4
// partial sums added in wave order (deterministic).  Returns the row's dot
// product in wave 0; other waves return 0.
template <typename T>
__device__ __forceinline__ double tile_dot(gptr<const T> Fcol0, int64_t m, const double* xv, int ncols, double* part) {
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = g;
    for (; j + 12 < ncols; j += 16) {
        a0 += (double)Fcol0[(int64_t)j * m] * xv[j];
        a1 += (double)Fcol0[(int64_t)(j + 4) * m] * xv[j + 4];
        a2 += (double)Fcol0[(int64_t)(j + 8) * m] * xv[j + 8];
        a3 += (double)Fcol0[(int64_t)(j + 12) * m] * xv[j + 12];
    }
    for (; j < ncols; j += 4) a0 += (double)Fcol0[(int64_t)j * m] * xv[j];
    part[g * 64 + lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    double r = 0.0;
    if (g == 0) r = (part[lane] + part[64 + lane]) + (part[128 + lane] + part[192 + lane]);
    __syncthreads();
    return r;
}

// tile_dot for NR right-hand sides (column c of xv at c * ldx; part holds NR x
// 256 doubles): each entry loaded once, each column's sums formed and combined
// as tile_dot does.  Wave 0 gets the results in out; columns >= nrc repeat
// column nrc - 1.
template <typename T, int NR>
__device__ __forceinline__ void tile_dot_n(gptr<const T> Fcol0, int64_t m, const double* xv, int ldx, int ncols,
                                           int nrc, double* part, double* out) {
    if constexpr (NR == 1) {
        out[0] = tile_dot<T>(Fcol0, m, xv, ncols, part);
    } else {
        const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
        const double* xc[NR];
        double a0[NR], a1[NR], a2[NR], a3[NR];
#pragma unroll
        for (int c = 0; c < NR; c++) {
            xc[c] = xv + min(c, nrc - 1) * ldx;
            a0[c] = a1[c] = a2[c] = a3[c] = 0.0;
        }
        int j = g;
        for (; j + 12 < ncols; j += 16) {
            const double f0 = (double)Fcol0[(int64_t)j * m], f1 = (double)Fcol0[(int64_t)(j + 4) * m];
            const double f2 = (double)Fcol0[(int64_t)(j + 8) * m], f3 = (double)Fcol0[(int64_t)(j + 12) * m];
#pragma unroll
            for (int c = 0; c < NR; c++) {
                a0[c] += f0 * xc[c][j];
                a1[c] += f1 * xc[c][j + 4];
                a2[c] += f2 * xc[c][j + 8];
                a3[c] += f3 * xc[c][j + 12];
            }
        }
        for (; j < ncols; j += 4) {
            const double f0 = (double)Fcol0[(int64_t)j * m];
#pragma unroll
            for (int c = 0; c < NR; c++) a0[c] += f0 * xc[c][j];
        }
#pragma unroll
        for (int c = 0; c < NR; c++) part[(c * 4 + g) * 64 + lane] = (a0[c] + a1[c]) + (a2[c] + a3[c]);
        __syncthreads();
        if (g == 0) {
#pragma unroll
            for (int c = 0; c < NR; c++)
                out[c] = (part[(c * 4) * 64 + lane] + part[(c * 4 + 1) * 64 + lane]) +
                         (part[(c * 4 + 2) * 64 + lane] + part[(c * 4 + 3) * 64 + lane]);
        }
        __syncthreads();
    }
}

// c[i] = z[i] - sum_{j<k} L[i, j] y[j] for rows i in [k, m); block (x: 64-row tile, y: front)
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_fwd_gemv(const FrontNum* fn, int slot0, int want_prec, double* vec,
                                                       int nrhs, int c0, int nrc, const uint8_t* skip) {
    extern __shared__ double ys[];
    __shared__ double part[kThreads * NR];
    const int s = slot0 + blockIdx.y;
    const FrontNum d = fn[s];
    if (d.prec != want_prec || (skip && skip[s])) return;
    const int m = d.m, k = d.k;
    const int i0 = k + blockIdx.x * kGemvRows;
    if (i0 >= m || k == 0) return;
    const gptr<const T> F = as_global((const T*)d.F);
    double* v = vec + d.voff * nrhs;
    for (int j = threadIdx.x; j < k; j += kThreads) {
        double t[NR];
        load_cols<NR>(t, nrc, [&](int c) { return v[j + (int64_t)(c0 + c) * m]; });
#pragma unroll
        for (int c = 0; c < NR; c++)
            if (c < nrc) ys[j + c * k] = t[c];
    }
    __syncthreads();
    const int i = min(i0 + (int)(threadIdx.x & 63), m - 1);  // clamped rows compute, never store
    double t[NR];
    tile_dot_n<T, NR>(F + i, m, ys, k, k, nrc, part, t);
    if (threadIdx.x < 64 && i0 + (int)threadIdx.x < m) {
#pragma unroll
        for (int c = 0; c < NR; c++)
            if (c < nrc) v[i + (int64_t)(c0 + c) * m] -= t[c];
    }
}

// t[i] = y[i] - sum_{j in [k,m)} U[i, j] x[colvar[j]] for rows i < k, in place in vec
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_bwd_gemv(const FrontNum* fn, int slot0, int want_prec, const double* x,
                                                       int64_t ldx, double* vec, int nrhs, int c0, int nrc,
                                                       const uint8_t* skip) {
    extern __shared__ double xs[];
    __shared__ double part[kThreads * NR];
    const int s = slot0 + blockIdx.y;
    const FrontNum d = fn[s];
    if (d.prec != want_prec || (skip && skip[s])) return;
    const int m = d.m, P = d.P, k = d.k;
    const int i0 = blockIdx.x * kGemvRows;
    if (i0 >= k || k == m) return;
    const gptr<const T> F = as_global((const T*)d.F);
    const gptr<const int32_t> colvar = as_global(iv_colvar(d.iv, P, m));
    double* v = vec + d.voff * nrhs;
    const int nc = m - k;
    for (int j = threadIdx.x; j < nc; j += kThreads) {
        const int var = colvar[k + j];
        double t[NR];
        load_cols<NR>(t, nrc, [&](int c) { return var >= 0 ? x[var + (int64_t)(c0 + c) * ldx] : 0.0; });
#pragma unroll
        for (int c = 0; c < NR; c++)
            if (c < nrc) xs[j + c * nc] = t[c];
    }
    __syncthreads();
    const int i = min(i0 + (int)(threadIdx.x & 63), k - 1);  // clamped rows compute, never store
    double t[NR];
    tile_dot_n<T, NR>(F + i + (int64_t)k * m, m, xs, nc, nc, nrc, part, t);
    if (threadIdx.x < 64 && i0 + (int)threadIdx.x < k) {
#pragma unroll
        for (int c = 0; c < NR; c++)
            if (c < nrc) v[i + (int64_t)(c0 + c) * m] -= t[c];
    }
}

// FUSE (one-wave blocks of small-front levels): the same block first forms
// t = y - U12 x[colvar[k:m]], which k_bwd_gemv does otherwise.
template <typename T, int TT, bool FUSE, int NR>
__global__ __launch_bounds__(TT, TT == 64 && NR > 1 ? 3 : 1) void k_bwd_tri(const FrontNum* fn, int slot0, int want_prec,
                                                                   double* x, int64_t ldx, const double* vec, int nrhs,
                                                                   int c0, int nrc, const uint8_t* skip) {
    extern __shared__ double ts[];
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec || (skip && skip[s])) return;
    const int m = d.m, P = d.P, k = d.k;
    const gptr<const T> F = as_global((const T*)d.F);
    const gptr<const int32_t> colvar = as_global(iv_colvar(d.iv, P, m));
    const double* v = vec + d.voff * nrhs;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr bool kStage = TT > 64;
    __shared__ T dblk[kStage ? kBS * kBS : 1];
    if constexpr (kStage) {
        if (wid > 0 && k > 0) {
            DiagStage<T, TT> st0;
            const int jb0 = max(0, k - kBS);
            st0.load(F, m, jb0, k - jb0);
            st0.store(dblk);
        }
    }
    constexpr int kCL = NR == 1 ? 1 : kSwRhs;  // columns a row's loads cover
    for (int i = tid; i < k; i += TT) {
        double t[kCL];
        load_cols<kCL>(t, nrc, [&](int c) { return v[i + (int64_t)(c0 + c) * m]; });
#pragma unroll
        for (int c = 0; c < kCL; c++)
            if (c < nrc) ts[i + c * k] = t[c];
    }
    // FUSE: the solution values of the columns [k, m), after ts
    double* const xs = ts + (int64_t)k * nrc;
    const int nc = m - k;
    if constexpr (FUSE) {
        if (nc > 0 && k > 0) {
            for (int j = tid; j < nc; j += TT) {
                const int var = colvar[k + j];
                double t[kCL];
                load_cols<kCL>(t, nrc, [&](int c) { return var >= 0 ? x[var + (int64_t)(c0 + c) * ldx] : 0.0; });
#pragma unroll
                for (int c = 0; c < kCL; c++)
                    if (c < nrc) xs[j + c * nc] = t[c];
            }
        }
    }
    __syncthreads();
    // the columns in groups of NR, as in the forward sweep
    for (int cg = 0; cg < nrc; cg += NR) {
        double* const tg = ts + (int64_t)cg * k;
        const int ng = min(NR, nrc - cg);
        if constexpr (FUSE) {
            if (nc > 0 && k > 0) {
                for (int i = tid; i < k; i += TT) {
                    double o[NR];
                    row_dot_tiled_n<T, NR>(F + i + (int64_t)k * m, m, xs + (int64_t)cg * nc, nc, nc, ng, o);
#pragma unroll
                    for (int c = 0; c < NR; c++)
                        if (c < ng) tg[i + c * k] -= o[c];
                }
                __syncthreads();
            }
        }
        constexpr int kCW = (NR > 1 && TT > 64) ? (NR < TT / 64 ? NR : TT / 64) : 1;  // waves with chains
        constexpr int kCN = NR / kCW;                                               // chains per wave
        for (int j1 = k; j1 > 0; j1 -= kBS) {
            const int j0 = max(0, j1 - kBS), bs = j1 - j0;
            if (wid < kCW && wid < ng) {
                T raw[kBS];  // clamped unconditional loads, as in the forward sweep
                const int lr = j0 + min(lane, bs - 1);
                if constexpr (kStage) {
#pragma unroll
                    for (int a = 0; a < kBS; a++) raw[a] = dblk[a * kBS + lane];
                } else {
#pragma unroll
                    for (int a = 0; a < kBS; a++) raw[a] = F[lr + (int64_t)(j0 + min(a, bs - 1)) * m];
                }
                __builtin_amdgcn_sched_barrier(0);
                double Ur[kBS];
#pragma unroll
                for (int a = 0; a < kBS; a++) Ur[a] = ((lane < bs) & (a >= lane) & (a < bs)) ? (double)raw[a] : 0.0;
                // each lane's reciprocal of itg own diagonal entry, taken in parallel
                // once per block: the sequential sweep then multiplies instead of
                // dividing (within 1.5 ulp of the quotient)
                const int ld = min(lane, bs - 1);
                const double rd = 1.0 / (double)(kStage ? dblk[ld * kBS + ld] : F[lr + (int64_t)lr * m]);
                // a wave's chains step together, as in the forward sweep
                double xl[kCN];
#pragma unroll
                for (int q = 0; q < kCN; q++) xl[q] = lane < bs ? tg[j0 + lane + min(wid + kCW * q, ng - 1) * k] : 0.0;
#pragma unroll
                for (int a = kBS - 1; a >= 0; a--) {
                    if (a < bs) {
                        // row a's value and diagonal reciprocal are broadcast from lane a
                        const double ra = readlane_d(rd, a);
#pragma unroll
                        for (int q = 0; q < kCN; q++) {
                            const double xa = readlane_d(xl[q], a) * ra;
                            if (lane == a) xl[q] = xa;
                            if (lane < a) xl[q] -= Ur[a] * xa;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kCN; q++)
                    if (wid + kCW * q < ng && lane < bs) tg[j0 + lane + (wid + kCW * q) * k] = xl[q];
            }
            __syncthreads();
            if constexpr (kStage) {
                const bool nxt = wid > 0 && j0 > 0;
                DiagStage<T, TT> st1;
                if (nxt) st1.load(F, m, max(0, j0 - kBS), j0 - max(0, j0 - kBS));
                for (int i = tid; i < j0; i += TT) {
                    const gptr<const T> Fi = F + i + (int64_t)j0 * m;
                    double o[NR];
                    block_dot_n<T, NR>(Fi, m, tg + j0, k, bs, ng, o);
#pragma unroll
                    for (int c = 0; c < NR; c++)
                        if (c < ng) tg[i + c * k] -= o[c];
                }
                if (nxt) st1.store(dblk);
            } else {
                for (int i = tid; i < j0; i += TT) {
                    const gptr<const T> Fi = F + i + (int64_t)j0 * m;
                    double o[NR];
                    block_dot_n<T, NR>(Fi, m, tg + j0, k, bs, ng, o);
#pragma unroll
                    for (int c = 0; c < NR; c++)
                        if (c < ng) tg[i + c * k] -= o[c];
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < k; i += TT) {
        const int var = colvar[i];
        if (var < 0) continue;
        for (int c = 0; c < nrc; c++) x[var + (int64_t)(c0 + c) * ldx] = ts[i + c * k];
    }
}

// ------------------------------------------------------------------ residual
// r = b - J x and, per right-hand side (blockIdx.y) and per system of a batch,
// the componentwise backward error omega = max_i |r_i| / (|J||x| + |b|)_i
// together with the four maxima of the normwise one (max |r_i|, max |x_i|,
// max |b_i| and max_i sum_j |J_ij|), 16 lanes per row.  Each quantity is a
// non-negative double kept as its bit pattern and combined with an unsigned
// atomic max (exact and order-independent); quantity q of (system, rhs) s sits at
// out[q * cnt + s].
constexpr int kResRows = 256;  // rows per residual block (16 lanes per row, 16 rows per pass)

__device__ __forceinline__ void res_flush(unsigned long long* out, int64_t cnt, int64_t s, const double* q) {
#pragma unroll
    for (int k = 0; k < kResQ; k++) atomicMax(out + k * cnt + s, (unsigned long long)__double_as_longlong(q[k]));
}

__global__ __launch_bounds__(kThreads) void k_residual(const int64_t* rp, const int32_t* ci, const double* val,
                                                       int64_t n, const double* x, int64_t ldx, const double* b,
                                                       int64_t ldb, double* r, int64_t ldr,
                                                       unsigned long long* out, int64_t cnt, const int32_t* row_seg,
                                                       int nrhs, double* part) {
    // Each block covers kResRows consecutive rows and folds their maxima into
    // part[(c * gridDim.x + block) * kResQ + q]; k_residual_fold then reduces the
    // blocks of each system, so no two blocks update one address (same-address
    // atomics serialize in L2).  In a batch, rows of one system are contiguous,
    // so only blocks that straddle two systems post zeros there and fall back to
    // per-thread maxima flushed with atomics at each system boundary.
    __shared__ double wmax[kResQ][kThreads / 64];
    const int c = blockIdx.y;
    const int sub = threadIdx.x & 15;
    const int64_t r0 = (int64_t)blockIdx.x * kResRows;
    const int64_t r1 = min(n, r0 + kResRows);
    const double* xc = x + (int64_t)c * ldx;
    const bool one_seg = !row_seg || row_seg[r0] == row_seg[r1 - 1];
    double q[kResQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int seg = -1;
    for (int64_t row0 = r0; row0 < r1; row0 += kThreads / 16) {
        const int64_t row = row0 + threadIdx.x / 16;
        double acc = 0.0, den = 0.0, asum = 0.0;
        if (row < r1) {
            // two entries per lane and pass, both loaded (and both x gathered)
            // before either is used; the sums take them in the same order as one
            // at a time
            const int64_t te = rp[row + 1];
            for (int64_t t = rp[row] + sub; t < te; t += 32) {
                const bool two = t + 16 < te;
                const double a0 = val[t], a1 = two ? val[t + 16] : 0.0;
                const int j0 = ci[t], j1 = two ? ci[t + 16] : j0;
                const double x0 = xc[j0], x1 = xc[j1];
                acc = fma(a0, x0, acc);
                den = fma(fabs(a0), fabs(x0), den);
                asum += fabs(a0);
                if (two) {
                    acc = fma(a1, x1, acc);
                    den = fma(fabs(a1), fabs(x1), den);
                    asum += fabs(a1);
                }
            }
        }
        for (int off = 8; off > 0; off >>= 1) {
            acc += __shfl_xor(acc, off, 16);
            den += __shfl_xor(den, off, 16);
            asum += __shfl_xor(asum, off, 16);
        }
        if (row < r1 && sub == 0) {
            const double bi = b[row + (int64_t)c * ldb];
            const double ri = bi - acc;
            r[row + (int64_t)c * ldr] = ri;
            const double dd = den + fabs(bi);
            double w = dd > 0.0 ? fabs(ri) / dd : (ri == 0.0 ? 0.0 : INFINITY);
            if (w != w) w = INFINITY;
            double v[kResQ] = {w, fabs(ri), fabs(xc[row]), fabs(bi), asum};
#pragma unroll
            for (int k = 1; k < kResQ; k++)
                if (v[k] != v[k]) v[k] = INFINITY;
            if (!one_seg) {
                const int sg = row_seg[row];
                if (sg != seg) {
                    if (seg >= 0) res_flush(out, cnt, (int64_t)seg * nrhs + c, q);
                    seg = sg;
#pragma unroll
                    for (int k = 0; k < kResQ; k++) q[k] = v[k];
                    continue;
                }
            }
#pragma unroll
            for (int k = 0; k < kResQ; k++) q[k] = fmax(q[k], v[k]);
        }
    }
    double* pb = part + ((int64_t)c * gridDim.x + blockIdx.x) * kResQ;
    if (!one_seg) {
        if (sub == 0 && seg >= 0) res_flush(out, cnt, (int64_t)seg * nrhs + c, q);
        if (threadIdx.x < kResQ) pb[threadIdx.x] = 0.0;
        return;
    }
#pragma unroll
    for (int k = 0; k < kResQ; k++) {
        for (int off = 32; off > 0; off >>= 1) q[k] = fmax(q[k], __shfl_xor(q[k], off));
        if ((threadIdx.x & 63) == 0) wmax[k][threadIdx.x >> 6] = q[k];
    }
    __syncthreads();
    if (threadIdx.x < kResQ) {
        double mx = wmax[threadIdx.x][0];
        for (int i = 1; i < kThreads / 64; i++) mx = fmax(mx, wmax[threadIdx.x][i]);
        pb[threadIdx.x] = mx;
    }
}

// Second stage: block (s, c) folds the per-block maxima of system s's row blocks
// for right-hand side c and posts them with one atomic max per quantity (blocks
// that straddle two systems posted zeros and their own atomics).
__global__ __launch_bounds__(kThreads) void k_residual_fold(const double* part, int nblk, const int64_t* seg_row0,
                                                            const int64_t* seg_n, int nrhs,
                                                            unsigned long long* out, int64_t cnt) {
    __shared__ double red[kResQ][kThreads / 64];
    const int s = blockIdx.x, c = blockIdx.y;
    const int64_t ns = seg_n[s];
    if (ns <= 0) return;
    const int b0 = (int)(seg_row0[s] / kResRows), b1 = (int)((seg_row0[s] + ns - 1) / kResRows);
    double q[kResQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = b0 + (int)threadIdx.x; b <= b1; b += kThreads) {
        const double* pb = part + ((int64_t)c * nblk + b) * kResQ;
#pragma unroll
        for (int k = 0; k < kResQ; k++) q[k] = fmax(q[k], pb[k]);
    }
#pragma unroll
    for (int k = 0; k < kResQ; k++) {
        for (int off = 32; off > 0; off >>= 1) q[k] = fmax(q[k], __shfl_xor(q[k], off));
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = q[k];
    }
    __syncthreads();
    if (threadIdx.x < kResQ) {
        double mx = red[threadIdx.x][0];
        for (int i = 1; i < kThreads / 64; i++) mx = fmax(mx, red[threadIdx.x][i]);
        atomicMax(out + threadIdx.x * cnt + (int64_t)s * nrhs + c, (unsigned long long)__double_as_longlong(mx));
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// x[:, c] += d[:, c] on the rows of systems still refining (active[seg * nrhs + c])
__global__ __launch_bounds__(kThreads) void k_axpy(int64_t n, double* x, int64_t ldx, const double* dvec,
                                                   int64_t ldd, const int32_t* active, const int32_t* row_seg,
                                                   int nrhs) {
    const int c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const int sg = row_seg ? row_seg[i] : 0;
        if (active[sg * nrhs + c]) x[i + c * ldx] += dvec[i + c * ldd];
    }
}

#define MF_CHECK_LAUNCH() (hipGetLastError())

// ------------------------------------------------------------------ Krylov vectors (FP64)
// y[:, c] = J x[:, c] (column c = blockIdx.y), 16 lanes per row
__global__ __launch_bounds__(kThreads) void k_spmv(const int64_t* rp, const int32_t* ci, const double* val, int64_t n,
                                                   const double* x, int64_t ldx, double* y, int64_t ldy) {
    const int64_t row = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 16;
    const int sub = threadIdx.x & 15;
    const double* xc = x + (int64_t)blockIdx.y * ldx;
    double acc = 0.0;
    if (row < n)
        for (int64_t t = rp[row] + sub; t < rp[row + 1]; t += 16) acc = fma(val[t], xc[ci[t]], acc);
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (row < n && sub == 0) y[row + (int64_t)blockIdx.y * ldy] = acc;
}

// Deterministic segmented multi-dot, stage 1: block (b, s) reduces chunk b of
// system s: part[(s * nblk + b) * nv + i] = sum over its rows of V[:, i] * w.
// A system's chunks depend only on its own size, so its dots are the same alone
// and in a batch.
constexpr int kDotBlocks = 512;
__global__ __launch_bounds__(kThreads) void k_mdot1(const double* V, int64_t ldv, int nv, const double* w,
                                                    const int64_t* seg_row0, const int64_t* seg_n, double* part) {
    __shared__ double red[kThreads / 64];
    const int sg = blockIdx.y;
    const int64_t n = seg_n[sg], base = seg_row0[sg];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = base + blockIdx.x * chunk, hi = base + min(n, (int64_t)(blockIdx.x + 1) * chunk);
    for (int i = 0; i < nv; i++) {
        double acc = 0.0;
        for (int64_t r = lo + threadIdx.x; r < hi; r += kThreads) acc = fma(V[r + i * ldv], w[r], acc);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < kThreads / 64; q++) t += red[q];
            part[((int64_t)sg * gridDim.x + blockIdx.x) * nv + i] = t;
        }
        __syncthreads();
    }
}
// stage 2: out[s * ostride + i] = sum_b part[(s * nb + b) * nv + i] in block order
__global__ void k_mdot2(const double* part, int nb, int nv, int nseg, int ostride, double* out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nv * nseg) return;
    const int sg = q / nv, i = q % nv;
    double t = 0.0;
    for (int b = 0; b < nb; b++) t += part[((int64_t)sg * nb + b) * nv + i];
    out[sg * ostride + i] = t;
}
// w -= V[:, 0:nv] h_seg   (coefficients of the row's system: h[seg * hstride + i])
__global__ __launch_bounds__(kThreads) void k_vsub(double* w, const double* V, int64_t ldv, int nv, const double* h,
                                                   int hstride, int64_t n, const int32_t* row_seg) {
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < n; r += (int64_t)gridDim.x * kThreads) {
        const double* hs = h + (row_seg ? row_seg[r] : 0) * hstride;
        double acc = w[r];
        for (int i = 0; i < nv; i++) acc -= V[r + i * ldv] * hs[i];
        w[r] = acc;
    }
}
// y = a_seg * x
__global__ __launch_bounds__(kThreads) void k_scale(double* y, const double* x, const double* a, int astride, int64_t n,
                                                    const int32_t* row_seg) {
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < n; r += (int64_t)gridDim.x * kThreads)
        y[r] = a[(row_seg ? row_seg[r] : 0) * astride] * x[r];
}
// x += V[:, 0:nv] c_seg
__global__ __launch_bounds__(kThreads) void k_vadd(double* x, const double* V, int64_t ldv, int nv, const double* c,
                                                   int cstride, int64_t n, const int32_t* row_seg) {
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < n; r += (int64_t)gridDim.x * kThreads) {
        const double* cs = c + (row_seg ? row_seg[r] : 0) * cstride;
        double acc = x[r];
        for (int i = 0; i < nv; i++) acc += V[r + i * ldv] * cs[i];
        x[r] = acc;
    }
}
__global__ __launch_bounds__(kThreads) void k_fill(double* y, double v, int64_t n) {
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < n; r += (int64_t)gridDim.x * kThreads) y[r] = v;
}

static unsigned vec_blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 2048); }

hipError_t launch_spmv(const DevSym& S, const double* val, int64_t n, const double* x, int64_t ldx, double* y,
                       int64_t ldy, int ncol, hipStream_t st) {
    if (n <= 0 || ncol <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spmv, dim3((unsigned)((n * 16 + kThreads - 1) / kThreads), (unsigned)ncol), dim3(kThreads), 0,
                       st, S.csr_rowptr, S.csr_colind, val, n, x, ldx, y, ldy);
    return MF_CHECK_LAUNCH();
}
// out[s * ostride + i] (device) = V_s[:, 0:nv]^T w_s per system; part: kDotBlocks * nseg * nv doubles
hipError_t launch_mdot(const DevSym& S, const double* V, int64_t ldv, int nv, const double* w, double* part,
                       double* out, int ostride, hipStream_t st) {
    hipLaunchKernelGGL(k_mdot1, dim3(kDotBlocks, S.nseg), dim3(kThreads), 0, st, V, ldv, nv, w, S.seg_row0, S.seg_n,
                       part);
    hipLaunchKernelGGL(k_mdot2, dim3((nv * S.nseg + 63) / 64), dim3(64), 0, st, part, kDotBlocks, nv, S.nseg, ostride,
                       out);
    return MF_CHECK_LAUNCH();
}
hipError_t launch_vsub(const DevSym& S, double* w, const double* V, int64_t ldv, int nv, const double* h, int hstride,
                       int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_vsub, dim3(vec_blocks(n)), dim3(kThreads), 0, st, w, V, ldv, nv, h, hstride, n, S.row_seg);
    return MF_CHECK_LAUNCH();
}
hipError_t launch_vadd(const DevSym& S, double* x, const double* V, int64_t ldv, int nv, const double* c,
                       int cstride, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_vadd, dim3(vec_blocks(n)), dim3(kThreads), 0, st, x, V, ldv, nv, c, cstride, n, S.row_seg);
    return MF_CHECK_LAUNCH();
}
hipError_t launch_scale(const DevSym& S, double* y, const double* x, const double* a, int astride, int64_t n,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(vec_blocks(n)), dim3(kThreads), 0, st, y, x, a, astride, n, S.row_seg);
    return MF_CHECK_LAUNCH();
}
hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(vec_blocks(n)), dim3(kThreads), 0, st, y, v, n);
    return MF_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ launchers

hipError_t launch_level_setup(const DevSym& S, FrontNum* fn, const FrontNum* tmpl, int slot0, int count, int level,
                              int32_t* overflow, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_setup, dim3((count + kThreads - 1) / kThreads), dim3(kThreads), 0, st, S, fn, tmpl,
                       slot0, count, level, overflow);
    return MF_CHECK_LAUNCH();
}
// first[0] = smallest CSR position holding NaN or Inf (left at ~0 if none)
__global__ __launch_bounds__(kThreads) void k_nonfinite(const double* v, int64_t nnz, unsigned long long* first) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kThreads)
        if (!isfinite(v[i])) atomicMin(first, (unsigned long long)i);
}
hipError_t launch_nonfinite(const double* v, int64_t nnz, unsigned long long* first, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, first, 1, ~0ull);
    if (nnz > 0)
        hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)std::min<int64_t>((nnz + kThreads - 1) / kThreads, 4096)),
                           dim3(kThreads), 0, st, v, nnz, first);
    return MF_CHECK_LAUNCH();
}
hipError_t launch_fill_i32(int32_t* y, int32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, y, v);
    return MF_CHECK_LAUNCH();
}

// Segmented copy with an offset per segment (start[s] = elements before segment
// s, start[nseg] = total): the device-side concatenation of the pattern maps of
// the systems of a batch.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_seg_copy(const SegCopy* __restrict__ segs, const int64_t* __restrict__ start,
                                                       int nseg, T* __restrict__ out) {
    const int64_t total = start[nseg];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads) {
        int lo = 0, hi = nseg - 1;  // last segment whose start is <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const SegCopy g = segs[lo];
        const int64_t o = i - start[lo];
        if constexpr (std::is_integral<T>::value) out[g.dst + o] = ((const T*)g.src)[o] + (T)g.add;
        else out[g.dst + o] = ((const T*)g.src)[o];  // values: copied bit for bit
    }
}
// The reverse: segment g of `in` (from g.src, g.count entries) to its own
// destination g.dst, for all segments in one launch.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_seg_scatter(const SegOut* __restrict__ segs,
                                                          const int64_t* __restrict__ start, int nseg,
                                                          const T* __restrict__ in) {
    const int64_t total = start[nseg];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads) {
        int lo = 0, hi = nseg - 1;  // last segment whose start is <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const SegOut g = segs[lo];
        const int64_t o = i - start[lo];
        ((T*)g.dst)[o] = in[g.src + o];
    }
}
template <typename T>
hipError_t launch_seg_scatter(const SegOut* segs, const int64_t* start, int nseg, int64_t total, const T* in,
                              hipStream_t st) {
    if (nseg > 0 && total > 0)
        hipLaunchKernelGGL(k_seg_scatter<T>, dim3((unsigned)std::min<int64_t>((total + kThreads - 1) / kThreads, 8192)),
                           dim3(kThreads), 0, st, segs, start, nseg, in);
    return MF_CHECK_LAUNCH();
}
template hipError_t launch_seg_scatter<double>(const SegOut*, const int64_t*, int, int64_t, const double*, hipStream_t);
template <typename T>
hipError_t launch_seg_copy(const SegCopy* segs, const int64_t* start, int nseg, int64_t total, T* out,
                           hipStream_t st) {
    if (nseg > 0 && total > 0)
        hipLaunchKernelGGL(k_seg_copy<T>, dim3((unsigned)std::min<int64_t>((total + kThreads - 1) / kThreads, 8192)),
                           dim3(kThreads), 0, st, segs, start, nseg, out);
    return MF_CHECK_LAUNCH();
}
template hipError_t launch_seg_copy<int32_t>(const SegCopy*, const int64_t*, int, int64_t, int32_t*, hipStream_t);
template hipError_t launch_seg_copy<int64_t>(const SegCopy*, const int64_t*, int, int64_t, int64_t*, hipStream_t);
template hipError_t launch_seg_copy<double>(const SegCopy*, const int64_t*, int, int64_t, double*, hipStream_t);

int panel_nb(int prec, int m) { return class_nb(front_class(m), prec); }

// cls_mmax[kNClass], cls_Pmax[kNClass]: per panel class of this precision in the level (0 = none)
// part 1: extend-add, value scatter and the panel rounds (after which every
// front's eliminated count, and so its delayed-out count, is final); part 2: the
// Schur GEMM and finalize; part 0: both.
template <typename T>
hipError_t launch_level_factor(const DevSym& S, FrontNum* fn, int slot0, int count, int mmax, const int* cls_mmax,
                               const int* cls_Pmax, const double* vals, int64_t u0, int64_t u1, double u, int prec,
                               const LevelTasks& tk, hipStream_t st, hipEvent_t* ev, bool bf16_schur,
                               std::vector<hipEvent_t>* pev, bool panel_full, int part) {
    if (count <= 0) return hipSuccess;
    if (mmax > 4096) return hipErrorInvalidValue;
    if (part != 2) {
        if (tk.ngather)
            hipLaunchKernelGGL(k_gather<T>, dim3(tk.ngather), dim3(kThreads), 0, st, S, fn, slot0, prec, tk.gather);
        if (u1 > u0)
            hipLaunchKernelGGL(k_scatter<T>, dim3((unsigned)((u1 - u0 + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                               st, S, fn, vals, u0, u1, prec);
        if (ev) (void)hipEventRecord(ev[0], st);
        int rounds = 0, Pmax = 0;
        for (int c = 0; c < kNClass; c++) {
            if (cls_mmax[c] <= 0) continue;
            const int nbc = class_nb(c, prec);
            rounds = std::max(rounds, (cls_Pmax[c] + nbc - 1) / nbc);
            Pmax = std::max(Pmax, cls_Pmax[c]);
        }
        {
            const size_t panel_lds = 2 * sizeof(int) * (size_t)Pmax;
            for (int t = 0; t < rounds; t++) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (pev && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
                    (void)hipEventRecord(e0, st);
                    pev->push_back(e0);
                    pev->push_back(e1);
                }
                // levels of class-0 fronts (order <= 512, window 32): 4 waves per front, one
                // per SIMD, with one or two rows per lane (same arithmetic as 8 waves),
                // unless panel_full asks for the 8-wave kernel
                if (panel_full)
                    hipLaunchKernelGGL(k_panel<T>, dim3(count), dim3(kPanelThreads), panel_lds, st, fn, slot0, u, prec);
                else if (mmax <= kPanelSmallThreads)
                    hipLaunchKernelGGL((k_panel_small<T, 1>), dim3(count), dim3(kPanelSmallThreads), panel_lds, st, fn,
                                       slot0, u, prec);
                else if (mmax <= 2 * kPanelSmallThreads)
                    hipLaunchKernelGGL((k_panel_small<T, 2>), dim3(count), dim3(kPanelSmallThreads), panel_lds, st, fn,
                                       slot0, u, prec);
                else
                    hipLaunchKernelGGL(k_panel<T>, dim3(count), dim3(kPanelThreads), panel_lds, st, fn, slot0, u, prec);
                if (e1) (void)hipEventRecord(e1, st);
                if (tk.nswap)
                    hipLaunchKernelGGL(k_swap_trsm<T>, dim3(tk.nswap), dim3(kThreads), 0, st, fn, slot0, prec, tk.swap,
                                       tk.swap_cols);
                if (tk.ng0) hipLaunchKernelGGL(k_gemm<T>, dim3(tk.ng0), dim3(kThreads), 0, st, fn, slot0, 0, prec, tk.g0);
            }
        }
    }
    if (part == 1) return MF_CHECK_LAUNCH();
    if (ev) (void)hipEventRecord(ev[1], st);
    if (tk.ng1) {
        if (bf16_schur && sizeof(T) == 4)
            hipLaunchKernelGGL(k_gemm_bf16, dim3(tk.ng1), dim3(kThreads), 0, st, fn, slot0, tk.g1);
        else
            hipLaunchKernelGGL(k_gemm<T>, dim3(tk.ng1), dim3(kThreads), 0, st, fn, slot0, 1, prec, tk.g1);
    }
    if (ev) (void)hipEventRecord(ev[2], st);
    hipLaunchKernelGGL(k_finalize<T>, dim3(count), dim3(kThreads), 0, st, S, fn, slot0, prec);
    if (ev) (void)hipEventRecord(ev[3], st);
    return MF_CHECK_LAUNCH();
}

template hipError_t launch_level_factor<double>(const DevSym&, FrontNum*, int, int, int, const int*, const int*,
                                                const double*, int64_t, int64_t, double, int, const LevelTasks&, hipStream_t,
                                                hipEvent_t*, bool, std::vector<hipEvent_t>*, bool, int);
template hipError_t launch_level_factor<float>(const DevSym&, FrontNum*, int, int, int, const int*, const int*,
                                               const double*, int64_t, int64_t, double, int, const LevelTasks&, hipStream_t,
                                               hipEvent_t*, bool, std::vector<hipEvent_t>*, bool, int);

// One right-hand side per pass, or up to kSwRhs of them (nrc, at most kSwRhs).
template <typename T, int NR>
static void level_fwd(const DevSym& S, const FrontNum* fn, int slot0, int count, int prec, const double* b,
                      int64_t ldb, double* vec, int nrhs, int c0, int nrc, int mmax, hipStream_t st,
                      const uint8_t* skip) {
    // levels of small fronts: one wave per front (the diagonal sweep is one wave's work anyway)
    // (and the L21 product in the same one-wave block)
    // (several right-hand sides: four at a time there, which keeps the one-wave
    // blocks at a register count that leaves room for more waves per SIMD)
    if (mmax <= kTriSmallOrder) {
        hipLaunchKernelGGL((k_fwd_tri<T, 64, true, (NR > 4 ? 4 : NR)>), dim3(count), dim3(64),
                           sizeof(double) * (size_t)mmax * nrc, st, S, fn, slot0, prec, b, ldb, vec, nrhs, c0, nrc,
                           skip);
        return;
    }
    hipLaunchKernelGGL((k_fwd_tri<T, kTriThreads, false, NR>), dim3(count), dim3(kTriThreads),
                       sizeof(double) * (size_t)mmax * nrc, st, S, fn, slot0, prec, b, ldb, vec, nrhs, c0, nrc, skip);
    hipLaunchKernelGGL((k_fwd_gemv<T, NR>), dim3((mmax + kGemvRows - 1) / kGemvRows, count), dim3(kThreads),
                       sizeof(double) * (size_t)mmax * nrc, st, fn, slot0, prec, vec, nrhs, c0, nrc, skip);
}
template <typename T, int NR>
static void level_bwd(const FrontNum* fn, int slot0, int count, int prec, double* x, int64_t ldx, const double* vec,
                      int nrhs, int c0, int nrc, int mmax, hipStream_t st, const uint8_t* skip) {
    if (mmax <= kTriSmallOrder) {  // U12 product and sweep in one one-wave block (four columns at a time)
        hipLaunchKernelGGL((k_bwd_tri<T, 64, true, (NR > 4 ? 4 : NR)>), dim3(count), dim3(64),
                           sizeof(double) * (size_t)mmax * nrc, st, fn, slot0, prec, x, ldx, vec, nrhs, c0, nrc, skip);
        return;
    }
    hipLaunchKernelGGL((k_bwd_gemv<T, NR>), dim3((mmax + kGemvRows - 1) / kGemvRows, count), dim3(kThreads),
                       sizeof(double) * (size_t)mmax * nrc, st, fn, slot0, prec, x, ldx, (double*)vec, nrhs, c0, nrc,
                       skip);
    hipLaunchKernelGGL((k_bwd_tri<T, kTriThreads, false, NR>), dim3(count), dim3(kTriThreads),
                       sizeof(double) * (size_t)mmax * nrc, st, fn, slot0, prec, x, ldx, vec, nrhs, c0, nrc, skip);
}

template <typename T>
hipError_t launch_level_fwd(const DevSym& S, const FrontNum* fn, int slot0, int count, int prec, const double* b,
                            int64_t ldb, double* vec, int nrhs, int c0, int nrc, int mmax, hipStream_t st,
                            const uint8_t* skip) {
    if (count <= 0) return hipSuccess;
    if (nrc < 1 || nrc > kSwRhs) return hipErrorInvalidValue;
    if (nrc == 1) level_fwd<T, 1>(S, fn, slot0, count, prec, b, ldb, vec, nrhs, c0, nrc, mmax, st, skip);
    else level_fwd<T, kSwRhs>(S, fn, slot0, count, prec, b, ldb, vec, nrhs, c0, nrc, mmax, st, skip);
    return MF_CHECK_LAUNCH();
}
template <typename T>
hipError_t launch_level_bwd(const FrontNum* fn, int slot0, int count, int prec, double* x, int64_t ldx,
                            const double* vec, int nrhs, int c0, int nrc, int mmax, hipStream_t st,
                            const uint8_t* skip) {
    if (count <= 0) return hipSuccess;
    if (nrc < 1 || nrc > kSwRhs) return hipErrorInvalidValue;
    if (nrc == 1) level_bwd<T, 1>(fn, slot0, count, prec, x, ldx, vec, nrhs, c0, nrc, mmax, st, skip);
    else level_bwd<T, kSwRhs>(fn, slot0, count, prec, x, ldx, vec, nrhs, c0, nrc, mmax, st, skip);
    return MF_CHECK_LAUNCH();
}
template hipError_t launch_level_fwd<double>(const DevSym&, const FrontNum*, int, int, int, const double*, int64_t,
                                             double*, int, int, int, int, hipStream_t, const uint8_t*);
template hipError_t launch_level_fwd<float>(const DevSym&, const FrontNum*, int, int, int, const double*, int64_t,
                                            double*, int, int, int, int, hipStream_t, const uint8_t*);
template hipError_t launch_level_bwd<double>(const FrontNum*, int, int, int, double*, int64_t, const double*, int,
                                             int, int, int, hipStream_t, const uint8_t*);
template hipError_t launch_level_bwd<float>(const FrontNum*, int, int, int, double*, int64_t, const double*, int,
                                            int, int, int, hipStream_t, const uint8_t*);

// ------------------------------------------------------------------ equilibration
// One Ruiz sweep over the CSR values scaled by the current dr, dc: rmax[i] =
// max_j |dr_i a_ij dc_j| (16 lanes per row) and cmax[j] = the same maximum over
// column j (atomic max on the bit patterns of non-negative doubles: exact and
// independent of the order of arrival).
__global__ __launch_bounds__(kThreads) void k_ruiz_max(const int64_t* rp, const int32_t* ci, const double* val,
                                                       int64_t n, const double* dr, const double* dc, double* rmax,
                                                       unsigned long long* cmax) {
    const int64_t row = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 16;
    const int sub = threadIdx.x & 15;
    double mx = 0.0;
    if (row < n) {
        const double di = dr[row];
        for (int64_t t = rp[row] + sub; t < rp[row + 1]; t += 16) {
            const int j = ci[t];
            const double a = fabs(di * val[t] * dc[j]);
            mx = fmax(mx, a);
            // a plain read first: any value it returns is at most the column's
            // current maximum, so the atomic is skipped only where it could not
            // raise it (most entries, once a column's large entries have landed)
            const unsigned long long ab = (unsigned long long)__double_as_longlong(a);
            if (ab > cmax[j]) atomicMax(cmax + j, ab);
        }
    }
    for (int off = 8; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 16));
    if (row < n && sub == 0) rmax[row] = mx;
}

// Nearest power of two to 1/sqrt(x) for x > 0 (1 otherwise): the scaled values are
// then exact multiples of the originals.
__device__ __forceinline__ double ruiz_factor(double x) {
    if (!(x > 0.0) || !(x <= DBL_MAX)) return 1.0;
    return ldexp(1.0, -(int)rint(0.5 * log2(x)));
}

__global__ __launch_bounds__(kThreads) void k_ruiz_update(int64_t n, double* dr, double* dc, const double* rmax,
                                                          const unsigned long long* cmax) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        dr[i] *= ruiz_factor(rmax[i]);
        dc[i] *= ruiz_factor(__longlong_as_double((long long)cmax[i]));
    }
}

// out = Dr A Dc, entrywise over the CSR (exact: the factors are powers of two).
__global__ __launch_bounds__(kThreads) void k_ruiz_apply(const int64_t* rp, const int32_t* ci, const double* val,
                                                         int64_t n, const double* dr, const double* dc, double* out) {
    const int64_t row = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 16;
    const int sub = threadIdx.x & 15;
    if (row >= n) return;
    const double di = dr[row];
    for (int64_t t = rp[row] + sub; t < rp[row + 1]; t += 16) out[t] = di * val[t] * dc[ci[t]];
}

// y[:, c] = d .* x[:, c] for nrhs columns (y may alias x).
__global__ __launch_bounds__(kThreads) void k_diag_scale(int64_t n, const double* d, const double* x, int64_t ldx,
                                                         double* y, int64_t ldy) {
    const int c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        y[i + c * ldy] = d[i] * x[i + c * ldx];
}

hipError_t launch_ruiz(const DevSym& S, const double* val, int64_t n, int sweeps, double* dr, double* dc,
                       double* rmax, unsigned long long* cmax, double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned vb = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
    const unsigned rb = (unsigned)((n * 16 + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_fill, dim3(vb), dim3(kThreads), 0, st, dr, 1.0, n);
    hipLaunchKernelGGL(k_fill, dim3(vb), dim3(kThreads), 0, st, dc, 1.0, n);
    for (int t = 0; t < sweeps; t++) {
        hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, cmax, (int)n, 0ull);
        hipLaunchKernelGGL(k_ruiz_max, dim3(rb), dim3(kThreads), 0, st, S.csr_rowptr, S.csr_colind, val, n, dr, dc,
                           rmax, cmax);
        hipLaunchKernelGGL(k_ruiz_update, dim3(vb), dim3(kThreads), 0, st, n, dr, dc, rmax, cmax);
    }
    hipLaunchKernelGGL(k_ruiz_apply, dim3(rb), dim3(kThreads), 0, st, S.csr_rowptr, S.csr_colind, val, n, dr, dc, out);
    return MF_CHECK_LAUNCH();
}

hipError_t launch_diag_scale(int64_t n, const double* d, const double* x, int64_t ldx, double* y, int64_t ldy,
                             int nrhs, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const unsigned vb = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_diag_scale, dim3(vb, nrhs), dim3(kThreads), 0, st, n, d, x, ldx, y, ldy);
    return MF_CHECK_LAUNCH();
}

// doubles of residual scratch (per-block maxima) for n rows and nrhs columns
size_t residual_part_size(int64_t n, int nrhs) {
    return (size_t)std::max<int64_t>((n + kResRows - 1) / kResRows, 1) * nrhs * kResQ;
}
hipError_t launch_residual(const DevSym& S, const double* val, int64_t n, const double* x, int64_t ldx,
                           const double* b, int64_t ldb, double* r, int64_t ldr, int nrhs,
                           unsigned long long* omega_bits, double* part, hipStream_t st) {
    // omega_bits holds kResQ blocks of nrhs * nseg entries (see k_residual)
    const int nom = nrhs * S.nseg;
    hipLaunchKernelGGL(k_fill_u64, dim3((kResQ * nom + 63) / 64), dim3(64), 0, st, omega_bits, kResQ * nom, 0ull);
    if (n > 0) {
        const int64_t blocks = (n + kResRows - 1) / kResRows;
        hipLaunchKernelGGL(k_residual, dim3((unsigned)blocks, nrhs), dim3(kThreads), 0, st, S.csr_rowptr,
                           S.csr_colind, val, n, x, ldx, b, ldb, r, ldr, omega_bits, (int64_t)nom, S.row_seg, nrhs,
                           part);
        hipLaunchKernelGGL(k_residual_fold, dim3((unsigned)S.nseg, nrhs), dim3(kThreads), 0, st, part, (int)blocks,
                           S.seg_row0, S.seg_n, nrhs, omega_bits, (int64_t)nom);
    }
    return MF_CHECK_LAUNCH();
}

hipError_t launch_axpy(const DevSym& S, int64_t n, double* x, int64_t ldx, const double* d, int64_t ldd,
                       const int32_t* active, int nrhs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_axpy, dim3(blocks, nrhs), dim3(kThreads), 0, st, n, x, ldx, d, ldd, active, S.row_seg, nrhs);
    return MF_CHECK_LAUNCH();
}

}  // namespace mf
