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
#include <cmath>

#include "mf_device.h"

namespace mf {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kGatherCols = 16;   // columns per gather work-group
constexpr int kTile = 64;         // GEMM tile (rows and columns)
constexpr int kKC = 32;           // GEMM K chunk staged through LDS
constexpr int kLdsPad = kTile + 1;

// Position of parent (pre-pivot) row i inside child c's contribution block, or -1.
// dseg: start of c's segment inside the parent's delayed-in block; dout: c's
// delayed-out count; im: c's inverse nominal map (indexed by parent nominal row).
__device__ __forceinline__ int child_pos(int i, int npiv_p, int din_p, int dseg, int dout, const int32_t* im) {
    if (i < npiv_p) {
        int t = im[i];
        return t >= 0 ? dout + t : -1;
    }
    int d = i - npiv_p;
    if (d < din_p) {
        d -= dseg;
        return (d >= 0 && d < dout) ? d : -1;
    }
    int t = im[i - din_p];
    return t >= 0 ? dout + t : -1;
}

__device__ __forceinline__ double load_front(const FrontNum& d, int64_t idx) {
    return d.prec ? (double)((const float*)d.F)[idx] : ((const double*)d.F)[idx];
}

// ------------------------------------------------------------------ assembly
// Owner-computes extend-add: every entry of the front is written exactly once,
// as the sum over children (in child order) of the matching CB entries.  Block
// (x: column tile, y: front).  Also resets the front's pivot bookkeeping.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(DevSym S, FrontNum* fn, int slot0, int want_prec) {
    const int s = slot0 + blockIdx.y;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m;
    const int j0 = blockIdx.x * kGatherCols;
    if (j0 >= m) return;
    T* F = (T*)d.F;
    if (blockIdx.x == 0) {
        int32_t* colperm = iv_colperm(d.iv, d.P, m);
        int32_t* rowperm = iv_rowperm(d.iv, d.P, m);
        for (int i = threadIdx.x; i < d.P; i += kThreads) {
            colperm[i] = i;
            rowperm[i] = i;
        }
    }
    const int cb = S.child_ptr[s], ce = S.child_ptr[s + 1];
    for (int i = threadIdx.x; i < m; i += kThreads) {
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
            if (ci >= 0) {
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
    T* F = (T*)d.F;
    const int64_t idx = r + (int64_t)c * d.m;
    F[idx] = (T)((double)F[idx] + v);
}

// ------------------------------------------------------------------ panel
// Threshold partial pivoting on the window of fully summed columns
// [t*NB, min(P, (t+1)*NB)).  Column q is accepted when its largest fully summed
// entry (rows [k, P)) is at least u times its largest entry over all remaining
// rows [k, m); otherwise it stays behind (delayed) and later pivots keep
// updating it.  Accepted pivots are swapped to position k (column swap over the
// whole front, row swap over the panel's columns).  The row swaps of the panel
// are summarised as (destination, source) pairs for the other columns.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_panel(FrontNum* fn, int slot0, int t, int NB, double u,
                                                    int want_prec) {
    extern __shared__ char smem[];
    __shared__ double red_a[kThreads / 64], red_f[kThreads / 64];
    __shared__ int red_i[kThreads / 64];
    __shared__ int npairs_s;
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P;
    const int wstart = t * NB;
    if (wstart >= P) return;
    const int wend = min(P, wstart + NB);
    T* F = (T*)d.F;
    T* urow = (T*)smem;                                        // pivot row segment, P entries
    int* lmap = (int*)(smem + sizeof(T) * (size_t)P);         // row position -> source, P entries
    int32_t* rowpiv = iv_rowpiv(d.iv, P, m);
    int32_t* colperm = iv_colperm(d.iv, P, m);
    int32_t* rowperm = iv_rowperm(d.iv, P, m);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int kd = d.k;
    const int kd0 = kd;
    for (int q = wstart; q < wend; q++) {
        const T* col = F + (int64_t)q * m;
        double aall = 0.0, afs = -1.0;
        int ifs = INT_MAX;
        for (int i = kd + tid; i < m; i += kThreads) {
            const double a = fabs((double)col[i]);
            if (!(a <= aall)) aall = (a != a) ? INFINITY : a;
            if (i < P && a > afs) {
                afs = a;
                ifs = i;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double oa = __shfl_xor(aall, off);
            aall = fmax(aall, oa);
            const double of = __shfl_xor(afs, off);
            const int oi = __shfl_xor(ifs, off);
            if (of > afs || (of == afs && oi < ifs)) {
                afs = of;
                ifs = oi;
            }
        }
        if (lane == 0) {
            red_a[wid] = aall;
            red_f[wid] = afs;
            red_i[wid] = ifs;
        }
        __syncthreads();
        aall = red_a[0];
        afs = red_f[0];
        ifs = red_i[0];
#pragma unroll
        for (int w = 1; w < kThreads / 64; w++) {
            aall = fmax(aall, red_a[w]);
            if (red_f[w] > afs || (red_f[w] == afs && red_i[w] < ifs)) {
                afs = red_f[w];
                ifs = red_i[w];
            }
        }
        __syncthreads();
        const bool accept = (afs > 0.0) && (afs <= DBL_MAX) && (afs >= u * aall);
        if (!accept) continue;  // uniform: column q stays behind as a delayed column
        const int r = ifs;
        if (q != kd)
            for (int i = tid; i < m; i += kThreads) {
                const T a = F[i + (int64_t)q * m];
                F[i + (int64_t)q * m] = F[i + (int64_t)kd * m];
                F[i + (int64_t)kd * m] = a;
            }
        if (tid == 0) {
            rowpiv[kd] = r;
            const int cq = colperm[q];
            colperm[q] = colperm[kd];
            colperm[kd] = cq;
            const int rr = rowperm[r];
            rowperm[r] = rowperm[kd];
            rowperm[kd] = rr;
        }
        __syncthreads();
        if (r != kd)
            for (int j = kd0 + tid; j < wend; j += kThreads) {
                const T a = F[r + (int64_t)j * m];
                F[r + (int64_t)j * m] = F[kd + (int64_t)j * m];
                F[kd + (int64_t)j * m] = a;
            }
        __syncthreads();
        for (int j = kd + 1 + tid; j < wend; j += kThreads) urow[j] = F[kd + (int64_t)j * m];
        __syncthreads();
        const T piv = F[kd + (int64_t)kd * m];
        for (int i = kd + 1 + tid; i < m; i += kThreads) {
            const T l = F[i + (int64_t)kd * m] / piv;
            F[i + (int64_t)kd * m] = l;
            for (int j = kd + 1; j < wend; j++) F[i + (int64_t)j * m] -= l * urow[j];
        }
        kd++;
        __syncthreads();
    }
    // composite row permutation of this panel on rows [kd0, P): (dest, source) pairs
    for (int i = kd0 + tid; i < P; i += kThreads) lmap[i] = i;
    if (tid == 0) npairs_s = 0;
    __syncthreads();
    if (tid == 0)
        for (int qq = kd0; qq < kd; qq++) {
            const int r = rowpiv[qq];
            const int a = lmap[qq];
            lmap[qq] = lmap[r];
            lmap[r] = a;
        }
    __syncthreads();
    int32_t* pairs = iv_pairs(d.iv, P, m);
    for (int i = kd0 + tid; i < P; i += kThreads) {
        const int src = lmap[i];
        if (src != i) {
            const int slot = atomicAdd(&npairs_s, 1);
            pairs[1 + 2 * slot] = i;
            pairs[2 + 2 * slot] = src;
        }
    }
    __syncthreads();
    if (tid == 0) {
        pairs[0] = npairs_s;
        fn[s].k = kd;
        fn[s].k0 = kd0;
    }
}

// Row swaps of the panel on every column outside the panel, then U12 rows of
// the new pivots (unit-lower triangular solve with L11) for columns >= wend.
// Block (x: 64-column tile, y: front); one wave per column at a time.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_swap_trsm(FrontNum* fn, int slot0, int t, int NB, int want_prec) {
    __shared__ T L11[kNBMax * kNBMax];
    const int s = slot0 + blockIdx.y;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P;
    const int wstart = t * NB;
    if (wstart >= P) return;
    const int wend = min(P, wstart + NB);
    const int kd0 = d.k0, kd1 = d.k, nb = kd1 - kd0;
    if (nb <= 0) return;
    const int c0 = blockIdx.x * kTile;
    if (c0 >= m) return;
    T* F = (T*)d.F;
    const int32_t* pairs = iv_pairs(d.iv, P, m);
    const int np = pairs[0];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int idx = tid; idx < nb * nb; idx += kThreads) {
        const int a = idx % nb, b = idx / nb;
        L11[a + b * kNBMax] = F[(kd0 + a) + (int64_t)(kd0 + b) * m];
    }
    const int d0 = lane < np ? pairs[1 + 2 * lane] : 0, s0 = lane < np ? pairs[2 + 2 * lane] : 0;
    const int d1 = lane + 64 < np ? pairs[1 + 2 * (lane + 64)] : 0,
              s1 = lane + 64 < np ? pairs[2 + 2 * (lane + 64)] : 0;
    for (int cc = wid; cc < kTile; cc += kThreads / 64) {
        const int j = c0 + cc;
        if (j >= m) break;
        if (j >= kd0 && j < wend) continue;
        T* colp = F + (int64_t)j * m;
        const T v0 = lane < np ? colp[s0] : T(0);
        const T v1 = lane + 64 < np ? colp[s1] : T(0);
        if (lane < np) colp[d0] = v0;
        if (lane + 64 < np) colp[d1] = v1;
    }
    __syncthreads();
    for (int cc = wid; cc < kTile; cc += kThreads / 64) {
        const int j = c0 + cc;
        if (j >= m) break;
        if (j < wend) continue;
        T* colp = F + (int64_t)j * m + kd0;
        double x = lane < nb ? (double)colp[lane] : 0.0;
        for (int a = 0; a < nb - 1; a++) {
            const double xa = __shfl(x, a);
            if (lane > a && lane < nb) x -= (double)L11[lane + a * kNBMax] * xa;
        }
        if (lane < nb) colp[lane] = (T)x;
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
// mode 0 (eager, after panel t): rows [k, m) x cols [wend, m) except the deferred
//        block rows >= P and cols >= P; K = the panel's pivots [k0, k).
// mode 1 (Schur): rows [P, m) x cols [P, m); K = all pivots [0, k).
// Block (x: column tile, y: row tile, z: front).  4 waves, each a 32x32 quarter
// made of 2x2 MFMA 16x16 blocks; K staged through LDS in chunks of 32.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gemm(FrontNum* fn, int slot0, int t, int NB, int mode,
                                                   int want_prec) {
    // A and B chunks, then (aliased) the C tile for the transposed epilogue
    __shared__ T smem_ab[2 * kKC * kLdsPad];
    static_assert(2 * kKC * kLdsPad >= kTile * kLdsPad, "C tile must fit in the A/B buffer");
    T* As = smem_ab;
    T* Bs = smem_ab + kKC * kLdsPad;
    T* Cs = smem_ab;
    const int s = slot0 + blockIdx.z;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P;
    int rlo, clo, ka, kb;
    if (mode == 0) {
        const int wstart = t * NB;
        if (wstart >= P) return;
        const int wend = min(P, wstart + NB);
        rlo = d.k;
        clo = wend;
        ka = d.k0;
        kb = d.k;
    } else {
        rlo = P;
        clo = P;
        ka = 0;
        kb = d.k;
    }
    if (kb <= ka) return;
    const int col0 = clo + blockIdx.x * kTile;
    const int row0 = (mode == 0 ? 0 : P) + blockIdx.y * kTile;
    if (col0 >= m || row0 >= m || row0 + kTile <= rlo) return;
    if (mode == 0 && row0 >= P && col0 >= P) return;
    const T* F = (const T*)d.F;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wi = wid & 1, wj = wid >> 1;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = acc_t{0, 0, 0, 0};
    for (int k0 = ka; k0 < kb; k0 += kKC) {
        const int kc = min(kKC, kb - k0);
        for (int idx = tid; idx < kKC * kTile; idx += kThreads) {
            const int r = idx % kTile, a = idx / kTile;
            const int row = row0 + r;
            As[a * kLdsPad + r] = (a < kc && row < m) ? F[row + (int64_t)(k0 + a) * m] : T(0);
        }
        for (int idx = tid; idx < kKC * kTile; idx += kThreads) {
            const int a = idx % kKC, c = idx / kKC;
            const int col = col0 + c;
            Bs[a * kLdsPad + c] = (a < kc && col < m) ? F[(k0 + a) + (int64_t)col * m] : T(0);
        }
        __syncthreads();
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
    T* Fw = (T*)d.F;
    for (int idx = tid; idx < kTile * kTile; idx += kThreads) {
        const int i = idx % kTile, j = idx / kTile;
        const int row = row0 + i, col = col0 + j;
        if (row < rlo || row >= m || col >= m) continue;
        if (mode == 0 && row >= P && col >= P) continue;
        Fw[row + (int64_t)col * m] -= Cs[j * kLdsPad + i];
    }
}

// Post-factorization bookkeeping: column variables in final order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_finalize(DevSym S, FrontNum* fn, int slot0, int want_prec) {
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P;
    const int32_t* rows = S.rows + S.rows_ptr[s];
    const int32_t* colperm = iv_colperm(d.iv, P, m);
    int32_t* colvar = iv_colvar(d.iv, P, m);
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
                    v = iv_colvar(dc.iv, dc.P, dc.m)[dc.k + off];
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
// Forward sweep of one level: z = rows of (b + children's CB vectors) in final
// row order; y = L11^{-1} z[0:k]; CB vector = z[k:m] - L21 y.  The front's block
// of `vec` receives [y; CB vector].  One block per front; z lives in LDS.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fwd(DevSym S, const FrontNum* fn, int slot0, int want_prec,
                                                  const double* b, int64_t ldb, double* vec, int nrhs, int c0,
                                                  int nrc) {
    extern __shared__ double zs[];
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P, k = d.k;
    const T* F = (const T*)d.F;
    const int32_t* rowperm = iv_rowperm(d.iv, P, m);
    const int32_t* rows = S.rows + S.rows_ptr[s];
    double* v = vec + d.voff * nrhs;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int cb = S.child_ptr[s], ce = S.child_ptr[s + 1];
    for (int i = tid; i < m; i += kThreads) {
        const int src = i < P ? rowperm[i] : i;
        for (int c = 0; c < nrc; c++)
            zs[i + c * m] = (src < d.npiv) ? b[rows[src] + (int64_t)(c0 + c) * ldb] : 0.0;
        int dseg = 0;
        for (int tt = cb; tt < ce; tt++) {
            const int cs = S.child_slot[tt];
            const FrontNum dc = fn[cs];
            const int dout = dc.P - dc.k;
            const int ci = child_pos(src, d.npiv, d.din, dseg, dout, S.imap + S.imap_off[cs]);
            if (ci >= 0) {
                const double* vc = vec + dc.voff * nrhs;
                for (int c = 0; c < nrc; c++) zs[i + c * m] += vc[dc.k + ci + (int64_t)(c0 + c) * dc.m];
            }
            dseg += dout;
        }
    }
    __syncthreads();
    constexpr int BS = 16;
    for (int j0 = 0; j0 < k; j0 += BS) {
        const int bs = min(BS, k - j0);
        if (wid == 0) {
            for (int c = 0; c < nrc; c++) {
                double x = lane < bs ? zs[j0 + lane + c * m] : 0.0;
#pragma unroll
                for (int a = 0; a < BS - 1; a++) {
                    if (a + 1 >= bs) break;
                    const double xa = __shfl(x, a);
                    if (lane > a && lane < bs) x -= (double)F[(j0 + lane) + (int64_t)(j0 + a) * m] * xa;
                }
                if (lane < bs) zs[j0 + lane + c * m] = x;
            }
        }
        __syncthreads();
        for (int i = j0 + bs + tid; i < m; i += kThreads) {
            for (int c = 0; c < nrc; c++) {
                double acc = zs[i + c * m];
                for (int a = 0; a < bs; a++) acc -= (double)F[i + (int64_t)(j0 + a) * m] * zs[j0 + a + c * m];
                zs[i + c * m] = acc;
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < m; i += kThreads)
        for (int c = 0; c < nrc; c++) v[i + (int64_t)(c0 + c) * m] = zs[i + c * m];
}

// Backward sweep of one level (root first): x_f = U11^{-1} (y - U12 x_cb), where
// x_cb is gathered from x at the front's remaining column variables.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd(const FrontNum* fn, int slot0, int want_prec, double* x,
                                                  int64_t ldx, const double* vec, int nrhs, int c0, int nrc) {
    extern __shared__ double xs[];
    const int s = slot0 + blockIdx.x;
    const FrontNum d = fn[s];
    if (d.prec != want_prec) return;
    const int m = d.m, P = d.P, k = d.k;
    const T* F = (const T*)d.F;
    const int32_t* colvar = iv_colvar(d.iv, P, m);
    const double* v = vec + d.voff * nrhs;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int i = tid; i < m; i += kThreads)
        for (int c = 0; c < nrc; c++)
            xs[i + c * m] = (i < k) ? v[i + (int64_t)(c0 + c) * m]
                                    : (colvar[i] >= 0 ? x[colvar[i] + (int64_t)(c0 + c) * ldx] : 0.0);
    __syncthreads();
    for (int i = tid; i < k; i += kThreads) {
        for (int c = 0; c < nrc; c++) {
            double acc = xs[i + c * m];
            for (int j = k; j < m; j++) acc -= (double)F[i + (int64_t)j * m] * xs[j + c * m];
            xs[i + c * m] = acc;
        }
    }
    __syncthreads();
    constexpr int BS = 16;
    for (int j1 = k; j1 > 0; j1 -= BS) {
        const int j0 = max(0, j1 - BS), bs = j1 - j0;
        if (wid == 0) {
            for (int c = 0; c < nrc; c++) {
                double xl = lane < bs ? xs[j0 + lane + c * m] : 0.0;
                for (int a = bs - 1; a >= 0; a--) {
                    if (lane == a) xl /= (double)F[(j0 + a) + (int64_t)(j0 + a) * m];
                    const double xa = __shfl(xl, a);
                    if (lane < a) xl -= (double)F[(j0 + lane) + (int64_t)(j0 + a) * m] * xa;
                }
                if (lane < bs) xs[j0 + lane + c * m] = xl;
            }
        }
        __syncthreads();
        for (int i = tid; i < j0; i += kThreads) {
            for (int c = 0; c < nrc; c++) {
                double acc = xs[i + c * m];
                for (int a = 0; a < bs; a++) acc -= (double)F[i + (int64_t)(j0 + a) * m] * xs[j0 + a + c * m];
                xs[i + c * m] = acc;
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < k; i += kThreads) {
        const int var = colvar[i];
        if (var < 0) continue;
        for (int c = 0; c < nrc; c++) x[var + (int64_t)(c0 + c) * ldx] = xs[i + c * m];
    }
}

// ------------------------------------------------------------------ residual
// r = b - J x and omega = max_i |r_i| / (|J||x| + |b|)_i per right-hand side
// (blockIdx.y), 16 lanes per row.  omega is accumulated as the bit pattern of a
// non-negative double with an unsigned atomic max.
__global__ __launch_bounds__(kThreads) void k_residual(const int64_t* rp, const int32_t* ci, const double* val,
                                                       int64_t n, const double* x, int64_t ldx, const double* b,
                                                       int64_t ldb, double* r, int64_t ldr,
                                                       unsigned long long* omega_bits) {
    __shared__ double wmax[kThreads / 64];
    const int c = blockIdx.y;
    const int64_t row = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 16;
    const int sub = threadIdx.x & 15;
    double acc = 0.0, den = 0.0;
    if (row < n) {
        const double* xc = x + (int64_t)c * ldx;
        for (int64_t t = rp[row] + sub; t < rp[row + 1]; t += 16) {
            const double a = val[t];
            const double xv = xc[ci[t]];
            acc = fma(a, xv, acc);
            den = fma(fabs(a), fabs(xv), den);
        }
    }
    for (int off = 8; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, 16);
        den += __shfl_xor(den, off, 16);
    }
    double w = 0.0;
    if (row < n && sub == 0) {
        const double bi = b[row + (int64_t)c * ldb];
        const double ri = bi - acc;
        r[row + (int64_t)c * ldr] = ri;
        const double dd = den + fabs(bi);
        w = dd > 0.0 ? fabs(ri) / dd : (ri == 0.0 ? 0.0 : INFINITY);
        if (w != w) w = INFINITY;
    }
    for (int off = 32; off > 0; off >>= 1) w = fmax(w, __shfl_xor(w, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = wmax[0];
        for (int i = 1; i < kThreads / 64; i++) mx = fmax(mx, wmax[i]);
        atomicMax(omega_bits + c, (unsigned long long)__double_as_longlong(mx));
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// x[:, c] += d[:, c]
__global__ __launch_bounds__(kThreads) void k_axpy(int64_t n, double* x, int64_t ldx, const double* dvec,
                                                   int64_t ldd) {
    const int c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        x[i + c * ldx] += dvec[i + c * ldd];
}

// Column copy y[:, c] = x[:, c]
__global__ __launch_bounds__(kThreads) void k_copy(int64_t n, const double* x, int64_t ldx, double* y,
                                                   int64_t ldy) {
    const int c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        y[i + c * ldy] = x[i + c * ldx];
}

// ------------------------------------------------------------------ launchers
#define MF_CHECK_LAUNCH() (hipGetLastError())

template <typename T>
hipError_t launch_level_factor(const DevSym& S, FrontNum* fn, int slot0, int count, int mmax, int Pmax,
                               const double* vals, int64_t u0, int64_t u1, int NB, double u, int prec,
                               hipStream_t st, hipEvent_t* ev) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather<T>, dim3((mmax + kGatherCols - 1) / kGatherCols, count), dim3(kThreads), 0, st, S,
                       fn, slot0, prec);
    if (u1 > u0)
        hipLaunchKernelGGL(k_scatter<T>, dim3((unsigned)((u1 - u0 + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                           st, S, fn, vals, u0, u1, prec);
    if (ev) (void)hipEventRecord(ev[0], st);
    const int npan = (Pmax + NB - 1) / NB;
    const size_t panel_lds = (sizeof(T) + sizeof(int)) * (size_t)Pmax;
    const int tiles = (mmax + kTile - 1) / kTile;
    for (int t = 0; t < npan; t++) {
        hipLaunchKernelGGL(k_panel<T>, dim3(count), dim3(kThreads), panel_lds, st, fn, slot0, t, NB, u, prec);
        hipLaunchKernelGGL(k_swap_trsm<T>, dim3(tiles, count), dim3(kThreads), 0, st, fn, slot0, t, NB, prec);
        hipLaunchKernelGGL(k_gemm<T>, dim3(tiles, tiles, count), dim3(kThreads), 0, st, fn, slot0, t, NB, 0, prec);
    }
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(k_gemm<T>, dim3(tiles, tiles, count), dim3(kThreads), 0, st, fn, slot0, 0, NB, 1, prec);
    if (ev) (void)hipEventRecord(ev[2], st);
    hipLaunchKernelGGL(k_finalize<T>, dim3(count), dim3(kThreads), 0, st, S, fn, slot0, prec);
    if (ev) (void)hipEventRecord(ev[3], st);
    return MF_CHECK_LAUNCH();
}

template hipError_t launch_level_factor<double>(const DevSym&, FrontNum*, int, int, int, int, const double*,
                                                int64_t, int64_t, int, double, int, hipStream_t, hipEvent_t*);
template hipError_t launch_level_factor<float>(const DevSym&, FrontNum*, int, int, int, int, const double*,
                                               int64_t, int64_t, int, double, int, hipStream_t, hipEvent_t*);

template <typename T>
hipError_t launch_level_fwd(const DevSym& S, const FrontNum* fn, int slot0, int count, int prec, const double* b,
                            int64_t ldb, double* vec, int nrhs, int c0, int nrc, int mmax, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd<T>, dim3(count), dim3(kThreads), sizeof(double) * (size_t)mmax * nrc, st, S, fn, slot0,
                       prec, b, ldb, vec, nrhs, c0, nrc);
    return MF_CHECK_LAUNCH();
}
template <typename T>
hipError_t launch_level_bwd(const FrontNum* fn, int slot0, int count, int prec, double* x, int64_t ldx,
                            const double* vec, int nrhs, int c0, int nrc, int mmax, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd<T>, dim3(count), dim3(kThreads), sizeof(double) * (size_t)mmax * nrc, st, fn, slot0,
                       prec, x, ldx, vec, nrhs, c0, nrc);
    return MF_CHECK_LAUNCH();
}
template hipError_t launch_level_fwd<double>(const DevSym&, const FrontNum*, int, int, int, const double*, int64_t,
                                             double*, int, int, int, int, hipStream_t);
template hipError_t launch_level_fwd<float>(const DevSym&, const FrontNum*, int, int, int, const double*, int64_t,
                                            double*, int, int, int, int, hipStream_t);
template hipError_t launch_level_bwd<double>(const FrontNum*, int, int, int, double*, int64_t, const double*, int,
                                             int, int, int, hipStream_t);
template hipError_t launch_level_bwd<float>(const FrontNum*, int, int, int, double*, int64_t, const double*, int,
                                            int, int, int, hipStream_t);

hipError_t launch_residual(const DevSym& S, const double* val, int64_t n, const double* x, int64_t ldx,
                           const double* b, int64_t ldb, double* r, int64_t ldr, int nrhs,
                           unsigned long long* omega_bits, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3((nrhs + 63) / 64), dim3(64), 0, st, omega_bits, nrhs, 0ull);
    if (n > 0) {
        const int64_t blocks = (n * 16 + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_residual, dim3((unsigned)blocks, nrhs), dim3(kThreads), 0, st, S.csr_rowptr,
                           S.csr_colind, val, n, x, ldx, b, ldb, r, ldr, omega_bits);
    }
    return MF_CHECK_LAUNCH();
}

hipError_t launch_axpy(int64_t n, double* x, int64_t ldx, const double* d, int64_t ldd, int nrhs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_axpy, dim3(blocks, nrhs), dim3(kThreads), 0, st, n, x, ldx, d, ldd);
    return MF_CHECK_LAUNCH();
}

hipError_t launch_copy(int64_t n, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_copy, dim3(blocks, nrhs), dim3(kThreads), 0, st, n, x, ldx, y, ldy);
    return MF_CHECK_LAUNCH();
}

}  // namespace mf
