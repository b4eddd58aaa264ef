// Device-side data layout shared by the kernels and the numeric driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mf {

// Panel width upper bound (options.panel_nb is clamped to it).
constexpr int kNBMax = 32;
// Largest front order: the tile work lists keep 64-row tile indices in 6 bits.
constexpr int kMaxFrontOrder = 4096;
// Most fronts in one tree level: the extend-add task code keeps the front in 16 bits.
constexpr int kMaxLevelFronts = 65535;

// Panel shape class of a front, from its order and precision: the window width
// NB and rows per thread RS (of a 512-thread block) are per front (never per
// launch), so a front's arithmetic does not depend on the other fronts it is
// batched with.  The widths are the widest windows whose registers fit without
// spilling in the kernel that holds all classes.
//   class 0: m <= 512  (NB 32, RS 1)     class 1: m <= 1024 (NB 32, RS 2)
//   class 2: m <= 1536 (FP64 NB 26, FP32 NB 32; RS 3)
//   class 3: m <= 2048 (FP64 NB 20, FP32 NB 32; RS 4)
//   class 4: m <= 4096 (FP64 NB 8, FP32 NB 16; RS 8)
constexpr int kNClass = 5;
__host__ __device__ inline int front_class(int m) {
    return m <= 512 ? 0 : (m <= 1024 ? 1 : (m <= 1536 ? 2 : (m <= 2048 ? 3 : 4)));
}
__host__ __device__ inline int class_nb(int cls, int prec) {
    if (cls <= 1) return 32;
    if (cls == 2) return prec ? 32 : 26;
    if (cls == 3) return prec ? 32 : 20;
    return prec ? 16 : 8;
}

// Per-front numeric state, indexed by "slot" (fronts in level order, so the
// fronts of one tree level are contiguous).  Written by the host before a level
// is assembled; k / k0 are updated by the factorization kernels.
// FrontNum::prec of a front that the planned schedule skips after a capacity overflow.
constexpr int32_t kSkipPrec = 2;
struct FrontNum {
    void* F;         // dense front, column-major m x m (double or float)
    int32_t* iv;     // rowpiv[P] | colperm[P] | rowperm[P] | colvar[m] | npairs, pairs[4*kNBMax]
    int64_t voff;    // element offset of this front's vector block (times nrhs) in the solve arena
    int32_t m;       // actual order (nominal + delayed-in)
    int32_t P;       // fully summed variables (nominal pivots + delayed-in)
    int32_t din;     // delayed-in count
    int32_t k;       // eliminated so far / in total
    int32_t k0;      // k at the start of the current panel
    int32_t prec;    // 0: double front, 1: float front (kSkipPrec: no kernel takes it)
    int32_t npiv;    // nominal pivots
    int32_t mnom;    // nominal order
    int32_t pcur;    // end of the not-yet-tried fully summed columns [k, pcur); [pcur, P) are delayed
    int32_t x0, x1;  // columns rejected by the last panel (already up to date): skipped by its updates
    int32_t pad_;
    void* W;         // panel scratch (2 m NB entries): staging of the column commit
};

// Per-level work lists of the tiled factorization kernels, built on the host
// once a level's front orders are known (one block per entry, no idle blocks for
// the small fronts of a level).  Entry = (slot - first slot of the level) << 12 |
// tile_a << 6 | tile_b, tiles of 64 (front orders are at most 4096).
struct LevelTasks {
    const int32_t* swap;  // (front, column tile of swap_cols) over [0, m); tile index in the low 12 bits
    int32_t nswap;
    int32_t swap_cols;    // 64, or 16 on levels of few fronts
    const int32_t* g0;    // (front, row tile, column tile) over [0, m)^2 minus the block >= P x >= P
    int32_t ng0;
    const int32_t* g1;    // (front, row tile, column tile) over the contribution block [P, m)^2
    int32_t ng1;
    const int32_t* gather;  // (front, group size, first column tile): see gather_task
    int32_t ngather;
};
__host__ __device__ inline int32_t task_code(int rel, int a, int b) { return (rel << 12) | (a << 6) | b; }

// Extend-add tasks: kGatherCols-column tiles (16), 1 << lg of them per block;
// tile index below 512 (orders up to 8192), lg in {0, 1, 2}.  Fronts with many
// children can also split their rows into chunks of kGatherChunkRows (one task
// per tile and chunk), so that no single block walks all rows past every child.
// Bits: tile 0-8, lg 9-10, chunked 11, chunk 12-15, front 16-31 (unsigned).
constexpr int kGatherTileCols = 16;
constexpr int kGatherChunkRows = 256;
constexpr int kGatherChunkKids = 8;  // fronts with more children than this are split by rows
__host__ __device__ inline int gather_lg(int m) { return m <= 64 ? 2 : (m <= 128 ? 1 : 0); }
__host__ __device__ inline int32_t gather_task(int rel, int lg, int tile, int chunk = -1) {
    const uint32_t c = chunk < 0 ? 0u : ((1u | ((uint32_t)chunk << 1)) << 11);
    return (int32_t)(((uint32_t)rel << 16) | c | ((uint32_t)lg << 9) | (uint32_t)tile);
}
__host__ __device__ inline int gather_task_rel(int32_t code) { return (int)((uint32_t)code >> 16); }
__host__ __device__ inline int gather_task_lg(int32_t code) { return (code >> 9) & 3; }
__host__ __device__ inline int gather_task_tile(int32_t code) { return code & 511; }
__host__ __device__ inline int gather_task_chunk(int32_t code) { return ((code >> 11) & 1) ? ((code >> 12) & 15) : -1; }

// Quantities of one residual pass, per (system, right-hand side): the
// componentwise backward error omega, then max |r_i|, max |x_i|, max |b_i| and
// the largest row sum of |J| (the pieces of the normwise backward error eta).
constexpr int kResQ = 5;

// Pattern data (slot-indexed), uploaded once per symbolic handle.
struct DevSym {
    int32_t nslots;
    const int32_t* parent;       // parent slot or -1
    const int32_t* child_ptr;    // nslots+1
    const int32_t* child_slot;   // children (slots) in increasing front order
    const int64_t* rows_ptr;     // nslots+1, into rows (slot order)
    const int32_t* rows;         // nominal front rows (original vars)
    const int64_t* imap_off;     // per child slot: offset of its inverse map (length mnom[parent])
    const int32_t* imap;
    const int32_t* ue_slot;      // unique original entries
    const int32_t* ue_row;
    const int32_t* ue_col;
    const int64_t* ue_src_ptr;
    const int32_t* ue_src;
    const int64_t* csr_rowptr;   // the matrix pattern (for residuals)
    const int32_t* csr_colind;
    int32_t nseg;                // systems (segments) in a batch; 1 for a single system
    const int32_t* row_seg;      // row -> segment (nullptr when nseg == 1)
    const int64_t* seg_row0;     // nseg: first row of each segment
    const int64_t* seg_n;        // nseg: rows of each segment
};

// One block of a segmented copy: out[dst + i] = src[i] + add for i < count.
struct SegCopy {
    const void* src;
    int64_t dst, count, add;
};
// One segment of a scatter out of a single array: count entries from in[src..]
// to dst.
struct SegOut {
    void* dst;
    int64_t src, count;
};

// Persistent sweeps (k_fwd_persist / k_bwd_persist): one launch per direction
// runs every front of every system from a ticket-ordered list of tasks.  Fronts
// of order <= kSwWhole are one task; larger fronts split into 64-row blocks of
// the fully summed part (forward and backward) and 64-row tiles of the
// contribution rows (forward).  Task = (slot, kind << 8 | block).
constexpr int kSwWhole = 256;
constexpr int kSwRhs = 8;       // right-hand sides per sweep launch
constexpr int kSwBundle = 8;    // consecutive whole-front tasks taken with one ticket
constexpr int kSwTopFronts = 64;  // levels with at most this many fronts (and all above) run persistently
constexpr int kSwListedMinOrder = 1024;  // ... in systems whose largest front has at least this order
enum SweepKind { kSwKindWhole = 0, kSwKindFs = 1, kSwKindCb = 2 };
__host__ __device__ inline int32_t sweep_code(int kind, int blk) { return (kind << 8) | blk; }
__host__ __device__ inline int sweep_kind(int32_t code) { return code >> 8; }
__host__ __device__ inline int sweep_blk(int32_t code) { return code & 255; }

__host__ __device__ inline int32_t* iv_rowpiv(int32_t* iv, int P, int m) { (void)m; return iv; }
__host__ __device__ inline int32_t* iv_colperm(int32_t* iv, int P, int m) { (void)m; return iv + P; }
__host__ __device__ inline int32_t* iv_rowperm(int32_t* iv, int P, int m) { (void)m; return iv + 2 * P; }
__host__ __device__ inline int32_t* iv_colvar(int32_t* iv, int P, int m) { return iv + 3 * P; }
// panel area: npairs, pairs[2 * 2 * kNBMax] | w, nmove, col_dst[kNBMax], mv_src[kNBMax], mv_dst[kNBMax]
__host__ __device__ inline int32_t* iv_pairs(int32_t* iv, int P, int m) { return iv + 3 * P + m; }
__host__ __device__ inline int32_t* iv_commit(int32_t* iv, int P, int m) { return iv + 3 * P + m + 1 + 4 * kNBMax; }
__host__ __device__ inline int64_t iv_size(int P, int m) { return 3 * (int64_t)P + m + 1 + 4 * kNBMax + 2 + 3 * kNBMax; }

}  // namespace mf
