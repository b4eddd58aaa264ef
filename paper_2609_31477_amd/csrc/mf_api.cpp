// C ABI of libmf: handles, the level-synchronous numeric driver and the
// refinement loop.  All device work is issued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <unordered_map>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "mf_device.h"
#include "mf_internal.h"
#include "mf_tasks.h"

namespace mf {

// kernel launchers (mf_kernels.hip)
// ev (nullable): 4 events recorded after assembly, panels, Schur GEMM and finalize;
// part 1: through the panel rounds, part 2: Schur GEMM and finalize, 0: all
template <typename T>
hipError_t launch_level_factor(const DevSym& S, FrontNum* fn, int slot0, int count, int mmax, const int* cls_mmax,
                               const int* cls_Pmax, const double* vals, int64_t u0, int64_t u1, double u, int prec,
                               const LevelTasks& tk, hipStream_t st, hipEvent_t* ev, bool bf16_schur,
                               std::vector<hipEvent_t>* pev, bool panel_full = false, int part = 0);
template <typename T>
hipError_t launch_level_fwd(const DevSym& S, const FrontNum* fn, int slot0, int count, int prec, const double* b,
                            int64_t ldb, double* vec, int nrhs, int c0, int nrc, int mmax, hipStream_t st,
                            const uint8_t* skip = nullptr);
template <typename T>
hipError_t launch_level_bwd(const FrontNum* fn, int slot0, int count, int prec, double* x, int64_t ldx,
                            const double* vec, int nrhs, int c0, int nrc, int mmax, hipStream_t st,
                            const uint8_t* skip = nullptr);
int panel_nb(int prec, int mmax);
hipError_t launch_spmv(const DevSym& S, const double* val, int64_t n, const double* x, int64_t ldx, double* y,
                       int64_t ldy, int ncol, hipStream_t st);
hipError_t launch_mdot(const DevSym& S, const double* V, int64_t ldv, int nv, const double* w, double* part,
                       double* out, int ostride, hipStream_t st);
hipError_t launch_vsub(const DevSym& S, double* w, const double* V, int64_t ldv, int nv, const double* h, int hstride,
                       int64_t n, hipStream_t st);
hipError_t launch_vadd(const DevSym& S, double* x, const double* V, int64_t ldv, int nv, const double* c,
                       int cstride, int64_t n, hipStream_t st);
hipError_t launch_scale(const DevSym& S, double* y, const double* x, const double* a, int astride, int64_t n,
                        hipStream_t st);
hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t st);
hipError_t launch_fill_i32(int32_t* y, int32_t v, hipStream_t st);
template <typename T>
hipError_t launch_seg_copy(const SegCopy* segs, const int64_t* start, int nseg, int64_t total, T* out,
                           hipStream_t st);
template <typename T>
hipError_t launch_seg_scatter(const SegOut* segs, const int64_t* start, int nseg, int64_t total, const T* in,
                              hipStream_t st);
hipError_t launch_nonfinite(const double* v, int64_t nnz, unsigned long long* first, hipStream_t st);
hipError_t launch_level_setup(const DevSym& S, FrontNum* fn, const FrontNum* tmpl, int slot0, int count, int level,
                              int32_t* overflow, hipStream_t st);
hipError_t launch_residual(const DevSym& S, const double* val, int64_t n, const double* x, int64_t ldx,
                           const double* b, int64_t ldb, double* r, int64_t ldr, int nrhs,
                           unsigned long long* omega_bits, double* part, hipStream_t st);
size_t residual_part_size(int64_t n, int nrhs);
hipError_t launch_sweep_persist(bool forward, const DevSym& S, const FrontNum* fn, const int32_t* tasks,
                                const int32_t* bptr, int nbund, const int32_t* ntask, const int32_t* need,
                                int32_t* ctr,
                                const double* b, int64_t ldb, double* x, int64_t ldx, double* vec, int nrhs, int c0,
                                int nrc, int grid, int cap, hipStream_t st);
hipError_t launch_axpy(const DevSym& S, int64_t n, double* x, int64_t ldx, const double* d, int64_t ldd,
                       const int32_t* active, int nrhs, hipStream_t st);
hipError_t launch_ruiz(const DevSym& S, const double* val, int64_t n, int sweeps, double* dr, double* dc,
                       double* rmax, unsigned long long* cmax, double* out, hipStream_t st);
hipError_t launch_diag_scale(int64_t n, const double* d, const double* x, int64_t ldx, double* y, int64_t ldy,
                             int nrhs, hipStream_t st);

namespace {
thread_local std::string g_err;

struct Fail {
    mf_status st;
    std::string msg;
};

#define HIPX(call)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            throw Fail{e_ == hipErrorOutOfMemory ? MF_ERR_OOM : MF_ERR_DEVICE,                         \
                       std::string(#call) + ": " + hipGetErrorString(e_)};                             \
    } while (0)

// Device and pinned host memory of the library's handles comes from a cache per
// device and goes back to it, not to the runtime: hipFree and hipHostFree
// synchronize the whole device, which would stall every other stream of a
// serving loop whenever one request's handle is released.  A block goes back to
// the cache only when nothing uses it any more: every entry point synchronizes
// its stream before it returns, so a handle's blocks are idle when it is
// released or when one of its calls replaces a buffer.  Sizes are rounded up to
// an eighth of their power of two; when the device runs out, the cached blocks
// are handed back to the runtime and the allocation is tried once more.
// hipFree synchronizes the device, which would invalidate a graph capture that
// another thread has in progress: captures hold this lock shared, and handing
// cached blocks back to the runtime holds it exclusively.
std::shared_mutex g_capture_mu;

class MemCache {
  public:
    hipError_t get(void** p, size_t n, bool host) {
        *p = nullptr;
        int dev = 0;
        if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) return e;
        const size_t b = bin(n);
        {
            // best fit among the idle blocks of at most 1.5 times the request
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(Key{dev, host, b});
            if (it != free_.end() && it->first.dev == dev && it->first.host == host &&
                it->first.bytes <= b + b / 2) {
                *p = it->second;
                idle_[host] -= it->first.bytes;
                live_[*p] = it->first;
                free_.erase(it);
                return hipSuccess;
            }
        }
        hipError_t e = raw_alloc(p, b, host);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            trim(dev, host, 0);
            e = raw_alloc(p, b, host);
        }
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> lk(mu_);
            live_[*p] = Key{dev, host, b};
        }
        return e;
    }
    hipError_t put(void* p) {
        if (!p) return hipSuccess;
        Key k;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = live_.find(p);
            if (it == live_.end()) return hipErrorInvalidValue;
            k = it->second;
            live_.erase(it);
            free_.emplace(k, p);
            idle_[k.host] += k.bytes;
            if (idle_[k.host] <= limit(k.host)) return hipSuccess;
        }
        trim(k.dev, k.host, limit(k.host) / 2);  // rare: too much idle memory kept
        return hipSuccess;
    }

  private:
    struct Key {
        int dev = 0;
        bool host = false;
        size_t bytes = 0;
        bool operator<(const Key& o) const {
            return dev != o.dev ? dev < o.dev : (host != o.host ? host < o.host : bytes < o.bytes);
        }
    };
    static size_t limit(bool host) { return host ? (size_t(1) << 30) : (size_t(16) << 30); }
    static size_t bin(size_t n) {
        n = std::max<size_t>(n, 256);
        int e = 63 - __builtin_clzll(n);
        const size_t step = (size_t)1 << std::max(e - 3, 8);
        return (n + step - 1) / step * step;
    }
    static hipError_t raw_alloc(void** p, size_t b, bool host) {
        return host ? hipHostMalloc(p, b, hipHostMallocDefault) : hipMalloc(p, b);
    }
    // hand idle blocks of one kind back to the runtime, largest first, until at
    // most `keep` bytes stay idle
    void trim(int dev, bool host, size_t keep) {
        std::vector<void*> out;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto it = free_.end(); it != free_.begin() && idle_[host] > keep;) {
                --it;
                if (it->first.dev != dev || it->first.host != host) continue;
                out.push_back(it->second);
                idle_[host] -= it->first.bytes;
                it = free_.erase(it);
            }
        }
        if (out.empty()) return;
        std::unique_lock<std::shared_mutex> nocap(g_capture_mu);
        for (void* q : out) (void)(host ? hipHostFree(q) : hipFree(q));
    }
    std::mutex mu_;
    std::multimap<Key, void*> free_;
    std::unordered_map<void*, Key> live_;
    size_t idle_[2] = {0, 0};
};
MemCache& mem_cache() {
    static MemCache* c = new MemCache();  // lives until the process ends
    return *c;
}
hipError_t dmalloc(void** p, size_t n) { return mem_cache().get(p, n, false); }
hipError_t hmalloc(void** p, size_t n, unsigned) { return mem_cache().get(p, n, true); }
hipError_t dfree(void* p) { return mem_cache().put(p); }
hipError_t hfree(void* p) { return mem_cache().put(p); }

constexpr size_t kMaxLds = 64 * 1024;
constexpr size_t kSweepStaticLds = 36 * 1024;  // static LDS of the sweep kernels, with margin

template <typename V>
void upload(V** dst, const std::vector<V>& src) {
    *dst = nullptr;
    size_t bytes = sizeof(V) * std::max<size_t>(src.size(), 1);
    HIPX(dmalloc((void**)dst, bytes));
    if (!src.empty()) HIPX(hipMemcpy(*dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice));
}

// Device copy of the pattern data, slot-indexed; owned by the symbolic handle.
struct SymDev {
    int device = -1;
    DevSym S{};
    std::vector<void*> allocs;
    std::vector<int32_t> slot_of;  // front id -> slot
    ~SymDev() {
        for (void* p : allocs) (void)dfree(p);
    }
    template <typename V>
    const V* put(const std::vector<V>& v) {
        V* p = nullptr;
        upload(&p, v);
        allocs.push_back(p);
        return p;
    }
    template <typename V>
    V* alloc(size_t n) {
        V* p = nullptr;
        HIPX(dmalloc((void**)&p, sizeof(V) * std::max<size_t>(n, 1)));
        allocs.push_back(p);
        return p;
    }
};

// Bump allocator over a list of device chunks (fronts or integer bookkeeping).
struct Arena {
    std::vector<std::pair<char*, size_t>> chunks;
    size_t ci = 0, off = 0;
    size_t grow_hint = 0;
    void reset() {
        ci = 0;
        off = 0;
    }
    size_t capacity() const {
        size_t c = 0;
        for (auto& k : chunks) c += k.second;
        return c;
    }
    char* alloc(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        while (ci < chunks.size()) {
            if (off + bytes <= chunks[ci].second) {
                char* p = chunks[ci].first + off;
                off += bytes;
                return p;
            }
            ci++;
            off = 0;
        }
        size_t sz = std::max(bytes, grow_hint);
        char* p = nullptr;
        HIPX(dmalloc((void**)&p, sz));
        chunks.emplace_back(p, sz);
        ci = chunks.size() - 1;
        off = bytes;
        return p;
    }
    void release() {
        for (auto& k : chunks) (void)dfree(k.first);
        chunks.clear();
        reset();
    }
};

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace mf

using namespace mf;

struct mf_sym {
    uint32_t magic = kSymMagic;
    Symbolic S;
    mf_options opt;
    std::shared_ptr<SymDev> dev;
    // a light batch: its systems' device pattern data, shared with their handles
    std::vector<std::shared_ptr<SymDev>> parts_dev;
};

struct mf_num {
    uint32_t magic = kNumMagic;
    mf_sym* sym = nullptr;
    mf_options opt;
    int device = -1;
    Arena fronts, ints, wsp;  // fronts, integer bookkeeping, per-level panel scratch
    FrontNum* d_fn = nullptr;
    FrontNum* h_fn = nullptr;  // pinned mirror
    double* d_vals = nullptr;
    int64_t vec_len = 0;       // sum of actual front orders
    double* d_vec = nullptr;
    size_t vec_cap = 0;        // doubles
    double* d_work = nullptr;  // r, d, x0 copies (3 * n * nrhs)
    size_t work_cap = 0;
    double* d_kry = nullptr;   // GMRES basis (n x (m+1)), w, and reduction scratch
    size_t kry_cap = 0;
    double* d_small = nullptr;  // device coefficients (dots, combination weights)
    double* h_small = nullptr;  // pinned mirror
    char* d_seg = nullptr;      // segment lists of the batch gathers and scatters
    char* h_seg = nullptr;      // pinned mirror
    size_t seg_cap = 0;         // bytes
    unsigned long long* d_omega = nullptr;
    double* d_respart = nullptr;            // residual per-block maxima
    size_t respart_cap = 0;
    unsigned long long* h_omega = nullptr;  // pinned
    int32_t* d_active = nullptr;            // per (system, rhs): still refining
    int32_t* h_active = nullptr;            // pinned
    int omega_cap = 0;
    size_t small_cap = 0;
    std::vector<mf_solve_info> seg_info;    // per system of the last solve
    std::vector<int64_t> seg_delayed;       // per system: delayed columns of the last factorization
    // Krylov vectors of several right-hand sides as one segmented vector (krylov_view)
    int kv_nrhs = 0;
    DevSym kv{};
    std::vector<void*> kv_alloc;
    // Persistent sweeps: per direction (0 forward, 1 backward) the ticket-ordered
    // task list of the current factors, built at the first solve after a factorization.
    struct SweepPlan {
        bool valid = false;
        int32_t* d_buf = nullptr;  // tasks | bundle pointers | per-slot task counts, both directions
        const int32_t* tasks[2] = {nullptr, nullptr};
        const int32_t* bptr[2] = {nullptr, nullptr};
        const int32_t* ntask[2] = {nullptr, nullptr};
        const int32_t* need = nullptr;  // forward: children of each slot inside the lists
        const uint8_t* d_listed = nullptr;  // per slot: run by the lists (skipped by the level launches)
        std::vector<int32_t> level_rest;    // per level: fronts left to the level launches
        bool any = false;                   // the lists are not empty
        int32_t nbund[2] = {0, 0};
        int64_t ntasks[2] = {0, 0};
        size_t cap = 0;            // ints of d_buf
        int32_t* d_ctr = nullptr;  // counters of both directions (2 + 3 nslots each)
        int32_t* h_err = nullptr;  // pinned: the two error words
        void free_device() {
            if (d_buf) (void)dfree(d_buf);
            if (d_ctr) (void)dfree(d_ctr);
            if (h_err) (void)hfree(h_err);
            d_buf = nullptr;
            d_ctr = nullptr;
            h_err = nullptr;
            cap = 0;
            valid = false;
        }
    } sweep;
    int sweep_grid = 0;
    unsigned long long* d_bad = nullptr;    // first CSR position of a non-finite value
    unsigned long long* h_bad = nullptr;    // pinned mirror
    double* d_cat = nullptr;                // batched solve: concatenated b and x
    size_t cat_cap = 0;
    int32_t* d_ones = nullptr;              // nseg ones: every system active
    int ones_cap = 0;
    bool factored = false;
    hipStream_t last_stream = nullptr;  // stream of the last call (idle when the call returned)
    bool stale = false;        // operator values replaced since the factorization (mf_set_operator)
    std::vector<int32_t> lvl_mmax[2], lvl_Pmax[2], lvl_cnt[2];  // per level per precision
    std::vector<std::array<int32_t, kNClass>> lvl_cls_mmax[2], lvl_cls_Pmax[2];  // per level, precision, panel class
    // equilibration: factors are of Dr J Dc (powers of two); residuals use J itself
    bool scaled = false;
    double* d_svals = nullptr;          // Dr J Dc values (nnz)
    double* d_dr = nullptr;             // n
    double* d_dc = nullptr;             // n
    double* d_rmax = nullptr;           // n
    unsigned long long* d_cmax = nullptr;  // n
    double* d_sb = nullptr;             // Dr b for the sweeps (n x nrhs)
    size_t sb_cap = 0;
    int32_t* d_tasks = nullptr;  // per-level tile work lists (LevelTasks)
    std::vector<int32_t> kid_scratch;  // children per front of the level being set up
    int32_t* h_tasks = nullptr;  // pinned staging
    size_t tasks_cap = 0;        // entries
    mf_factor_info info{};
    // Planned schedule.  A factorization that synchronizes once per level learns
    // every front's delayed-in count; the plan gives each front a capacity (that
    // count plus slack) and fixes from it all storage, tile lists and launch
    // shapes, so the next factorizations on this handle enqueue every level at
    // once and synchronize only at the end.  A front that outgrows its capacity
    // flags the run, which is then repeated with per-level synchronization.
    struct Plan {
        bool valid = false;
        int32_t prec = -1;
        std::vector<int32_t> din_cap;  // per slot
        FrontNum* d_tmpl = nullptr;    // per slot: storage pointers, offsets, din = capacity
        int32_t* d_tasks = nullptr;    // tile lists of all levels
        std::vector<LevelTasks> tasks; // per level, pointing into d_tasks
        std::vector<int32_t> lvl_mmax[2], lvl_Pmax[2], lvl_cnt[2];
        std::vector<std::array<int32_t, kNClass>> lvl_cls_mmax[2], lvl_cls_Pmax[2];
        int64_t vec_len = 0;
        int32_t* d_flag = nullptr;  // overflow flag
        int32_t* h_flag = nullptr;  // pinned mirror
        // plan = 2: the planned launches captured once into a graph and replayed;
        // the capture bakes in the values buffer and the pivot threshold
        hipGraphExec_t graph = nullptr;
        hipStream_t cap_stream = nullptr;  // private stream to capture on (the caller's may be the null stream)
        const double* graph_vals = nullptr;
        double graph_u = -1.0;
        void drop_graph() {
            if (graph) (void)hipGraphExecDestroy(graph);
            graph = nullptr;
            graph_vals = nullptr;
            graph_u = -1.0;
        }
        void free_device() {
            drop_graph();
            if (cap_stream) (void)hipStreamDestroy(cap_stream);
            cap_stream = nullptr;
            if (d_tmpl) (void)dfree(d_tmpl);
            if (d_tasks) (void)dfree(d_tasks);
            if (d_flag) (void)dfree(d_flag);
            if (h_flag) (void)hfree(h_flag);
            d_tmpl = nullptr;
            d_tasks = nullptr;
            d_flag = nullptr;
            h_flag = nullptr;
            valid = false;
        }
    } plan;
    int32_t plan_fallbacks = 0;
    hipEvent_t ev_level = nullptr;  // end of a level's panel rounds (synchronizing schedule)
    // Launch-shape tuner (options.tune): per tree level, the panel block (4 or 8
    // waves for fronts of order <= 512) and the swap tile width (16 or 64
    // columns).  Neither changes any result.  Trial factorization c runs shape c
    // on every level and times each level with events; after the last trial each
    // level keeps its fastest shape.
    struct Tuner {
        static constexpr int kShapes = 4;  // bit 0: 8-wave panel; bit 1: 16-column swap tiles
        int32_t prec = -1;
        int trials = 0;
        std::vector<std::array<float, kShapes>> ms;  // per level and shape
        std::vector<int8_t> pick;                    // per level, once done
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool done() const { return trials >= kShapes; }
        void reset(int nlevels, int p) {
            prec = p;
            trials = 0;
            ms.assign(nlevels, {});
            pick.assign(nlevels, -1);
        }
    } tuner;
    ~mf_num() {
        for (void* p : kv_alloc) (void)dfree(p);
        sweep.free_device();
        if (d_bad) (void)dfree(d_bad);
        if (h_bad) (void)hfree(h_bad);
        if (ev_level) (void)hipEventDestroy(ev_level);
        if (tuner.e0) (void)hipEventDestroy(tuner.e0);
        if (tuner.e1) (void)hipEventDestroy(tuner.e1);
        plan.free_device();
        fronts.release();
        ints.release();
        wsp.release();
        if (d_fn) (void)dfree(d_fn);
        if (h_fn) (void)hfree(h_fn);
        if (d_vals) (void)dfree(d_vals);
        if (d_vec) (void)dfree(d_vec);
        if (d_work) (void)dfree(d_work);
        if (d_kry) (void)dfree(d_kry);
        if (d_small) (void)dfree(d_small);
        if (h_small) (void)hfree(h_small);
        if (d_seg) (void)dfree(d_seg);
        if (h_seg) (void)hfree(h_seg);
        if (d_omega) (void)dfree(d_omega);
        if (d_respart) (void)dfree(d_respart);
        if (h_omega) (void)hfree(h_omega);
        if (d_active) (void)dfree(d_active);
        if (d_cat) (void)dfree(d_cat);
        if (d_ones) (void)dfree(d_ones);
        if (h_active) (void)hfree(h_active);
        if (d_tasks) (void)dfree(d_tasks);
        if (d_svals) (void)dfree(d_svals);
        if (d_dr) (void)dfree(d_dr);
        if (d_dc) (void)dfree(d_dc);
        if (d_rmax) (void)dfree(d_rmax);
        if (d_cmax) (void)dfree(d_cmax);
        if (d_sb) (void)dfree(d_sb);
        if (h_tasks) (void)hfree(h_tasks);
    }
};

namespace {

mf_status fail(mf_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

void resolve_refine(mf_options& o) {
    if (o.refine < 0) o.refine = (o.prec == MF_FP64) ? 1 : 3;
}

// The unique-entry maps and the CSR pattern of a light batch, concatenated on
// the device from its systems' own device copies (one segmented copy per array,
// each (system, level) block shifted to its batch slots and sources).
void build_light_maps(mf_sym* h, SymDev& D) {
    const Symbolic& S = h->S;
    DevSym& d = D.S;
    for (const auto& P : h->parts_dev)
        if (!P || P->device != D.device)
            throw Fail{MF_ERR_ARG, "a batch analyzed on one device is factored on another"};
    const int nq = (int)h->parts_dev.size();
    std::vector<SegCopy> slot, row, col, sptr, src, rp, ci;
    for (const Symbolic::UeBlock& b : S.ue_blocks) {
        const DevSym& P = h->parts_dev[b.part]->S;
        slot.push_back({P.ue_slot + b.u0, b.dst_u, b.cnt, b.slot_delta});
        row.push_back({P.ue_row + b.u0, b.dst_u, b.cnt, 0});
        col.push_back({P.ue_col + b.u0, b.dst_u, b.cnt, 0});
        sptr.push_back({P.ue_src_ptr + b.u0, b.dst_u, b.cnt, b.dst_s - b.s0});
        src.push_back({P.ue_src + b.s0, b.dst_s, b.scnt, S.seg_nnz0[b.part]});
    }
    for (int q = 0; q < nq; q++) {
        const DevSym& P = h->parts_dev[q]->S;
        const int64_t nz = (q + 1 < nq ? S.seg_nnz0[q + 1] : S.nnz) - S.seg_nnz0[q];
        rp.push_back({P.csr_rowptr, S.seg_row0[q], S.seg_n[q], S.seg_nnz0[q]});
        ci.push_back({P.csr_colind, S.seg_nnz0[q], nz, S.seg_row0[q]});
    }
    auto run = [&](const std::vector<SegCopy>& segs, auto* out) {
        std::vector<int64_t> start(segs.size() + 1, 0);
        for (size_t i = 0; i < segs.size(); i++) start[i + 1] = start[i] + segs[i].count;
        HIPX(launch_seg_copy(D.put(segs), D.put(start), (int)segs.size(), start.back(), out, nullptr));
    };
    int32_t* ue_slot = D.alloc<int32_t>(S.n_ue);
    int32_t* ue_row = D.alloc<int32_t>(S.n_ue);
    int32_t* ue_col = D.alloc<int32_t>(S.n_ue);
    int64_t* ue_src_ptr = D.alloc<int64_t>(S.n_ue + 1);
    int32_t* ue_src = D.alloc<int32_t>(S.n_src);
    int64_t* rowptr = D.alloc<int64_t>(S.n + 1);
    int32_t* colind = D.alloc<int32_t>(S.nnz);
    run(slot, ue_slot);
    run(row, ue_row);
    run(col, ue_col);
    run(sptr, ue_src_ptr);
    run(src, ue_src);
    run(rp, rowptr);
    run(ci, colind);
    HIPX(hipMemcpy(ue_src_ptr + S.n_ue, &S.n_src, sizeof(int64_t), hipMemcpyHostToDevice));
    HIPX(hipMemcpy(rowptr + S.n, &S.nnz, sizeof(int64_t), hipMemcpyHostToDevice));
    HIPX(hipStreamSynchronize(nullptr));
    d.ue_slot = ue_slot;
    d.ue_row = ue_row;
    d.ue_col = ue_col;
    d.ue_src_ptr = ue_src_ptr;
    d.ue_src = ue_src;
    d.csr_rowptr = rowptr;
    d.csr_colind = colind;
}

std::mutex g_symdev_mu;  // device pattern data is built once per handle, also when batches share it

void ensure_device_symbolic(mf_sym* h) {
    int dev = 0;
    HIPX(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_symdev_mu);
    if (h->dev && h->dev->device == dev) return;
    const Symbolic& S = h->S;
    auto D = std::make_unique<SymDev>();
    D->device = dev;
    const int nf = S.nf;
    D->slot_of.assign(nf, -1);
    for (int32_t i = 0; i < nf; i++) D->slot_of[S.level_fronts[i]] = i;
    std::vector<int32_t> parent(nf), child_ptr(nf + 1, 0), child_slot;
    std::vector<int64_t> rows_ptr(nf + 1, 0), imap_off(nf + 1, 0);
    std::vector<int32_t> rows, imap;
    child_slot.reserve(S.child_idx.size());
    rows.reserve(S.rows.size());
    imap.reserve(S.imap.size());
    for (int32_t sl = 0; sl < nf; sl++) {
        int32_t f = S.level_fronts[sl];
        parent[sl] = S.front_parent[f] >= 0 ? D->slot_of[S.front_parent[f]] : -1;
        for (int32_t t = S.child_ptr[f]; t < S.child_ptr[f + 1]; t++) child_slot.push_back(D->slot_of[S.child_idx[t]]);
        child_ptr[sl + 1] = (int32_t)child_slot.size();
        rows.insert(rows.end(), S.rows.begin() + S.rows_ptr[f], S.rows.begin() + S.rows_ptr[f + 1]);
        rows_ptr[sl + 1] = (int64_t)rows.size();
        imap.insert(imap.end(), S.imap.begin() + S.imap_off[f], S.imap.begin() + S.imap_off[f + 1]);
        imap_off[sl + 1] = (int64_t)imap.size();
    }
    DevSym& d = D->S;
    d.nslots = nf;
    d.parent = D->put(parent);
    d.child_ptr = D->put(child_ptr);
    d.child_slot = D->put(child_slot);
    d.rows_ptr = D->put(rows_ptr);
    d.rows = D->put(rows);
    d.imap_off = D->put(imap_off);
    d.imap = D->put(imap);
    if (S.light) {
        build_light_maps(h, *D);
    } else {
        std::vector<int32_t> ue_slot(S.ue_front.size());
        for (size_t i = 0; i < ue_slot.size(); i++) ue_slot[i] = D->slot_of[S.ue_front[i]];
        d.ue_slot = D->put(ue_slot);
        d.ue_row = D->put(S.ue_row);
        d.ue_col = D->put(S.ue_col);
        d.ue_src_ptr = D->put(S.ue_src_ptr);
        d.ue_src = D->put(S.ue_src);
        d.csr_rowptr = D->put(S.rowptr);
        d.csr_colind = D->put(S.colind);
    }
    d.nseg = (int32_t)S.seg_n.size();
    d.seg_row0 = D->put(S.seg_row0);
    d.seg_n = D->put(S.seg_n);
    d.row_seg = nullptr;
    if (d.nseg > 1) {
        std::vector<int32_t> rs(S.n);
        for (int32_t q = 0; q < d.nseg; q++)
            for (int64_t i = 0; i < S.seg_n[q]; i++) rs[S.seg_row0[q] + i] = q;
        d.row_seg = D->put(rs);
    }
    h->dev = std::move(D);
}

int front_prec(const mf_options& o, bool is_root) { return (o.prec == MF_FP64 || is_root) ? 0 : 1; }

// Children of each front of the level [s0, s1) (slot order).
void level_kids(const Symbolic& S, int s0, int s1, std::vector<int32_t>& out) {
    out.resize((size_t)std::max(s1 - s0, 0));
    for (int sl = s0; sl < s1; sl++) {
        const int f = S.level_fronts[sl];
        out[sl - s0] = S.child_ptr[f + 1] - S.child_ptr[f];
    }
}

// Appended to t (the planned schedule collects every level's lists).
LevelTasks build_level_tasks(const FrontNum* hf, int count, std::vector<int32_t>& t, int sw_force = 0,
                             const int32_t* nkid = nullptr) {
    const LevelTasks tk = level_task_count(hf, count, sw_force, nkid);
    const size_t base = t.size();
    t.resize(base + level_task_total(tk));
    if (fill_level_tasks(hf, count, tk, nkid, t.data() + base, level_task_total(tk)) != level_task_total(tk))
        throw Fail{MF_ERR_STATE, "internal: task list count mismatch"};
    return tk;
}

// Point a level's lists at their device copy starting at d.
LevelTasks place_tasks(LevelTasks tk, const int32_t* d) {
    tk.swap = d;
    tk.g0 = d + tk.nswap;
    tk.g1 = d + tk.nswap + tk.ng0;
    tk.gather = d + tk.nswap + tk.ng0 + tk.ng1;
    return tk;
}

// Uploaded once per level by the synchronizing schedule: the previous level has
// been synchronized, so the pinned staging can be reused.
LevelTasks upload_level_tasks(mf_num* N, const FrontNum* hf, int count, hipStream_t st, int sw_force = 0,
                              const int32_t* nkid = nullptr) {
    // written straight into the pinned staging buffer, then one copy
    const LevelTasks tk = level_task_count(hf, count, sw_force, nkid);
    const size_t total = level_task_total(tk);
    if (total > N->tasks_cap) {
        if (N->d_tasks) HIPX(dfree(N->d_tasks));
        if (N->h_tasks) HIPX(hfree(N->h_tasks));
        N->d_tasks = nullptr;
        N->h_tasks = nullptr;
        N->tasks_cap = 0;
        const size_t cap = total + total / 2 + 1024;
        HIPX(dmalloc((void**)&N->d_tasks, sizeof(int32_t) * cap));
        HIPX(hmalloc((void**)&N->h_tasks, sizeof(int32_t) * cap, hipHostMallocDefault));
        N->tasks_cap = cap;
    }
    if (fill_level_tasks(hf, count, tk, nkid, N->h_tasks, N->tasks_cap) != total)
        throw Fail{MF_ERR_STATE, "internal: task list count mismatch"};
    if (total) HIPX(hipMemcpyAsync(N->d_tasks, N->h_tasks, sizeof(int32_t) * total, hipMemcpyHostToDevice, st));
    return place_tasks(tk, N->d_tasks);
}

// Flops of eliminating p pivots from a front of order m: sum over i in [m-p, m)
// of i + 2 i^2, in closed form (exact in 64-bit integers for orders below 2^20).
double front_flops(int64_t m, int64_t p) {
    auto s1 = [](int64_t n) { return n * (n - 1) / 2; };                // sum of i, i < n
    auto s2 = [](int64_t n) { return (n - 1) * n * (2 * n - 1) / 6; };  // sum of i^2, i < n
    const int64_t a = m - p;
    return (double)(s1(m) - s1(a)) + 2.0 * (double)(s2(m) - s2(a));
}

// Slack of a planned front over the delayed-in count it was planned from.
int plan_capacity(int din) { return din + 16 + din / 2; }

// Build the plan from the delayed-in counts of the factorization just finished
// (h_fn).  Capacities never shrink on a handle, so a plan rebuilt after an
// overflow covers both runs.  Storage is laid out afresh from the arenas' start:
// the finished factors stay where they are until the next factorization writes.
void build_plan(mf_num* N) {
    const Symbolic& S = N->sym->S;
    const mf_options& o = N->opt;
    const int nf = S.nf;
    mf_num::Plan& pl = N->plan;
    const FrontNum* hf = N->h_fn;
    const bool grow = pl.prec == o.prec && (int)pl.din_cap.size() == nf;
    std::vector<int32_t> cap(nf);
    for (int sl = 0; sl < nf; sl++) {
        const int c = plan_capacity(hf[sl].din);
        cap[sl] = grow ? std::max(pl.din_cap[sl], c) : c;
    }
    pl.free_device();
    std::vector<FrontNum> tm(std::max(nf, 1));
    for (int p = 0; p < 2; p++) {
        pl.lvl_mmax[p].assign(S.nlevels, 0);
        pl.lvl_Pmax[p].assign(S.nlevels, 0);
        pl.lvl_cnt[p].assign(S.nlevels, 0);
        pl.lvl_cls_mmax[p].assign(S.nlevels, {});
        pl.lvl_cls_Pmax[p].assign(S.nlevels, {});
    }
    N->fronts.reset();
    N->ints.reset();
    std::vector<int32_t> tasks;
    std::vector<size_t> toff(S.nlevels);
    pl.tasks.assign(S.nlevels, LevelTasks{});
    int64_t voff = 0;
    for (int L = 0; L < S.nlevels; L++) {
        const int s0 = S.level_ptr[L], s1 = S.level_ptr[L + 1];
        N->wsp.reset();
        for (int sl = s0; sl < s1; sl++) {
            const int f = S.level_fronts[sl];
            FrontNum& t = tm[sl];
            t = FrontNum{};
            t.npiv = S.npiv[f];
            t.mnom = S.mnom[f];
            t.din = cap[sl];
            t.m = t.mnom + cap[sl];  // capacity; the level setup writes the actual order
            t.P = t.npiv + cap[sl];
            t.pcur = t.P;
            t.prec = front_prec(o, S.front_parent[f] < 0);
            const size_t esz = t.prec ? 4 : 8;
            t.F = N->fronts.alloc(std::max<size_t>(esz * (size_t)t.m * (size_t)t.m, 8));
            t.iv = (int32_t*)N->ints.alloc(sizeof(int32_t) * (size_t)iv_size(t.P, t.m));
            t.voff = voff;
            voff += t.m;
            // any class the actual order falls in has a window of at most kNBMax
            t.W = N->wsp.alloc((size_t)2 * t.m * kNBMax * esz);
            const int p = t.prec;
            const int cls = front_class(t.m);
            pl.lvl_cls_mmax[p][L][cls] = std::max(pl.lvl_cls_mmax[p][L][cls], t.m);
            pl.lvl_cls_Pmax[p][L][cls] = std::max(pl.lvl_cls_Pmax[p][L][cls], t.P);
            pl.lvl_mmax[p][L] = std::max(pl.lvl_mmax[p][L], t.m);
            pl.lvl_Pmax[p][L] = std::max(pl.lvl_Pmax[p][L], t.P);
            pl.lvl_cnt[p][L]++;
        }
        for (int p = 0; p < 2; p++)
            if (pl.lvl_cnt[p][L] &&
                ((size_t)pl.lvl_Pmax[p][L] * 2 * sizeof(int) > kMaxLds || pl.lvl_mmax[p][L] > kMaxFrontOrder))
                return;  // capacities beyond the kernels' limits: keep synchronizing per level
        toff[L] = tasks.size();
        const int shape = (o.tune && N->tuner.done()) ? N->tuner.pick[L] : -1;
        std::vector<int32_t> kids;
        level_kids(S, s0, s1, kids);
        pl.tasks[L] = build_level_tasks(tm.data() + s0, s1 - s0, tasks, shape < 0 ? 0 : ((shape & 2) ? 16 : 64),
                                        kids.data());
    }
    HIPX(dmalloc((void**)&pl.d_tmpl, sizeof(FrontNum) * tm.size()));
    HIPX(hipMemcpy(pl.d_tmpl, tm.data(), sizeof(FrontNum) * tm.size(), hipMemcpyHostToDevice));
    HIPX(dmalloc((void**)&pl.d_tasks, sizeof(int32_t) * std::max<size_t>(tasks.size(), 1)));
    if (!tasks.empty())
        HIPX(hipMemcpy(pl.d_tasks, tasks.data(), sizeof(int32_t) * tasks.size(), hipMemcpyHostToDevice));
    for (int L = 0; L < S.nlevels; L++) pl.tasks[L] = place_tasks(pl.tasks[L], pl.d_tasks + toff[L]);
    HIPX(dmalloc((void**)&pl.d_flag, sizeof(int32_t)));
    HIPX(hmalloc((void**)&pl.h_flag, sizeof(int32_t), hipHostMallocDefault));
    pl.vec_len = voff;
    pl.din_cap = cap;
    pl.prec = o.prec;
    pl.valid = true;
}

// Factor info of a finished run from its fronts' final bookkeeping (h_fn).
mf_factor_info finished_info(const mf_num* N) {
    const Symbolic& S = N->sym->S;
    const FrontNum* hf = N->h_fn;
    mf_factor_info info{};
    info.factor_flops = S.nominal_flops;
    for (int sl = 0; sl < S.nf; sl++) {
        const FrontNum& fr = hf[sl];
        const size_t esz = fr.prec ? 4 : 8;
        info.factor_bytes += (int64_t)(esz * (size_t)fr.m * (size_t)fr.m);
        info.max_front = std::max(info.max_front, fr.m);
        info.actual_flops += front_flops(fr.m, fr.P);
        const double cb = (double)(fr.m - fr.P);
        info.schur_flops += 2.0 * cb * cb * (double)fr.k;
        const int dout = fr.P - fr.k;
        info.delayed_pivots += dout;
        const int f = S.level_fronts[sl];
        if (S.front_parent[f] < 0) {
            info.root_order = std::max(info.root_order, fr.m);
            if (dout > 0)
                throw Fail{MF_ERR_SINGULAR, "root front " + std::to_string(f) + " (order " + std::to_string(fr.m) +
                                                "): no acceptable pivot for column position " + std::to_string(fr.k) +
                                                " (numerically singular or non-finite)"};
        }
    }
    info.levels = S.nlevels;
    return info;
}

// Delayed columns per system of a batch (one entry for a single system), from the
// finished factorization's bookkeeping (h_fn).
void seg_delays(mf_num* N) {
    const Symbolic& S = N->sym->S;
    const int nseg = (int)S.seg_n.size();
    N->seg_delayed.assign(nseg, 0);
    for (int sl = 0; sl < S.nf; sl++) {
        const int f = S.level_fronts[sl];
        if (S.rows_ptr[f + 1] == S.rows_ptr[f]) continue;
        const int64_t var = S.rows[S.rows_ptr[f]];
        const int q = nseg == 1 ? 0
                                : (int)(std::upper_bound(S.seg_row0.begin(), S.seg_row0.end(), var) -
                                        S.seg_row0.begin()) - 1;
        N->seg_delayed[q] += N->h_fn[sl].P - N->h_fn[sl].k;
    }
}

// Values are scanned for NaN and Inf before any front is built; the position of
// the first one is read back with the first synchronization of the factorization.
void check_finite(const mf_num* N) {
    if (*N->h_bad != ~0ull)
        throw Fail{MF_ERR_ARG, "values_dev[" + std::to_string(*N->h_bad) + "] is NaN or Inf"};
}

// The planned schedule: every level enqueued at once, one synchronization at the
// end.  Returns -1 when it finished, else the first level where a front outgrew
// its capacity: the levels below it are finished (factors, bookkeeping in h_fn,
// storage in the plan's layout) and the caller continues from that level.
int factor_planned(mf_num* N, const double* fvals, hipStream_t st) {
    mf_sym* H = N->sym;
    const Symbolic& S = H->S;
    SymDev& D = *H->dev;
    const mf_options& o = N->opt;
    mf_num::Plan& pl = N->plan;
    auto enqueue = [&](hipStream_t q) {
        HIPX(launch_fill_i32(pl.d_flag, INT_MAX, q));
        for (int L = 0; L < S.nlevels; L++) {
            const int s0 = S.level_ptr[L], s1 = S.level_ptr[L + 1];
            const bool full = o.tune && N->tuner.done() && (N->tuner.pick[L] & 1);
            HIPX(launch_level_setup(D.S, N->d_fn, pl.d_tmpl, s0, s1 - s0, L, pl.d_flag, q));
            const int64_t u0 = S.level_ue_ptr[L], u1 = S.level_ue_ptr[L + 1];
            if (pl.lvl_cnt[0][L])
                HIPX(launch_level_factor<double>(D.S, N->d_fn, s0, s1 - s0, pl.lvl_mmax[0][L],
                                                 pl.lvl_cls_mmax[0][L].data(), pl.lvl_cls_Pmax[0][L].data(), fvals,
                                                 u0, u1, o.pivot_u, 0, pl.tasks[L], q, nullptr, false, nullptr, full));
            if (pl.lvl_cnt[1][L])
                HIPX(launch_level_factor<float>(D.S, N->d_fn, s0, s1 - s0, pl.lvl_mmax[1][L],
                                                pl.lvl_cls_mmax[1][L].data(), pl.lvl_cls_Pmax[1][L].data(), fvals,
                                                u0, u1, o.pivot_u, 1, pl.tasks[L], q, nullptr, o.prec == MF_BF16,
                                                nullptr, full));
        }
    };
    if (o.plan == 2) {
        if (!pl.graph || pl.graph_vals != fvals || pl.graph_u != o.pivot_u) {
            pl.drop_graph();
            if (!pl.cap_stream) HIPX(hipStreamCreateWithFlags(&pl.cap_stream, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            std::shared_lock<std::shared_mutex> cap(g_capture_mu);
            // relaxed: allocations and frees of other threads (other handles, other
            // libraries) cannot invalidate this capture
            HIPX(hipStreamBeginCapture(pl.cap_stream, hipStreamCaptureModeRelaxed));
            try {
                enqueue(pl.cap_stream);
            } catch (...) {
                (void)hipStreamEndCapture(pl.cap_stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIPX(hipStreamEndCapture(pl.cap_stream, &g));
            const hipError_t ie = hipGraphInstantiate(&pl.graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPX(ie);
            pl.graph_vals = fvals;
            pl.graph_u = o.pivot_u;
        }
        HIPX(hipGraphLaunch(pl.graph, st));
    } else {
        enqueue(st);
    }
    HIPX(hipMemcpyAsync(N->h_fn, N->d_fn, sizeof(FrontNum) * S.nf, hipMemcpyDeviceToHost, st));
    HIPX(hipMemcpyAsync(pl.h_flag, pl.d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    check_finite(N);
    if (*pl.h_flag != INT_MAX) {
        N->plan_fallbacks++;
        if (*pl.h_flag < 0 || *pl.h_flag >= S.nlevels) throw Fail{MF_ERR_STATE, "internal: bad overflow level"};
        return *pl.h_flag;
    }
    for (int p = 0; p < 2; p++) {
        N->lvl_mmax[p] = pl.lvl_mmax[p];
        N->lvl_Pmax[p] = pl.lvl_Pmax[p];
        N->lvl_cnt[p] = pl.lvl_cnt[p];
        N->lvl_cls_mmax[p] = pl.lvl_cls_mmax[p];
        N->lvl_cls_Pmax[p] = pl.lvl_cls_Pmax[p];
    }
    N->vec_len = pl.vec_len;
    N->info = finished_info(N);
    seg_delays(N);
    N->info.planned = o.plan == 2 ? 2 : 1;
    N->info.tuned = (o.tune && N->tuner.done()) ? 1 : 0;
    N->info.plan_fallbacks = N->plan_fallbacks;
    N->factored = true;
    return -1;
}

// The handle's own copy of the operator values (one array, or one per system of a
// batch), scanned for NaN and Inf; the scan's result is read back by the next
// synchronization on the stream (check_finite).
// The segment lists of one batch gather or scatter, written to the pinned
// staging buffer (every entry point returns with its stream synchronized, so the
// buffer is free again when the next call writes it).  Layout: for each list,
// the segments, then their start offsets (prefix sums, nseg + 1 entries).
struct SegLists {
    size_t bytes = 0;
    template <typename S>
    static size_t need(size_t nseg) {
        return ((sizeof(S) * nseg + 15) & ~size_t(15)) + ((sizeof(int64_t) * (nseg + 1) + 15) & ~size_t(15));
    }
};
char* seg_staging(mf_num* N, size_t bytes) {
    if (bytes > N->seg_cap) {
        if (N->d_seg) HIPX(dfree(N->d_seg));
        if (N->h_seg) HIPX(hfree(N->h_seg));
        N->d_seg = nullptr;
        N->h_seg = nullptr;
        HIPX(dmalloc((void**)&N->d_seg, bytes));
        HIPX(hmalloc((void**)&N->h_seg, bytes, hipHostMallocDefault));
        N->seg_cap = bytes;
    }
    return N->h_seg;
}
// Writes the list (segments and starts) at byte offset off of the staging
// buffer; returns the total count and advances off.
template <typename S>
int64_t put_segments(mf_num* N, size_t& off, const std::vector<S>& segs, const S** d_segs, const int64_t** d_start) {
    S* hs = (S*)(N->h_seg + off);
    std::copy(segs.begin(), segs.end(), hs);
    *d_segs = (const S*)(N->d_seg + off);
    off += (sizeof(S) * segs.size() + 15) & ~size_t(15);
    int64_t* st = (int64_t*)(N->h_seg + off);
    st[0] = 0;
    for (size_t q = 0; q < segs.size(); q++) st[q + 1] = st[q] + segs[q].count;
    *d_start = (const int64_t*)(N->d_seg + off);
    off += (sizeof(int64_t) * (segs.size() + 1) + 15) & ~size_t(15);
    return st[segs.size()];
}

void load_values(mf_num* N, const double* values_dev, const double* const* seg_values, hipStream_t st) {
    const Symbolic& S = N->sym->S;
    if (!N->d_vals) HIPX(dmalloc((void**)&N->d_vals, sizeof(double) * std::max<int64_t>(S.nnz, 1)));
    if (!N->d_bad) {
        HIPX(dmalloc((void**)&N->d_bad, sizeof(unsigned long long)));
        HIPX(hmalloc((void**)&N->h_bad, sizeof(unsigned long long), hipHostMallocDefault));
    }
    if (seg_values) {
        // every system's values into the batch's array in one launch
        std::vector<SegCopy> segs;
        for (size_t q = 0; q < S.seg_n.size(); q++) {
            const int64_t nz = (q + 1 < S.seg_n.size() ? S.seg_nnz0[q + 1] : S.nnz) - S.seg_nnz0[q];
            if (nz) segs.push_back(SegCopy{seg_values[q], S.seg_nnz0[q], nz, 0});
        }
        if (!segs.empty()) {
            const size_t bytes = SegLists::need<SegCopy>(segs.size());
            seg_staging(N, bytes);
            size_t off = 0;
            const SegCopy* ds;
            const int64_t* dst;
            const int64_t total = put_segments(N, off, segs, &ds, &dst);
            HIPX(hipMemcpyAsync(N->d_seg, N->h_seg, off, hipMemcpyHostToDevice, st));
            HIPX(launch_seg_copy<double>(ds, dst, (int)segs.size(), total, N->d_vals, st));
        }
    } else if (S.nnz && values_dev != N->d_vals) {
        HIPX(hipMemcpyAsync(N->d_vals, values_dev, sizeof(double) * S.nnz, hipMemcpyDeviceToDevice, st));
    }
    HIPX(launch_nonfinite(N->d_vals, S.nnz, N->d_bad, st));
    HIPX(hipMemcpyAsync(N->h_bad, N->d_bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
}

void do_factor(mf_num* N, const double* values_dev, hipStream_t st, const double* const* seg_values = nullptr) {
    N->sweep.valid = false;
    mf_sym* H = N->sym;
    const Symbolic& S = H->S;
    ensure_device_symbolic(H);
    SymDev& D = *H->dev;
    const int nf = S.nf;
    const mf_options& o = N->opt;
    if (!N->d_fn) {
        HIPX(dmalloc((void**)&N->d_fn, sizeof(FrontNum) * std::max(nf, 1)));
        HIPX(hmalloc((void**)&N->h_fn, sizeof(FrontNum) * std::max(nf, 1), hipHostMallocDefault));
    }
    load_values(N, values_dev, seg_values, st);
    N->stale = false;
    // equilibration (values only: the pattern and the analysis are unchanged)
    const double* fvals = N->d_vals;
    N->scaled = o.scale > 0 && S.n > 0;
    if (N->scaled) {
        if (!N->d_svals) {
            HIPX(dmalloc((void**)&N->d_svals, sizeof(double) * std::max<int64_t>(S.nnz, 1)));
            HIPX(dmalloc((void**)&N->d_dr, sizeof(double) * S.n));
            HIPX(dmalloc((void**)&N->d_dc, sizeof(double) * S.n));
            HIPX(dmalloc((void**)&N->d_rmax, sizeof(double) * S.n));
            HIPX(dmalloc((void**)&N->d_cmax, sizeof(unsigned long long) * S.n));
        }
        HIPX(launch_ruiz(D.S, N->d_vals, S.n, o.scale, N->d_dr, N->d_dc, N->d_rmax, N->d_cmax, N->d_svals, st));
        fvals = N->d_svals;
    }
    const bool use_plan = o.plan != 0 && o.profile == 0 && N->plan.valid && N->plan.prec == o.prec &&
                          !(o.tune && !N->tuner.done());  // tuner trials run level by level
    // first level factored here: above 0 when a planned run overflowed there (the
    // levels below it are finished in the plan's storage, which the arenas keep)
    int L0 = 0;
    if (use_plan) {
        L0 = factor_planned(N, fvals, st);
        if (L0 < 0) return;
    }
    if (N->fronts.chunks.empty()) {
        double tot = 0;
        for (int f = 0; f < nf; f++) tot += (double)S.mnom[f] * S.mnom[f];
        size_t esz = (o.prec == MF_FP64) ? 8 : 4;
        N->fronts.grow_hint = (size_t)(tot * esz * 1.25) + (64u << 20);
        N->ints.grow_hint = (size_t)(sizeof(int32_t) * (S.rows.size() * 4 + (size_t)nf * (3 + 7 * kNBMax))) + (16u << 20);
        N->wsp.grow_hint = (64u << 20);
    }
    if (L0 == 0) {
        N->fronts.reset();
        N->ints.reset();
    }
    for (int p = 0; p < 2; p++) {
        if (L0 == 0) {
            N->lvl_mmax[p].assign(S.nlevels, 0);
            N->lvl_Pmax[p].assign(S.nlevels, 0);
            N->lvl_cnt[p].assign(S.nlevels, 0);
            N->lvl_cls_mmax[p].assign(S.nlevels, {});
            N->lvl_cls_Pmax[p].assign(S.nlevels, {});
            continue;
        }
        const mf_num::Plan& pl = N->plan;
        N->lvl_mmax[p] = pl.lvl_mmax[p];
        N->lvl_Pmax[p] = pl.lvl_Pmax[p];
        N->lvl_cnt[p] = pl.lvl_cnt[p];
        N->lvl_cls_mmax[p] = pl.lvl_cls_mmax[p];
        N->lvl_cls_Pmax[p] = pl.lvl_cls_Pmax[p];
        for (int L = L0; L < S.nlevels; L++) {
            N->lvl_mmax[p][L] = N->lvl_Pmax[p][L] = N->lvl_cnt[p][L] = 0;
            N->lvl_cls_mmax[p][L] = {};
            N->lvl_cls_Pmax[p][L] = {};
        }
    }
    std::vector<int32_t> dout(nf, 0);
    FrontNum* hf = N->h_fn;
    for (int sl = 0; sl < S.level_ptr[L0]; sl++) dout[sl] = hf[sl].P - hf[sl].k;
    const bool prof = o.profile != 0;
    hipEvent_t ev[2][5] = {};
    if (prof)
        for (int p = 0; p < 2; p++)
            for (int e = 0; e < 5; e++) HIPX(hipEventCreate(&ev[p][e]));
    struct EvGuard {
        hipEvent_t (*e)[5];
        bool on;
        ~EvGuard() {
            if (on)
                for (int p = 0; p < 2; p++)
                    for (int k = 0; k < 5; k++) (void)hipEventDestroy(e[p][k]);
        }
    } evg{ev, prof};
    std::vector<hipEvent_t> pev;  // (start, end) of every panel launch (profile mode)
    // launch-shape tuner: trials run on this (level by level) schedule only
    if (o.tune && (N->tuner.prec != o.prec || (int)N->tuner.pick.size() != S.nlevels))
        N->tuner.reset(S.nlevels, o.prec);
    const bool tuning = o.tune && !prof && !N->tuner.done();
    const bool tuned = o.tune && N->tuner.done();
    if (tuning && !N->tuner.e0) {
        HIPX(hipEventCreate(&N->tuner.e0));
        HIPX(hipEventCreate(&N->tuner.e1));
    }
    int64_t voff = L0 ? N->plan.vec_len : 0;  // after every vector block of the plan
    mf_factor_info info{};
    info.factor_flops = S.nominal_flops;
    int64_t front_bytes = 0;
    for (int L = L0; L < S.nlevels; L++) {
        const int s0 = S.level_ptr[L], s1 = S.level_ptr[L + 1];
        for (int sl = s0; sl < s1; sl++) {
            const int f = S.level_fronts[sl];
            int din = 0;
            for (int t = S.child_ptr[f]; t < S.child_ptr[f + 1]; t++) din += dout[D.slot_of[S.child_idx[t]]];
            FrontNum& fr = hf[sl];
            fr.npiv = S.npiv[f];
            fr.mnom = S.mnom[f];
            fr.din = din;
            fr.m = S.mnom[f] + din;
            fr.P = S.npiv[f] + din;
            fr.k = 0;
            fr.k0 = 0;
            fr.pcur = fr.P;
            fr.x0 = 0;
            fr.x1 = 0;
            fr.pad_ = 0;
            fr.prec = front_prec(o, S.front_parent[f] < 0);
            const size_t esz = fr.prec ? 4 : 8;
            const size_t fb = esz * (size_t)fr.m * (size_t)fr.m;
            fr.F = N->fronts.alloc(std::max<size_t>(fb, 8));
            front_bytes += (int64_t)fb;
            fr.iv = (int32_t*)N->ints.alloc(sizeof(int32_t) * (size_t)iv_size(fr.P, fr.m));
            fr.voff = voff;
            voff += fr.m;
            const int p = fr.prec;
            const int cls = front_class(fr.m);
            N->lvl_cls_mmax[p][L][cls] = std::max(N->lvl_cls_mmax[p][L][cls], fr.m);
            N->lvl_cls_Pmax[p][L][cls] = std::max(N->lvl_cls_Pmax[p][L][cls], fr.P);
            N->lvl_mmax[p][L] = std::max(N->lvl_mmax[p][L], fr.m);
            N->lvl_Pmax[p][L] = std::max(N->lvl_Pmax[p][L], fr.P);
            N->lvl_cnt[p][L]++;
            info.max_front = std::max(info.max_front, fr.m);
            info.actual_flops += front_flops(fr.m, fr.P);
        }
        for (int p = 0; p < 2; p++) {
            if (!N->lvl_cnt[p][L]) continue;
            size_t lds = (size_t)N->lvl_Pmax[p][L] * 2 * sizeof(int);
            if (N->lvl_mmax[p][L] > kMaxFrontOrder)
                throw Fail{MF_ERR_ARG, "front of order " + std::to_string(N->lvl_mmax[p][L]) +
                                           " (nominal plus delayed-in) exceeds the limit of " +
                                           std::to_string(kMaxFrontOrder)};
            if (lds > kMaxLds)
                throw Fail{MF_ERR_ARG, "front with " + std::to_string(N->lvl_Pmax[p][L]) +
                                           " fully summed variables exceeds the panel kernel's LDS budget"};
        }
        if (s1 - s0 > kMaxLevelFronts)
            throw Fail{MF_ERR_ARG, "tree level with " + std::to_string(s1 - s0) + " fronts (limit " +
                                       std::to_string(kMaxLevelFronts) + "; split the batch)"};
        // panel scratch (reused level by level): m x NB entries per front
        N->wsp.reset();
        for (int sl = s0; sl < s1; sl++) {
            FrontNum& fr = hf[sl];
            const int nbp = panel_nb(fr.prec, fr.m);
            fr.W = N->wsp.alloc((size_t)2 * fr.m * nbp * (fr.prec ? 4 : 8));
        }
        HIPX(hipMemcpyAsync(N->d_fn + s0, hf + s0, sizeof(FrontNum) * (s1 - s0), hipMemcpyHostToDevice, st));
        const int shape = tuning ? N->tuner.trials : (tuned ? N->tuner.pick[L] : -1);
        level_kids(S, s0, s1, N->kid_scratch);
        const LevelTasks tk = upload_level_tasks(N, hf + s0, s1 - s0, st, shape < 0 ? 0 : ((shape & 2) ? 16 : 64),
                                                 N->kid_scratch.data());
        const bool full = shape >= 0 && (shape & 1);
        const int64_t u0 = S.level_ue_ptr[L], u1 = S.level_ue_ptr[L + 1];
        if (tuning) HIPX(hipEventRecord(N->tuner.e0, st));
        // Outside profiling and tuning the level runs in two parts: the host waits only
        // for the panel rounds (after which every delayed-out count is final) and sets
        // up the next level while the Schur GEMM and finalize of this one run.  Every
        // buffer the next set-up rewrites is either host memory this level no longer
        // reads or device memory written in stream order after this level's kernels.
        const bool split = !prof && !tuning;
        auto launch = [&](int part) {
            // fronts of both precisions may share a level; each kernel skips the other kind
            if (N->lvl_cnt[0][L]) {
                if (prof) HIPX(hipEventRecord(ev[0][0], st));
                HIPX(launch_level_factor<double>(D.S, N->d_fn, s0, s1 - s0, N->lvl_mmax[0][L],
                                                 N->lvl_cls_mmax[0][L].data(), N->lvl_cls_Pmax[0][L].data(), fvals,
                                                 u0, u1, o.pivot_u, 0, tk, st, prof ? &ev[0][1] : nullptr, false,
                                                 prof ? &pev : nullptr, full, part));
            }
            if (N->lvl_cnt[1][L]) {
                if (prof) HIPX(hipEventRecord(ev[1][0], st));
                HIPX(launch_level_factor<float>(D.S, N->d_fn, s0, s1 - s0, N->lvl_mmax[1][L],
                                                N->lvl_cls_mmax[1][L].data(), N->lvl_cls_Pmax[1][L].data(), fvals,
                                                u0, u1, o.pivot_u, 1, tk, st, prof ? &ev[1][1] : nullptr,
                                                o.prec == MF_BF16, prof ? &pev : nullptr, full, part));
            }
        };
        launch(split ? 1 : 0);
        if (tuning) HIPX(hipEventRecord(N->tuner.e1, st));
        HIPX(hipMemcpyAsync(hf + s0, N->d_fn + s0, sizeof(FrontNum) * (s1 - s0), hipMemcpyDeviceToHost, st));
        if (split) {
            if (!N->ev_level) HIPX(hipEventCreateWithFlags(&N->ev_level, hipEventDisableTiming));
            HIPX(hipEventRecord(N->ev_level, st));
            launch(2);
            HIPX(hipEventSynchronize(N->ev_level));
        } else {
            HIPX(hipStreamSynchronize(st));
        }
        if (L == 0) check_finite(N);
        if (tuning) HIPX(hipEventElapsedTime(&N->tuner.ms[L][N->tuner.trials], N->tuner.e0, N->tuner.e1));
        info.levels++;
        if (prof)
            for (int p = 0; p < 2; p++) {
                if (!N->lvl_cnt[p][L]) continue;
                float ms[4];
                for (int e = 0; e < 4; e++) HIPX(hipEventElapsedTime(&ms[e], ev[p][e], ev[p][e + 1]));
                info.t_assemble_ms += ms[0];
                info.t_panel_ms += ms[1];
                info.t_schur_ms += ms[2];
                info.t_finalize_ms += ms[3];
                info.schur_launches++;
            }
        if (prof) {
            for (size_t q = 0; q + 1 < pev.size(); q += 2) {
                float ms = 0.f;
                HIPX(hipEventElapsedTime(&ms, pev[q], pev[q + 1]));
                info.t_panel_kernel_ms += ms;
                info.panel_launches++;
            }
            for (hipEvent_t e : pev) (void)hipEventDestroy(e);
            pev.clear();
            // nominal panel work of this level (windows of the front's class width, no delays):
            // for each pivot of a window, scale the column below it and update the rest of the window
            for (int sl = s0; sl < s1; sl++) {
                const FrontNum& fr = hf[sl];
                const int cls = front_class(fr.m);
                const int nbp = panel_nb(fr.prec, fr.m);
                for (int k0 = 0; k0 < fr.P; k0 += nbp) {
                    const int w = std::min(nbp, fr.P - k0);
                    for (int t = 0; t < w; t++) {
                        const double rows = (double)(fr.m - k0 - t - 1);
                        info.panel_flops += rows + 2.0 * rows * (double)(w - t - 1);
                    }
                }
            }
        }
        for (int sl = s0; sl < s1; sl++) {
            const FrontNum& fr = hf[sl];
            dout[sl] = fr.P - fr.k;
            {
                const double cb = (double)(fr.m - fr.P);
                info.schur_flops += 2.0 * cb * cb * (double)fr.k;
            }
            info.delayed_pivots += dout[sl];
            const int f = S.level_fronts[sl];
            if (S.front_parent[f] < 0) {
                info.root_order = std::max(info.root_order, fr.m);
                if (dout[sl] > 0)
                    throw Fail{MF_ERR_SINGULAR, "root front " + std::to_string(f) + " (order " + std::to_string(fr.m) +
                                                    "): no acceptable pivot for column position " +
                                                    std::to_string(fr.k) + " (numerically singular or non-finite)"};
            }
        }
    }
    N->vec_len = voff;
    info.factor_bytes = front_bytes;
    if (L0 > 0) info = finished_info(N);  // the levels below L0 are only in h_fn
    info.plan_fallbacks = N->plan_fallbacks;
    info.tuned = tuned ? 1 : 0;
    if (tuning && ++N->tuner.trials == mf_num::Tuner::kShapes)
        for (int L = 0; L < S.nlevels; L++) {
            int best = 0;
            for (int c = 1; c < mf_num::Tuner::kShapes; c++)
                if (N->tuner.ms[L][c] < N->tuner.ms[L][best]) best = c;
            N->tuner.pick[L] = (int8_t)best;
        }
    if (S.nlevels == 0) {
        HIPX(hipStreamSynchronize(st));
        check_finite(N);
    }
    N->info = info;
    seg_delays(N);
    N->factored = true;
    if (o.plan != 0) build_plan(N);
}

void ensure_solve_buffers(mf_num* N, int nrhs) {
    const Symbolic& S = N->sym->S;
    const int64_t n = S.n;
    const int nseg = (int)S.seg_n.size();
    size_t need = (size_t)std::max<int64_t>(N->vec_len, 1) * nrhs;
    if (need > N->vec_cap) {
        if (N->d_vec) HIPX(dfree(N->d_vec));
        N->d_vec = nullptr;
        HIPX(dmalloc((void**)&N->d_vec, sizeof(double) * need));
        N->vec_cap = need;
    }
    size_t wneed = (size_t)std::max<int64_t>(n, 1) * nrhs * 2;
    if (wneed > N->work_cap) {
        if (N->d_work) HIPX(dfree(N->d_work));
        N->d_work = nullptr;
        HIPX(dmalloc((void**)&N->d_work, sizeof(double) * wneed));
        N->work_cap = wneed;
    }
    if (nrhs * nseg > N->omega_cap) {
        if (N->d_omega) HIPX(dfree(N->d_omega));
        if (N->h_omega) HIPX(hfree(N->h_omega));
        if (N->d_active) HIPX(dfree(N->d_active));
        if (N->h_active) HIPX(hfree(N->h_active));
        N->d_omega = nullptr;
        N->h_omega = nullptr;
        N->d_active = nullptr;
        N->h_active = nullptr;
        const int cnt = nrhs * nseg;
        HIPX(dmalloc((void**)&N->d_omega, sizeof(unsigned long long) * kResQ * cnt));
        HIPX(hmalloc((void**)&N->h_omega, sizeof(unsigned long long) * kResQ * cnt, hipHostMallocDefault));
        HIPX(dmalloc((void**)&N->d_active, sizeof(int32_t) * cnt));
        HIPX(hmalloc((void**)&N->h_active, sizeof(int32_t) * cnt, hipHostMallocDefault));
        N->omega_cap = cnt;
    }
}

// Task lists of the persistent sweeps for the current factors (h_fn): the
// forward list goes up the tree level by level, the backward list down; a front
// of order <= kSwWhole is one task (runs of them share a ticket, kSwBundle at
// most), a larger one is its fully summed 64-row blocks (forward: in order, then
// its contribution tiles; backward: last block first).  A front with nothing to
// eliminate still gets one task, which releases its dependants.
void build_sweep_plan(mf_num* N) {
    const Symbolic& S = N->sym->S;
    const FrontNum* hf = N->h_fn;
    const int ns = S.nf;
    std::vector<int32_t> tk[2], bp[2], nt[2], hm(std::max(ns, 1)), hk(std::max(ns, 1));
    for (int sl = 0; sl < ns; sl++) {
        hm[sl] = hf[sl].m;
        hk[sl] = hf[sl].k;
    }
    // Each system of a batch lists its own upper tree: the levels, from the top
    // down, where it has at most kSwTopFronts fronts.  The choice depends only on
    // the system, so its arithmetic is the same alone and in any batch.
    const int nseg = (int)S.seg_n.size();
    std::vector<int32_t> seg_of(std::max(ns, 1), 0);
    for (int sl = 0; sl < ns; sl++) {
        const int f = S.level_fronts[sl];
        if (nseg > 1 && S.rows_ptr[f + 1] > S.rows_ptr[f]) {
            const int64_t var = S.rows[S.rows_ptr[f]];
            seg_of[sl] = (int)(std::upper_bound(S.seg_row0.begin(), S.seg_row0.end(), var) - S.seg_row0.begin()) - 1;
        }
    }
    std::vector<int32_t> cnt((size_t)nseg * (S.nlevels + 1), 0), first(nseg, S.nlevels), mmax(nseg, 0);
    for (int L = 0; L < S.nlevels; L++)
        for (int sl = S.level_ptr[L]; sl < S.level_ptr[L + 1]; sl++) {
            cnt[(size_t)seg_of[sl] * (S.nlevels + 1) + L]++;
            mmax[seg_of[sl]] = std::max(mmax[seg_of[sl]], hm[sl]);
        }
    for (int q = 0; q < nseg; q++) {
        // only systems with fronts large enough for several work-groups per front to
        // pay for the cross-group waits (measured: the 64-system batch of small
        // meshes sweeps faster level by level)
        if (mmax[q] < kSwListedMinOrder) continue;
        const int32_t* c = cnt.data() + (size_t)q * (S.nlevels + 1);
        int T = S.nlevels;
        while (T > 0 && c[T - 1] <= kSwTopFronts) T--;
        first[q] = T;
    }
    std::vector<uint8_t> listed(std::max(ns, 1), 0);
    mf_num::SweepPlan& P0 = N->sweep;
    P0.level_rest.assign(S.nlevels, 0);
    P0.any = false;
    for (int L = 0; L < S.nlevels; L++)
        for (int sl = S.level_ptr[L]; sl < S.level_ptr[L + 1]; sl++) {
            listed[sl] = L >= first[seg_of[sl]] ? 1 : 0;
            if (listed[sl]) P0.any = true;
            else P0.level_rest[L]++;
        }
    if (!sweep_lists(S.nlevels, S.level_ptr.data(), hm.data(), hk.data(), ns, tk, bp, nt, listed.data()))
        throw Fail{MF_ERR_ARG, "front too large for the sweep task code"};
    // forward: a listed front waits for its listed children only (the others
    // finished in the level launches before the list)
    std::vector<int32_t> need(std::max(ns, 1), 0);
    for (int sl = 0; sl < ns; sl++) {
        if (!listed[sl]) continue;
        const int f = S.level_fronts[sl];
        for (int q = S.child_ptr[f]; q < S.child_ptr[f + 1]; q++)
            if (listed[N->sym->dev->slot_of[S.child_idx[q]]]) need[sl]++;
    }
    mf_num::SweepPlan& P = N->sweep;
    size_t need_ints = 0;
    for (int dir = 0; dir < 2; dir++) need_ints += tk[dir].size() + bp[dir].size() + nt[dir].size();
    need_ints += need.size() + (listed.size() + 3) / 4;
    if (need_ints > P.cap) {
        if (P.d_buf) HIPX(dfree(P.d_buf));
        P.d_buf = nullptr;
        P.cap = 0;
        HIPX(dmalloc((void**)&P.d_buf, sizeof(int32_t) * need_ints));
        P.cap = need_ints;
    }
    if (!P.d_ctr) {
        HIPX(dmalloc((void**)&P.d_ctr, sizeof(int32_t) * 2 * (2 + 3 * (size_t)std::max(ns, 1))));
        HIPX(hmalloc((void**)&P.h_err, sizeof(int32_t) * 2, hipHostMallocDefault));
        P.h_err[0] = P.h_err[1] = 0;
    }
    std::vector<int32_t> host;
    host.reserve(need_ints);
    size_t off[2][3];
    for (int dir = 0; dir < 2; dir++) {
        off[dir][0] = host.size();
        host.insert(host.end(), tk[dir].begin(), tk[dir].end());
        off[dir][1] = host.size();
        host.insert(host.end(), bp[dir].begin(), bp[dir].end());
        off[dir][2] = host.size();
        host.insert(host.end(), nt[dir].begin(), nt[dir].end());
        P.nbund[dir] = (int32_t)bp[dir].size() - 1;
        P.ntasks[dir] = (int64_t)tk[dir].size() / 2;
    }
    const size_t need_off = host.size();
    host.insert(host.end(), need.begin(), need.end());
    const size_t listed_off = host.size();
    host.resize(host.size() + (listed.size() + 3) / 4, 0);
    std::memcpy(host.data() + listed_off, listed.data(), listed.size());
    HIPX(hipMemcpy(P.d_buf, host.data(), sizeof(int32_t) * host.size(), hipMemcpyHostToDevice));
    for (int dir = 0; dir < 2; dir++) {
        P.tasks[dir] = P.d_buf + off[dir][0];
        P.bptr[dir] = P.d_buf + off[dir][1];
        P.ntask[dir] = P.d_buf + off[dir][2];
    }
    P.need = P.d_buf + need_off;
    P.d_listed = (const uint8_t*)(P.d_buf + listed_off);
    if (!N->sweep_grid) {
        int cus = 0;
        HIPX(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, N->device));
        N->sweep_grid = std::max(1, cus) * 3;  // about 48 KB of LDS per work-group: 3 per CU
    }
    P.valid = true;
}

// A persistent sweep that ran into its wait limit (never expected: every wait is
// for a task taken earlier by a running work-group) leaves wrong vectors.
void check_sweep_errors(const mf_num* N) {
    const mf_num::SweepPlan& P = N->sweep;
    if (P.h_err && (P.h_err[0] || P.h_err[1]))
        throw Fail{MF_ERR_DEVICE, "persistent sweep wait limit reached (forward " + std::to_string(P.h_err[0]) +
                                      ", backward " + std::to_string(P.h_err[1]) + ")"};
}

// x = M^{-1} b with the multifrontal factors (forward then backward sweep).
void apply_inverse(mf_num* N, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, hipStream_t st) {
    const Symbolic& S = N->sym->S;
    const DevSym& DS = N->sym->dev->S;
    // with equilibration the factors are of Dr J Dc: x = Dc (Dr J Dc)^{-1} Dr b
    if (N->scaled) {
        const size_t need = (size_t)S.n * nrhs;
        if (need > N->sb_cap) {
            if (N->d_sb) HIPX(dfree(N->d_sb));
            N->d_sb = nullptr;
            HIPX(dmalloc((void**)&N->d_sb, sizeof(double) * need));
            N->sb_cap = need;
        }
        HIPX(launch_diag_scale(S.n, N->d_dr, b, ldb, N->d_sb, S.n, nrhs, st));
        b = N->d_sb;
        ldb = S.n;
    }
    // persistent sweeps for the upper tree (levels >= T), one launch per level and
    // direction below it
    bool hybrid = false;
    if (N->opt.sweep == 1 && S.nlevels > 0) {
        if (!N->sweep.valid) build_sweep_plan(N);
        hybrid = N->sweep.any;
    }
    mf_num::SweepPlan& P = N->sweep;
    const uint8_t* skip = hybrid ? P.d_listed : nullptr;
    auto level_runs = [&](int L) { return !hybrid || P.level_rest[L] > 0; };
    const size_t cstride = 2 + 3 * (size_t)std::max(S.nf, 1);
    int32_t* cf = P.d_ctr;
    int32_t* cb = P.d_ctr ? P.d_ctr + cstride : nullptr;
    constexpr int kCap = 1 << 20;  // polls of one wait (a device-coherent load and a short sleep each): about a second
    if (hybrid) {
        HIPX(launch_fill_i32(cf + 1, 0, st));  // error words (the launches clear everything else)
        HIPX(launch_fill_i32(cb + 1, 0, st));
    }
    int mm = 1;
    for (int p = 0; p < 2; p++)
        for (int L = 0; L < S.nlevels; L++) mm = std::max(mm, N->lvl_mmax[p][L]);
    // vectors of the largest front per right-hand side in dynamic LDS, beside the
    // sweep kernels' static LDS (the staged 64 x 64 diagonal block, at most 32 KB,
    // and small buffers), within the device's limit per block
    int lds_block = 0;
    HIPX(hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, N->device));
    if ((size_t)lds_block <= kSweepStaticLds) throw Fail{MF_ERR_DEVICE, "device LDS per block too small for the sweeps"};
    const size_t budget = (size_t)lds_block - kSweepStaticLds;
    if ((size_t)mm * sizeof(double) > budget)
        throw Fail{MF_ERR_ARG, "front of order " + std::to_string(mm) + " exceeds the solve kernel's LDS budget"};
    for (int c0 = 0; c0 < nrhs;) {
        // right-hand-side chunk so that the largest front's vectors fit in LDS
        int nrc = (int)std::max<size_t>(1, budget / (sizeof(double) * (size_t)mm));
        nrc = std::min(nrc, nrhs - c0);
        nrc = std::min(nrc, kSwRhs);  // the sweep kernels take at most kSwRhs columns per pass
        for (int L = 0; L < S.nlevels; L++) {
            if (!level_runs(L)) continue;
            const int s0 = S.level_ptr[L], cnt = S.level_ptr[L + 1] - s0;
            if (N->lvl_cnt[0][L])
                HIPX(launch_level_fwd<double>(DS, N->d_fn, s0, cnt, 0, b, ldb, N->d_vec, nrhs, c0, nrc,
                                              N->lvl_mmax[0][L], st, skip));
            if (N->lvl_cnt[1][L])
                HIPX(launch_level_fwd<float>(DS, N->d_fn, s0, cnt, 1, b, ldb, N->d_vec, nrhs, c0, nrc,
                                             N->lvl_mmax[1][L], st, skip));
        }
        if (hybrid) {
            HIPX(launch_sweep_persist(true, DS, N->d_fn, P.tasks[0], P.bptr[0], P.nbund[0], P.ntask[0], P.need, cf,
                                      b, ldb, x, ldx, N->d_vec, nrhs, c0, nrc, N->sweep_grid, kCap, st));
            HIPX(launch_sweep_persist(false, DS, N->d_fn, P.tasks[1], P.bptr[1], P.nbund[1], P.ntask[1], P.need, cb,
                                      b, ldb, x, ldx, N->d_vec, nrhs, c0, nrc, N->sweep_grid, kCap, st));
        }
        for (int L = S.nlevels - 1; L >= 0; L--) {
            if (!level_runs(L)) continue;
            const int s0 = S.level_ptr[L], cnt = S.level_ptr[L + 1] - s0;
            if (N->lvl_cnt[0][L])
                HIPX(launch_level_bwd<double>(N->d_fn, s0, cnt, 0, x, ldx, N->d_vec, nrhs, c0, nrc,
                                              N->lvl_mmax[0][L], st, skip));
            if (N->lvl_cnt[1][L])
                HIPX(launch_level_bwd<float>(N->d_fn, s0, cnt, 1, x, ldx, N->d_vec, nrhs, c0, nrc,
                                             N->lvl_mmax[1][L], st, skip));
        }
        c0 += nrc;
    }
    if (hybrid) {
        HIPX(hipMemcpyAsync(P.h_err, cf + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPX(hipMemcpyAsync(P.h_err + 1, cb + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    if (N->scaled) HIPX(launch_diag_scale(S.n, N->d_dc, x, ldx, x, ldx, nrhs, st));
}

double omega_of_bits(unsigned long long b) {
    double w;
    std::memcpy(&w, &b, sizeof(w));
    return w;
}

// r = b - J x; om[seg * nrhs + c] = omega of system seg, right-hand side c, and
// (if eta is given) the normwise backward error
// eta = ||r||_inf / (||J||_inf ||x||_inf + ||b||_inf) at the same positions.
void residual(mf_num* N, const double* b, int64_t ldb, const double* x, int64_t ldx, double* r, int nrhs,
              hipStream_t st, std::vector<double>& om, std::vector<double>* eta = nullptr) {
    const Symbolic& S = N->sym->S;
    const int nseg = (int)S.seg_n.size();
    const int cnt = nrhs * nseg;
    const size_t pneed = residual_part_size(S.n, nrhs);
    if (pneed > N->respart_cap) {
        if (N->d_respart) HIPX(dfree(N->d_respart));
        N->d_respart = nullptr;
        HIPX(dmalloc((void**)&N->d_respart, sizeof(double) * pneed));
        N->respart_cap = pneed;
    }
    HIPX(launch_residual(N->sym->dev->S, N->d_vals, S.n, x, ldx, b, ldb, r, S.n, nrhs, N->d_omega, N->d_respart, st));
    HIPX(hipMemcpyAsync(N->h_omega, N->d_omega, sizeof(unsigned long long) * (eta ? kResQ : 1) * cnt,
                        hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    check_sweep_errors(N);
    om.resize((size_t)cnt);
    for (int q = 0; q < cnt; q++) om[q] = omega_of_bits(N->h_omega[q]);
    if (eta) {
        eta->resize((size_t)cnt);
        for (int q = 0; q < cnt; q++) {
            const double rm = omega_of_bits(N->h_omega[cnt + q]), xm = omega_of_bits(N->h_omega[2 * cnt + q]);
            const double bm = omega_of_bits(N->h_omega[3 * cnt + q]), jm = omega_of_bits(N->h_omega[4 * cnt + q]);
            const double den = jm * xm + bm;
            (*eta)[q] = den > 0.0 ? rm / den : (rm == 0.0 ? 0.0 : INFINITY);
        }
    }
}

// Krylov vectors of nrhs columns: the n x nrhs block (leading dimension n) is
// treated as one long vector whose segment v = c * nseg + s holds system s's rows
// of column c.  Every (system, column) pair is then an independent GMRES
// instance, and the segmented vector kernels run all of them in lockstep.
const DevSym& krylov_view(mf_num* N, int nrhs) {
    const DevSym& DS = N->sym->dev->S;
    if (nrhs == 1) return DS;
    if (N->kv_nrhs == nrhs) return N->kv;
    for (void* p : N->kv_alloc) HIPX(dfree(p));
    N->kv_alloc.clear();
    N->kv_nrhs = 0;
    const Symbolic& S = N->sym->S;
    const int64_t n = S.n;
    const int nseg = (int)S.seg_n.size();
    std::vector<int64_t> r0((size_t)nseg * nrhs), nn((size_t)nseg * nrhs);
    std::vector<int32_t> rs((size_t)n * nrhs);
    for (int c = 0; c < nrhs; c++)
        for (int s = 0; s < nseg; s++) {
            const int v = c * nseg + s;
            r0[v] = (int64_t)c * n + S.seg_row0[s];
            nn[v] = S.seg_n[s];
            std::fill(rs.begin() + r0[v], rs.begin() + r0[v] + nn[v], v);
        }
    int64_t* d_r0 = nullptr;
    int64_t* d_nn = nullptr;
    int32_t* d_rs = nullptr;
    upload(&d_r0, r0);
    N->kv_alloc.push_back(d_r0);
    upload(&d_nn, nn);
    N->kv_alloc.push_back(d_nn);
    upload(&d_rs, rs);
    N->kv_alloc.push_back(d_rs);
    N->kv = DS;
    N->kv.nseg = nseg * nrhs;
    N->kv.seg_row0 = d_r0;
    N->kv.seg_n = d_nn;
    N->kv.row_seg = d_rs;
    N->kv_nrhs = nrhs;
    return N->kv;
}

void ensure_krylov(mf_num* N, int mres, int nrhs) {
    const Symbolic& S = N->sym->S;
    const int64_t len = S.n * nrhs;
    const int nq = (int)S.seg_n.size() * nrhs;
    // V (mres + 1 vectors) | w | trial x | trial r | reduction scratch
    size_t need = (size_t)len * (mres + 4) + (size_t)512 * nq * (mres + 2);
    if (need > N->kry_cap) {
        if (N->d_kry) HIPX(dfree(N->d_kry));
        N->d_kry = nullptr;
        HIPX(dmalloc((void**)&N->d_kry, sizeof(double) * need));
        N->kry_cap = need;
    }
    size_t sneed = (size_t)2 * nq * (mres + 2);
    if (sneed > N->small_cap) {
        if (N->d_small) HIPX(dfree(N->d_small));
        if (N->h_small) HIPX(hfree(N->h_small));
        N->d_small = nullptr;
        N->h_small = nullptr;
        HIPX(dmalloc((void**)&N->d_small, sizeof(double) * sneed));
        HIPX(hmalloc((void**)&N->h_small, sizeof(double) * sneed, hipHostMallocDefault));
        N->small_cap = sneed;
    }
    if (!N->d_ones || N->ones_cap < nq) {
        if (N->d_ones) HIPX(dfree(N->d_ones));
        N->d_ones = nullptr;
        HIPX(dmalloc((void**)&N->d_ones, sizeof(int32_t) * nq));
        std::vector<int32_t> ones(nq, 1);
        HIPX(hipMemcpy(N->d_ones, ones.data(), sizeof(int32_t) * nq, hipMemcpyHostToDevice));
        N->ones_cap = nq;
    }
}

// Per-segment dots of V[:, 0:nv] with w (segments of VS), returned on the host:
// out[seg * stride + i].
void mdot_host(mf_num* N, const DevSym& VS, const double* V, int64_t ldv, int nv, const double* w, double* part,
               int stride, std::vector<double>& out, hipStream_t st) {
    HIPX(launch_mdot(VS, V, ldv, nv, w, part, N->d_small, stride, st));
    HIPX(hipMemcpyAsync(N->h_small, N->d_small, sizeof(double) * VS.nseg * stride, hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    check_sweep_errors(N);
    out.assign(N->h_small, N->h_small + (size_t)VS.nseg * stride);
}

// per-system coefficients to the device (second half of the small buffer)
double* put_small(mf_num* N, const std::vector<double>& v, hipStream_t st) {
    const size_t off = N->small_cap / 2;
    for (size_t i = 0; i < v.size(); i++) N->h_small[off + i] = v[i];
    HIPX(hipMemcpyAsync(N->d_small + off, N->h_small + off, sizeof(double) * v.size(), hipMemcpyHostToDevice, st));
    return N->d_small + off;
}

// y = R^{-1} g of the first jq columns of one system's rotated Hessenberg matrix.
void hessenberg_solve(const std::vector<double>& Hq, const std::vector<double>& gq, int jq, int ldh, double* y) {
    for (int i = jq - 1; i >= 0; i--) {
        double t = gq[i];
        for (int k = i + 1; k < jq; k++) t -= Hq[(size_t)i + (size_t)k * ldh] * y[k];
        const double rii = Hq[(size_t)i + (size_t)i * ldh];
        y[i] = rii != 0.0 ? t / rii : 0.0;
    }
}

// GMRES(m) on M^{-1} J d = M^{-1} r, one instance per (system, right-hand side)
// of the batch, all run in lockstep on the concatenated n x nrhs vectors (ld n):
// one multi-column sweep pair and one multi-column SpMV per inner step serve every
// instance.  Classical Gram-Schmidt with one reorthogonalization, Givens
// rotations on the host.  An instance's numbers depend only on its own rows and
// column.  It stops when its preconditioned residual falls by tol, or, with
// target > 0, as soon as the refined iterate x + d of the current Krylov space
// meets the componentwise backward-error target (its true residual against b, one
// SpMV per check: much cheaper than the sweep pair each further iteration or
// outer step costs).  act and the result are in residual order (seg * nrhs + c);
// returns the inner iterations per instance.
std::vector<int> gmres_correction(mf_num* N, const double* r, double* d, int nrhs, int mres, double tol,
                                  const std::vector<char>& act, hipStream_t st, const double* b, int64_t ldb,
                                  const double* x, int64_t ldx, double target) {
    const Symbolic& S = N->sym->S;
    const int64_t n = S.n;
    const int nseg = (int)S.seg_n.size();
    const int nq = nseg * nrhs;
    const int64_t len = n * nrhs;
    const DevSym& DS = N->sym->dev->S;
    const DevSym& VS = krylov_view(N, nrhs);
    const int stride = mres + 2;
    double* V = N->d_kry;
    double* w = V + (size_t)len * (mres + 1);
    double* xt = w + len;
    double* rt = xt + len;
    double* part = rt + len;
    auto ro = [&](int v) { return (v % nseg) * nrhs + v / nseg; };  // instance -> residual order
    std::vector<int> iters(nq, 0);
    apply_inverse(N, r, n, w, n, nrhs, st);  // w = M^{-1} r
    std::vector<double> dots, beta(nq), coef((size_t)nq * stride, 0.0);
    mdot_host(N, VS, w, len, 1, w, part, stride, dots, st);
    std::vector<char> live(nq, 0);
    for (int q = 0; q < nq; q++) {
        beta[q] = std::sqrt(dots[(size_t)q * stride]);
        live[q] = act[ro(q)] && beta[q] > 0.0 && std::isfinite(beta[q]);
        coef[(size_t)q * stride] = live[q] ? 1.0 / beta[q] : 0.0;
    }
    HIPX(launch_fill(d, 0.0, len, st));
    HIPX(launch_scale(VS, V, w, put_small(N, coef, st), stride, len, st));
    std::vector<std::vector<double>> H(nq, std::vector<double>((size_t)(mres + 1) * mres, 0.0)), cs(nq), sn(nq),
        g(nq);
    std::vector<int> jdone(nq, 0);
    for (int q = 0; q < nq; q++) {
        cs[q].assign(mres, 0.0);
        sn[q].assign(mres, 0.0);
        g[q].assign(mres + 1, 0.0);
        g[q][0] = beta[q];
    }
    std::vector<char> running = live;
    std::vector<double> h((size_t)nq * stride), h2;
    for (int j = 0; j < mres; j++) {
        bool any = false;
        for (int q = 0; q < nq; q++) any = any || running[q];
        if (!any) break;
        double* vj = V + (size_t)len * j;
        double* vj1 = V + (size_t)len * (j + 1);
        HIPX(launch_spmv(DS, N->d_vals, n, vj, n, vj1, n, nrhs, st));  // vj1 = J vj (temporary)
        apply_inverse(N, vj1, n, w, n, nrhs, st);                       // w = M^{-1} J vj
        mdot_host(N, VS, V, len, j + 1, w, part, stride, h, st);
        HIPX(launch_vsub(VS, w, V, len, j + 1, put_small(N, h, st), stride, len, st));
        mdot_host(N, VS, V, len, j + 1, w, part, stride, h2, st);  // reorthogonalize
        HIPX(launch_vsub(VS, w, V, len, j + 1, put_small(N, h2, st), stride, len, st));
        for (size_t i = 0; i < h.size(); i++) h[i] += h2[i];
        mdot_host(N, VS, w, len, 1, w, part, stride, dots, st);
        for (int q = 0; q < nq; q++) {
            const double hn = std::sqrt(dots[(size_t)q * stride]);
            h[(size_t)q * stride + j + 1] = hn;
            coef[(size_t)q * stride] = hn > 0.0 ? 1.0 / hn : 0.0;
        }
        HIPX(launch_scale(VS, vj1, w, put_small(N, coef, st), stride, len, st));
        for (int q = 0; q < nq; q++) {
            if (!running[q]) continue;
            double* hq = h.data() + (size_t)q * stride;
            const double hn = hq[j + 1];
            for (int i = 0; i < j; i++) {
                const double t = cs[q][i] * hq[i] + sn[q][i] * hq[i + 1];
                hq[i + 1] = -sn[q][i] * hq[i] + cs[q][i] * hq[i + 1];
                hq[i] = t;
            }
            const double den = std::hypot(hq[j], hq[j + 1]);
            cs[q][j] = den > 0 ? hq[j] / den : 1.0;
            sn[q][j] = den > 0 ? hq[j + 1] / den : 0.0;
            hq[j] = den;
            hq[j + 1] = 0.0;
            g[q][j + 1] = -sn[q][j] * g[q][j];
            g[q][j] = cs[q][j] * g[q][j];
            for (int i = 0; i <= j; i++) H[q][(size_t)i + (size_t)j * (mres + 1)] = hq[i];
            jdone[q] = j + 1;
            if (std::fabs(g[q][j + 1]) <= tol * beta[q] || !(hn > 0.0)) running[q] = 0;
        }
        if (target > 0.0 && b && x) {
            // the check is worth its SpMV only once some instance's preconditioned
            // residual has fallen to within kCheckGate of the target (on these
            // Jacobians omega met the target only below that, and a check costs
            // about a sixth of the sweep pair that one more inner step costs)
            constexpr double kCheckGate = 1e4;
            bool anyr = false;
            for (int q = 0; q < nq; q++)
                anyr = anyr || (running[q] && std::fabs(g[q][j + 1]) <= kCheckGate * target * beta[q]);
            if (anyr) {
                // trial iterate x + V y of every instance still running (the others add 0)
                std::fill(coef.begin(), coef.end(), 0.0);
                for (int q = 0; q < nq; q++)
                    if (running[q]) hessenberg_solve(H[q], g[q], j + 1, mres + 1, coef.data() + (size_t)q * stride);
                HIPX(launch_fill(d, 0.0, len, st));
                HIPX(launch_vadd(VS, d, V, len, j + 1, put_small(N, coef, st), stride, len, st));
                HIPX(hipMemcpy2DAsync(xt, sizeof(double) * n, x, sizeof(double) * ldx, sizeof(double) * n, nrhs,
                                      hipMemcpyDeviceToDevice, st));
                HIPX(launch_axpy(DS, n, xt, n, d, n, N->d_ones, nrhs, st));
                std::vector<double> omt;
                residual(N, b, ldb, xt, n, rt, nrhs, st, omt);
                // each instance acts on its own gate only, so that its iterations do
                // not depend on the systems or columns it runs beside
                for (int q = 0; q < nq; q++)
                    if (running[q] && std::fabs(g[q][j + 1]) <= kCheckGate * target * beta[q] && omt[ro(q)] <= target)
                        running[q] = 0;
            }
        }
    }
    // y = R^{-1} g per instance, d = V y
    std::fill(coef.begin(), coef.end(), 0.0);
    int jmax = 0;
    std::vector<int> out(nq, 0);
    for (int q = 0; q < nq; q++) {
        if (!live[q]) continue;
        const int jq = jdone[q];
        out[ro(q)] = jq;
        jmax = std::max(jmax, jq);
        hessenberg_solve(H[q], g[q], jq, mres + 1, coef.data() + (size_t)q * stride);
    }
    HIPX(launch_fill(d, 0.0, len, st));  // (trial iterates left their d behind)
    if (jmax > 0) HIPX(launch_vadd(VS, d, V, len, jmax, put_small(N, coef, st), stride, len, st));
    return out;
}

// Solve and refine.  b, x: n x nrhs (ld) over the whole (possibly batched) system.
// Every system of a batch refines on its own: its update stops as soon as its own
// omega meets the target, so its result equals the one it gets when solved alone.
void do_solve(mf_num* N, const double* b, double* x, int nrhs, int64_t ld, hipStream_t st, mf_solve_info* info) {
    const Symbolic& S = N->sym->S;
    const mf_options& o = N->opt;
    const int64_t n = S.n;
    const int nseg = (int)S.seg_n.size();
    ensure_solve_buffers(N, nrhs);
    double* r = N->d_work;
    double* dv = N->d_work + (size_t)n * nrhs;
    apply_inverse(N, b, ld, x, ld, nrhs, st);
    std::vector<double> om, et;
    residual(N, b, ld, x, ld, r, nrhs, st, om, &et);
    N->seg_info.assign(nseg, mf_solve_info{});
    for (int q = 0; q < nseg; q++) {
        mf_solve_info& si = N->seg_info[q];
        for (int c = 0; c < nrhs; c++) {
            si.omega0 = std::max(si.omega0, om[(size_t)q * nrhs + c]);
            si.eta = std::max(si.eta, et[(size_t)q * nrhs + c]);
        }
        si.omega = si.omega0;
        si.delayed_pivots = q < (int)N->seg_delayed.size() ? N->seg_delayed[q] : 0;
    }
    std::vector<char> active((size_t)nseg * nrhs);
    // with a replaced operator the factors are only a preconditioner: plain
    // refinement may diverge, so the correction is always the Krylov one
    const int refine = (N->stale && o.refine > 0) ? 2 : o.refine;
    // refine 3: classical steps while each cuts the worst active omega at least
    // tenfold, the Krylov correction from the first step that does not
    bool krylov = refine == 2;
    int it = 0;
    while (refine > 0 && it < o.max_outer) {
        bool any = false;
        double before = 0.0;
        for (size_t q = 0; q < active.size(); q++) {
            active[q] = !(om[q] <= o.target_omega);
            any = any || active[q];
            if (active[q]) before = std::max(before, om[q] == om[q] ? om[q] : INFINITY);
        }
        if (!any) break;
        const bool classical = refine == 1 || (refine == 3 && !krylov);
        if (classical) {
            apply_inverse(N, r, n, dv, n, nrhs, st);
        } else {
            const int mres = std::max(1, std::min(o.gmres_m, 200));
            ensure_krylov(N, mres, nrhs);
            const std::vector<int> its = gmres_correction(N, r, dv, nrhs, mres, o.gmres_tol, active, st, b, ld, x, ld,
                                                          o.target_omega);
            for (int q = 0; q < nseg; q++)
                for (int c = 0; c < nrhs; c++) N->seg_info[q].inner_iters += its[(size_t)q * nrhs + c];
        }
        for (size_t q = 0; q < active.size(); q++) N->h_active[q] = active[q];
        HIPX(hipMemcpyAsync(N->d_active, N->h_active, sizeof(int32_t) * active.size(), hipMemcpyHostToDevice, st));
        HIPX(launch_axpy(N->sym->dev->S, n, x, ld, dv, n, N->d_active, nrhs, st));
        residual(N, b, ld, x, ld, r, nrhs, st, om, &et);
        it++;
        if (refine == 3 && classical) {
            double after = 0.0;
            for (size_t q = 0; q < active.size(); q++)
                if (active[q]) after = std::max(after, om[q] == om[q] ? om[q] : INFINITY);
            if (!(after <= 0.1 * before)) krylov = true;
        }
        for (int q = 0; q < nseg; q++) {
            bool stepped = false;
            double wq = 0.0, eq = 0.0;
            for (int c = 0; c < nrhs; c++) {
                stepped = stepped || active[(size_t)q * nrhs + c];
                wq = std::max(wq, om[(size_t)q * nrhs + c]);
                eq = std::max(eq, et[(size_t)q * nrhs + c]);
            }
            if (stepped) N->seg_info[q].outer_iters++;
            N->seg_info[q].omega = wq;
            N->seg_info[q].eta = eq;
        }
    }
    mf_solve_info inf{};
    for (int q = 0; q < nseg; q++) {
        inf.omega = std::max(inf.omega, N->seg_info[q].omega);
        inf.omega0 = std::max(inf.omega0, N->seg_info[q].omega0);
        inf.eta = std::max(inf.eta, N->seg_info[q].eta);
        inf.outer_iters = std::max(inf.outer_iters, N->seg_info[q].outer_iters);
        inf.inner_iters += N->seg_info[q].inner_iters;
        inf.delayed_pivots += N->seg_info[q].delayed_pivots;
    }
    if (info) *info = inf;
    if (!(inf.omega <= o.target_omega) && refine > 0)
        throw Fail{MF_ERR_NOT_CONVERGED, "refinement stopped at omega = " + std::to_string(inf.omega)};
}

// Solve with the fallback of the reduced-precision path: when GMRES-IR on FP32 or
// BF16 factors stops above the target, the handle is factored again in FP64 (from
// its own copy of the values) and the system solved with FP64 refinement.
void solve_with_fallback(mf_num* N, const double* b, double* x, int nrhs, int64_t ld, hipStream_t st,
                         mf_solve_info* info) {
    try {
        do_solve(N, b, x, nrhs, ld, st, info);
        return;
    } catch (const Fail& f) {
        if (f.st != MF_ERR_NOT_CONVERGED || !N->opt.fallback || (N->opt.prec == MF_FP64 && !N->stale)) throw;
    }
    N->opt.prec = MF_FP64;
    N->opt.refine = 1;
    N->opt.plan = 0;
    N->opt.tune = 0;
    N->factored = false;
    do_factor(N, N->d_vals, st);
    do_solve(N, b, x, nrhs, ld, st, info);
    for (auto& si : N->seg_info) si.fp64_fallback = 1;
    if (info) info->fp64_fallback = 1;
}

}  // namespace

extern "C" {

void mf_default_options(mf_options* o) {
    if (!o) return;
    o->prec = MF_FP64;
    o->pivot_u = 0.01;
    o->leaf_max = 64;
    o->target_omega = 1e-12;
    o->max_outer = 10;
    o->gmres_m = 30;
    o->gmres_tol = 1e-12;
    o->refine = -1;
    o->panel_nb = 32;
    o->profile = 0;
    o->scale = 1;
    o->plan = 0;
    o->tune = 0;
    o->fallback = 1;
    o->sweep = 1;
}

const char* mf_last_error(void) { return g_err.c_str(); }

mf_status mf_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t nroot, const int32_t* root_idx,
                     const mf_options* opt, mf_sym_t* out) {
    if (!out) return fail(MF_ERR_ARG, "out is null");
    *out = nullptr;
    try {
        auto h = std::make_unique<mf_sym>();
        if (opt)
            h->opt = *opt;
        else
            mf_default_options(&h->opt);
        analyze_pattern(h->S, n, rowptr, colind, nroot, root_idx, h->opt.leaf_max);
        *out = h.release();
        return MF_OK;
    } catch (const std::invalid_argument& e) {
        return fail(MF_ERR_ARG, e.what());
    } catch (const std::bad_alloc&) {
        return fail(MF_ERR_OOM, "host allocation failed in mf_analyze");
    } catch (const std::exception& e) {
        return fail(MF_ERR_ARG, e.what());
    }
}

mf_status mf_symbolic_export(mf_sym_t h, mf_symbolic_view* v) {
    if (!h || h->magic != kSymMagic || !v) return fail(MF_ERR_ARG, "bad symbolic handle");
    const Symbolic& S = h->S;
    v->n = S.n;
    v->nfronts = S.nf;
    v->leaf_max = S.leaf_max;
    v->spec_version = kSpecVersion;
    v->nlevels = S.nlevels;
    v->perm = S.perm.data();
    v->front_ptr = S.front_ptr.data();
    v->front_parent = S.front_parent.data();
    v->rows_ptr = S.rows_ptr.data();
    v->rows = S.rows.data();
    v->var_etree = S.var_etree.data();
    v->nominal_flops = S.nominal_flops;
    v->nominal_nnz_lu = S.nominal_nnz_lu;
    return MF_OK;
}

static mf_status factor_common(mf_sym_t h, const double* values_dev, const double* const* seg_values,
                               const mf_options* opt, void* stream, mf_num_t* inout) {
    if (!h || h->magic != kSymMagic) return fail(MF_ERR_ARG, "bad symbolic handle");
    if (!inout) return fail(MF_ERR_ARG, "inout is null");
    if (!seg_values && !values_dev && h->S.nnz > 0) return fail(MF_ERR_ARG, "values_dev is null");
    if (seg_values)
        for (size_t q = 0; q < h->S.seg_n.size(); q++)
            if (!seg_values[q] && h->S.seg_n[q] > 0) return fail(MF_ERR_ARG, "values_dev[i] is null");
    mf_num* N = *inout;
    if (N && (N->magic != kNumMagic || N->sym != h))
        return fail(MF_ERR_PATTERN, "numeric handle belongs to another symbolic handle");
    std::unique_ptr<mf_num> fresh;
    if (!N) {
        fresh = std::make_unique<mf_num>();
        N = fresh.get();
        N->sym = h;
    }
    N->opt = h->opt;
    if (opt) {
        N->opt.prec = opt->prec;
        N->opt.pivot_u = opt->pivot_u;
        N->opt.target_omega = opt->target_omega;
        N->opt.max_outer = opt->max_outer;
        N->opt.gmres_m = opt->gmres_m;
        N->opt.gmres_tol = opt->gmres_tol;
        N->opt.refine = opt->refine;
        N->opt.panel_nb = opt->panel_nb;
        N->opt.profile = opt->profile;
        N->opt.scale = opt->scale;
        N->opt.plan = opt->plan;
        N->opt.tune = opt->tune;
        N->opt.fallback = opt->fallback;
        N->opt.sweep = opt->sweep;
    }
    resolve_refine(N->opt);
    if (N->opt.prec < MF_FP64 || N->opt.prec > MF_BF16) return fail(MF_ERR_ARG, "bad precision");
    if (N->opt.refine > 3) return fail(MF_ERR_ARG, "bad refinement mode (0..3, or -1 for the default)");
    if (!(N->opt.pivot_u >= 0.0 && N->opt.pivot_u <= 1.0)) return fail(MF_ERR_ARG, "pivot_u must be in [0, 1]");
    if (N->opt.scale < 0 || N->opt.scale > 64) return fail(MF_ERR_ARG, "scale must be in [0, 64] sweeps");
    if (N->opt.sweep < 0 || N->opt.sweep > 1) return fail(MF_ERR_ARG, "sweep must be 0 or 1");
    N->factored = false;
    N->last_stream = (hipStream_t)stream;
    try {
        HIPX(hipGetDevice(&N->device));
        do_factor(N, values_dev, (hipStream_t)stream, seg_values);
        HIPX(hipStreamSynchronize((hipStream_t)stream));  // every call returns with its stream idle
    } catch (const Fail& f) {
        // also on errors (a level's Schur update may still be running when the
        // bookkeeping read after its panel rounds reports a singular root)
        (void)hipStreamSynchronize((hipStream_t)stream);
        if (fresh) *inout = fresh.release();  // keep the handle so the caller can release it
        return fail(f.st, f.msg);
    } catch (const std::bad_alloc&) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        if (fresh) *inout = fresh.release();
        return fail(MF_ERR_OOM, "host allocation failed in mf_factor");
    }
    if (fresh) *inout = fresh.release();
    return MF_OK;
}

mf_status mf_factor(mf_sym_t h, const double* values_dev, const mf_options* opt, void* stream, mf_num_t* inout) {
    return factor_common(h, values_dev, nullptr, opt, stream, inout);
}

mf_status mf_batch_analyze(int32_t count, const mf_sym_t* syms, mf_sym_t* out) {
    if (!out) return fail(MF_ERR_ARG, "out is null");
    *out = nullptr;
    if (count < 1 || !syms) return fail(MF_ERR_ARG, "count must be >= 1");
    std::vector<const Symbolic*> parts;
    for (int32_t i = 0; i < count; i++) {
        if (!syms[i] || syms[i]->magic != kSymMagic) return fail(MF_ERR_ARG, "bad symbolic handle in batch");
        if (syms[i]->S.seg_n.size() != 1) return fail(MF_ERR_ARG, "nested batches are not supported");
        parts.push_back(&syms[i]->S);
    }
    try {
        auto h = std::make_unique<mf_sym>();
        h->opt = syms[0]->opt;
        // With a device present, each system's pattern data goes to the device
        // once (kept with its handle, shared with every batch it joins) and the
        // batch's maps are concatenated there; the host merges only per-front data.
        int dev = -1, ndev = 0;
        const bool light = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 && hipGetDevice(&dev) == hipSuccess;
        if (light) {
            for (int32_t i = 0; i < count; i++) {
                mf_sym* p = const_cast<mf_sym*>(syms[i]);
                ensure_device_symbolic(p);
                h->parts_dev.push_back(p->dev);
            }
        } else {
            (void)hipGetLastError();  // no device: the host merge below needs none
        }
        merge_symbolic(h->S, parts, light);
        *out = h.release();
        return MF_OK;
    } catch (const Fail& f) {
        return fail(f.st, f.msg);
    } catch (const std::invalid_argument& e) {
        return fail(MF_ERR_ARG, e.what());
    } catch (const std::bad_alloc&) {
        return fail(MF_ERR_OOM, "host allocation failed in mf_batch_analyze");
    }
}

mf_status mf_factor_batched(mf_sym_t batch, const double* const* values_dev, const mf_options* opt, void* stream,
                            mf_num_t* inout) {
    if (!values_dev) return fail(MF_ERR_ARG, "values_dev is null");
    return factor_common(batch, nullptr, values_dev, opt, stream, inout);
}

mf_status mf_get_factor_info(mf_num_t N, mf_factor_info* info) {
    if (!N || N->magic != kNumMagic || !info) return fail(MF_ERR_ARG, "bad numeric handle");
    if (!N->factored) return fail(MF_ERR_STATE, "not factored");
    *info = N->info;
    return MF_OK;
}

mf_status mf_solve(mf_num_t N, const double* b_dev, double* x_dev, int32_t nrhs, int64_t ld, void* stream,
                   mf_solve_info* info) {
    if (!N || N->magic != kNumMagic) return fail(MF_ERR_ARG, "bad numeric handle");
    if (!N->factored) return fail(MF_ERR_STATE, "mf_solve before a successful mf_factor");
    const int64_t n = N->sym->S.n;
    if (nrhs < 0) return fail(MF_ERR_ARG, "bad nrhs");
    if (nrhs == 0 || n == 0) {
        if (info) *info = mf_solve_info{};
        return MF_OK;
    }
    if (ld < n) return fail(MF_ERR_ARG, "ld < n");
    if (!b_dev || !x_dev || b_dev == x_dev) return fail(MF_ERR_ARG, "b_dev and x_dev must be distinct device buffers");
    N->last_stream = (hipStream_t)stream;
    try {
        solve_with_fallback(N, b_dev, x_dev, nrhs, ld, (hipStream_t)stream, info);
        HIPX(hipStreamSynchronize((hipStream_t)stream));
    } catch (const Fail& f) {
        return fail(f.st, f.msg);
    } catch (const std::bad_alloc&) {
        return fail(MF_ERR_OOM, "host allocation failed in mf_solve");
    }
    return MF_OK;
}

static mf_status set_operator_common(mf_num_t N, const double* values_dev, const double* const* seg_values,
                                     const mf_options* opt, void* stream) {
    if (!N || N->magic != kNumMagic) return fail(MF_ERR_ARG, "bad numeric handle");
    if (!N->factored) return fail(MF_ERR_STATE, "mf_set_operator before a successful factorization");
    const Symbolic& S = N->sym->S;
    const bool batch = S.seg_n.size() > 1;
    if (batch != (seg_values != nullptr))
        return fail(MF_ERR_ARG, batch ? "a batch handle takes mf_set_operator_batched"
                                      : "a single-system handle takes mf_set_operator");
    if (!seg_values && !values_dev && S.nnz > 0) return fail(MF_ERR_ARG, "values_dev is null");
    if (seg_values)
        for (size_t q = 0; q < S.seg_n.size(); q++)
            if (!seg_values[q] && S.seg_n[q] > 0) return fail(MF_ERR_ARG, "values_dev[i] is null");
    if (opt) {
        if (!(opt->target_omega > 0.0) || opt->max_outer < 0 || opt->gmres_m < 1 || !(opt->gmres_tol >= 0.0)
            || opt->refine > 3)
            return fail(MF_ERR_ARG, "bad refinement options");
        N->opt.target_omega = opt->target_omega;
        N->opt.max_outer = opt->max_outer;
        N->opt.gmres_m = opt->gmres_m;
        N->opt.gmres_tol = opt->gmres_tol;
        N->opt.fallback = opt->fallback;
        if (opt->refine >= 0) N->opt.refine = opt->refine;
    }
    try {
        const hipStream_t st = (hipStream_t)stream;
        load_values(N, values_dev, seg_values, st);
        HIPX(hipStreamSynchronize(st));
        N->stale = true;
        check_finite(N);
    } catch (const Fail& f) {
        N->factored = false;  // the operator copy is unusable: factor again before solving
        return fail(f.st, f.msg);
    } catch (const std::bad_alloc&) {
        N->factored = false;
        return fail(MF_ERR_OOM, "host allocation failed in mf_set_operator");
    }
    return MF_OK;
}

mf_status mf_set_operator(mf_num_t N, const double* values_dev, const mf_options* opt, void* stream) {
    return set_operator_common(N, values_dev, nullptr, opt, stream);
}

mf_status mf_set_operator_batched(mf_num_t N, const double* const* values_dev, const mf_options* opt, void* stream) {
    if (!values_dev) return fail(MF_ERR_ARG, "values_dev is null");
    return set_operator_common(N, nullptr, values_dev, opt, stream);
}

// ---------------------------------------------------------------- no-allocation solve
// Callers that cannot allocate (graph capture, tight serving loops) get the solve's
// scratch from one statically sized device array per GPU instead of the handle's
// buffers.  Host code never takes the array's name as a device address: it asks
// the runtime for this GPU's copy once and keeps that pointer.
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchMaxDevices = 64;
constexpr int kScratchMaxCounts = 4096;  // (system, right-hand side) pairs
double* g_scratch_ptr[kScratchMaxDevices] = {};
unsigned long long g_host_omega[kResQ * kScratchMaxCounts];  // readback staging (pageable, static)
int32_t g_host_active[kScratchMaxCounts];
}  // namespace
}  // extern "C"

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
// This device's copy of the scratch array (looked up once per device).
double* scratch_for_current_device(int* dev_out) {
    int dev = 0;
    HIPX(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchMaxDevices) throw Fail{MF_ERR_DEVICE, "device index beyond the scratch table"};
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Fail{MF_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_ptr[dev] = (double*)p;
    }
    *dev_out = dev;
    return g_scratch_ptr[dev];
}

// Carve the solve's buffers out of the scratch array for the duration of one
// call; the handle's own buffers (and their capacities) are put back afterwards.
struct ScratchSolve {
    mf_num* N;
    double *vec, *work, *sb, *respart;
    unsigned long long *omega, *homega;
    int32_t *active, *hactive;
    size_t vec_cap, work_cap, sb_cap, respart_cap;
    int omega_cap;
    int sweep;
    explicit ScratchSolve(mf_num* n)
        : N(n), vec(n->d_vec), work(n->d_work), sb(n->d_sb), respart(n->d_respart), omega(n->d_omega),
          homega(n->h_omega), active(n->d_active), hactive(n->h_active), vec_cap(n->vec_cap), work_cap(n->work_cap),
          sb_cap(n->sb_cap), respart_cap(n->respart_cap), omega_cap(n->omega_cap), sweep(n->opt.sweep) {}
    ~ScratchSolve() {
        N->d_vec = vec;
        N->d_work = work;
        N->d_sb = sb;
        N->d_respart = respart;
        N->d_omega = omega;
        N->h_omega = homega;
        N->d_active = active;
        N->h_active = hactive;
        N->vec_cap = vec_cap;
        N->work_cap = work_cap;
        N->sb_cap = sb_cap;
        N->respart_cap = respart_cap;
        N->omega_cap = omega_cap;
        N->opt.sweep = sweep;
    }
};
}  // namespace

extern "C" {

mf_status mf_solve_noalloc(mf_num_t N, const double* b_dev, double* x_dev, int32_t nrhs, int64_t ld, void* stream,
                           mf_solve_info* info) {
    if (!N || N->magic != kNumMagic) return fail(MF_ERR_ARG, "bad numeric handle");
    if (!N->factored) return fail(MF_ERR_STATE, "mf_solve_noalloc before a successful mf_factor");
    const Symbolic& S = N->sym->S;
    const int64_t n = S.n;
    if (nrhs < 0) return fail(MF_ERR_ARG, "bad nrhs");
    if (nrhs == 0 || n == 0) {
        if (info) *info = mf_solve_info{};
        return MF_OK;
    }
    if (ld < n) return fail(MF_ERR_ARG, "ld < n");
    if (!b_dev || !x_dev || b_dev == x_dev) return fail(MF_ERR_ARG, "b_dev and x_dev must be distinct device buffers");
    if (N->opt.refine > 1 || (N->stale && N->opt.refine > 0))
        return fail(MF_ERR_ARG, "mf_solve_noalloc refines with FP64 iterative refinement only (refine 0 or 1, "
                                "operator not replaced): GMRES-IR needs its Krylov basis; use mf_solve");
    const int nseg = (int)S.seg_n.size();
    const int cnt = nseg * nrhs;
    if (cnt > kScratchMaxCounts) return fail(MF_ERR_ARG, "too many (system, right-hand side) pairs for mf_solve_noalloc");
    auto al = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
    const size_t b_vec = al(sizeof(double) * (size_t)std::max<int64_t>(N->vec_len, 1) * nrhs);
    const size_t b_work = al(sizeof(double) * (size_t)n * nrhs * 2);
    const size_t b_sb = N->scaled ? al(sizeof(double) * (size_t)n * nrhs) : 0;
    const size_t b_part = al(sizeof(double) * residual_part_size(n, nrhs));
    const size_t b_om = al(sizeof(unsigned long long) * kResQ * cnt);
    const size_t b_act = al(sizeof(int32_t) * cnt);
    const size_t total = b_vec + b_work + b_sb + b_part + b_om + b_act;
    if (total > kScratchBytes)
        return fail(MF_ERR_ARG, "mf_solve_noalloc needs " + std::to_string(total) + " bytes of scratch, above its " +
                                    std::to_string(kScratchBytes) + "-byte limit (use mf_solve)");
    try {
        int dev = 0;
        char* base = (char*)scratch_for_current_device(&dev);
        ScratchSolve keep(N);  // restores the handle's buffers on every exit
        size_t off = 0;
        auto take = [&](size_t bytes) {
            char* p = base + off;
            off += bytes;
            return p;
        };
        N->d_vec = (double*)take(b_vec);
        N->vec_cap = b_vec / sizeof(double);
        N->d_work = (double*)take(b_work);
        N->work_cap = b_work / sizeof(double);
        if (N->scaled) {
            N->d_sb = (double*)take(b_sb);
            N->sb_cap = b_sb / sizeof(double);
        }
        N->d_respart = (double*)take(b_part);
        N->respart_cap = b_part / sizeof(double);
        N->d_omega = (unsigned long long*)take(b_om);
        N->h_omega = g_host_omega;
        N->d_active = (int32_t*)take(b_act);
        N->h_active = g_host_active;
        N->omega_cap = cnt;
        N->opt.sweep = 0;  // the persistent sweeps keep task lists in handle memory
        N->last_stream = (hipStream_t)stream;
        do_solve(N, b_dev, x_dev, nrhs, ld, (hipStream_t)stream, info);
        HIPX(hipStreamSynchronize((hipStream_t)stream));
    } catch (const Fail& f) {
        return fail(f.st, f.msg);
    } catch (const std::bad_alloc&) {
        return fail(MF_ERR_OOM, "host allocation failed in mf_solve_noalloc");
    }
    return MF_OK;
}

mf_status mf_solve_batched(mf_num_t N, const double* const* b_dev, double* const* x_dev, const int32_t* nrhs,
                           void* stream, mf_solve_info* info) {
    if (!N || N->magic != kNumMagic) return fail(MF_ERR_ARG, "bad numeric handle");
    if (!N->factored) return fail(MF_ERR_STATE, "mf_solve_batched before a successful mf_factor_batched");
    if (!b_dev || !x_dev) return fail(MF_ERR_ARG, "bad arguments");
    const Symbolic& S = N->sym->S;
    const int nseg = (int)S.seg_n.size();
    int nmax = 0;
    bool ragged = false;
    for (int q = 0; q < nseg; q++) {
        const int nr = nrhs ? nrhs[q] : 1;
        if (nr < 0) return fail(MF_ERR_ARG, "nrhs[" + std::to_string(q) + "] < 0");
        ragged = ragged || (q > 0 && nr != (nrhs ? nrhs[0] : 1));
        nmax = std::max(nmax, nr);
        if (S.seg_n[q] > 0 && nr > 0 && (!b_dev[q] || !x_dev[q] || b_dev[q] == x_dev[q]))
            return fail(MF_ERR_ARG, "b_dev[i] and x_dev[i] must be distinct device buffers");
    }
    if (info)
        for (int q = 0; q < nseg; q++) info[q] = mf_solve_info{};
    if (nmax == 0 || S.n == 0) return MF_OK;
    hipStream_t st = (hipStream_t)stream;
    N->last_stream = st;
    try {
        const size_t need = (size_t)S.n * nmax * 2;
        if (need > N->cat_cap) {
            if (N->d_cat) HIPX(dfree(N->d_cat));
            N->d_cat = nullptr;
            HIPX(dmalloc((void**)&N->d_cat, sizeof(double) * need));
            N->cat_cap = need;
        }
        double* B = N->d_cat;
        double* X = N->d_cat + (size_t)S.n * nmax;
        // systems with fewer right-hand sides get zero columns: their solution is
        // exactly zero with omega 0, so they never refine
        if (ragged) HIPX(launch_fill(B, 0.0, S.n * nmax, st));
        // every system's columns in (one gather launch) and out (one scatter launch)
        std::vector<SegCopy> gin;
        std::vector<SegOut> sout;
        for (int q = 0; q < nseg; q++) {
            const int nr = nrhs ? nrhs[q] : 1;
            for (int c = 0; c < nr && S.seg_n[q]; c++) {
                const int64_t col = (int64_t)c * S.n + S.seg_row0[q], own = (int64_t)c * S.seg_n[q];
                gin.push_back(SegCopy{b_dev[q] + own, col, S.seg_n[q], 0});
                sout.push_back(SegOut{x_dev[q] + own, col, S.seg_n[q]});
            }
        }
        seg_staging(N, SegLists::need<SegCopy>(gin.size()) + SegLists::need<SegOut>(sout.size()));
        size_t off = 0;
        const SegCopy* d_gin = nullptr;
        const SegOut* d_sout = nullptr;
        const int64_t *d_gst = nullptr, *d_sst = nullptr;
        const int64_t ntot = put_segments(N, off, gin, &d_gin, &d_gst);
        put_segments(N, off, sout, &d_sout, &d_sst);
        if (!gin.empty()) {
            HIPX(hipMemcpyAsync(N->d_seg, N->h_seg, off, hipMemcpyHostToDevice, st));
            HIPX(launch_seg_copy<double>(d_gin, d_gst, (int)gin.size(), ntot, B, st));
        }
        mf_status rc = MF_OK;
        std::string msg;
        try {
            solve_with_fallback(N, B, X, nmax, S.n, st, nullptr);
        } catch (const Fail& f) {
            if (f.st != MF_ERR_NOT_CONVERGED) throw;
            rc = f.st;
            msg = f.msg;
        }
        if (!sout.empty()) HIPX(launch_seg_scatter<double>(d_sout, d_sst, (int)sout.size(), ntot, X, st));
        HIPX(hipStreamSynchronize(st));
        if (info)
            for (int q = 0; q < nseg; q++) info[q] = N->seg_info[q];
        if (rc != MF_OK) return fail(rc, msg);
    } catch (const Fail& f) {
        return fail(f.st, f.msg);
    } catch (const std::bad_alloc&) {
        return fail(MF_ERR_OOM, "host allocation failed in mf_solve_batched");
    }
    return MF_OK;
}

mf_status mf_debug_front(mf_num_t N, int32_t front, int32_t* meta, double* F_host, int32_t* iv_host) {
    if (!N || N->magic != kNumMagic || !meta) return fail(MF_ERR_ARG, "bad arguments");
    if (!N->factored) return fail(MF_ERR_STATE, "not factored");
    const Symbolic& S = N->sym->S;
    if (front < 0 || front >= S.nf) return fail(MF_ERR_ARG, "front out of range");
    try {
        HIPX(hipDeviceSynchronize());
        const int sl = N->sym->dev->slot_of[front];
        const FrontNum fr = N->h_fn[sl];
        int32_t mm[8] = {fr.m, fr.P, fr.din, fr.k, fr.npiv, fr.mnom, fr.prec, sl};
        std::memcpy(meta, mm, sizeof(mm));
        const size_t cnt = (size_t)fr.m * fr.m;
        if (F_host) {
            if (fr.prec == 0) {
                HIPX(hipMemcpy(F_host, fr.F, sizeof(double) * cnt, hipMemcpyDeviceToHost));
            } else {
                std::vector<float> tmp(cnt);
                HIPX(hipMemcpy(tmp.data(), fr.F, sizeof(float) * cnt, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < cnt; i++) F_host[i] = tmp[i];
            }
        }
        if (iv_host) HIPX(hipMemcpy(iv_host, fr.iv, sizeof(int32_t) * (3 * (size_t)fr.P + fr.m), hipMemcpyDeviceToHost));
    } catch (const Fail& f) {
        return fail(f.st, f.msg);
    }
    return MF_OK;
}

int64_t mf_footprint_bytes(mf_sym_t h, const mf_options* opt, double margin) {
    if (!h || h->magic != kSymMagic) return -1;
    const Symbolic& S = h->S;
    const int prec = opt ? opt->prec : h->opt.prec;
    double b = 0;
    for (int f = 0; f < S.nf; f++) {
        double m = S.mnom[f];
        b += m * m * ((prec == MF_FP64 || S.front_parent[f] < 0) ? 8.0 : 4.0);
        b += 4.0 * (4.0 * m + 1 + 4 * kNBMax);
    }
    b += 12.0 * S.nnz + 8.0 * S.n * 4;  // values copy, pattern, vectors
    return (int64_t)(b * (1.0 + std::max(0.0, margin)));
}

void mf_release(void* handle) {
    if (!handle) return;
    uint32_t magic;
    std::memcpy(&magic, handle, sizeof(magic));
    if (magic == kSymMagic) {
        mf_sym* h = (mf_sym*)handle;
        h->magic = 0;
        delete h;
    } else if (magic == kNumMagic) {
        mf_num* N = (mf_num*)handle;
        // its calls returned with their streams idle; this only guards against a
        // caller that released the handle from another thread mid-call
        (void)hipStreamSynchronize(N->last_stream);
        N->magic = 0;
        delete N;
    }
}

}  // extern "C"
