// C ABI of the ALE Newton assembly (include/ale.h): problem set-up on the host
// (device copies, quadrature tables, the fixed-order summation lists that take
// element values to CSR entries and residual rows) and the assembly calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ale.h"
#include "ale_internal.h"

namespace mf {
void set_error(const std::string& msg);
}

namespace {

constexpr uint32_t kAleMagic = 0x41u << 24 | 0x4c45u;

struct AFail {
    mf_status st;
    std::string msg;
};

#define AHIP(call)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            throw AFail{e_ == hipErrorOutOfMemory ? MF_ERR_OOM : MF_ERR_DEVICE,                        \
                        std::string(#call) + ": " + hipGetErrorString(e_)};                            \
    } while (0)

mf_status afail(mf_status st, const std::string& msg) {
    mf::set_error(msg);
    return st;
}

template <typename V>
V* upload(const std::vector<V>& h, std::vector<void*>& owned) {
    V* d = nullptr;
    AHIP(hipMalloc((void**)&d, sizeof(V) * std::max<size_t>(h.size(), 1)));
    owned.push_back(d);
    if (!h.empty()) AHIP(hipMemcpy(d, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice));
    return d;
}

// The quadrature tables: the 7-point degree-5 triangle rule (weights summing to
// the reference area 1/2) with the P1 and P2 bases at its points, and 3-point
// Gauss-Legendre on [0, 1] for the Gamma edges.
ale::Tables make_tables() {
    ale::Tables T{};
    const double r = std::sqrt(15.0);
    const double a = (6.0 - r) / 21.0, b = (6.0 + r) / 21.0;
    const double wa = (155.0 - r) / 1200.0, wb = (155.0 + r) / 1200.0;
    const double pts[7][2] = {{1.0 / 3, 1.0 / 3}, {a, a}, {1 - 2 * a, a}, {a, 1 - 2 * a},
                              {b, b}, {1 - 2 * b, b}, {b, 1 - 2 * b}};
    const double w[7] = {9.0 / 40, wa, wa, wa, wb, wb, wb};
    const double dL[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
    const int edges[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    for (int q = 0; q < 7; q++) {
        const double L[3] = {1.0 - pts[q][0] - pts[q][1], pts[q][0], pts[q][1]};
        T.vw[q] = 0.5 * w[q];
        for (int v = 0; v < 3; v++) {
            T.L[q][v] = L[v];
            T.phi[q][v] = L[v] * (2.0 * L[v] - 1.0);
            for (int c = 0; c < 2; c++) T.dphi[q][v][c] = (4.0 * L[v] - 1.0) * dL[v][c];
        }
        for (int e = 0; e < 3; e++) {
            const int i = edges[e][0], j = edges[e][1];
            T.phi[q][3 + e] = 4.0 * L[i] * L[j];
            for (int c = 0; c < 2; c++) T.dphi[q][3 + e][c] = 4.0 * (L[j] * dL[i][c] + L[i] * dL[j][c]);
        }
    }
    const double g = std::sqrt(0.6);
    const double t[3] = {0.5 - 0.5 * g, 0.5, 0.5 + 0.5 * g};
    const double ew[3] = {5.0 / 18, 8.0 / 18, 5.0 / 18};
    for (int q = 0; q < 3; q++) {
        T.ew[q] = ew[q];
        T.psi[q][0] = (1 - t[q]) * (1 - 2 * t[q]);
        T.psi[q][1] = t[q] * (2 * t[q] - 1);
        T.psi[q][2] = 4 * t[q] * (1 - t[q]);
        T.lin[q][0] = 1 - t[q];
        T.lin[q][1] = t[q];
    }
    return T;
}

// Lists of (destination, element-scratch index) pairs, ordered by destination
// and, within one destination, by enumeration order (a counting sort), so every
// sum is taken in one fixed order.
struct Lists {
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
};

template <typename Enum>
Lists build_lists(int64_t m, Enum&& enumerate) {
    Lists L;
    L.ptr.assign(m + 1, 0);
    enumerate([&](int64_t dst, int64_t) { L.ptr[dst + 1]++; });
    for (int64_t i = 0; i < m; i++) L.ptr[i + 1] += L.ptr[i];
    L.idx.resize(L.ptr[m]);
    std::vector<int64_t> next(L.ptr.begin(), L.ptr.end() - 1);
    enumerate([&](int64_t dst, int64_t src) { L.idx[next[dst]++] = (int32_t)src; });
    return L;
}

}  // namespace

struct ale_problem {
    uint32_t magic = kAleMagic;
    int device = -1;
    int64_t n = 0, nnz = 0;
    ale::Dev D{};
    ale::Tables T{};
    std::vector<void*> owned;
    int64_t *jptr = nullptr, *rptr = nullptr;
    int32_t *jidx = nullptr, *ridx = nullptr, *gv = nullptr;
    double* jcst = nullptr;
    int32_t ngv = 0;
    int64_t bytes = 0;
    ~ale_problem() {
        for (void* p : owned) (void)hipFree(p);
    }
};

namespace {

void create(const ale_desc* d, ale_problem* P) {
    const int64_t n = d->n;
    const int32_t nn = d->nnodes, nv = d->nvert, ne = d->nelem, ng = d->nedge;
    if (n < 1 || n > INT32_MAX || nn < 3 || nv < 3 || ne < 1 || ng < 0)
        throw AFail{MF_ERR_ARG, "bad problem sizes"};
    if (!d->tri || !d->vtx || (ng && (!d->gedge || !d->gvtx)) || !d->u_dof || !d->p_dof || !d->x_dof ||
        !d->lam_dof || !d->s_dof || !d->gamma_vertex || !d->u_bc || !d->u_prev || !d->x_ref || !d->x_prev ||
        !d->lam_s || !d->rowptr || !d->colind)
        throw AFail{MF_ERR_ARG, "null array in the problem description"};
    const int64_t nnz = d->rowptr[n];
    if (d->rowptr[0] != 0 || nnz < 1 || nnz > INT32_MAX) throw AFail{MF_ERR_ARG, "bad rowptr"};
    if (!(d->dt > 0.0)) throw AFail{MF_ERR_ARG, "dt must be positive"};
    auto chk = [&](int64_t v, int64_t hi, const char* what) {
        if (v < -1 || v >= hi) throw AFail{MF_ERR_ARG, std::string(what) + " out of range"};
    };
    for (int64_t i = 0; i < 6LL * ne; i++) chk(d->tri[i], nn, "tri");
    for (int64_t i = 0; i < 3LL * ne; i++) chk(d->vtx[i], nv, "vtx");
    for (int64_t i = 0; i < 3LL * ng; i++) chk(d->gedge[i], nn, "gedge");
    for (int64_t i = 0; i < 2LL * ng; i++) chk(d->gvtx[i], nv, "gvtx");
    for (int64_t i = 0; i < 6LL * ne; i++)
        if (d->tri[i] < 0) throw AFail{MF_ERR_ARG, "tri has a negative node"};
    for (int64_t i = 0; i < 3LL * ne; i++)
        if (d->vtx[i] < 0) throw AFail{MF_ERR_ARG, "vtx has a negative vertex"};
    for (int64_t i = 0; i < 2LL * nn; i++) chk(d->u_dof[i], n, "u_dof"), chk(d->lam_dof[i], n, "lam_dof");
    for (int64_t i = 0; i < nv; i++) {
        chk(d->p_dof[i], n, "p_dof");
        if (d->p_dof[i] < 0) throw AFail{MF_ERR_ARG, "every vertex carries a pressure unknown"};
    }
    for (int64_t i = 0; i < 2LL * nv; i++) chk(d->x_dof[i], n, "x_dof");
    for (int c = 0; c < 2; c++)
        if (d->s_dof[c] < 0 || d->s_dof[c] >= n) throw AFail{MF_ERR_ARG, "s_dof out of range"};
    for (int64_t v = 0; v < nv; v++)
        if (d->gamma_vertex[v] && (d->x_dof[2 * v] < 0 || d->x_dof[2 * v + 1] < 0))
            throw AFail{MF_ERR_ARG, "a Gamma vertex needs both position unknowns"};
    for (int64_t r = 0; r < n; r++)
        if (d->rowptr[r + 1] < d->rowptr[r]) throw AFail{MF_ERR_ARG, "rowptr not monotone"};

    // CSR position of (row, col) in the pattern
    auto pos = [&](int64_t r, int64_t c) -> int64_t {
        const int32_t* a = d->colind + d->rowptr[r];
        const int32_t* b = d->colind + d->rowptr[r + 1];
        const int32_t* it = std::lower_bound(a, b, (int32_t)c);
        if (it == b || *it != c)
            throw AFail{MF_ERR_PATTERN, "coupling (" + std::to_string(r) + ", " + std::to_string(c) +
                                            ") is not in the pattern"};
        return d->rowptr[r] + (it - a);
    };
    const int64_t* ud = d->u_dof;
    const int64_t* xd = d->x_dof;
    const int64_t* ld = d->lam_dof;
    auto vrow = [&](int64_t e, int r) -> int64_t {      // triangle output row r
        return r < 12 ? ud[2 * d->tri[6 * e + (r >> 1)] + (r & 1)] : d->p_dof[d->vtx[3 * e + r - 12]];
    };
    auto vcol = [&](int64_t e, int j) -> int64_t {      // triangle input j
        if (j < 12) return ud[2 * d->tri[6 * e + (j >> 1)] + (j & 1)];
        if (j < 15) return d->p_dof[d->vtx[3 * e + j - 12]];
        return xd[2 * d->vtx[3 * e + ((j - 15) >> 1)] + ((j - 15) & 1)];
    };
    auto srow = [&](int64_t e, int r) -> int64_t {      // pseudo-solid row (not on Gamma vertices)
        const int v = d->vtx[3 * e + (r >> 1)];
        return d->gamma_vertex[v] ? -1 : xd[2 * v + (r & 1)];
    };
    auto scol = [&](int64_t e, int j) -> int64_t { return xd[2 * d->vtx[3 * e + (j >> 1)] + (j & 1)]; };
    auto erow = [&](int64_t g, int r) -> int64_t {      // edge output row
        if (r < 6) return ud[2 * d->gedge[3 * g + (r >> 1)] + (r & 1)];
        if (r < 12) return ld[2 * d->gedge[3 * g + ((r - 6) >> 1)] + (r & 1)];
        return d->s_dof[r - 12];
    };
    auto ecol = [&](int64_t g, int j) -> int64_t {      // edge input
        if (j < 6) return ud[2 * d->gedge[3 * g + (j >> 1)] + (j & 1)];
        if (j < 12) return ld[2 * d->gedge[3 * g + ((j - 6) >> 1)] + (j & 1)];
        return xd[2 * d->gvtx[2 * g + ((j - 12) >> 1)] + (j & 1)];
    };
    // structurally nonzero local blocks: triangle p rows do not see p; edge u rows
    // see lambda and x, lambda rows u and x, s rows lambda and x
    auto vol_nz = [](int r, int j) { return !(r >= 12 && j >= 12 && j < 15); };
    auto edg_nz = [](int r, int j) {
        const int rk = r < 6 ? 0 : (r < 12 ? 1 : 2), ck = j < 6 ? 0 : (j < 12 ? 1 : 2);
        const int rc = r < 12 ? (r & 1) : r - 12, cc = j & 1;
        if (ck == 2) return true;                       // the edge's length and velocity
        return (rk == 1 ? ck == 0 : ck == 1) && cc == rc;
    };

    ale::Dev& D = P->D;
    D.nelem = ne;
    D.nedge = ng;
    D.off_volJ = 0;
    D.off_volR = D.off_volJ + (int64_t)ne * ale::kVolIn * ale::kVolOut;
    D.off_solJ = D.off_volR + (int64_t)ne * ale::kVolOut;
    D.off_solR = D.off_solJ + (int64_t)ne * ale::kSolIn * ale::kSolOut;
    D.off_edgJ = D.off_solR + (int64_t)ne * ale::kSolOut;
    D.off_edgR = D.off_edgJ + (int64_t)ng * ale::kEdgIn * ale::kEdgOut;
    const int64_t nloc = D.off_edgR + (int64_t)ng * ale::kEdgOut;
    if (nloc > INT32_MAX) throw AFail{MF_ERR_ARG, "problem too large for 32-bit scratch indices"};

    Lists J = build_lists(nnz, [&](auto&& emit) {
        for (int64_t e = 0; e < ne; e++)
            for (int j = 0; j < ale::kVolIn; j++) {
                const int64_t c = vcol(e, j);
                if (c < 0) continue;
                for (int r = 0; r < ale::kVolOut; r++) {
                    const int64_t rr = vrow(e, r);
                    if (rr >= 0 && vol_nz(r, j)) emit(pos(rr, c), D.off_volJ + ale::kVolOut * (ale::kVolIn * e + j) + r);
                }
            }
        for (int64_t e = 0; e < ne; e++)
            for (int j = 0; j < ale::kSolIn; j++) {
                const int64_t c = scol(e, j);
                if (c < 0) continue;
                for (int r = 0; r < ale::kSolOut; r++) {
                    const int64_t rr = srow(e, r);
                    if (rr >= 0) emit(pos(rr, c), D.off_solJ + ale::kSolOut * (ale::kSolIn * e + j) + r);
                }
            }
        for (int64_t g = 0; g < ng; g++)
            for (int j = 0; j < ale::kEdgIn; j++) {
                const int64_t c = ecol(g, j);
                if (c < 0) continue;
                for (int r = 0; r < ale::kEdgOut; r++) {
                    const int64_t rr = erow(g, r);
                    if (rr >= 0 && edg_nz(r, j))
                        emit(pos(rr, c), D.off_edgJ + ale::kEdgOut * (ale::kEdgIn * g + j) + r);
                }
            }
    });
    Lists R = build_lists(n, [&](auto&& emit) {
        for (int64_t e = 0; e < ne; e++)
            for (int r = 0; r < ale::kVolOut; r++) {
                const int64_t rr = vrow(e, r);
                if (rr >= 0) emit(rr, D.off_volR + ale::kVolOut * e + r);
            }
        for (int64_t e = 0; e < ne; e++)
            for (int r = 0; r < ale::kSolOut; r++) {
                const int64_t rr = srow(e, r);
                if (rr >= 0) emit(rr, D.off_solR + ale::kSolOut * e + r);
            }
        for (int64_t g = 0; g < ng; g++)
            for (int r = 0; r < ale::kEdgOut; r++) {
                const int64_t rr = erow(g, r);
                if (rr >= 0) emit(rr, D.off_edgR + ale::kEdgOut * g + r);
            }
    });
    // entries no element assembles: x - X - s rows and the spring diagonal
    std::vector<double> cst(nnz, 0.0);
    std::vector<int32_t> gvl;
    for (int64_t v = 0; v < nv; v++)
        if (d->gamma_vertex[v]) {
            gvl.push_back((int32_t)v);
            for (int c = 0; c < 2; c++) {
                cst[pos(xd[2 * v + c], xd[2 * v + c])] += 1.0;
                cst[pos(xd[2 * v + c], d->s_dof[c])] += -1.0;
            }
        }
    for (int c = 0; c < 2; c++) cst[pos(d->s_dof[c], d->s_dof[c])] += d->k;

    auto i32 = [](const int64_t* a, int64_t m) {
        std::vector<int32_t> o(m);
        for (int64_t i = 0; i < m; i++) o[i] = (int32_t)a[i];
        return o;
    };
    auto& own = P->owned;
    AHIP(hipGetDevice(&P->device));
    D.tri = upload(std::vector<int32_t>(d->tri, d->tri + 6LL * ne), own);
    D.vtx = upload(std::vector<int32_t>(d->vtx, d->vtx + 3LL * ne), own);
    D.gedge = upload(std::vector<int32_t>(d->gedge, d->gedge + 3LL * ng), own);
    D.gvtx = upload(std::vector<int32_t>(d->gvtx, d->gvtx + 2LL * ng), own);
    D.u_dof = upload(i32(d->u_dof, 2LL * nn), own);
    D.p_dof = upload(i32(d->p_dof, nv), own);
    D.x_dof = upload(i32(d->x_dof, 2LL * nv), own);
    D.lam_dof = upload(i32(d->lam_dof, 2LL * nn), own);
    D.gamma_vertex = upload(std::vector<uint8_t>(d->gamma_vertex, d->gamma_vertex + nv), own);
    D.u_bc = upload(std::vector<double>(d->u_bc, d->u_bc + 2LL * nn), own);
    D.u_prev = upload(std::vector<double>(d->u_prev, d->u_prev + 2LL * nn), own);
    D.x_ref = upload(std::vector<double>(d->x_ref, d->x_ref + 2LL * nv), own);
    D.x_prev = upload(std::vector<double>(d->x_prev, d->x_prev + 2LL * nv), own);
    D.lam_s = upload(std::vector<double>(d->lam_s, d->lam_s + ne), own);
    D.s_dof[0] = (int32_t)d->s_dof[0];
    D.s_dof[1] = (int32_t)d->s_dof[1];
    D.nu = d->nu;
    D.dt = d->dt;
    D.k = d->k;
    D.loc = upload(std::vector<double>(nloc, 0.0), own);
    P->jptr = upload(J.ptr, own);
    P->jidx = upload(J.idx, own);
    P->rptr = upload(R.ptr, own);
    P->ridx = upload(R.idx, own);
    P->jcst = upload(cst, own);
    P->gv = upload(gvl, own);
    P->ngv = (int32_t)gvl.size();
    P->n = n;
    P->nnz = nnz;
    P->T = make_tables();
    P->bytes = (int64_t)(sizeof(double) * (nloc + nnz) + sizeof(int64_t) * (nnz + n + 2) +
                         sizeof(int32_t) * (J.idx.size() + R.idx.size()) +
                         sizeof(int32_t) * (9LL * ne + 5LL * ng + 4LL * nn + 3LL * nv) +
                         sizeof(double) * (4LL * nn + 4LL * nv + ne));
}

mf_status check_handle(ale_t p) {
    if (!p || p->magic != kAleMagic) return afail(MF_ERR_ARG, "bad ALE problem handle");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return afail(MF_ERR_ARG, "the ALE problem lives on another device");
    return MF_OK;
}

}  // namespace

extern "C" {

mf_status ale_create(const ale_desc* desc, ale_t* out) {
    if (!out) return afail(MF_ERR_ARG, "out is null");
    *out = nullptr;
    if (!desc) return afail(MF_ERR_ARG, "desc is null");
    try {
        auto P = std::make_unique<ale_problem>();
        create(desc, P.get());
        *out = P.release();
        return MF_OK;
    } catch (const AFail& f) {
        return afail(f.st, f.msg);
    } catch (const std::bad_alloc&) {
        return afail(MF_ERR_OOM, "host allocation failed in ale_create");
    }
}

mf_status ale_residual(ale_t p, const double* U_dev, double* R_dev, void* stream) {
    if (mf_status s = check_handle(p)) return s;
    if (!U_dev || !R_dev || U_dev == R_dev) return afail(MF_ERR_ARG, "U_dev and R_dev must be distinct device buffers");
    const hipStream_t st = (hipStream_t)stream;
    try {
        AHIP(ale::launch_elements(p->D, p->T, U_dev, false, st));
        AHIP(ale::launch_sum(p->n, p->rptr, p->ridx, nullptr, p->D.loc, R_dev, st));
        AHIP(ale::launch_fixup(p->D, p->gv, p->ngv, U_dev, R_dev, st));
    } catch (const AFail& f) {
        return afail(f.st, f.msg);
    }
    return MF_OK;
}

mf_status ale_jacobian(ale_t p, const double* U_dev, double* values_dev, double* R_dev, void* stream) {
    if (mf_status s = check_handle(p)) return s;
    if (!U_dev || !values_dev) return afail(MF_ERR_ARG, "U_dev and values_dev are required");
    if (R_dev && (R_dev == U_dev || R_dev == values_dev)) return afail(MF_ERR_ARG, "R_dev must be its own buffer");
    const hipStream_t st = (hipStream_t)stream;
    try {
        AHIP(ale::launch_elements(p->D, p->T, U_dev, true, st));
        AHIP(ale::launch_sum(p->nnz, p->jptr, p->jidx, p->jcst, p->D.loc, values_dev, st));
        if (R_dev) {
            AHIP(ale::launch_sum(p->n, p->rptr, p->ridx, nullptr, p->D.loc, R_dev, st));
            AHIP(ale::launch_fixup(p->D, p->gv, p->ngv, U_dev, R_dev, st));
        }
    } catch (const AFail& f) {
        return afail(f.st, f.msg);
    }
    return MF_OK;
}

int64_t ale_device_bytes(ale_t p) { return (p && p->magic == kAleMagic) ? p->bytes : -1; }

void ale_release(ale_t p) {
    if (p && p->magic == kAleMagic) {
        p->magic = 0;
        delete p;
    }
}

}  // extern "C"
