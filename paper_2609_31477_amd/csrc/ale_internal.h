// Device-side description of an ALE problem and the launchers of its assembly
// kernels (ale_kernels.hip), used by the host code in ale_api.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ale {

// Local inputs and outputs of the element kernels (their order is the layout
// of the element scratch):
//   triangle inputs  u (node i, component c) -> 2i + c (12), p (vertex v) -> 12 + v,
//                    x (vertex v, component c) -> 15 + 2v + c          (21)
//   triangle rows    u -> 2i + c (12), p -> 12 + v                     (15)
//   solid inputs and rows  x (vertex v, component c) -> 2v + c          (6)
//   edge inputs      u (edge node j, c) -> 2j + c, lambda -> 6 + 2j + c,
//                    x (end v, c) -> 12 + 2v + c                        (16)
//   edge rows        u -> 2j + c, lambda -> 6 + 2j + c, s_c -> 12 + c   (14)
constexpr int kVolIn = 21, kVolOut = 15;
constexpr int kSolIn = 6, kSolOut = 6;
constexpr int kEdgIn = 16, kEdgOut = 14;
constexpr int kVolQ = 7, kEdgQ = 3;

struct Tables {
    double vw[kVolQ];           // triangle rule weights (sum 1/2)
    double L[kVolQ][3];         // P1 values
    double phi[kVolQ][6];       // P2 values
    double dphi[kVolQ][6][2];   // P2 reference gradients
    double ew[kEdgQ];           // edge rule weights (sum 1)
    double psi[kEdgQ][3];       // P2 edge values (end, end, midpoint)
    double lin[kEdgQ][2];       // P1 edge values
};

struct Dev {
    int32_t nelem, nedge;
    const int32_t* tri;
    const int32_t* vtx;
    const int32_t* gedge;
    const int32_t* gvtx;
    const int32_t* u_dof;
    const int32_t* p_dof;
    const int32_t* x_dof;
    const int32_t* lam_dof;
    const uint8_t* gamma_vertex;
    const double* u_bc;
    const double* u_prev;
    const double* x_ref;
    const double* x_prev;
    const double* lam_s;
    int32_t s_dof[2];
    double nu, dt, k;
    double* loc;                // element scratch
    int64_t off_volJ, off_volR, off_solJ, off_solR, off_edgJ, off_edgR;
};

hipError_t launch_elements(const Dev& D, const Tables& T, const double* U, bool jacobian, hipStream_t st);
hipError_t launch_sum(int64_t m, const int64_t* ptr, const int32_t* idx, const double* cst, const double* loc,
                      double* out, hipStream_t st);
hipError_t launch_fixup(const Dev& D, const int32_t* gv, int32_t ngv, const double* U, double* R, hipStream_t st);

}  // namespace ale
