// Declarations of the adjoint kernels (adjoint_kernels.hip).
#pragma once

#include "edf_internal.h"

namespace edf {

struct QoiBox {
  double b[6];  // x0, x1, y0, y1, z0, z1 (z is depth)
};

template <typename T>
void launch_transpose(const Geom& g, const double* src, T* dst, int S, const int* mask,
                      hipStream_t st);
void launch_qoi(const Geom& g, const Phys& ph, const QoiBox& S, const double* phi, const double* u,
                double* dJ, double* part, int S_n, const int* mask, hipStream_t st);
void launch_adjoint_rhs(const Geom& g, const Phys& ph, const double* phi, const double* u,
                        const double* lam, double* b, int S_n, const int* mask, hipStream_t st);
int launch_param_grad(const Geom& g, const Phys& ph, const double* dts, const FieldParams& fp,
                      const double* xi, const double* phi, const double* K, const double* u,
                      const double* uo, const double* lam, const QoiBox& S, int with_qoi,
                      double* part, int S_n, const int* mask, hipStream_t st);
void launch_sum4(int nb, const double* part, double* out, int S_n, const int* mask,
                 hipStream_t st);
void launch_gather_state(size_t n, const double* src, size_t stride_s, const int* idx,
                         double* dst, int S_n, hipStream_t st);
void launch_scatter_state(size_t n, const double* src, double* dst, size_t stride_s,
                          const int* idx, int S_n, hipStream_t st);

}  // namespace edf
