// Generalised polynomial chaos surrogate of the salt mass fraction (Section 3.1 and
// the appendix): Legendre basis of the field parameters, projection of the sample
// fields onto it with quadrature weights (eq. PCEcoef), mean and variance from the
// coefficients (eqs. PCEcoef2, var), and the exceedance probability of the surrogate
// sampled at many parameter points (eq. PCEpoint and Section 3.2).
//
// All of it is FP64 on the vector units.  The projection is a [n_coef x S] x [S x N]
// product that reads every sample field once (HBM bound); the exceedance is an
// [N x n_coef] x [n_coef x N_s] product fused with the threshold count (ALU bound).
// FP64 matrix cores have the same peak rate as FP64 vector FMAs on this chip, so the
// contractions use plain FMAs with the point-side basis values broadcast from LDS.
#include <hip/hip_ext.h>

#include "gpc.h"

namespace edf {

// psi_n(x) by the recursion (k + 1) psi_{k+1} = (2k + 1) x psi_k - k psi_{k-1}
__device__ __forceinline__ double legendre(int n, double x) {
  double a = 1.0, b = x;
  if (n == 0) return a;
  for (int k = 1; k < n; ++k) {
    const double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    a = b;
    b = c;
  }
  return b;
}

// W[q][i] = w_i Psi_q(theta_i) / Q_q
__global__ __launch_bounds__(kBlock) void k_gpc_weights(int S, int M, int nc, const double* theta,
                                                        int ldt, const double* w, const int* idx,
                                                        const double* Q, double* W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * nc) return;
  const int q = e / S, i = e % S;
  double psi = 1.0;
  for (int j = 0; j < M; ++j) psi *= legendre(idx[q * M + j], theta[(size_t)i * ldt + j]);
  W[(size_t)q * S + i] = w[i] * psi / Q[q];
}

void launch_gpc_weights(int S, int M, int nc, const double* theta, int ldt, const double* w,
                        const int* idx, const double* Q, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_gpc_weights, dim3(ceil_div(S * nc, kBlock)), dim3(kBlock), 0, st, S, M,
                     nc, theta, ldt, w, idx, Q, W);
}

// C[q][v] = sum_i W[q][i] F[i][v]: one vertex per thread, kProjChunk coefficients per
// thread in registers (blockIdx.y selects the chunk), the samples' values read once
constexpr int kProjChunk = 32;

__global__ __launch_bounds__(kBlock) void k_gpc_project(int S, int Nc, int nc, const double* W,
                                                        const double* F, double* C) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int q0 = blockIdx.y * kProjChunk;
  if (v >= Nc) return;
  double acc[kProjChunk];
#pragma unroll
  for (int q = 0; q < kProjChunk; ++q) acc[q] = 0.0;
  for (int i = 0; i < S; ++i) {
    const double f = F[(size_t)i * Nc + v];
#pragma unroll
    for (int q = 0; q < kProjChunk; ++q)
      if (q0 + q < nc) acc[q] += W[(size_t)(q0 + q) * S + i] * f;
  }
#pragma unroll
  for (int q = 0; q < kProjChunk; ++q)
    if (q0 + q < nc) C[(size_t)(q0 + q) * Nc + v] = acc[q];
}

void launch_gpc_project(int S, int Nc, int nc, const double* W, const double* F, double* C,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  dim3 grid(ceil_div(Nc, kBlock), ceil_div(nc, kProjChunk));
  if (ev0)
    hipExtLaunchKernelGGL(k_gpc_project, grid, dim3(kBlock), 0, st, ev0, ev1, 0, S, Nc, nc, W, F,
                          C);
  else
    hipLaunchKernelGGL(k_gpc_project, grid, dim3(kBlock), 0, st, S, Nc, nc, W, F, C);
}

// mean = C[0], var = sum_{q >= 1} Q_q C[q]^2
__global__ __launch_bounds__(kBlock) void k_gpc_moments(int Nc, int nc, const double* C,
                                                        const double* Q, double* mean,
                                                        double* var) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= Nc) return;
  double s = 0.0;
  for (int q = 1; q < nc; ++q) {
    const double c = C[(size_t)q * Nc + v];
    s += Q[q] * c * c;
  }
  mean[v] = C[v];
  var[v] = s;
}

void launch_gpc_moments(int Nc, int nc, const double* C, const double* Q, double* mean,
                        double* var, hipStream_t st) {
  hipLaunchKernelGGL(k_gpc_moments, dim3(ceil_div(Nc, kBlock)), dim3(kBlock), 0, st, Nc, nc, C, Q,
                     mean, var);
}

// Exceedance counts: a block holds kBlock vertices' coefficients in registers (NC
// padded to a multiple of 8 with zeros) and walks its chunk of points in tiles of
// kTilePts: the tile's basis values Psi_q(theta_s) are formed in LDS (1D Legendre
// values first, then the products), then every thread evaluates the surrogate at the
// tile's points with FMAs on broadcast LDS reads and counts values above the threshold.
constexpr int kTilePts = 64;

template <int NC>
__global__ __launch_bounds__(kBlock) void k_gpc_exceed(int Nc, int nc, int M, int pmax,
                                                       const double* C, const int* idx,
                                                       const double* theta, int Ns, int chunk,
                                                       double thr, int* partial) {
  __shared__ double basis[kTilePts][NC];
  __shared__ double leg[kTilePts][kGpcMaxM][kGpcMaxDeg + 1];
  __shared__ int sidx[NC * kGpcMaxM];
  const int tid = threadIdx.x;
  const int v = blockIdx.x * blockDim.x + tid;
  for (int e = tid; e < NC * M; e += blockDim.x) sidx[e] = e < nc * M ? idx[e] : 0;
  double c[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) c[q] = (v < Nc && q < nc) ? C[(size_t)q * Nc + v] : 0.0;
  const int s_begin = blockIdx.y * chunk;
  const int s_end = min(Ns, s_begin + chunk);
  int count = 0;
  for (int s0 = s_begin; s0 < s_end; s0 += kTilePts) {
    const int nt = min(kTilePts, s_end - s0);
    __syncthreads();  // the previous tile's basis values are no longer read
    for (int e = tid; e < nt * M; e += blockDim.x) {
      const int s = e / M, j = e % M;
      const double x = theta[(size_t)(s0 + s) * M + j];
      double a = 1.0, b = x;
      leg[s][j][0] = 1.0;
      if (pmax >= 1) leg[s][j][1] = x;
      for (int k = 1; k < pmax; ++k) {
        const double cc = ((2 * k + 1) * x * b - k * a) / (k + 1);
        a = b;
        b = cc;
        leg[s][j][k + 1] = cc;
      }
    }
    __syncthreads();
    for (int e = tid; e < nt * NC; e += blockDim.x) {
      const int s = e / NC, q = e % NC;
      double psi = 0.0;
      if (q < nc) {
        psi = 1.0;
        for (int j = 0; j < M; ++j) psi *= leg[s][j][sidx[q * M + j]];
      }
      basis[s][q] = psi;
    }
    __syncthreads();
    int s = 0;
    for (; s + 4 <= nt; s += 4) {  // four independent chains per thread
      double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        v0 = fma(c[q], basis[s][q], v0);
        v1 = fma(c[q], basis[s + 1][q], v1);
        v2 = fma(c[q], basis[s + 2][q], v2);
        v3 = fma(c[q], basis[s + 3][q], v3);
      }
      count += (v0 > thr) + (v1 > thr) + (v2 > thr) + (v3 > thr);
    }
    for (; s < nt; ++s) {
      double val = 0.0;
#pragma unroll
      for (int q = 0; q < NC; ++q) val = fma(c[q], basis[s][q], val);
      count += val > thr ? 1 : 0;
    }
  }
  if (v < Nc) partial[(size_t)blockIdx.y * Nc + v] = count;
}

template <int NC>
static void exceed_nc(dim3 grid, int Nc, int nc, int M, int pmax, const double* C, const int* idx,
                      const double* theta, int Ns, int chunk, double thr, int* partial,
                      hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0)
    hipExtLaunchKernelGGL(k_gpc_exceed<NC>, grid, dim3(kBlock), 0, st, ev0, ev1, 0, Nc, nc, M,
                          pmax, C, idx, theta, Ns, chunk, thr, partial);
  else
    hipLaunchKernelGGL(k_gpc_exceed<NC>, grid, dim3(kBlock), 0, st, Nc, nc, M, pmax, C, idx,
                       theta, Ns, chunk, thr, partial);
}

int gpc_exceed_padded(int nc) {
  const int steps[] = {8, 16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128};
  for (int p : steps)
    if (nc <= p) return p;
  return -1;
}

void launch_gpc_exceed(int Nc, int nc, int M, int pmax, const double* C, const int* idx,
                       const double* theta, int Ns, int chunk, int n_chunks, double thr,
                       int* partial, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 grid(ceil_div(Nc, kBlock), n_chunks);
  switch (gpc_exceed_padded(nc)) {
#define EDF_NC(P)                                                                                \
  case P:                                                                                        \
    exceed_nc<P>(grid, Nc, nc, M, pmax, C, idx, theta, Ns, chunk, thr, partial, st, ev0, ev1);   \
    break;
    EDF_NC(8) EDF_NC(16) EDF_NC(24) EDF_NC(32) EDF_NC(40) EDF_NC(48) EDF_NC(56) EDF_NC(64)
    EDF_NC(80) EDF_NC(96) EDF_NC(112) EDF_NC(128)
#undef EDF_NC
    default:
      break;
  }
}

// prob[v] = sum over chunks of the counts / N_s (integer sums: exact, order-free)
__global__ __launch_bounds__(kBlock) void k_gpc_count(int Nc, int n_chunks, int Ns,
                                                      const int* partial, double* prob) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= Nc) return;
  long long n = 0;
  for (int y = 0; y < n_chunks; ++y) n += partial[(size_t)y * Nc + v];
  prob[v] = (double)n / (double)Ns;
}

void launch_gpc_count(int Nc, int n_chunks, int Ns, const int* partial, double* prob,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_gpc_count, dim3(ceil_div(Nc, kBlock)), dim3(kBlock), 0, st, Nc, n_chunks, Ns,
                     partial, prob);
}

}  // namespace edf
