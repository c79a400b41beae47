// Generalised polynomial chaos surrogate of the salt mass fraction (Section 3.1 and
// the appendix): Legendre basis of the field parameters, projection of the sample
// fields onto it with quadrature weights (eq. PCEcoef), mean and variance from the
// coefficients (eqs. PCEcoef2, var), and the exceedance probability of the surrogate
// sampled at many parameter points (eq. PCEpoint and Section 3.2).
//
// All of it is FP64.  The projection is a [n_coef x S] x [S x N] product that reads
// every sample field once (HBM bound, vector FMAs); the exceedance is an
// [N x n_coef] x [n_coef x N_s] product fused with the threshold count (compute
// bound), run on the FP64 matrix cores.
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
// thread in registers (blockIdx.y selects the chunk); the samples are taken in tiles of
// kProjTile whose weights are staged in LDS (read back as broadcasts), and the tile's
// field values are loaded eight at a time so that enough loads are in flight
constexpr int kProjChunk = 32;
constexpr int kProjTile = 64;

__global__ __launch_bounds__(kBlock) void k_gpc_project(int S, int Nc, int nc, const double* W,
                                                        const double* F, double* C) {
  __shared__ double w[kProjTile][kProjChunk];
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int q0 = blockIdx.y * kProjChunk;
  double acc[kProjChunk];
#pragma unroll
  for (int q = 0; q < kProjChunk; ++q) acc[q] = 0.0;
  for (int i0 = 0; i0 < S; i0 += kProjTile) {
    const int ni = min(kProjTile, S - i0);
    __syncthreads();
    for (int e = threadIdx.x; e < kProjTile * kProjChunk; e += blockDim.x) {
      const int i = e / kProjChunk, q = e % kProjChunk;
      w[i][q] = (i < ni && q0 + q < nc) ? W[(size_t)(q0 + q) * S + i0 + i] : 0.0;
    }
    __syncthreads();
    if (v < Nc) {
      int i = 0;
      for (; i + 8 <= ni; i += 8) {
        double f[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) f[u] = F[(size_t)(i0 + i + u) * Nc + v];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < kProjChunk; ++q) acc[q] += w[i + u][q] * f[u];
      }
      for (; i < ni; ++i) {
        const double f = F[(size_t)(i0 + i) * Nc + v];
#pragma unroll
        for (int q = 0; q < kProjChunk; ++q) acc[q] += w[i][q] * f;
      }
    }
  }
  if (v >= Nc) return;
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

// Basis table of a batch of surrogate points: B[q][s] = Psi_q(theta_s) for q < nc,
// zero for the padding terms q < ncp and the padding points s < ldb (one thread per
// point and term; the recursion is the one of k_gpc_weights)
__global__ __launch_bounds__(kBlock) void k_gpc_basis(int n, int ldb, int nc, int M,
                                                      const int* idx, const double* theta,
                                                      double* B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (s >= ldb) return;
  double psi = 0.0;
  if (q < nc && s < n) {
    psi = 1.0;
    for (int j = 0; j < M; ++j) psi *= legendre(idx[q * M + j], theta[(size_t)s * M + j]);
  }
  B[(size_t)q * ldb + s] = psi;
}

void launch_gpc_basis(int n, int ldb, int nc, int ncp, int M, const int* idx, const double* theta,
                      double* B, hipStream_t st) {
  hipLaunchKernelGGL(k_gpc_basis, dim3(ceil_div(ldb, kBlock), ncp), dim3(kBlock), 0, st, n, ldb,
                     nc, M, idx, theta, B);
}

// Exceedance counts on the matrix cores.  The surrogate values of 16 vertices at 16
// points are one 16x16 tile of the product [vertices x q] x [q x points], built by
// v_mfma_f64_16x16x4f64 over q in steps of 4 (FP64 throughout).  Lane l supplies
// A[l % 16][l / 16] (a vertex's coefficient) and B[l / 16][l % 16] (a point's basis
// value) and receives D[l / 16 + 4 v][l % 16], v = 0..3.  A wave keeps the coefficients
// of its kRowBlocks x 16 vertices in registers (one value per lane, row block and step of
// 4 terms), a block of four waves walks its chunk of points in tiles of kTilePts: the
// tile's columns of the basis table are copied to LDS ([q][point], point fastest; the
// next tile's are fetched into registers during the products), every wave runs kTilePts / 16 x kRowBlocks independent 16 x 16 accumulations (each basis
// value read from LDS feeds kRowBlocks products), compares the values with the threshold
// and counts per lane; the counts of the 16 lanes that share a vertex are summed by
// shuffles at the end.
constexpr int kTilePts = 64;
constexpr int kRowBlocks = 2;
constexpr int kExceedRows = 4 * 16 * kRowBlocks;  // vertices per workgroup
constexpr int kMaxKb = kGpcMaxCoef / 4;
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// this thread's share of the columns [s0, s0 + kTilePts) of the basis table, 16 bytes
// per load (element e = q * kTilePts / 2 + pair)
template <int P>
__device__ __forceinline__ void load_basis_tile(v2d (&nxt)[P], const double* B, int ldb, int s0,
                                                int ncp, int tid) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int e = tid + p * kBlock;
    const int q = min(e / (kTilePts / 2), ncp - 1), sp = 2 * (e % (kTilePts / 2));
    nxt[p] = *reinterpret_cast<const v2d*>(B + (size_t)q * ldb + s0 + sp);
  }
}

template <int KB>  // at most KB steps of 4 terms (register array length)
__global__ __launch_bounds__(kBlock) void k_gpc_exceed(int Nc, int nc, const double* C,
                                                       const double* B, int ldb, int n, int chunk,
                                                       int chunk0, double thr, int* partial) {
  extern __shared__ double basis[];  // [ncp][kTilePts]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kb_n = (nc + 3) / 4;  // steps of 4 terms
  const int ncp = 4 * kb_n;
  // this lane's A operand for every row block and step: coefficient (l / 16 + 4 kb) of
  // vertex l % 16 of the row block
  const int row0 = blockIdx.x * kExceedRows + wave * 16 * kRowBlocks;
  double a[kRowBlocks][KB];
#pragma unroll
  for (int r = 0; r < kRowBlocks; ++r) {
    const int vrow = row0 + 16 * r + (lane & 15);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int q = 4 * kb + (lane >> 4);
      a[r][kb] = (kb < kb_n && q < nc && vrow < Nc) ? C[(size_t)q * Nc + vrow] : 0.0;
    }
  }
  const int s_begin = blockIdx.y * chunk;
  const int s_end = min(n, s_begin + chunk);
  int cnt[kRowBlocks][4] = {};
  // up to 48 terms (KB <= 12) the next tile's columns of the basis table are loaded into
  // registers while the current tile's products run, and stored to LDS after them; with
  // more terms those registers would halve the waves per SIMD, and the tile is copied
  // between two barriers.  A tile starts at a multiple of kTilePts below n <= ldb, so its
  // 16-byte loads stay in the table.
  constexpr bool kPrefetch = KB <= 12;
  constexpr int kPref = kPrefetch ? (KB * 4 * (kTilePts / 2) + kBlock - 1) / kBlock : 1;
  v2d nxt[kPref];
  if (kPrefetch && s_begin < s_end) load_basis_tile<kPref>(nxt, B, ldb, s_begin, ncp, tid);
  for (int s0 = s_begin; s0 < s_end; s0 += kTilePts) {
    const int nt = min(kTilePts, s_end - s0);
    __syncthreads();  // the previous tile's basis values are no longer read
    if constexpr (kPrefetch) {
#pragma unroll
      for (int p = 0; p < kPref; ++p) {
        const int e = tid + p * kBlock;
        if (e < ncp * (kTilePts / 2)) {
          const int q = e / (kTilePts / 2), sp = 2 * (e % (kTilePts / 2));
          *reinterpret_cast<v2d*>(basis + q * kTilePts + sp) = nxt[p];
        }
      }
    } else {
      for (int e = tid; e < ncp * (kTilePts / 2); e += blockDim.x) {
        const int q = e / (kTilePts / 2), sp = 2 * (e % (kTilePts / 2));
        *reinterpret_cast<v2d*>(basis + q * kTilePts + sp) =
            *reinterpret_cast<const v2d*>(B + (size_t)q * ldb + s0 + sp);
      }
    }
    __syncthreads();
    if (kPrefetch && s0 + kTilePts < s_end)
      load_basis_tile<kPref>(nxt, B, ldb, s0 + kTilePts, ncp, tid);
    constexpr int kCols = kTilePts / 16;  // independent 16-point accumulations
    v4d d[kRowBlocks][kCols];
#pragma unroll
    for (int r = 0; r < kRowBlocks; ++r)
#pragma unroll
      for (int t = 0; t < kCols; ++t) d[r][t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      if (kb < kb_n) {
        const int q = 4 * kb + (lane >> 4);
#pragma unroll
        for (int t = 0; t < kCols; ++t) {
          const double b = basis[q * kTilePts + 16 * t + (lane & 15)];
#pragma unroll
          for (int r = 0; r < kRowBlocks; ++r)
            d[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][kb], b, d[r][t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kCols; ++t) {
      const bool point = 16 * t + (lane & 15) < nt;
#pragma unroll
      for (int r = 0; r < kRowBlocks; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) cnt[r][v] += (point && d[r][t][v] > thr) ? 1 : 0;
    }
  }
  // lanes with the same l / 16 hold the same four vertices: sum over l % 16
#pragma unroll
  for (int r = 0; r < kRowBlocks; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) cnt[r][v] += __shfl_xor(cnt[r][v], off, 16);
  if ((lane & 15) == 0)
#pragma unroll
    for (int r = 0; r < kRowBlocks; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + 16 * r + (lane >> 4) + 4 * v;
        if (row < Nc) partial[(size_t)(chunk0 + blockIdx.y) * Nc + row] = cnt[r][v];
      }
}

void launch_gpc_exceed(int Nc, int nc, const double* C, const double* B, int ldb, int n, int chunk,
                       int chunk0, int n_chunks, double thr, int* partial, hipStream_t st,
                       hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 grid(ceil_div(Nc, kExceedRows), n_chunks);
  const int ncp = 4 * ((nc + 3) / 4);
  const size_t lds = sizeof(double) * (size_t)ncp * kTilePts;
  const int kb_n = ncp / 4;
  auto kern = kb_n <= 2    ? k_gpc_exceed<2>
              : kb_n <= 4  ? k_gpc_exceed<4>
              : kb_n <= 8  ? k_gpc_exceed<8>
              : kb_n <= 12 ? k_gpc_exceed<12>
              : kb_n <= 16 ? k_gpc_exceed<16>
              : kb_n <= 24 ? k_gpc_exceed<24>
                           : k_gpc_exceed<kMaxKb>;
  if (ev0)
    hipExtLaunchKernelGGL(kern, grid, dim3(kBlock), lds, st, ev0, ev1, 0, Nc, nc, C, B, ldb, n,
                          chunk, chunk0, thr, partial);
  else
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), lds, st, Nc, nc, C, B, ldb, n, chunk, chunk0, thr,
                       partial);
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
