// BiCGStab (right preconditioned, Section 2.3: the Newton systems are solved by
// BiCGStab with a multigrid preconditioner) for a batch of independent samples,
// plus the vector kernels of the Newton iteration and the sample statistics.
//
// Every sample keeps its own scalars (rho, alpha, omega, ...) in device memory
// and its own active flag; a finished sample is skipped by every later kernel.
// Reductions are two-pass and deterministic: each workgroup writes its partial
// sums in a fixed order, and one wave per sample adds the partials in a fixed
// order.
#include "fv_common.h"

namespace edf {

constexpr int kRedMax = 1024;  // partial sums per sample and quantity

int reduce_blocks(size_t n) {
  const size_t b = (n + kBlock * 4 - 1) / (kBlock * 4);
  return (int)(b < 1 ? 1 : (b > kRedMax ? kRedMax : b));
}

// ---------------------------------------------------------------------------
// y = A x (FP64 stencil), optional fused dots: (d1, y) and (d2, y) or (y, y)
// ---------------------------------------------------------------------------
enum DotMode { kDotNone = 0, kDotOne = 1, kDotTS = 2 };

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_spmv(Geom g, const double* A_all, const double* x_all,
                                                 double* y_all, const double* d_all, double* part,
                                                 const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  // one thread per vertex in natural order: the Krylov vectors x, y, d are read and
  // written contiguously; the stencil rows of a wave's 64 vertices are two runs of 32
  // positions of two colours
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = g.N, Np = g.off[8];
  double acc[2] = {0.0, 0.0};
  if (v < g.N) {
    const int i = v % g.nx, j = (v / g.nx) % g.ny, k = v / (g.nx * g.ny);
    const int t = colour_encode_sel(g, i, j, k);
    const double* A = A_all + (size_t)s * kPlanes * Np + sidx<double>(t, 0, kPlanes);
    const char* x = reinterpret_cast<const char*>(reinterpret_cast<const double2*>(x_all) + (size_t)s * N);
    const int plane = g.nx * g.ny;
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int o = nb_index(dx, dy, dz);
          // a neighbour outside the grid has a zero block: any vertex of the sample will do,
          // so the index is clamped (below 0 wraps to a large unsigned value)
          const unsigned w = min((unsigned)(v + dx + g.nx * dy + plane * dz), (unsigned)(g.N - 1));
          const double2 xv = *reinterpret_cast<const double2*>(x + w * (unsigned)sizeof(double2));
          const Block2<double> a = load_block(A, o * 4);
          r0 += a.a00 * xv.x + a.a01 * xv.y;
          r1 += a.a10 * xv.x + a.a11 * xv.y;
        }
      }
    }
    reinterpret_cast<double2*>(y_all)[(size_t)s * N + v] = make_double2(r0, r1);
    if (MODE != kDotNone) {
      const double2 d = reinterpret_cast<const double2*>(d_all)[(size_t)s * N + v];
      acc[0] = d.x * r0 + d.y * r1;
      if (MODE == kDotTS) acc[1] = r0 * r0 + r1 * r1;
    }
  }
  if (MODE == kDotOne) {
    double a1[1] = {acc[0]};
    block_partial<1>(a1, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
  } else if (MODE == kDotTS) {
    block_partial<2>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
  }
}

void launch_spmv(const Geom& g, const JacOp& J, const double* x, double* y, int S,
                 const int* mask, hipStream_t st) {
  if (!J.A) {
    launch_jx(g, J.ph, J.dts, J.phi, J.K, J.u, x, y, nullptr, nullptr, 0, S, mask, nullptr, S, st);
    return;
  }
  dim3 grid(ceil_div(g.N, kBlock), S);
  hipLaunchKernelGGL(k_spmv<kDotNone>, grid, dim3(kBlock), 0, st, g, J.A, x, y,
                     (const double*)nullptr, (double*)nullptr, mask, (const int*)nullptr);
}

// ---------------------------------------------------------------------------
// per-sample scalar updates (one wave per sample)
// ---------------------------------------------------------------------------
enum Phase { kInit = 0, kAlpha = 1, kS = 2, kOmega = 3, kUpdate = 4 };

// BiCGStab restarts when |(r^, r)| <= kBreakdown |r^| |r| (or omega or (r^, v) vanish)
constexpr double kBreakdown = 1e-12;
constexpr int kMaxRestarts = 8;

__global__ __launch_bounds__(64) void k_bicg_finalize(int phase, int nb, const double* part,
                                                      KrylovScalars* ks_all, int* active,
                                                      const double* rtol, const int* gate) {
  const int s = blockIdx.x;
  if (phase == kInit) {
    if (gate && !gate[s]) {
      if (threadIdx.x == 0) active[s] = 0;
      return;
    }
  } else if (!active[s]) {
    return;
  }
  const int lane = threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  for (int b = lane; b < nb; b += 64) {
    a0 += part[((size_t)s * nb + b) * 4 + 0];
    a1 += part[((size_t)s * nb + b) * 4 + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a0 += __shfl_down(a0, off, 64);
    a1 += __shfl_down(a1, off, 64);
  }
  if (lane != 0) return;
  KrylovScalars& k = ks_all[s];
  switch (phase) {
    case kInit:
      k.bb = a0;
      k.rr = a0;
      k.rho = a0;  // (r^, r) with r^ = r = b
      k.rho_old = 1.0;
      k.alpha = 1.0;
      k.omega = 1.0;
      k.beta = 0.0;
      k.tol2 = rtol[s] * rtol[s] * a0;
      k.ss = 0.0;
      k.hh = a0;
      k.it = 0;
      k.restart = 0;
      k.restarts = 0;
      k.state = (a0 > 0.0 && a0 == a0) ? 0 : (a0 == 0.0 ? 1 : 2);
      active[s] = k.state == 0;
      break;
    case kAlpha:
      k.restart = 0;  // the restart (if any) took place in the p update before this
      k.rv = a0;
      k.alpha = (a0 != 0.0) ? k.rho / a0 : 0.0;
      break;
    case kS:
      k.ss = a0;
      break;
    case kOmega:
      k.ts = a0;
      k.tt = a1;
      k.omega = (k.ss <= k.tol2 || a1 == 0.0) ? 0.0 : a0 / a1;
      break;
    case kUpdate: {
      k.rho_old = k.rho;
      k.rho = a0;
      k.rr = a1;
      k.it += 1;
      const bool finite = (a1 == a1) && (a1 < 1e300);
      if (!finite) {
        k.state = 2;
      } else if (a1 <= k.tol2 || k.ss <= k.tol2) {
        k.state = 1;
      } else if (k.omega == 0.0 || k.rv == 0.0 ||
                 !(fabs(k.rho) > kBreakdown * sqrt(k.hh * a1))) {
        // (near) breakdown: (r^, r) or omega has vanished; restart from the iterate
        // reached so far with r^ = p = r (at most kMaxRestarts times)
        if (k.restarts < kMaxRestarts) {
          k.restart = 1;
          k.restarts += 1;
          k.rho = a1;
          k.hh = a1;
          k.beta = 0.0;
        } else {
          k.state = 2;
        }
      } else {
        k.beta = (k.rho / k.rho_old) * (k.alpha / k.omega);
      }
      if (k.state != 0) active[s] = 0;
      break;
    }
  }
}

static void finalize(int phase, int nb, const double* part, KrylovScalars* ks, int* active,
                     const double* rtol, int S, hipStream_t st, const int* gate = nullptr) {
  hipLaunchKernelGGL(k_bicg_finalize, dim3(S), dim3(64), 0, st, phase, nb, part, ks, active, rtol,
                     gate);
}

// ---------------------------------------------------------------------------
// BiCGStab phases
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bicg_init(size_t n, const double* b, double* x,
                                                      double* r, double* rh, double* p, double* v,
                                                      double* part, const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const size_t o = (size_t)s * n;
  double acc[1] = {0.0};
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const double be = b[o + e];
    x[o + e] = 0.0;
    r[o + e] = be;
    rh[o + e] = be;
    p[o + e] = 0.0;
    v[o + e] = 0.0;
    acc[0] += be * be;
  }
  block_partial<1>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
}

void launch_bicg_init(size_t n, const double* b, double* x, double* r, double* rh, double* p,
                      double* v, double* part, KrylovScalars* ks, const double* rtol, int* active,
                      int S, const int* mask, hipStream_t st) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_bicg_init, dim3(nb, S), dim3(kBlock), 0, st, n, b, x, r, rh, p, v, part,
                     mask);
  // `mask` gates which samples solve; their active flags start from the initial residual
  finalize(kInit, nb, part, ks, active, rtol, S, st, mask);
}

__global__ __launch_bounds__(kBlock) void k_bicg_p(size_t n, const double* r, const double* v,
                                                   double* p, double* rh, const KrylovScalars* ks,
                                                   const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const double beta = ks[s].beta, omega = ks[s].omega;
  const size_t o = (size_t)s * n;
  if (ks[s].restart) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
      p[o + e] = r[o + e];
      rh[o + e] = r[o + e];
    }
    return;
  }
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[o + e] = r[o + e] + beta * (p[o + e] - omega * v[o + e]);
}

void launch_bicg_p(size_t n, const double* r, const double* v, double* p, double* rh,
                   const KrylovScalars* ks, int S, const int* mask, SampleList sl, hipStream_t st) {
  hipLaunchKernelGGL(k_bicg_p, dim3(reduce_blocks(n), sl.rows(S)), dim3(kBlock), 0, st, n, r, v,
                     p, rh, ks, mask, sl.idx);
}

void launch_bicg_alpha(const Geom& g, const JacOp& J, const double* ph, double* v,
                       const double* rh, double* part, KrylovScalars* ks, int S, const int* mask,
                       SampleList sl, hipStream_t st) {
  int nb = ceil_div(g.N, kBlock);
  if (J.A)
    hipLaunchKernelGGL(k_spmv<kDotOne>, dim3(nb, sl.rows(S)), dim3(kBlock), 0, st, g, J.A, ph, v,
                       rh, part, mask, sl.idx);
  else
    nb = launch_jx(g, J.ph, J.dts, J.phi, J.K, J.u, ph, v, rh, part, 1, S, mask, sl.idx,
                   sl.rows(S), st);
  finalize(kAlpha, nb, part, ks, const_cast<int*>(mask), nullptr, S, st);  // mask is `active`
}

__global__ __launch_bounds__(kBlock) void k_bicg_s(size_t n, const double* r, const double* v,
                                                   double* sv, double* part,
                                                   const KrylovScalars* ks, const int* mask,
                                                   const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const double alpha = ks[s].alpha;
  const size_t o = (size_t)s * n;
  double acc[1] = {0.0};
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const double se = r[o + e] - alpha * v[o + e];
    sv[o + e] = se;
    acc[0] += se * se;
  }
  block_partial<1>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
}

void launch_bicg_s(size_t n, const double* r, const double* v, double* s, double* part,
                   KrylovScalars* ks, int S, const int* mask, SampleList sl, hipStream_t st) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_bicg_s, dim3(nb, sl.rows(S)), dim3(kBlock), 0, st, n, r, v, s, part, ks,
                     mask, sl.idx);
  finalize(kS, nb, part, ks, const_cast<int*>(mask), nullptr, S, st);
}

void launch_bicg_omega(const Geom& g, const JacOp& J, const double* sh, const double* s,
                       double* t, double* part, KrylovScalars* ks, int S, const int* mask,
                       SampleList sl, hipStream_t st) {
  int nb = ceil_div(g.N, kBlock);
  if (J.A)
    hipLaunchKernelGGL(k_spmv<kDotTS>, dim3(nb, sl.rows(S)), dim3(kBlock), 0, st, g, J.A, sh, t, s,
                       part, mask, sl.idx);
  else
    nb = launch_jx(g, J.ph, J.dts, J.phi, J.K, J.u, sh, t, s, part, 2, S, mask, sl.idx,
                   sl.rows(S), st);
  finalize(kOmega, nb, part, ks, const_cast<int*>(mask), nullptr, S, st);
}

__global__ __launch_bounds__(kBlock) void k_bicg_update(size_t n, const double* ph,
                                                        const double* sh, const double* sv,
                                                        const double* t, const double* rh,
                                                        double* x, double* r, double* part,
                                                        const KrylovScalars* ks, const int* mask,
                                                        const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const double alpha = ks[s].alpha, omega = ks[s].omega;
  const size_t o = (size_t)s * n;
  double acc[2] = {0.0, 0.0};
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    x[o + e] += alpha * ph[o + e] + omega * sh[o + e];
    const double re = sv[o + e] - omega * t[o + e];
    r[o + e] = re;
    acc[0] += rh[o + e] * re;
    acc[1] += re * re;
  }
  block_partial<2>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
}

void launch_bicg_update(size_t n, const double* ph, const double* sh, const double* s,
                        const double* t, const double* rh, double* x, double* r, double* part,
                        KrylovScalars* ks, int* active, int S, const int* mask, SampleList sl,
                        hipStream_t st) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_bicg_update, dim3(nb, sl.rows(S)), dim3(kBlock), 0, st, n, ph, sh, s, t, rh,
                     x, r, part, ks, mask, sl.idx);
  finalize(kUpdate, nb, part, ks, active, nullptr, S, st);
}

// ---------------------------------------------------------------------------
// Newton helpers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_sq_norm(size_t n, const double* x, double* part,
                                                    const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const size_t o = (size_t)s * n;
  double acc[1] = {0.0};
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    acc[0] += x[o + e] * x[o + e];
  block_partial<1>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
}

__global__ __launch_bounds__(64) void k_sum_partials(int nb, const double* part, double* out,
                                                     const int* mask) {
  const int s = blockIdx.x;
  if (mask && !mask[s]) return;
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) a += part[((size_t)s * nb + b) * 4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  if (threadIdx.x == 0) out[s] = a;
}

void launch_sq_norm(size_t n, const double* x, double* part, double* out, int S, const int* mask,
                    hipStream_t st) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_sq_norm, dim3(nb, S), dim3(kBlock), 0, st, n, x, part, mask);
  hipLaunchKernelGGL(k_sum_partials, dim3(S), dim3(64), 0, st, nb, part, out, mask);
}

// per-sample minimum and maximum of c (admissibility check of a converged step):
// out[s] = (min c, max c); block partials in part[s][b][0..1]
__global__ __launch_bounds__(kBlock) void k_c_range(size_t N, const double* u, double* part,
                                                    const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const double2* u2 = reinterpret_cast<const double2*>(u) + (size_t)s * N;
  double lo = 1e300, hi = -1e300;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N;
       e += (size_t)gridDim.x * blockDim.x) {
    const double c = u2[e].y;
    lo = fmin(lo, c);
    hi = fmax(hi, c);
  }
  __shared__ double sl[kBlock / 64], shh[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
  }
  if (lane == 0) {
    sl[wave] = lo;
    shh[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      lo = fmin(lo, sl[w]);
      hi = fmax(hi, shh[w]);
    }
    part[((size_t)s * gridDim.x + blockIdx.x) * 4 + 0] = lo;
    part[((size_t)s * gridDim.x + blockIdx.x) * 4 + 1] = hi;
  }
}

__global__ __launch_bounds__(64) void k_range_finalize(int nb, const double* part, double* out,
                                                       const int* mask) {
  const int s = blockIdx.x;
  if (mask && !mask[s]) return;
  double lo = 1e300, hi = -1e300;
  for (int b = threadIdx.x; b < nb; b += 64) {
    lo = fmin(lo, part[((size_t)s * nb + b) * 4 + 0]);
    hi = fmax(hi, part[((size_t)s * nb + b) * 4 + 1]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
  }
  if (threadIdx.x == 0) {
    out[2 * s] = lo;
    out[2 * s + 1] = hi;
  }
}

void launch_c_range(const Geom& g, const double* u, double* part, double* out, int S,
                    const int* mask, hipStream_t st) {
  const int nb = reduce_blocks(2 * (size_t)g.N);
  hipLaunchKernelGGL(k_c_range, dim3(nb, S), dim3(kBlock), 0, st, (size_t)g.N, u, part, mask);
  hipLaunchKernelGGL(k_range_finalize, dim3(S), dim3(64), 0, st, nb, part, out, mask);
}

// out = u + lam_s * (p_unit * d_p, d_c): Newton update in physical units
__global__ __launch_bounds__(kBlock) void k_axpy_state(size_t N, const double* u, const double* d,
                                                       const double* lam, double p_unit,
                                                       double* out, const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const double l = lam[s];
  const size_t o = (size_t)s * N;
  const double2* u2 = reinterpret_cast<const double2*>(u) + o;
  const double2* d2 = reinterpret_cast<const double2*>(d) + o;
  double2* o2 = reinterpret_cast<double2*>(out) + o;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N;
       e += (size_t)gridDim.x * blockDim.x) {
    const double2 a = u2[e], b = d2[e];
    o2[e] = make_double2(a.x + l * p_unit * b.x, a.y + l * b.y);
  }
}

void launch_axpy_state(size_t N, const double* u, const double* d, const double* lam,
                       double p_unit, double* out, int S, const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_state, dim3(reduce_blocks(2 * N), S), dim3(kBlock), 0, st, N, u, d,
                     lam, p_unit, out, mask);
}

__global__ __launch_bounds__(kBlock) void k_masked_copy(size_t n, const double* a, double* b,
                                                        const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const size_t o = (size_t)s * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    b[o + e] = a[o + e];
}

void launch_masked_copy(size_t n, const double* a, double* b, int S, const int* mask,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_masked_copy, dim3(reduce_blocks(n), S), dim3(kBlock), 0, st, n, a, b,
                     mask);
}

// the sample list of a launch over several groups' levels of one grid: segment q gives
// the slots off_q + src_q[j] (or off_q + j when src_q is null), j < n_q, one after the other
__global__ __launch_bounds__(kBlock) void k_concat_lists(ListSegs L, int* dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int q = 0; q < L.nseg; ++q) {
    if (i < L.seg[q].n) {
      dst[L.seg[q].at + i] = L.seg[q].off + (L.seg[q].src ? L.seg[q].src[i] : i);
      return;
    }
    i -= L.seg[q].n;
  }
}

void launch_concat_lists(const ListSegs& L, int total, int* dst, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_concat_lists, dim3(ceil_div(total, kBlock)), dim3(kBlock), 0, st, L, dst);
}

// out = 2 u - u_prev: the linear extrapolation of a sample's last two states (Newton's
// starting point candidate of the next step)
__global__ __launch_bounds__(kBlock) void k_extrapolate(size_t n, const double* u,
                                                        const double* u_prev, double* out,
                                                        const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const size_t o = (size_t)s * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    out[o + e] = 2.0 * u[o + e] - u_prev[o + e];
}

void launch_extrapolate(size_t n, const double* u, const double* u_prev, double* out, int S,
                        const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_extrapolate, dim3(reduce_blocks(n), S), dim3(kBlock), 0, st, n, u, u_prev,
                     out, mask);
}

// ---------------------------------------------------------------------------
// statistics over samples (Section 3: eqs. pdestat, numer_var; Section 3.2)
// ---------------------------------------------------------------------------
// c of every sample of a group at the common vertices (nested, every r-th vertex)
__global__ __launch_bounds__(kBlock) void k_gather_common(Geom gf, int cx, int cy, int cz,
                                                          const double* u, double* out) {
  const int s = blockIdx.y;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int Nc = cx * cy * cz;
  if (v >= Nc) return;
  const int rx = (gf.nx - 1) / (cx - 1), ry = (gf.ny - 1) / (cy - 1), rz = (gf.nz - 1) / (cz - 1);
  const int I = v % cx, J = (v / cx) % cy, K = v / (cx * cy);
  const size_t vf = (size_t)I * rx + (size_t)gf.nx * ((size_t)J * ry + (size_t)gf.ny * K * rz);
  out[(size_t)s * Nc + v] = reinterpret_cast<const double2*>(u)[(size_t)s * gf.N + vf].y;
}

void launch_gather_common(const Geom& gf, int cx, int cy, int cz, const double* u, double* out,
                          int S, hipStream_t st) {
  dim3 grid(ceil_div(cx * cy * cz, kBlock), S);
  hipLaunchKernelGGL(k_gather_common, grid, dim3(kBlock), 0, st, gf, cx, cy, cz, u, out);
}

// one thread per common vertex, samples summed in index order (deterministic)
__global__ __launch_bounds__(kBlock) void k_moments(int Nc, int S, const double* f, const double* w,
                                                    double thr, double* mean, double* var,
                                                    double* exc) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= Nc) return;
  double m = 0.0, e = 0.0;
  for (int s = 0; s < S; ++s) {
    const double c = f[(size_t)s * Nc + v];
    m += w[s] * c;
    e += (c > thr) ? w[s] : 0.0;
  }
  double q = 0.0;
  for (int s = 0; s < S; ++s) {
    const double d = m - f[(size_t)s * Nc + v];
    q += w[s] * d * d;
  }
  mean[v] = m;
  var[v] = q;
  exc[v] = e;
}

// The same sums taken over the samples in chunks (fields f [n][Nc] of the samples s0 ..
// s0 + n - 1, weights w indexed by sample), each chunk added to the running sums in sample
// order, so that the result is bitwise that of k_moments.  Pass 0: mean and exceedance;
// pass 1 (after every chunk of pass 0): the variance about the finished mean.
__global__ __launch_bounds__(kBlock) void k_moments_chunk(int pass, int Nc, int s0, int n,
                                                          const double* f, const double* w,
                                                          double thr, double* mean, double* var,
                                                          double* exc) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= Nc) return;
  if (pass == 0) {
    double m = s0 == 0 ? 0.0 : mean[v], e = s0 == 0 ? 0.0 : exc[v];
    for (int s = 0; s < n; ++s) {
      const double c = f[(size_t)s * Nc + v];
      m += w[s0 + s] * c;
      e += (c > thr) ? w[s0 + s] : 0.0;
    }
    mean[v] = m;
    exc[v] = e;
  } else {
    const double m = mean[v];
    double q = s0 == 0 ? 0.0 : var[v];
    for (int s = 0; s < n; ++s) {
      const double d = m - f[(size_t)s * Nc + v];
      q += w[s0 + s] * d * d;
    }
    var[v] = q;
  }
}

void launch_moments_chunk(int pass, int Nc, int s0, int n, const double* f, const double* w,
                          double thr, double* mean, double* var, double* exc, hipStream_t st) {
  hipLaunchKernelGGL(k_moments_chunk, dim3(ceil_div(Nc, kBlock)), dim3(kBlock), 0, st, pass, Nc,
                     s0, n, f, w, thr, mean, var, exc);
}

// weights of the statistics in place: w[s] = 0 for a failed sample (flag[s] != 0), then
// every weight divided by their sum, taken in sample order (as the host does it for
// edf_moments); *sum_out = that sum.  One thread: S is the number of samples.
__global__ void k_normalise_weights(int S, double* w, const int* flag, double* sum_out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double sum = 0.0;
  for (int s = 0; s < S; ++s) {
    if (flag[s]) w[s] = 0.0;
    sum += w[s];
  }
  if (sum > 0.0)
    for (int s = 0; s < S; ++s) w[s] /= sum;
  *sum_out = sum;
}

void launch_normalise_weights(int S, double* w, const int* flag, double* sum_out, hipStream_t st) {
  hipLaunchKernelGGL(k_normalise_weights, dim3(1), dim3(1), 0, st, S, w, flag, sum_out);
}

void launch_moments(int Nc, int S, const double* f, const double* w, double thr, double* mean,
                    double* var, double* exc, hipStream_t st) {
  hipLaunchKernelGGL(k_moments, dim3(ceil_div(Nc, kBlock)), dim3(kBlock), 0, st, Nc, S, f, w, thr,
                     mean, var, exc);
}

}  // namespace edf
