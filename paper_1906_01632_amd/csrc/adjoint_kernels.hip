// Kernels of the discrete adjoint: gradient of the salt mass in a subregion at
// the final time with respect to the field parameters xi.
//
// Every implicit-Euler step n solves R~^n(u^n; u^{n-1}, xi) = 0 (scaled residual).
// With J(u^N, xi) the salt mass phi rho(c) c integrated over the box S with the
// lumped control volumes, the adjoint states solve, backwards in n,
//   (dR~^n/du~^n)^T lambda^n = [n = N] dJ/du~^N - (dR~^{n+1}/du~^n)^T lambda^{n+1},
// and dJ/dxi = dJ/dxi|_explicit - sum_n (lambda^n)^T dR~^n/dxi.
// dR~^{n+1}/du^n comes only from the storage terms (a diagonal in c); dR/dxi acts
// through phi_e (storage, salt diffusion) and K_e (Darcy fluxes) of every hexahedron.
// Rows replaced by Dirichlet conditions depend neither on xi nor on u^{n-1}.
#include <cmath>

#include "adjoint.h"
#include "fv_common.h"

namespace edf {

// ---------------------------------------------------------------------------
// transposed stencil: (A^T)_{v,o} = (A_{v+o, -o})^T, blockwise
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_transpose(Geom g, const double* src_all, T* dst_all,
                                                      const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t >= g.off[8] || !colour_decode(g, t, i, j, k)) return;
  const size_t Np = g.off[8];
  const double* src = src_all + (size_t)s * kPlanes * Np;
  T* dst = dst_all + (size_t)s * kPlanes * Np + sidx<T>(t, 0, kPlanes);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int o = nb_index(dx, dy, dz);
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        double b00 = 0, b01 = 0, b10 = 0, b11 = 0;
        if (ii >= 0 && jj >= 0 && kk >= 0 && ii < g.nx && jj < g.ny && kk < g.nz) {
          const int tw = colour_encode(g, ii, jj, kk);
          const int ob = nb_index(-dx, -dy, -dz);
          const double* w = src + sidx<double>(tw, 0, kPlanes);
          b00 = w[soff<double>(ob * 4)];
          b01 = w[soff<double>(ob * 4 + 1)];
          b10 = w[soff<double>(ob * 4 + 2)];
          b11 = w[soff<double>(ob * 4 + 3)];
        }
        dst[soff<T>(o * 4 + 0)] = (T)b00;
        dst[soff<T>(o * 4 + 1)] = (T)b10;
        dst[soff<T>(o * 4 + 2)] = (T)b01;
        dst[soff<T>(o * 4 + 3)] = (T)b11;
      }
}

template <typename T>
void launch_transpose(const Geom& g, const double* src, T* dst, int S, const int* mask,
                      hipStream_t st) {
  dim3 grid(ceil_div(g.off[8], kBlock), S);
  hipLaunchKernelGGL(k_transpose<T>, grid, dim3(kBlock), 0, st, g, src, dst, mask);
}
template void launch_transpose<double>(const Geom&, const double*, double*, int, const int*,
                                       hipStream_t);
template void launch_transpose<float>(const Geom&, const double*, float*, int, const int*,
                                      hipStream_t);

// ---------------------------------------------------------------------------
// octant of vertex v in the hexahedron where v is corner (ax, ay, az): its overlap
// with the box S
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ovl(double lo, double hi, double s0, double s1) {
  return fmax(0.0, fmin(hi, s1) - fmax(lo, s0));
}

__device__ __forceinline__ double octant_in_box(const Geom& g, const QoiBox& S, int i, int j, int k,
                                                int ax, int ay, int az) {
  const double x = i * g.hx, y = j * g.hy, z = k * g.hz;
  const double x0 = ax ? x - 0.5 * g.hx : x, y0 = ay ? y - 0.5 * g.hy : y,
               z0 = az ? z - 0.5 * g.hz : z;
  return ovl(x0, x0 + 0.5 * g.hx, S.b[0], S.b[1]) * ovl(y0, y0 + 0.5 * g.hy, S.b[2], S.b[3]) *
         ovl(z0, z0 + 0.5 * g.hz, S.b[4], S.b[5]);
}

template <int Q>
__device__ __forceinline__ void block_sum4(double (&v)[Q], double* part) {
  __shared__ double sh[Q][kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
    if (lane == 0) sh[q][wave] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double a = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) a += sh[q][w];
      part[q] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// J = sum_v W_v rho(c_v) c_v, W_v = sum_e phi_e |o(e,v) ∩ S|; dJ/du~ = (0, W_v (rho0 + 2 drho c_v))
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_qoi(Geom g, Phys ph, QoiBox S, const double* phi_all,
                                                const double* u_all, double* dJ_all, double* part,
                                                const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (v < g.N) {
    const int i = v % g.nx, j = (v / g.nx) % g.ny, k = v / (g.nx * g.ny);
    const size_t cells = (size_t)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
    const double* phi = phi_all + s * cells;
    double W = 0.0;
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax) {
          const int hi = i - ax, hj = j - ay, hk = k - az;
          if (hi < 0 || hj < 0 || hk < 0 || hi > g.nx - 2 || hj > g.ny - 2 || hk > g.nz - 2) continue;
          const size_t e = hi + (size_t)(g.nx - 1) * (hj + (size_t)(g.ny - 1) * hk);
          W += phi[e] * octant_in_box(g, S, i, j, k, ax, ay, az);
        }
    const double c = reinterpret_cast<const double2*>(u_all)[(size_t)s * g.N + v].y;
    acc[0] = W * (ph.rho0 + ph.drho * c) * c;
    reinterpret_cast<double2*>(dJ_all)[(size_t)s * g.N + v] =
        make_double2(0.0, W * (ph.rho0 + 2.0 * ph.drho * c));
  }
  block_sum4<1>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
}

// b~_c(v) = row_c m_v [drho lam_l + (rho0 + 2 drho c_v) lam_s] (rows of step n+1 that are
// finite-volume rows), b~_p = 0: the right-hand side -(dR~^{n+1}/du~^n)^T lambda^{n+1}
__global__ __launch_bounds__(kBlock) void k_adjoint_rhs(Geom g, Phys ph, const double* phi_all,
                                                        const double* u_all, const double* lam_all,
                                                        double* b_all, const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.N) return;
  const int i = v % g.nx, j = (v / g.nx) % g.ny, k = v / (g.nx * g.ny);
  const size_t cells = (size_t)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  const double* phi = phi_all + s * cells;
  double msum = 0.0;
  for (int az = 0; az < 2; ++az)
    for (int ay = 0; ay < 2; ++ay)
      for (int ax = 0; ax < 2; ++ax) {
        const int hi = i - ax, hj = j - ay, hk = k - az;
        if (hi < 0 || hj < 0 || hk < 0 || hi > g.nx - 2 || hj > g.ny - 2 || hk > g.nz - 2) continue;
        msum += phi[hi + (size_t)(g.nx - 1) * (hj + (size_t)(g.ny - 1) * hk)];
      }
  const double m = msum * g.hx * g.hy * g.hz * 0.125;
  const double c = reinterpret_cast<const double2*>(u_all)[(size_t)s * g.N + v].y;
  const double2 lam = reinterpret_cast<const double2*>(lam_all)[(size_t)s * g.N + v];
  double cD;
  const double ll = is_pin(g, i, j, k) ? 0.0 : lam.x;
  const double ls = is_cdir(g, i, j, k, cD) ? 0.0 : lam.y;
  reinterpret_cast<double2*>(b_all)[(size_t)s * g.N + v] =
      make_double2(0.0, ph.row_c * m * (ph.drho * ll + (ph.rho0 + 2.0 * ph.drho * c) * ls));
}

void launch_qoi(const Geom& g, const Phys& ph, const QoiBox& S, const double* phi, const double* u,
                double* dJ, double* part, int S_n, const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(g.N, kBlock), S_n);
  hipLaunchKernelGGL(k_qoi, grid, dim3(kBlock), 0, st, g, ph, S, phi, u, dJ, part, mask);
}

void launch_adjoint_rhs(const Geom& g, const Phys& ph, const double* phi, const double* u,
                        const double* lam, double* b, int S_n, const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(g.N, kBlock), S_n);
  hipLaunchKernelGGL(k_adjoint_rhs, grid, dim3(kBlock), 0, st, g, ph, phi, u, lam, b, mask);
}

// ---------------------------------------------------------------------------
// per hexahedron: d phi_e / d xi_m and d K_e / d xi_m for the field models
// ---------------------------------------------------------------------------
__device__ __forceinline__ void field_derivs(const FieldParams& fp, const double* q, double x,
                                             double y, double z, double phi, double* dphi,
                                             double* dK_over_K) {
  const double pm = fp.phi_mean;
  const double px = M_PI * x / fp.lx, py = M_PI * y / fp.ly, pz = M_PI * z / fp.lz;
  for (int m = 0; m < 4; ++m) dphi[m] = dK_over_K[m] = 0.0;
  double extra[4] = {0, 0, 0, 0};  // d ln K / d xi_m beyond Kozeny-Carman
  switch (fp.model) {
    case 1:
      dphi[0] = 0.2 * pm * cos(px) * cos(py);
      break;
    case 2:
      dphi[0] = 0.2 * pm * cos(px) * cos(py);
      dphi[1] = 0.2 * pm * sin(px) * sin(py);
      extra[2] = 0.5 * cos(pz);
      extra[3] = 0.5 * sin(px) * cos(pz);
      break;
    case 3: {
      const double sx = sin(px), sy = sin(py), sz = sin(pz);
      dphi[0] = 0.01 * (sx + sx * sy);
      dphi[1] = 0.01 * (sy + sx * sz);
      dphi[2] = 0.01 * sz;
      break;
    }
    default:
      return;
  }
  (void)q;
  // Kozeny-Carman: d ln K / d phi = 3/phi + 2/(1 - phi)
  const double dlnK = 3.0 / phi + 2.0 / (1.0 - phi);
  for (int m = 0; m < 4; ++m) dK_over_K[m] = dlnK * dphi[m] + extra[m];
}

// corner w of a hexahedron: bit 0 = x, bit 1 = y, bit 2 = z
__device__ __forceinline__ double tri_w(int w, int D, int s0b, int s1b) {
  // trilinear weight of corner w at the face point of face (D, start bits in the
  // other two directions s0b, s1b): 1/2 in D, 3/4 on the start's side, else 1/4
  double f = 1.0;
  int oi = 0;
  for (int e = 0; e < 3; ++e) {
    const int bit = (w >> e) & 1;
    if (e == D) {
      f *= 0.5;
    } else {
      const int sb = oi == 0 ? s0b : s1b;
      f *= bit == sb ? 0.75 : 0.25;
      ++oi;
    }
  }
  return f;
}

__device__ __forceinline__ double tri_dw(int w, int D, int s0b, int s1b) {
  double f = ((w >> D) & 1) ? 1.0 : -1.0;
  int oi = 0;
  for (int e = 0; e < 3; ++e) {
    if (e == D) continue;
    const int bit = (w >> e) & 1;
    const int sb = oi == 0 ? s0b : s1b;
    f *= bit == sb ? 0.75 : 0.25;
    ++oi;
  }
  return f;
}

// contribution of one hexahedron to dJ/dxi: -(lambda^T dR~/dphi_e) dphi_e/dxi
// - (lambda^T dR~/dK_e) dK_e/dxi (+ dJ/dphi_e dphi_e/dxi at the final state)
__global__ __launch_bounds__(kBlock) void k_param_grad(Geom g, Phys ph0, const double* dts,
                                                       FieldParams fp, const double* xi,
                                                       const double* phi_all, const double* K_all,
                                                       const double* u_all, const double* uo_all,
                                                       const double* lam_all, QoiBox S, int with_qoi,
                                                       double* part, const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int cx = g.nx - 1, cy = g.ny - 1, cz = g.nz - 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < cx * cy * cz) {
    const double dt = dts ? dts[s] : ph0.dt;
    const double srow = dt * ph0.row_c;
    const int hi = e % cx, hj = (e / cx) % cy, hk = e / (cx * cy);
    const size_t cells = (size_t)cx * cy * cz;
    const double phi = phi_all[s * cells + e], K = K_all[s * cells + e];
    const double2* u = reinterpret_cast<const double2*>(u_all) + (size_t)s * g.N;
    const double2* uo = reinterpret_cast<const double2*>(uo_all) + (size_t)s * g.N;
    const double2* lm = reinterpret_cast<const double2*>(lam_all) + (size_t)s * g.N;
    double P[8], C[8], Co[8], Ll[8], Ls[8];
    double Gq = 0.0;
    for (int w = 0; w < 8; ++w) {
      const int i = hi + (w & 1), j = hj + ((w >> 1) & 1), k = hk + (w >> 2);
      const size_t v = i + (size_t)g.nx * (j + (size_t)g.ny * k);
      P[w] = u[v].x;
      C[w] = u[v].y;
      Co[w] = uo[v].y;
      double cD;
      Ll[w] = is_pin(g, i, j, k) ? 0.0 : lm[v].x;
      Ls[w] = is_cdir(g, i, j, k, cD) ? 0.0 : lm[v].y;
      if (with_qoi)
        Gq += octant_in_box(g, S, i, j, k, w & 1, (w >> 1) & 1, w >> 2) *
              (ph0.rho0 + ph0.drho * C[w]) * C[w];
    }
    const double h[3] = {g.hx, g.hy, g.hz};
    const double area[3] = {g.hy * g.hz * 0.25, g.hx * g.hz * 0.25, g.hx * g.hy * 0.25};
    double GK = 0.0, Gphi = 0.0;
    // storage: d m_v / d phi_e = V/8
    const double vo = g.hx * g.hy * g.hz * 0.125;
    for (int w = 0; w < 8; ++w) {
      const double rc = ph0.rho0 + ph0.drho * C[w], rco = ph0.rho0 + ph0.drho * Co[w];
      Gphi += srow * vo / dt * (Ll[w] * (rc - rco) + Ls[w] * (rc * C[w] - rco * Co[w]));
    }
    // fluxes through the 12 faces
    for (int D = 0; D < 3; ++D)
      for (int sb = 0; sb < 4; ++sb) {
        const int s0b = sb & 1, s1b = sb >> 1;
        // start corner: bit D = 0, the other two directions from (s0b, s1b)
        int a = 0, oi = 0;
        for (int ee = 0; ee < 3; ++ee) {
          if (ee == D) continue;
          a |= (oi == 0 ? s0b : s1b) << ee;
          ++oi;
        }
        const int b = a | (1 << D);
        double cf = 0.0, dp = 0.0, dc = 0.0;
        for (int w = 0; w < 8; ++w) {
          const double Nw = tri_w(w, D, s0b, s1b), dNw = tri_dw(w, D, s0b, s1b);
          cf += Nw * C[w];
          dp += dNw * P[w];
          dc += dNw * C[w];
        }
        dp /= h[D];
        dc /= h[D];
        const double gD = D == 2 ? ph0.g : 0.0;
        const double rf = ph0.rho0 + ph0.drho * cf;
        const double Q1 = -(1.0 / ph0.mu) * (dp - rf * gD) * area[D];  // Q / K
        const double cup = (K * Q1 >= 0.0) ? C[a] : C[b];
        const double fl_K = rf * Q1;                                       // d(liquid flux)/dK
        const double fs_K = (ph0.rho0 + ph0.drho * cup) * cup * Q1;        // d(salt flux)/dK
        const double fs_phi = -rf * ph0.Dm * dc * area[D];                 // d(salt flux)/dphi
        GK += srow * ((Ll[a] - Ll[b]) * fl_K + (Ls[a] - Ls[b]) * fs_K);
        Gphi += srow * (Ls[a] - Ls[b]) * fs_phi;
      }
    const double xc = (hi + 0.5) * g.hx, yc = (hj + 0.5) * g.hy, zc = (hk + 0.5) * g.hz;
    double dphi[4], dKK[4];
    field_derivs(fp, xi + (size_t)s * (fp.n_xi > 0 ? fp.n_xi : 1), xc, yc, zc, phi, dphi, dKK);
    for (int m = 0; m < 4; ++m) acc[m] = -(Gphi * dphi[m] + GK * K * dKK[m]) + Gq * dphi[m];
  }
  block_sum4<4>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
}

int launch_param_grad(const Geom& g, const Phys& ph, const double* dts, const FieldParams& fp,
                      const double* xi, const double* phi, const double* K, const double* u,
                      const double* uo, const double* lam, const QoiBox& S, int with_qoi,
                      double* part, int S_n, const int* mask, hipStream_t st) {
  const int cells = (g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  const int nb = ceil_div(cells, kBlock);
  hipLaunchKernelGGL(k_param_grad, dim3(nb, S_n), dim3(kBlock), 0, st, g, ph, dts, fp, xi, phi, K,
                     u, uo, lam, S, with_qoi, part, mask);
  return nb;
}

// out[s][q] = sum of the nb partials (q < 4), one wave per sample, fixed order
__global__ __launch_bounds__(64) void k_sum4(int nb, const double* part, double* out,
                                             const int* mask) {
  const int s = blockIdx.x;
  if (mask && !mask[s]) return;
  double a[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += 64)
    for (int q = 0; q < 4; ++q) a[q] += part[((size_t)s * nb + b) * 4 + q];
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a[q] += __shfl_down(a[q], off, 64);
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) out[4 * s + q] = a[q];
}

void launch_sum4(int nb, const double* part, double* out, int S_n, const int* mask,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_sum4, dim3(S_n), dim3(64), 0, st, nb, part, out, mask);
}

// dst[s] = src[s * stride_s + idx[s] * n .. + n): per-sample gather of one state from a
// trajectory buffer (idx < 0: skip)
__global__ __launch_bounds__(kBlock) void k_gather_state(size_t n, const double* src,
                                                         size_t stride_s, const int* idx,
                                                         double* dst) {
  const int s = blockIdx.y;
  const int k = idx[s];
  if (k < 0) return;
  const double* a = src + (size_t)s * stride_s + (size_t)k * n;
  double* b = dst + (size_t)s * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

__global__ __launch_bounds__(kBlock) void k_scatter_state(size_t n, const double* src,
                                                          double* dst, size_t stride_s,
                                                          const int* idx) {
  const int s = blockIdx.y;
  const int k = idx[s];
  if (k < 0) return;
  const double* a = src + (size_t)s * n;
  double* b = dst + (size_t)s * stride_s + (size_t)k * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

void launch_gather_state(size_t n, const double* src, size_t stride_s, const int* idx,
                         double* dst, int S_n, hipStream_t st) {
  const int nb = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_gather_state, dim3(nb, S_n), dim3(kBlock), 0, st, n, src, stride_s, idx,
                     dst);
}

void launch_scatter_state(size_t n, const double* src, double* dst, size_t stride_s,
                          const int* idx, int S_n, hipStream_t st) {
  const int nb = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_scatter_state, dim3(nb, S_n), dim3(kBlock), 0, st, n, src, dst, stride_s,
                     idx);
}

}  // namespace edf
