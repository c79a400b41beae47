// Geometric multigrid kernels: 8-colour block Gauss-Seidel, residual, transfer
// operators and the dense coarsest-grid solve.  T is the V-cycle precision
// (double, or float inside the FP64 outer iteration).
//
// The V-cycle preconditions BiCGStab (Section 2.3: BiCGStab with a multigrid
// V-cycle; Section 5.1: a hierarchy of nested grids with the Jacobian assembled
// on every grid).  The paper smooths with ILU_beta, a sequential recurrence; here
// the smoother is block Gauss-Seidel over the 8 colours (i%2, j%2, k%2), which
// are independent sets of the 27-point stencil, so every colour is one fully
// parallel pass.  Prolongation is trilinear interpolation from the nested coarse
// vertices, restriction its transpose.
#include <hip/hip_ext.h>

#include "fv_common.h"

namespace edf {

// ---------------------------------------------------------------------------
// Per-vertex operations.  Pointers are those of one sample; the V-cycle vectors
// (b, x, r: [Np][2] of T on every level) are in the colour-major order of the
// stencil rows, so a wave reads and writes its own vertices contiguously and the
// neighbours of a run of one colour are runs of the neighbouring colours.  The
// helpers serve both the one-launch-per-sweep kernels (large grids) and the fused
// kernel that runs the bottom of the V-cycle in one workgroup per sample.
// ---------------------------------------------------------------------------

// block Gauss-Seidel update of vertex q of colour col: x_v += D_v^{-1} (b - A x)_v.
// ZC >= 0: the first forward sweep of a V-cycle level, whose x is still zero, for
// colour col = ZC: x_v = D_v^{-1} (b - A x)_v with the zero terms left out, so it reads
// neither the vertex's own x nor the stencil blocks of the colours not yet swept.
template <typename T, bool NT, int ZC = -1>
__device__ __forceinline__ void smooth_vertex(const Geom& g, int col, int q, const T* A_s,
                                              const T* D_s, const T* b_s, T* x_s) {
  using T2 = typename V2<T>::type;
  int i, j, k;
  colour_decode_in(g, col, q, i, j, k);
  const int t = g.off[col] + q;
  const T* A = A_s + sidx<T>(t, 0, kPlanes);
  T2* x = reinterpret_cast<T2*>(x_s);
  const T2 bv = reinterpret_cast<const T2*>(b_s)[t];
  const NbrMap nm = nbr_map(g, col, i, j, k);
  T r0 = bv.x, r1 = bv.y;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (ZC >= 0 && !zero_start_reads(ZC, dx, dy, dz)) continue;
        const T2 xv = load_nbr(x, g, nm, dx, dy, dz);
        const Block2<T> a = load_block<NT>(A, nb_index(dx, dy, dz) * 4);
        r0 -= a.a00 * xv.x + a.a01 * xv.y;
        r1 -= a.a10 * xv.x + a.a11 * xv.y;
      }
    }
  }
  const Block2<T> d = load_block<NT>(D_s + sidx<T>(t, 0, 4), 0);
  T2 xv;
  if (ZC >= 0) {
    xv.x = d.a00 * r0 + d.a01 * r1;
    xv.y = d.a10 * r0 + d.a11 * r1;
  } else {
    xv = x[t];
    xv.x += d.a00 * r0 + d.a01 * r1;
    xv.y += d.a10 * r0 + d.a11 * r1;
  }
  x[t] = xv;
}

// residual r = b - A x at colour-major position t after the pre-smoothing sweeps, zero
// in Dirichlet rows (their equations are solved exactly by the smoother and carry no
// coarse-grid correction) and in the rows of the last colour swept (colour 7: block
// Gauss-Seidel has just solved them with all their neighbours final, so their residual
// is zero up to rounding)
template <typename T, bool NT>
__device__ __forceinline__ void residual_vertex(const Geom& g, int t, const T* A_s,
                                                const T* b_s, const T* x_s, T* r_s) {
  using T2 = typename V2<T>::type;
  if (t >= g.off[7]) {
    if (t - g.off[7] < g.cnt[7]) {
      T2 z;
      z.x = 0;
      z.y = 0;
      reinterpret_cast<T2*>(r_s)[t] = z;
    }
    return;
  }
  int col, i, j, k;
  if (!colour_decode_wave(g, t, col, i, j, k)) return;
  const NbrMap nm = nbr_map(g, col, i, j, k);
  const T* A = A_s + sidx<T>(t, 0, kPlanes);
  const T2* x = reinterpret_cast<const T2*>(x_s);
  T a0 = 0, a1 = 0;  // (A x)_v; b is read after the sweep over the neighbours
#pragma unroll 1  // one z-plane of neighbours at a time keeps the register count low
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const T2 xv = load_nbr(x, g, nm, dx, dy, dz);
        const Block2<T> a = load_block<NT>(A, nb_index(dx, dy, dz) * 4);
        a0 += a.a00 * xv.x + a.a01 * xv.y;
        a1 += a.a10 * xv.x + a.a11 * xv.y;
      }
    }
  }
  const T2 bv = reinterpret_cast<const T2*>(b_s)[t];
  double cD;
  T2 out;
  out.x = is_pin(g, i, j, k) ? T(0) : bv.x - a0;
  out.y = is_cdir(g, i, j, k, cD) ? T(0) : bv.y - a1;
  reinterpret_cast<T2*>(r_s)[t] = out;
}

// Residual after a single forward sweep from x = 0, at position t of colour C < 7
// (vertex i, j, k).  That sweep left D_v x_v + (sum over the neighbours of the colours
// below C of A_vo x_{v+o}) = b_v, so r_v = -(sum over the neighbours of the colours above
// C of A_vo x_{v+o}): only those stencil blocks are read, and neither b nor x_v.
// Dirichlet rows are zero as in residual_vertex.
template <typename T, bool NT, int C>
__device__ __forceinline__ void residual_upper_vertex(const Geom& g, int t, int i, int j, int k,
                                                      const T* A_s, const T* x_s, T* r_s) {
  using T2 = typename V2<T>::type;
  const NbrMap nm = nbr_map(g, C, i, j, k);
  const T* A = A_s + sidx<T>(t, 0, kPlanes);
  const T2* x = reinterpret_cast<const T2*>(x_s);
  T a0 = 0, a1 = 0;
  // one z-plane of neighbours at a time keeps the register count low; the planes above
  // and below share their pattern of blocks
  auto plane = [&](int dz, auto mz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (nbr_colour(C, dx, dy, decltype(mz)::value) <= C) continue;
        const T2 xv = load_nbr(x, g, nm, dx, dy, dz);
        const Block2<T> a = load_block<NT>(A, nb_index(dx, dy, dz) * 4);
        a0 += a.a00 * xv.x + a.a01 * xv.y;
        a1 += a.a10 * xv.x + a.a11 * xv.y;
      }
    }
  };
#pragma unroll 1
  for (int dz = -1; dz <= 1; dz += 2) plane(dz, std::integral_constant<int, 1>());
  plane(0, std::integral_constant<int, 0>());
  double cD;
  T2 out;
  out.x = is_pin(g, i, j, k) ? T(0) : -a0;
  out.y = is_cdir(g, i, j, k, cD) ? T(0) : -a1;
  reinterpret_cast<T2*>(r_s)[t] = out;
}

// residual_vertex after a single forward sweep from x = 0 (same result up to rounding)
template <typename T, bool NT>
__device__ __forceinline__ void residual_after_zero_sweep(const Geom& g, int t, const T* A_s,
                                                          const T* x_s, T* r_s) {
  using T2 = typename V2<T>::type;
  int col, i, j, k;
  if (!colour_decode_wave(g, t, col, i, j, k)) return;
  switch (col) {
    case 0: residual_upper_vertex<T, NT, 0>(g, t, i, j, k, A_s, x_s, r_s); break;
    case 1: residual_upper_vertex<T, NT, 1>(g, t, i, j, k, A_s, x_s, r_s); break;
    case 2: residual_upper_vertex<T, NT, 2>(g, t, i, j, k, A_s, x_s, r_s); break;
    case 3: residual_upper_vertex<T, NT, 3>(g, t, i, j, k, A_s, x_s, r_s); break;
    case 4: residual_upper_vertex<T, NT, 4>(g, t, i, j, k, A_s, x_s, r_s); break;
    case 5: residual_upper_vertex<T, NT, 5>(g, t, i, j, k, A_s, x_s, r_s); break;
    case 6: residual_upper_vertex<T, NT, 6>(g, t, i, j, k, A_s, x_s, r_s); break;
    default: {  // colour 7, the last swept: zero residual
      T2 z;
      z.x = 0;
      z.y = 0;
      reinterpret_cast<T2*>(r_s)[t] = z;
    }
  }
}

// The first forward sweep from x = 0 of colour 0 reads no neighbour: x_v = D_v^{-1} b_v.
// The kernel that writes b (the V-cycle entry, the restriction) does it on the spot.
template <typename T>
__device__ __forceinline__ void zero_start_colour0(const T* D_s, int t, typename V2<T>::type b,
                                                   T* x_s) {
  using T2 = typename V2<T>::type;
  const Block2<T> d = load_block<false>(D_s + sidx<T>(t, 0, 4), 0);
  T2 xv;
  xv.x = d.a00 * b.x + d.a01 * b.y;
  xv.y = d.a10 * b.x + d.a11 * b.y;
  reinterpret_cast<T2*>(x_s)[t] = xv;
}

// restriction b_c = (1/8) P^T r_f of the scaled residual at coarse position t (the
// 1/8 converts the fine row scaling to the coarse one: rows are scaled by
// 1/(hx hy hz)).  x_c: with Dc, the zero-start sweep of colour 0 (zero_start_colour0);
// without, cleared when not null.
template <typename T>
__device__ __forceinline__ void restrict_vertex(const Geom& gf, const Geom& gc, int t,
                                                const T* rf_s, T* bc_s, T* xc_s,
                                                const T* Dc_s = nullptr) {
  using T2 = typename V2<T>::type;
  int cc, I, J, K;
  if (!colour_decode_wave(gc, t, cc, I, J, K)) return;
  const T2* rf = reinterpret_cast<const T2*>(rf_s);
  T a0 = 0, a1 = 0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    const int k = 2 * K + dz;
    if (k < 0 || k >= gf.nz) continue;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int j = 2 * J + dy;
      if (j < 0 || j >= gf.ny) continue;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int i = 2 * I + dx;
        if (i < 0 || i >= gf.nx) continue;
        const T w = (dx ? T(0.5) : T(1)) * (dy ? T(0.5) : T(1)) * (dz ? T(0.5) : T(1));
        const T2 r = rf[colour_encode(gf, i, j, k)];
        a0 += w * r.x;
        a1 += w * r.y;
      }
    }
  }
  double cD;
  T2 out;
  out.x = is_pin(gc, I, J, K) ? T(0) : T(0.125) * a0;
  out.y = is_cdir(gc, I, J, K, cD) ? T(0) : T(0.125) * a1;
  reinterpret_cast<T2*>(bc_s)[t] = out;
  if (Dc_s) {
    if (cc == 0) zero_start_colour0<T>(Dc_s, t, out, xc_s);
  } else if (xc_s) {  // the coarse correction starts from zero
    T2 z;
    z.x = 0;
    z.y = 0;
    reinterpret_cast<T2*>(xc_s)[t] = z;
  }
}

// prolongation and correction x_f += P x_c (trilinear) at fine position t, none in
// Dirichlet rows
template <typename T>
__device__ __forceinline__ void prolong_vertex(const Geom& gf, const Geom& gc, int t,
                                               const T* xc_s, T* xf_s) {
  using T2 = typename V2<T>::type;
  int cf, i, j, k;
  if (!colour_decode_wave(gf, t, cf, i, j, k)) return;
  const T2* xc = reinterpret_cast<const T2*>(xc_s);
  const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1,
            k1 = (k + 1) >> 1;
  const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
  T a0 = 0, a1 = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int I = (c & 1) ? i1 : i0, J = (c & 2) ? j1 : j0, K = (c & 4) ? k1 : k0;
    // the second parent of an even index coincides with the first: count it once
    if (((c & 1) && !(i & 1)) || ((c & 2) && !(j & 1)) || ((c & 4) && !(k & 1))) continue;
    const T2 e = xc[colour_encode_sel(gc, I, J, K)];
    const T w = wi * wj * wk;
    a0 += w * e.x;
    a1 += w * e.y;
  }
  T2* xf = reinterpret_cast<T2*>(xf_s);
  T2 x = xf[t];
  double cD;
  if (!is_pin(gf, i, j, k)) x.x += a0;
  if (!is_cdir(gf, i, j, k, cD)) x.y += a1;
  xf[t] = x;
}

// ---------------------------------------------------------------------------
// one launch per colour sweep / transfer (large grids)
// ---------------------------------------------------------------------------
// The colour sweeps run in workgroups of one wave: the lanes are independent (no LDS,
// no barrier), and a sweep over few positions (a coarse level, a single sample) then
// spreads over more CUs than with 256-lane workgroups (one 129^3 colour: 1072
// workgroups instead of 268 on 256 CUs).  The residual and the transfers, whose
// neighbour reads lose locality in one-wave workgroups, keep 256 lanes.
constexpr int kSweepBlock = 64;
// Matrices of at most this many bytes (all samples of a level) are read with plain
// loads: the small levels' matrices can stay in the last-level cache across sweeps
// and V-cycles, where the large levels' are streamed.
constexpr double kCachedMatrixBytes = 128.0 * 1024 * 1024;

template <typename T>
bool stream_matrix(const Geom& g, int S) {
  return (double)S * kPlanes * g.off[8] * sizeof(T) > kCachedMatrixBytes;
}

// ZC: -1 for a sweep of any colour col, else the zero-start sweep of colour col = ZC
template <typename T, bool NT, int ZC>
__global__ __launch_bounds__(kSweepBlock) void k_smooth(Geom g, int col, const T* A_all, const T* Dinv_all,
                                                   const T* b_all, T* x_all, const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.cnt[col]) return;
  const size_t Np = g.off[8];
  smooth_vertex<T, NT, ZC>(g, col, q, A_all + (size_t)s * kPlanes * Np,
                           Dinv_all + (size_t)s * 4 * Np, b_all + (size_t)s * 2 * Np,
                           x_all + (size_t)s * 2 * Np);
}

template <typename T, bool NT>
auto smooth_kernel(int colour, bool zero_start) {
  if (zero_start) {
    switch (colour) {
      case 0: return k_smooth<T, NT, 0>;
      case 1: return k_smooth<T, NT, 1>;
      case 2: return k_smooth<T, NT, 2>;
      case 3: return k_smooth<T, NT, 3>;
      case 4: return k_smooth<T, NT, 4>;
      case 5: return k_smooth<T, NT, 5>;
      case 6: return k_smooth<T, NT, 6>;
      default: return k_smooth<T, NT, 7>;
    }
  }
  return k_smooth<T, NT, -1>;
}

template <typename T>
void launch_smooth(const Geom& g, int colour, const T* A, const T* Dinv, const T* b, T* x, int S,
                   const int* mask, const int* list, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                   bool zero_start) {
  const int n = g.cnt[colour];
  if (n <= 0) return;
  dim3 grid(ceil_div(n, kSweepBlock), S);
  auto kern = stream_matrix<T>(g, S) ? smooth_kernel<T, true>(colour, zero_start)
                                     : smooth_kernel<T, false>(colour, zero_start);
  if (ev0)  // timed launch: events recorded around this kernel only
    hipExtLaunchKernelGGL(kern, grid, dim3(kSweepBlock), 0, st, ev0, ev1, 0, g, colour, A, Dinv, b, x,
                          mask, list);
  else
    hipLaunchKernelGGL(kern, grid, dim3(kSweepBlock), 0, st, g, colour, A, Dinv, b, x, mask, list);
}

// ZS: the level had a single pre-smoothing sweep, from x = 0
template <typename T, bool NT, bool ZS>
__global__ __launch_bounds__(kBlock) void k_residual(Geom g, const T* A_all, const T* b_all,
                                                     const T* x_all, T* r_all, const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.off[8]) return;
  const size_t Np = g.off[8];
  if (ZS)
    residual_after_zero_sweep<T, NT>(g, t, A_all + (size_t)s * kPlanes * Np,
                                     x_all + (size_t)s * 2 * Np, r_all + (size_t)s * 2 * Np);
  else
    residual_vertex<T, NT>(g, t, A_all + (size_t)s * kPlanes * Np, b_all + (size_t)s * 2 * Np,
                           x_all + (size_t)s * 2 * Np, r_all + (size_t)s * 2 * Np);
}

template <typename T>
void launch_residual(const Geom& g, const T* A, const T* b, const T* x, T* r, int S,
                     const int* mask, const int* list, hipStream_t st, bool zero_sweep) {
  dim3 grid(ceil_div(g.off[8], kBlock), S);
  const bool nt = stream_matrix<T>(g, S);
  auto kern = zero_sweep ? (nt ? k_residual<T, true, true> : k_residual<T, false, true>)
                         : (nt ? k_residual<T, true, false> : k_residual<T, false, false>);
  hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, st, g, A, b, x, r, mask, list);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(Geom gf, Geom gc, const T* rf_all, T* bc_all,
                                                     T* xc_all, const T* Dc_all, const int* mask,
                                                     const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= gc.off[8]) return;
  // x_c and D_c are optional: offset them only when given
  restrict_vertex<T>(gf, gc, t, rf_all + (size_t)s * 2 * gf.off[8],
                     bc_all + (size_t)s * 2 * gc.off[8],
                     xc_all ? xc_all + (size_t)s * 2 * gc.off[8] : nullptr,
                     Dc_all ? Dc_all + (size_t)s * 4 * gc.off[8] : nullptr);
}

template <typename T>
void launch_restrict(const Geom& gf, const Geom& gc, const T* rf, T* bc, T* xc, const T* Dc,
                     int S, const int* mask, const int* list, hipStream_t st) {
  dim3 grid(ceil_div(gc.off[8], kBlock), S);
  hipLaunchKernelGGL(k_restrict<T>, grid, dim3(kBlock), 0, st, gf, gc, rf, bc, xc, Dc, mask,
                     list);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(Geom gf, Geom gc, const T* xc_all, T* xf_all,
                                                    const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= gf.off[8]) return;
  prolong_vertex<T>(gf, gc, t, xc_all + (size_t)s * 2 * gc.off[8],
                    xf_all + (size_t)s * 2 * gf.off[8]);
}

template <typename T>
void launch_prolong(const Geom& gf, const Geom& gc, const T* xc, T* xf, int S, const int* mask,
                    const int* list, hipStream_t st) {
  dim3 grid(ceil_div(gf.off[8], kBlock), S);
  hipLaunchKernelGGL(k_prolong<T>, grid, dim3(kBlock), 0, st, gf, gc, xc, xf, mask, list);
}

// ---------------------------------------------------------------------------
// finest level with an FP16 matrix (EDF_PREC_MIXED_F16).  The FP32 matrix is scaled
// by its diagonal-block inverses, A16_vo = D_v^{-1} A_vo, so the stored entries are
// O(1) whatever the physical units and the diagonal blocks are exactly the identity
// (not read back).  The smoother then needs no block inverse: with bh = D^{-1} b
// (formed once at V-cycle entry), x_v = bh_v - sum_{o != diag} A16_vo x_{v+o}; the
// residual is unscaled with the FP32 diagonal blocks D.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_scale_f16(Geom g, const float* A32_all,
                                                      _Float16* A16_all, float* D_all,
                                                      const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int col, i, j, k;
  if (t >= g.off[8] || !colour_decode_wave(g, t, col, i, j, k)) return;
  const size_t Np = g.off[8];
  const float* a = A32_all + (size_t)s * kPlanes * Np + sidx<float>(t, 0, kPlanes);
  _Float16* h = A16_all + (size_t)s * kPlanes * Np + sidx<_Float16>(t, 0, kPlanes);
  const double d00 = a[soff<float>(kDiag * 4)], d01 = a[soff<float>(kDiag * 4 + 1)],
               d10 = a[soff<float>(kDiag * 4 + 2)], d11 = a[soff<float>(kDiag * 4 + 3)];
  const double det = d00 * d11 - d01 * d10;
  const double id = det != 0.0 ? 1.0 / det : 0.0;
  const double i00 = d11 * id, i01 = -d01 * id, i10 = -d10 * id, i11 = d00 * id;
  for (int o = 0; o < 27; ++o) {
    const double b00 = a[soff<float>(o * 4)], b01 = a[soff<float>(o * 4 + 1)],
                 b10 = a[soff<float>(o * 4 + 2)], b11 = a[soff<float>(o * 4 + 3)];
    double s00 = i00 * b00 + i01 * b10, s01 = i00 * b01 + i01 * b11;
    double s10 = i10 * b00 + i11 * b10, s11 = i10 * b01 + i11 * b11;
    if (o == kDiag) {
      s00 = 1.0;
      s01 = 0.0;
      s10 = 0.0;
      s11 = 1.0;
    }
    h[soff<_Float16>(o * 4)] = (_Float16)s00;
    h[soff<_Float16>(o * 4 + 1)] = (_Float16)s01;
    h[soff<_Float16>(o * 4 + 2)] = (_Float16)s10;
    h[soff<_Float16>(o * 4 + 3)] = (_Float16)s11;
  }
  float* d = D_all + (size_t)s * 4 * Np + sidx<float>(t, 0, 4);
  d[soff<float>(0)] = (float)d00;
  d[soff<float>(1)] = (float)d01;
  d[soff<float>(2)] = (float)d10;
  d[soff<float>(3)] = (float)d11;
}

void launch_scale_f16(const Geom& g, const float* A32, _Float16* A16, float* D32, int S,
                      const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(g.off[8], kBlock), S);
  hipLaunchKernelGGL(k_scale_f16, grid, dim3(kBlock), 0, st, g, A32, A16, D32, mask);
}

// ZC as in k_smooth: -1, or the zero-start sweep of colour col = ZC
template <bool NT, int ZC>
__global__ __launch_bounds__(kSweepBlock) void k_smooth_f16(Geom g, int col, const _Float16* A_all,
                                                       const float* bh_all, float* x_all,
                                                       const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.cnt[col]) return;
  const size_t Np = g.off[8];
  int i, j, k;
  colour_decode_in(g, col, q, i, j, k);
  const int t = g.off[col] + q;
  const _Float16* A = A_all + (size_t)s * kPlanes * Np + sidx<_Float16>(t, 0, kPlanes);
  float2* x = reinterpret_cast<float2*>(x_all + (size_t)s * 2 * Np);
  const float2 bv = reinterpret_cast<const float2*>(bh_all + (size_t)s * 2 * Np)[t];
  const NbrMap nm = nbr_map(g, col, i, j, k);
  float r0 = bv.x, r1 = bv.y;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int o = nb_index(dx, dy, dz);
        if (o == kDiag) continue;  // the unit diagonal block
        if (ZC >= 0 && !zero_start_reads(ZC, dx, dy, dz)) continue;
        const float2 xv = load_nbr(x, g, nm, dx, dy, dz);
        const Block2<float> a = load_block<NT>(A, o * 4);
        r0 -= a.a00 * xv.x + a.a01 * xv.y;
        r1 -= a.a10 * xv.x + a.a11 * xv.y;
      }
    }
  }
  x[t] = make_float2(r0, r1);
}

template <bool NT>
auto smooth_f16_kernel(int colour, bool zero_start) {
  if (zero_start) {
    switch (colour) {
      case 0: return k_smooth_f16<NT, 0>;
      case 1: return k_smooth_f16<NT, 1>;
      case 2: return k_smooth_f16<NT, 2>;
      case 3: return k_smooth_f16<NT, 3>;
      case 4: return k_smooth_f16<NT, 4>;
      case 5: return k_smooth_f16<NT, 5>;
      case 6: return k_smooth_f16<NT, 6>;
      default: return k_smooth_f16<NT, 7>;
    }
  }
  return k_smooth_f16<NT, -1>;
}

void launch_smooth_f16(const Geom& g, int colour, const _Float16* A16, const float* bh, float* x,
                       int S, const int* mask, const int* list, hipStream_t st, hipEvent_t ev0,
                       hipEvent_t ev1,
                       bool zero_start) {
  const int n = g.cnt[colour];
  if (n <= 0) return;
  dim3 grid(ceil_div(n, kSweepBlock), S);
  const bool stream = (double)S * kPlanes * g.off[8] * sizeof(_Float16) > kCachedMatrixBytes;
  auto kern = stream ? smooth_f16_kernel<true>(colour, zero_start)
                     : smooth_f16_kernel<false>(colour, zero_start);
  if (ev0)
    hipExtLaunchKernelGGL(kern, grid, dim3(kSweepBlock), 0, st, ev0, ev1, 0, g, colour, A16, bh, x,
                          mask, list);
  else
    hipLaunchKernelGGL(kern, grid, dim3(kSweepBlock), 0, st, g, colour, A16, bh, x, mask, list);
}

// r = D (bh - A16 x) after a single forward sweep from x = 0 at position t of colour
// C < 7: that sweep left x_v = bh_v - (sum over the colours below C of A16_vo x_{v+o}), so
// r_v = -D_v (sum over the colours above C of A16_vo x_{v+o})
template <bool NT, int C>
__device__ __forceinline__ void residual_f16_upper_vertex(const Geom& g, int t, int i, int j,
                                                          int k, const _Float16* A_s,
                                                          const float* D_s, const float* x_s,
                                                          float* r_s) {
  const NbrMap nm = nbr_map(g, C, i, j, k);
  const _Float16* A = A_s + sidx<_Float16>(t, 0, kPlanes);
  const float2* x = reinterpret_cast<const float2*>(x_s);
  float a0 = 0.f, a1 = 0.f;
  auto plane = [&](int dz, auto mz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (nbr_colour(C, dx, dy, decltype(mz)::value) <= C) continue;
        const float2 xv = load_nbr(x, g, nm, dx, dy, dz);
        const Block2<float> a = load_block<NT>(A, nb_index(dx, dy, dz) * 4);
        a0 += a.a00 * xv.x + a.a01 * xv.y;
        a1 += a.a10 * xv.x + a.a11 * xv.y;
      }
    }
  };
#pragma unroll 1
  for (int dz = -1; dz <= 1; dz += 2) plane(dz, std::integral_constant<int, 1>());
  plane(0, std::integral_constant<int, 0>());
  const Block2<float> d = load_block<NT>(D_s + sidx<float>(t, 0, 4), 0);
  double cD;
  float2 out;
  out.x = is_pin(g, i, j, k) ? 0.f : -(d.a00 * a0 + d.a01 * a1);
  out.y = is_cdir(g, i, j, k, cD) ? 0.f : -(d.a10 * a0 + d.a11 * a1);
  reinterpret_cast<float2*>(r_s)[t] = out;
}

// ZS: the level had a single pre-smoothing sweep, from x = 0
template <bool NT, bool ZS>
__global__ __launch_bounds__(kBlock) void k_residual_f16(Geom g, const _Float16* A_all,
                                                         const float* D_all, const float* bh_all,
                                                         const float* x_all, float* r_all,
                                                         const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t Np = g.off[8];
  if (t >= g.off[7]) {  // the last colour swept: zero residual (see residual_vertex)
    if (t < g.off[8] && t - g.off[7] < g.cnt[7])
      reinterpret_cast<float2*>(r_all + (size_t)s * 2 * Np)[t] = make_float2(0.f, 0.f);
    return;
  }
  int col, i, j, k;
  if (!colour_decode_wave(g, t, col, i, j, k)) return;
  if (ZS) {
    const _Float16* A = A_all + (size_t)s * kPlanes * Np;
    const float* D = D_all + (size_t)s * 4 * Np;
    const float* x = x_all + (size_t)s * 2 * Np;
    float* r = r_all + (size_t)s * 2 * Np;
    switch (col) {
      case 0: residual_f16_upper_vertex<NT, 0>(g, t, i, j, k, A, D, x, r); break;
      case 1: residual_f16_upper_vertex<NT, 1>(g, t, i, j, k, A, D, x, r); break;
      case 2: residual_f16_upper_vertex<NT, 2>(g, t, i, j, k, A, D, x, r); break;
      case 3: residual_f16_upper_vertex<NT, 3>(g, t, i, j, k, A, D, x, r); break;
      case 4: residual_f16_upper_vertex<NT, 4>(g, t, i, j, k, A, D, x, r); break;
      case 5: residual_f16_upper_vertex<NT, 5>(g, t, i, j, k, A, D, x, r); break;
      default: residual_f16_upper_vertex<NT, 6>(g, t, i, j, k, A, D, x, r); break;
    }
    return;
  }
  const NbrMap nm = nbr_map(g, col, i, j, k);
  const _Float16* A = A_all + (size_t)s * kPlanes * Np + sidx<_Float16>(t, 0, kPlanes);
  const float2* x = reinterpret_cast<const float2*>(x_all + (size_t)s * 2 * Np);
  float a0 = 0.f, a1 = 0.f;  // (A16 x)_v
#pragma unroll 1
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const float2 xv = load_nbr(x, g, nm, dx, dy, dz);
        if (dx == 0 && dy == 0 && dz == 0) {
          a0 += xv.x;
          a1 += xv.y;
        } else {
          const Block2<float> a = load_block<NT>(A, nb_index(dx, dy, dz) * 4);
          a0 += a.a00 * xv.x + a.a01 * xv.y;
          a1 += a.a10 * xv.x + a.a11 * xv.y;
        }
      }
    }
  }
  const float2 bv = reinterpret_cast<const float2*>(bh_all + (size_t)s * 2 * Np)[t];
  const Block2<float> d = load_block<NT>(D_all + (size_t)s * 4 * Np + sidx<float>(t, 0, 4), 0);
  const float u0 = bv.x - a0, u1 = bv.y - a1;
  double cD;
  float2 out;
  out.x = is_pin(g, i, j, k) ? 0.f : d.a00 * u0 + d.a01 * u1;
  out.y = is_cdir(g, i, j, k, cD) ? 0.f : d.a10 * u0 + d.a11 * u1;
  reinterpret_cast<float2*>(r_all + (size_t)s * 2 * Np)[t] = out;
}

void launch_residual_f16(const Geom& g, const _Float16* A16, const float* D32, const float* bh,
                         const float* x, float* r, int S, const int* mask, const int* list,
                         hipStream_t st, bool zero_sweep) {
  dim3 grid(ceil_div(g.off[8], kBlock), S);
  const bool stream = (double)S * kPlanes * g.off[8] * sizeof(_Float16) > kCachedMatrixBytes;
  auto kern = zero_sweep ? (stream ? k_residual_f16<true, true> : k_residual_f16<false, true>)
                         : (stream ? k_residual_f16<true, false> : k_residual_f16<false, false>);
  hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, st, g, A16, D32, bh, x, r, mask, list);
}

__global__ __launch_bounds__(kBlock) void k_to_colour_scaled(Geom g, const double* in_all,
                                                             const float* D_all, float* out_all,
                                                             float* x_all, const int* mask,
                                                             const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int col, i, j, k;
  if (t >= g.off[8] || !colour_decode_wave(g, t, col, i, j, k)) return;
  const size_t v = i + (size_t)g.nx * (j + (size_t)g.ny * k);
  const double2 b = reinterpret_cast<const double2*>(in_all)[(size_t)s * g.N + v];
  const float* d = D_all + (size_t)s * 4 * g.off[8] + sidx<float>(t, 0, 4);
  const double d00 = d[soff<float>(0)], d01 = d[soff<float>(1)], d10 = d[soff<float>(2)],
               d11 = d[soff<float>(3)];
  const double det = d00 * d11 - d01 * d10;
  const double id = det != 0.0 ? 1.0 / det : 0.0;
  const float2 bh =
      make_float2((float)((d11 * b.x - d01 * b.y) * id), (float)((d00 * b.y - d10 * b.x) * id));
  reinterpret_cast<float2*>(out_all)[(size_t)s * g.off[8] + t] = bh;
  // the zero-start sweep of colour 0 with the unit-diagonal FP16 matrix: x = bh
  if (x_all && col == 0) reinterpret_cast<float2*>(x_all)[(size_t)s * g.off[8] + t] = bh;
}

void launch_to_colour_scaled(const Geom& g, const double* in, const float* D32, float* out,
                             float* x, int S, const int* mask, const int* list, hipStream_t st) {
  hipLaunchKernelGGL(k_to_colour_scaled, dim3(ceil_div(g.off[8], kBlock), S), dim3(kBlock), 0, st,
                     g, in, D32, out, x, mask, list);
}

// ---------------------------------------------------------------------------
// fills and precision casts
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* x, size_t n, T value, const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  T* xs = x + (size_t)s * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    xs[e] = value;
}

template <typename T>
void launch_fill(T* x, size_t per_sample, int S, const int* mask, T value, hipStream_t st) {
  const int nb = (int)std::min<size_t>(ceil_div((int)std::min<size_t>(per_sample, 1u << 30), kBlock), 4096);
  dim3 grid(nb > 0 ? nb : 1, S);
  hipLaunchKernelGGL(k_fill<T>, grid, dim3(kBlock), 0, st, x, per_sample, value, mask);
}

// V-cycle entry and exit on the finest level: Krylov vectors (FP64, natural vertex
// order [N][2]) to and from the V-cycle vectors (T, colour-major [Np][2])
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_colour(Geom g, const double* in_all, T* out_all,
                                                      const T* D_all, T* x_all, const int* mask,
                                                      const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int col, i, j, k;
  if (t >= g.off[8] || !colour_decode_wave(g, t, col, i, j, k)) return;
  const size_t v = i + (size_t)g.nx * (j + (size_t)g.ny * k);
  const double2 a = reinterpret_cast<const double2*>(in_all)[(size_t)s * g.N + v];
  typename V2<T>::type b;
  b.x = (T)a.x;
  b.y = (T)a.y;
  reinterpret_cast<typename V2<T>::type*>(out_all)[(size_t)s * g.off[8] + t] = b;
  if (D_all && col == 0)
    zero_start_colour0<T>(D_all + (size_t)s * 4 * g.off[8], t, b, x_all + (size_t)s * 2 * g.off[8]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_from_colour(Geom g, const T* in_all, double* out_all,
                                                        const int* mask, const int* list) {
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.N) return;
  const int i = v % g.nx, j = (v / g.nx) % g.ny, k = v / (g.nx * g.ny);
  const typename V2<T>::type a =
      reinterpret_cast<const typename V2<T>::type*>(in_all)[(size_t)s * g.off[8] +
                                                           colour_encode_sel(g, i, j, k)];
  reinterpret_cast<double2*>(out_all)[(size_t)s * g.N + v] = make_double2((double)a.x, (double)a.y);
}

template <typename T>
void launch_to_colour(const Geom& g, const double* in, T* out, const T* D, T* x, int S,
                      const int* mask, const int* list, hipStream_t st) {
  hipLaunchKernelGGL(k_to_colour<T>, dim3(ceil_div(g.off[8], kBlock), S), dim3(kBlock), 0, st, g,
                     in, out, D, x, mask, list);
}

template <typename T>
void launch_from_colour(const Geom& g, const T* in, double* out, int S, const int* mask,
                        const int* list, hipStream_t st) {
  hipLaunchKernelGGL(k_from_colour<T>, dim3(ceil_div(g.N, kBlock), S), dim3(kBlock), 0, st, g,
                     in, out, mask, list);
}

// ---------------------------------------------------------------------------
// coarsest grid: dense matrix (natural unknown order 2v+var), explicit inverse by
// Gauss-Jordan elimination with partial pivoting, applied as a dense product
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_coarse_dense(Geom g, const double* A_all, double* M_all,
                                                         const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int col, i, j, k;
  if (t >= g.off[8] || !colour_decode_wave(g, t, col, i, j, k)) return;
  const size_t N = g.N, n = 2 * N;
  const double* A = A_all + (size_t)s * kPlanes * g.off[8] + sidx<double>(t, 0, kPlanes);
  double* M = M_all + (size_t)s * n * n;
  const size_t v = i + (size_t)g.nx * (j + (size_t)g.ny * k);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        if (ii < 0 || jj < 0 || kk < 0 || ii >= g.nx || jj >= g.ny || kk >= g.nz) continue;
        const size_t w = ii + (size_t)g.nx * (jj + (size_t)g.ny * kk);
        const int o = nb_index(dx, dy, dz);
        for (int e = 0; e < 2; ++e)
          for (int var = 0; var < 2; ++var)
            M[(2 * v + e) * n + 2 * w + var] = A[soff<double>(o * 4 + e * 2 + var)];
      }
}

void launch_coarse_dense(const Geom& g, const double* A, double* M, int S, const int* mask,
                         hipStream_t st) {
  const size_t n = 2 * (size_t)g.N;
  launch_fill<double>(M, n * n, S, mask, 0.0, st);
  dim3 grid(ceil_div(g.off[8], kBlock), S);
  hipLaunchKernelGGL(k_coarse_dense, grid, dim3(kBlock), 0, st, g, A, M, mask);
}

constexpr int kGJThreads = 1024;

__global__ __launch_bounds__(kGJThreads) void k_gauss_jordan(int n, double* M_all, int* piv_all,
                                                             int* status, const int* mask) {
  const int s = blockIdx.x;
  if (mask && !mask[s]) return;
  double* M = M_all + (size_t)s * n * n;
  int* piv = piv_all + (size_t)s * n;
  __shared__ double rowk[kMaxCoarse];
  __shared__ double colk[kMaxCoarse];
  __shared__ double red_v[kGJThreads];
  __shared__ int red_i[kGJThreads];
  __shared__ double s_pivinv;
  __shared__ int s_p;
  const int tid = threadIdx.x, nt = blockDim.x;
  bool singular = false;
  for (int k = 0; k < n; ++k) {
    // pivot: largest |M[i][k]|, i >= k, smallest i on ties
    double bv = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += nt) {
      const double a = fabs(M[(size_t)i * n + k]);
      if (a > bv) {
        bv = a;
        bi = i;
      }
    }
    red_v[tid] = bv;
    red_i[tid] = bi;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) {
        const double ov = red_v[tid + w];
        const int oi = red_i[tid + w];
        if (ov > red_v[tid] || (ov == red_v[tid] && oi < red_i[tid])) {
          red_v[tid] = ov;
          red_i[tid] = oi;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      s_p = red_i[0];
      piv[k] = s_p;
    }
    __syncthreads();
    const int p = s_p;
    if (p != k)
      for (int j = tid; j < n; j += nt) {
        const double a = M[(size_t)k * n + j];
        M[(size_t)k * n + j] = M[(size_t)p * n + j];
        M[(size_t)p * n + j] = a;
      }
    __syncthreads();
    if (tid == 0) {
      const double d = M[(size_t)k * n + k];
      s_pivinv = d != 0.0 ? 1.0 / d : 0.0;
    }
    __syncthreads();
    const double pivinv = s_pivinv;
    if (pivinv == 0.0) singular = true;
    for (int j = tid; j < n; j += nt) rowk[j] = (j == k) ? pivinv : M[(size_t)k * n + j] * pivinv;
    for (int i = tid; i < n; i += nt) colk[i] = (i == k) ? 0.0 : M[(size_t)i * n + k];
    __syncthreads();
    const int nn = n * n;
    for (int idx = tid; idx < nn; idx += nt) {
      const int i = idx / n, j = idx - i * n;
      if (i == k)
        M[idx] = rowk[j];
      else if (j == k)
        M[idx] = -colk[i] * pivinv;
      else
        M[idx] -= colk[i] * rowk[j];
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int i = tid; i < n; i += nt) {
        const double a = M[(size_t)i * n + k];
        M[(size_t)i * n + k] = M[(size_t)i * n + p];
        M[(size_t)i * n + p] = a;
      }
    __syncthreads();
  }
  if (tid == 0 && status) status[s] = singular ? 1 : 0;
}

void launch_gauss_jordan(int n, double* M, int* piv, int* status, int S, const int* mask,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_gauss_jordan, dim3(S), dim3(kGJThreads), 0, st, n, M, piv, status, mask);
}

// ---------------------------------------------------------------------------
// bottom of the V-cycle in one launch: one workgroup per sample runs the smoothed
// levels l0..n-2 of F and the dense coarse solve on level n-1, with workgroup
// barriers between the sweeps (all levels are small: at most kFuseMaxN vertices).
// When the levels' vectors fit, they live in LDS for the whole launch, so that a sweep
// waits only for its matrix reads.
// ---------------------------------------------------------------------------
constexpr int kFusedThreads = 1024;

// One vertical-line sweep of column colour cc inside the fused bottom (the workgroup's
// threads over the level's columns): first every (column, k) at once, r_k = b_k - (the
// other columns' couplings) A x and e_k = M_k^{-1} r_k, G_k = M_k^{-1} L_k, C_k into the
// LDS values scr [10][nz][columns]; then one thread per column runs d_k = e_k - G_k d_{k-1}
// and x_k = d_k - C_k x_{k+1}.  The rows of each k-parity are taken in a loop of their own,
// so that the vertex colour (cc + 4 parity) is the same across a wave.  The same
// arithmetic as k_line_sweep, as a phase of the fused launch.
template <typename T>
__device__ __forceinline__ void bottom_line_sweep(const Geom& g, int cc, const T* A, const T* F,
                                                  const T* b_s, T* x_s, T* scr, int tid, int nt) {
  using T2 = typename V2<T>::type;
  const int mx = g.mx[cc], ncol = mx * g.my[cc], nz = g.nz;
  auto L_at = [&](int v, int k, int c) -> T& { return scr[((size_t)v * nz + k) * ncol + c]; };
  const T2* b = reinterpret_cast<const T2*>(b_s);
  T2* x = reinterpret_cast<T2*>(x_s);
  for (int par = 0; par < 2; ++par) {
    const int rows = par ? nz / 2 : (nz + 1) / 2;
    const int col = cc + 4 * par;
    for (int idx = tid; idx < ncol * rows; idx += nt) {
      const int q = idx % ncol, k = par + 2 * (idx / ncol);
      const int i = 2 * (q % mx) + (cc & 1), j = 2 * (q / mx) + (cc >> 1);
      const int t = line_pos(g, cc, q, k);
      const NbrMap nm = nbr_map(g, col, i, j, k);
      const T* a = A + sidx<T>(t, 0, kPlanes);
      const T2 bv = b[t];
      T r0 = bv.x, r1 = bv.y;
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;  // the column itself: solved below
            const T2 xv = load_nbr(x, g, nm, dx, dy, dz);
            const Block2<T> blk = load_block<false>(a, nb_index(dx, dy, dz) * 4);
            r0 -= blk.a00 * xv.x + blk.a01 * xv.y;
            r1 -= blk.a10 * xv.x + blk.a11 * xv.y;
          }
        }
      }
      const Block2<T> l = load_block<false>(a, kLineL * 4);
      const T* f = F + sidx<T>(t, 0, kLineFactors);
      const Block2<T> mi = load_block<false>(f, 0);
      const Block2<T> c = load_block<false>(f, 4);
      L_at(0, k, q) = mi.a00 * r0 + mi.a01 * r1;
      L_at(1, k, q) = mi.a10 * r0 + mi.a11 * r1;
      L_at(2, k, q) = mi.a00 * l.a00 + mi.a01 * l.a10;
      L_at(3, k, q) = mi.a00 * l.a01 + mi.a01 * l.a11;
      L_at(4, k, q) = mi.a10 * l.a00 + mi.a11 * l.a10;
      L_at(5, k, q) = mi.a10 * l.a01 + mi.a11 * l.a11;
      L_at(6, k, q) = c.a00;
      L_at(7, k, q) = c.a01;
      L_at(8, k, q) = c.a10;
      L_at(9, k, q) = c.a11;
    }
  }
  __syncthreads();
  for (int q = tid; q < ncol; q += nt) {
    T d0 = 0, d1 = 0;
    for (int k = 0; k < nz; ++k) {  // d_k = e_k - G_k d_{k-1}, kept in place of e_k
      const T n0 = L_at(0, k, q) - (L_at(2, k, q) * d0 + L_at(3, k, q) * d1);
      const T n1 = L_at(1, k, q) - (L_at(4, k, q) * d0 + L_at(5, k, q) * d1);
      d0 = n0;
      d1 = n1;
      L_at(0, k, q) = n0;
      L_at(1, k, q) = n1;
    }
    T y0 = 0, y1 = 0;
    for (int k = nz - 1; k >= 0; --k) {  // x_k = d_k - C_k x_{k+1}
      const T n0 = L_at(0, k, q) - (L_at(6, k, q) * y0 + L_at(7, k, q) * y1);
      const T n1 = L_at(1, k, q) - (L_at(8, k, q) * y0 + L_at(9, k, q) * y1);
      y0 = n0;
      y1 = n1;
      T2 o;
      o.x = n0;
      o.y = n1;
      x[line_pos(g, cc, q, k)] = o;
    }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kFusedThreads) void k_vcycle_bottom(const FusedLevels<T>* __restrict__ Fp,
                                                                 const int* mask, const int* list) {
  // the levels' x, b and r in LDS when F.lds_off says so (the dynamic LDS of the launch)
  extern __shared__ double lds_vec[];
  const FusedLevels<T>& F = *Fp;
  const int s = list ? list[blockIdx.x] : blockIdx.x;
  if (mask && !mask[s]) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const bool in_lds = F.lds_off[0] >= 0;
  T* lds = reinterpret_cast<T*>(lds_vec);
  auto A = [&](int l) { return F.A[l] + (size_t)s * kPlanes * F.g[l].off[8]; };
  auto D = [&](int l) { return F.D[l] + (size_t)s * 4 * F.g[l].off[8]; };
  auto X = [&](int l) {
    return in_lds ? lds + F.lds_off[l] : F.x[l] + (size_t)s * 2 * F.g[l].off[8];
  };
  auto B = [&](int l) {
    return in_lds ? lds + F.lds_off[l] + 2 * F.g[l].off[8] : F.b[l] + (size_t)s * 2 * F.g[l].off[8];
  };
  auto Rv = [&](int l) {
    return in_lds ? lds + F.lds_off[l] + 4 * F.g[l].off[8] : F.r[l] + (size_t)s * 2 * F.g[l].off[8];
  };
  // vertical-line smoothing of the levels with line factors (LF), points otherwise
  auto line = [&](int l) { return F.line_lds >= 0 && F.LF[l] != nullptr; };
  auto LF = [&](int l) { return F.LF[l] + (size_t)s * kLineFactors * F.g[l].off[8]; };
  T* scr = lds + (F.line_lds >= 0 ? F.line_lds : 0);
  const int last = F.n - 1;
  // x = 0 on the first fused level (the finer levels' restriction clears the others);
  // in LDS the first level's right-hand side is brought in from device memory
  for (int e = tid; e < 2 * F.g[0].off[8]; e += nt) {
    X(0)[e] = T(0);
    if (in_lds) B(0)[e] = F.b[0][(size_t)s * 2 * F.g[0].off[8] + e];
  }
  __syncthreads();
  for (int l = 0; l < last; ++l) {
    const Geom& g = F.g[l];
    for (int it = 0; it < F.nu1; ++it) {
      if (line(l)) {
        for (int cc = 0; cc < 4; ++cc) bottom_line_sweep<T>(g, cc, A(l), LF(l), B(l), X(l), scr, tid, nt);
        continue;
      }
      for (int c = 0; c < 8; ++c) {
        for (int q = tid; q < g.cnt[c]; q += nt)
          smooth_vertex<T, false>(g, c, q, A(l), D(l), B(l), X(l));
        __syncthreads();
      }
    }
    for (int t = tid; t < g.off[8]; t += nt)
      residual_vertex<T, false>(g, t, A(l), B(l), X(l), Rv(l));
    __syncthreads();
    for (int t = tid; t < F.g[l + 1].off[8]; t += nt)
      restrict_vertex<T>(g, F.g[l + 1], t, Rv(l), B(l + 1), X(l + 1));
    __syncthreads();
  }
  {  // coarsest level: x = M^{-1} b, one wave per row; M is in the natural unknown
     // order 2v + var, so b is gathered into that order first
    __shared__ double bn[kMaxCoarse];
    const Geom& gc = F.g[last];
    const int n = F.nc, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    const double* Minv = F.Minv + (size_t)s * n * n;
    const T* b = B(last);
    T* x = X(last);
    auto pos = [&](int e) {  // natural unknown e -> colour-major unknown
      const int v = e >> 1;
      const int i = v % gc.nx, j = (v / gc.nx) % gc.ny, k = v / (gc.nx * gc.ny);
      return 2 * colour_encode_sel(gc, i, j, k) + (e & 1);
    };
    for (int e = tid; e < n; e += nt) bn[e] = (double)b[pos(e)];
    __syncthreads();
    for (int row = wave; row < n; row += nw) {
      double acc = 0.0;
      for (int j = lane; j < n; j += 64) acc += Minv[(size_t)row * n + j] * bn[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
      if (lane == 0) x[pos(row)] = (T)acc;
    }
    __syncthreads();
  }
  for (int l = last - 1; l >= 0; --l) {
    const Geom& g = F.g[l];
    for (int t = tid; t < g.off[8]; t += nt) prolong_vertex<T>(g, F.g[l + 1], t, X(l + 1), X(l));
    __syncthreads();
    for (int it = 0; it < F.nu2; ++it) {
      if (line(l)) {
        for (int cc = 3; cc >= 0; --cc) bottom_line_sweep<T>(g, cc, A(l), LF(l), B(l), X(l), scr, tid, nt);
        continue;
      }
      for (int c = 7; c >= 0; --c) {
        for (int q = tid; q < g.cnt[c]; q += nt)
          smooth_vertex<T, false>(g, c, q, A(l), D(l), B(l), X(l));
        __syncthreads();
      }
    }
  }
  if (in_lds)  // the first level's correction goes back for the finer level's prolongation
    for (int e = tid; e < 2 * F.g[0].off[8]; e += nt)
      F.x[0][(size_t)s * 2 * F.g[0].off[8] + e] = X(0)[e];
}

// dynamic LDS the kernel may take: the device's per-workgroup limit less the static
// part (the coarse right-hand side) and a margin; 0 if the device does not grant it
constexpr size_t kBottomStaticLds = kMaxCoarse * sizeof(double);

template <typename T>
size_t vcycle_bottom_lds_limit() {
  static size_t limit = [] {
    int dev = 0, per_block = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess ||
        (size_t)per_block <= kBottomStaticLds + 1024)
      return (size_t)0;
    const size_t want = (size_t)per_block - kBottomStaticLds - 1024;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vcycle_bottom<T>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)want);
    return e == hipSuccess ? want : (size_t)0;
  }();
  return limit;
}

template <typename T>
void launch_vcycle_bottom(const FusedLevels<T>* F, size_t lds_bytes, int S, const int* mask,
                          const int* list, hipStream_t st) {
  hipLaunchKernelGGL(k_vcycle_bottom<T>, dim3(S), dim3(kFusedThreads), lds_bytes, st, F, mask,
                     list);
}

// explicit instantiations
#define EDF_INST(T)                                                                              \
  template void launch_smooth<T>(const Geom&, int, const T*, const T*, const T*, T*, int,        \
                                 const int*, const int*, hipStream_t, hipEvent_t, hipEvent_t,    \
                                 bool);                                                          \
  template void launch_residual<T>(const Geom&, const T*, const T*, const T*, T*, int,           \
                                   const int*, const int*, hipStream_t, bool);                   \
  template void launch_restrict<T>(const Geom&, const Geom&, const T*, T*, T*, const T*, int,    \
                                   const int*, const int*, hipStream_t);                         \
  template void launch_prolong<T>(const Geom&, const Geom&, const T*, T*, int, const int*,       \
                                  const int*, hipStream_t);                                      \
  template void launch_fill<T>(T*, size_t, int, const int*, T, hipStream_t);                     \
  template void launch_to_colour<T>(const Geom&, const double*, T*, const T*, T*, int,           \
                                    const int*, const int*, hipStream_t);                        \
  template void launch_from_colour<T>(const Geom&, const T*, double*, int, const int*,           \
                                      const int*, hipStream_t);                                  \
  template void launch_vcycle_bottom<T>(const FusedLevels<T>*, size_t, int, const int*,         \
                                        const int*, hipStream_t);                                \
  template size_t vcycle_bottom_lds_limit<T>();
EDF_INST(double)
EDF_INST(float)
template void launch_fill<int>(int*, size_t, int, const int*, int, hipStream_t);

}  // namespace edf
