// Vertical-line (z-column) block Gauss-Seidel smoother of the multigrid V-cycle.
//
// The paper smooths with ILU_beta (Section 2.3), whose point of strength is strong
// directional coupling.  In the Elder problem the sinking brine fingers and the rising
// fresh water make the salt equation convection-dominated mostly along z, where a point
// smoother leaves the error of long vertical couplings in place.  This smoother solves
// each vertical column of 2x2-block unknowns exactly (block tridiagonal along z, the
// couplings to the other 8 neighbouring columns taken from their current values), and
// orders the columns in 4 colours (i % 2, j % 2): the 27-point stencil couples a column
// only with columns of other colours, so every colour is one parallel pass.
//
// Column q of colour cc is (i, j) = (2 (q % mx) + (cc & 1), 2 (q / mx) + (cc >> 1)) with
// mx = g.mx[cc], my = g.my[cc]; its vertex at height k has vertex colour cc + 4 (k & 1)
// and place q + mx my (k >> 1) in that colour (mx and my depend on the x and y parity
// only), so for a fixed k the columns of a wave read consecutive stencil rows.
//
// The matrix is stored in M: the vectors' type T, or FP16 on a finest level of the
// FP32 V-cycle (EDF_PREC_MIXED_F16).  The FP16 matrix is D^{-1} A, scaled by its
// diagonal-block inverses (identity diagonal blocks, O(1) entries), and b holds D^{-1} b,
// so the sweep solves the same system scaled row by row; its residual is unscaled by D.
#include <hip/hip_ext.h>

#include <type_traits>

#include "fv_common.h"

namespace edf {


// ---------------------------------------------------------------------------
// block LU of each column's tridiagonal part, from the top: M_k = D_k - L_k C_{k-1},
// C_k = M_k^{-1} U_k (C_{-1} = 0); F[0..3] = M_k^{-1}, F[4..7] = C_k, computed in FP64
// ---------------------------------------------------------------------------
template <typename M, typename T>
__global__ __launch_bounds__(64) void k_line_factor(Geom g, const M* A_all, T* F_all,
                                                    const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int cc = blockIdx.z;
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q >= g.mx[cc] * g.my[cc]) return;
  const size_t Np = g.off[8];
  const M* A = A_all + (size_t)s * kPlanes * Np;
  T* F = F_all + (size_t)s * kLineFactors * Np;
  // the FP16 matrix is scaled by its diagonal-block inverses: its diagonal blocks are I
  constexpr bool unit = std::is_same<M, _Float16>::value;
  double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
  for (int k = 0; k < g.nz; ++k) {
    const int t = line_pos(g, cc, q, k);
    const M* a = A + sidx<M>(t, 0, kPlanes);
    auto val = [&](int o, int e) { return (double)a[soff<M>(o * 4 + e)]; };
    const double l00 = val(kLineL, 0), l01 = val(kLineL, 1), l10 = val(kLineL, 2),
                 l11 = val(kLineL, 3);
    const double d00 = unit ? 1.0 : val(kDiag, 0), d01 = unit ? 0.0 : val(kDiag, 1),
                 d10 = unit ? 0.0 : val(kDiag, 2), d11 = unit ? 1.0 : val(kDiag, 3);
    const double m00 = d00 - (l00 * c00 + l01 * c10);
    const double m01 = d01 - (l00 * c01 + l01 * c11);
    const double m10 = d10 - (l10 * c00 + l11 * c10);
    const double m11 = d11 - (l10 * c01 + l11 * c11);
    const double det = m00 * m11 - m01 * m10;
    const double id = det != 0.0 ? 1.0 / det : 0.0;
    const double i00 = m11 * id, i01 = -m01 * id, i10 = -m10 * id, i11 = m00 * id;
    const double u00 = val(kLineU, 0), u01 = val(kLineU, 1), u10 = val(kLineU, 2),
                 u11 = val(kLineU, 3);
    c00 = i00 * u00 + i01 * u10;
    c01 = i00 * u01 + i01 * u11;
    c10 = i10 * u00 + i11 * u10;
    c11 = i10 * u01 + i11 * u11;
    T* f = F + sidx<T>(t, 0, kLineFactors);
    f[soff<T>(0)] = (T)i00;
    f[soff<T>(1)] = (T)i01;
    f[soff<T>(2)] = (T)i10;
    f[soff<T>(3)] = (T)i11;
    f[soff<T>(4)] = (T)c00;
    f[soff<T>(5)] = (T)c01;
    f[soff<T>(6)] = (T)c10;
    f[soff<T>(7)] = (T)c11;
  }
}

template <typename M, typename T>
void launch_line_factor_m(const Geom& g, const M* A, T* F, int S, const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(g.mx[0] * g.my[0], 64), S, 4);
  hipLaunchKernelGGL((k_line_factor<M, T>), grid, dim3(64), 0, st, g, A, F, mask);
}

template <typename T>
void launch_line_factor(const Geom& g, const T* A, T* F, int S, const int* mask, hipStream_t st) {
  launch_line_factor_m<T, T>(g, A, F, S, mask, st);
}

void launch_line_factor_f16(const Geom& g, const _Float16* A, float* F, int S, const int* mask,
                            hipStream_t st) {
  launch_line_factor_m<_Float16, float>(g, A, F, S, mask, st);
}

// ---------------------------------------------------------------------------
// one sweep of column colour cc: for every column, r_k = b_k - sum over the other
// columns' neighbours of A x, then the column's block tridiagonal system is solved with
// the factors (forward: d_k = M_k^{-1} (r_k - L_k d_{k-1}), stored in x; backward:
// x_k = d_k - C_k x_{k+1}).  ZC >= 0: the first forward sweep of a level whose x is zero
// on entry, for cc = ZC: only the columns of the colours already swept are read.
// ---------------------------------------------------------------------------
template <typename T, typename M, bool NT, int ZC>
__global__ __launch_bounds__(64) void k_line_smooth(Geom g, int cc, const M* A_all,
                                                    const T* F_all, const T* b_all, T* x_all,
                                                    const int* mask, const int* list) {
  using T2 = typename V2<T>::type;
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int mx = g.mx[cc];
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q >= mx * g.my[cc]) return;
  const int i = 2 * (q % mx) + (cc & 1), j = 2 * (q / mx) + (cc >> 1);
  const size_t Np = g.off[8];
  const M* A = A_all + (size_t)s * kPlanes * Np;
  const T* F = F_all + (size_t)s * kLineFactors * Np;
  const T2* b = reinterpret_cast<const T2*>(b_all + (size_t)s * 2 * Np);
  T2* x = reinterpret_cast<T2*>(x_all + (size_t)s * 2 * Np);
  T d0 = 0, d1 = 0;
  for (int k = 0; k < g.nz; ++k) {
    const int col = cc + 4 * (k & 1);
    const int t = line_pos(g, cc, q, k);
    const NbrMap nm = nbr_map(g, col, i, j, k);
    const M* a = A + sidx<M>(t, 0, kPlanes);
    const T2 bv = b[t];
    T r0 = bv.x, r1 = bv.y;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx == 0 && dy == 0) continue;  // the column itself: solved below
          if (ZC >= 0 && !line_zero_start_reads(ZC, dx, dy)) continue;
          const T2 xv = load_nbr(x, g, nm, dx, dy, dz);
          const Block2<T> blk = load_block<NT>(a, nb_index(dx, dy, dz) * 4);
          r0 -= blk.a00 * xv.x + blk.a01 * xv.y;
          r1 -= blk.a10 * xv.x + blk.a11 * xv.y;
        }
      }
    }
    const Block2<T> l = load_block<NT>(a, kLineL * 4);
    r0 -= l.a00 * d0 + l.a01 * d1;
    r1 -= l.a10 * d0 + l.a11 * d1;
    const Block2<T> mi = load_block<NT>(F + sidx<T>(t, 0, kLineFactors), 0);
    d0 = mi.a00 * r0 + mi.a01 * r1;
    d1 = mi.a10 * r0 + mi.a11 * r1;
    T2 dv;
    dv.x = d0;
    dv.y = d1;
    x[t] = dv;
  }
  T y0 = 0, y1 = 0;
  for (int k = g.nz - 1; k >= 0; --k) {
    const int t = line_pos(g, cc, q, k);
    const Block2<T> c = load_block<NT>(F + sidx<T>(t, 0, kLineFactors), 4);
    const T2 dv = x[t];
    const T n0 = dv.x - (c.a00 * y0 + c.a01 * y1);
    const T n1 = dv.y - (c.a10 * y0 + c.a11 * y1);
    y0 = n0;
    y1 = n1;
    T2 o;
    o.x = n0;
    o.y = n1;
    x[t] = o;
  }
}

// ---------------------------------------------------------------------------
// The same sweep with the work split by what depends on what: a workgroup takes COLS
// consecutive columns of colour cc.  Phase 1 (all 4 waves, every (column, k) at once):
// r_k = b_k - (the other columns' couplings) A x, then e_k = M_k^{-1} r_k, G_k = M_k^{-1} L_k
// and C_k go to LDS.  Phase 2 (one lane per column): the recurrences d_k = e_k - G_k d_{k-1}
// (downwards) and x_k = d_k - C_k x_{k+1} (upwards, written to x), which touch LDS only.  The
// rows of one k-parity share a vertex colour, so each wave takes 64 / COLS rows of one
// parity (k, k + 2, ...) and its neighbour colours stay wave-uniform.  COLS (8, 16 or 32)
// trades the LDS of a workgroup (10 values per row and column) against the rows a wave
// gathers at once; the autotuner picks it per level.  The per-thread column walk above
// serialises the neighbour gathers of a whole column in one lane, which leaves the GPU
// idle when few samples are active.
// ---------------------------------------------------------------------------
constexpr int kLineThreads = 256;      // 4 waves

template <typename T, typename M, bool NT, int ZC, int COLS>
__global__ __launch_bounds__(kLineThreads) void k_line_sweep(Geom g, int cc, const M* A_all,
                                                             const T* F_all, const T* b_all,
                                                             T* x_all, const int* mask,
                                                             const int* list) {
  using T2 = typename V2<T>::type;
  extern __shared__ double line_lds_raw[];
  T* lds = reinterpret_cast<T*>(line_lds_raw);
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const int mx = g.mx[cc], ncol = mx * g.my[cc];
  constexpr int RPW = 64 / COLS;  // rows per wave
  const int q0 = xcd_tile(blockIdx.x, blockIdx.y, gridDim.x) * COLS;
  const int nz = g.nz;
  const size_t Np = g.off[8];
  const M* A = A_all + (size_t)s * kPlanes * Np;
  const T* F = F_all + (size_t)s * kLineFactors * Np;
  const T2* b = reinterpret_cast<const T2*>(b_all + (size_t)s * 2 * Np);
  T2* x = reinterpret_cast<T2*>(x_all + (size_t)s * 2 * Np);
  // LDS, value-major so that the lanes of a row read consecutive words: [value][k][column]
  auto L_at = [&](int v, int k, int c) -> T& { return lds[((size_t)v * nz + k) * COLS + c]; };
  // the wave index as a scalar, so that the rows' colour is known to be wave-uniform
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cl = lane % COLS, rsub = lane / COLS;  // column, row within the wave
  const int n_even = (nz + 1) / 2, n_odd = nz / 2;
  const int g_even = (n_even + RPW - 1) / RPW, g_odd = (n_odd + RPW - 1) / RPW;  // row groups
  for (int grp = wave; grp < g_even + g_odd; grp += kLineThreads / 64) {
    const int par = grp < g_even ? 0 : 1;
    const int m = RPW * (par ? grp - g_even : grp) + rsub;
    const int k = par + 2 * m;
    const int q = q0 + cl;
    if (k >= nz || q >= ncol) continue;
    const int i = 2 * (q % mx) + (cc & 1), j = 2 * (q / mx) + (cc >> 1);
    const int col = cc + 4 * par;  // the same for the whole wave
    const int t = line_pos(g, cc, q, k);
    const NbrMap nm = nbr_map(g, col, i, j, k);
    const M* a = A + sidx<M>(t, 0, kPlanes);
    const T2 bv = b[t];
    T r0 = bv.x, r1 = bv.y;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx == 0 && dy == 0) continue;
          if (ZC >= 0 && !line_zero_start_reads(ZC, dx, dy)) continue;
          const T2 xv = load_nbr(x, g, nm, dx, dy, dz);
          const Block2<T> blk = load_block<NT>(a, nb_index(dx, dy, dz) * 4);
          r0 -= blk.a00 * xv.x + blk.a01 * xv.y;
          r1 -= blk.a10 * xv.x + blk.a11 * xv.y;
        }
      }
    }
    const Block2<T> l = load_block<NT>(a, kLineL * 4);
    const T* f = F + sidx<T>(t, 0, kLineFactors);
    const Block2<T> mi = load_block<NT>(f, 0);
    const Block2<T> c = load_block<NT>(f, 4);
    L_at(0, k, cl) = mi.a00 * r0 + mi.a01 * r1;
    L_at(1, k, cl) = mi.a10 * r0 + mi.a11 * r1;
    L_at(2, k, cl) = mi.a00 * l.a00 + mi.a01 * l.a10;
    L_at(3, k, cl) = mi.a00 * l.a01 + mi.a01 * l.a11;
    L_at(4, k, cl) = mi.a10 * l.a00 + mi.a11 * l.a10;
    L_at(5, k, cl) = mi.a10 * l.a01 + mi.a11 * l.a11;
    L_at(6, k, cl) = c.a00;
    L_at(7, k, cl) = c.a01;
    L_at(8, k, cl) = c.a10;
    L_at(9, k, cl) = c.a11;
  }
  __syncthreads();
  if (threadIdx.x >= COLS) return;
  const int q = q0 + threadIdx.x;
  if (q >= ncol) return;
  const int c = threadIdx.x;
  T d0 = 0, d1 = 0;
  for (int k = 0; k < nz; ++k) {  // d_k = e_k - G_k d_{k-1}, kept in place of e_k
    const T n0 = L_at(0, k, c) - (L_at(2, k, c) * d0 + L_at(3, k, c) * d1);
    const T n1 = L_at(1, k, c) - (L_at(4, k, c) * d0 + L_at(5, k, c) * d1);
    d0 = n0;
    d1 = n1;
    L_at(0, k, c) = n0;
    L_at(1, k, c) = n1;
  }
  T y0 = 0, y1 = 0;
  for (int k = nz - 1; k >= 0; --k) {  // x_k = d_k - C_k x_{k+1}
    const T n0 = L_at(0, k, c) - (L_at(6, k, c) * y0 + L_at(7, k, c) * y1);
    const T n1 = L_at(1, k, c) - (L_at(8, k, c) * y0 + L_at(9, k, c) * y1);
    y0 = n0;
    y1 = n1;
    T2 o;
    o.x = n0;
    o.y = n1;
    x[line_pos(g, cc, q, k)] = o;
  }
}

template <typename T, typename M, bool NT, int COLS>
auto line_sweep_kernel_c(int cc, bool zero_start) {
  if (zero_start) {
    switch (cc) {
      case 0: return k_line_sweep<T, M, NT, 0, COLS>;
      case 1: return k_line_sweep<T, M, NT, 1, COLS>;
      case 2: return k_line_sweep<T, M, NT, 2, COLS>;
      default: return k_line_sweep<T, M, NT, 3, COLS>;
    }
  }
  return k_line_sweep<T, M, NT, -1, COLS>;
}

template <typename T, typename M, bool NT>
auto line_sweep_kernel(int cc, bool zero_start, int cols) {
  switch (cols) {
    case 8: return line_sweep_kernel_c<T, M, NT, 8>(cc, zero_start);
    case 32: return line_sweep_kernel_c<T, M, NT, 32>(cc, zero_start);
    default: return line_sweep_kernel_c<T, M, NT, 16>(cc, zero_start);
  }
}

template <typename T>
size_t line_sweep_lds(const Geom& g, int cols) {
  return (size_t)kLineVals * g.nz * cols * sizeof(T);
}

template <typename T>
bool line_cols_valid(const Geom& g, int cols) {
  return (cols == 8 || cols == 16 || cols == 32) && line_sweep_lds<T>(g, cols) <= kLineLdsMax;
}

template <typename T, typename M, bool NT>
auto line_smooth_kernel(int cc, bool zero_start) {
  if (zero_start) {
    switch (cc) {
      case 0: return k_line_smooth<T, M, NT, 0>;
      case 1: return k_line_smooth<T, M, NT, 1>;
      case 2: return k_line_smooth<T, M, NT, 2>;
      default: return k_line_smooth<T, M, NT, 3>;
    }
  }
  return k_line_smooth<T, M, NT, -1>;
}

// matrices of more than this many bytes (all samples of a level) are streamed with
// non-temporal loads, as in the point smoother
constexpr double kLineCachedBytes = 128.0 * 1024 * 1024;

template <typename T, typename M>
void launch_line_smooth_m(const Geom& g, int cc, const M* A, const T* F, const T* b, T* x, int S,
                          const int* mask, const int* list, hipStream_t st, hipEvent_t ev0,
                          hipEvent_t ev1, bool zero_start, int cols) {
  const int n = g.mx[cc] * g.my[cc];
  if (n <= 0) return;
  const bool nt = (double)S * kPlanes * g.off[8] * sizeof(M) > kLineCachedBytes;
  if (!line_cols_valid<T>(g, cols)) cols = 16;
  const size_t lds = line_sweep_lds<T>(g, cols);
  if (lds <= kLineLdsMax) {
    dim3 grid(ceil_div(n, cols), S);
    auto kern = nt ? line_sweep_kernel<T, M, true>(cc, zero_start, cols)
                   : line_sweep_kernel<T, M, false>(cc, zero_start, cols);
    if (ev0)
      hipExtLaunchKernelGGL(kern, grid, dim3(kLineThreads), lds, st, ev0, ev1, 0, g, cc, A, F, b, x,
                            mask, list);
    else
      hipLaunchKernelGGL(kern, grid, dim3(kLineThreads), lds, st, g, cc, A, F, b, x, mask, list);
    return;
  }
  dim3 grid(ceil_div(n, 64), S);
  auto kern = nt ? line_smooth_kernel<T, M, true>(cc, zero_start)
                 : line_smooth_kernel<T, M, false>(cc, zero_start);
  if (ev0)
    hipExtLaunchKernelGGL(kern, grid, dim3(64), 0, st, ev0, ev1, 0, g, cc, A, F, b, x, mask, list);
  else
    hipLaunchKernelGGL(kern, grid, dim3(64), 0, st, g, cc, A, F, b, x, mask, list);
}

template <typename T>
void launch_line_smooth(const Geom& g, int cc, const T* A, const T* F, const T* b, T* x, int S,
                        const int* mask, const int* list, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1, bool zero_start, int cols) {
  launch_line_smooth_m<T, T>(g, cc, A, F, b, x, S, mask, list, st, ev0, ev1, zero_start, cols);
}

void launch_line_smooth_f16(const Geom& g, int cc, const _Float16* A, const float* F,
                            const float* b, float* x, int S, const int* mask, const int* list,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, bool zero_start,
                            int cols) {
  launch_line_smooth_m<float, _Float16>(g, cc, A, F, b, x, S, mask, list, st, ev0, ev1,
                                        zero_start, cols);
}

// ---------------------------------------------------------------------------
// residual after a single forward line sweep from x = 0, at position t (vertex colour
// col, column colour cc = col & 3): that sweep left T_col x_col + (the columns of the
// colours below cc) = b, so r = -(sum over the neighbours in columns of colours above cc
// of A x); the last column colour (3) has zero residual.  Dirichlet rows are zero.
// ---------------------------------------------------------------------------
template <typename T, typename M, bool NT, int CC>
__device__ __forceinline__ void line_residual_upper(const Geom& g, int t, int col, int i, int j,
                                                    int k, const M* A_s, const T* D_s,
                                                    const T* x_s, T* r_s) {
  using T2 = typename V2<T>::type;
  const NbrMap nm = nbr_map(g, col, i, j, k);
  const M* A = A_s + sidx<M>(t, 0, kPlanes);
  const T2* x = reinterpret_cast<const T2*>(x_s);
  T a0 = 0, a1 = 0;
#pragma unroll 1  // one z-plane of neighbours at a time keeps the register count low
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if ((dx == 0 && dy == 0) || line_column_colour(CC, dx, dy) <= CC) continue;
        const T2 xv = load_nbr(x, g, nm, dx, dy, dz);
        const Block2<T> a = load_block<NT>(A, nb_index(dx, dy, dz) * 4);
        a0 += a.a00 * xv.x + a.a01 * xv.y;
        a1 += a.a10 * xv.x + a.a11 * xv.y;
      }
    }
  }
  if (D_s) {  // the scaled system's residual back to the unscaled rows: r = D (D^{-1} r)
    const Block2<T> d = load_block<false>(D_s + sidx<T>(t, 0, 4), 0);
    const T s0 = d.a00 * a0 + d.a01 * a1, s1 = d.a10 * a0 + d.a11 * a1;
    a0 = s0;
    a1 = s1;
  }
  double cD;
  T2 out;
  out.x = is_pin(g, i, j, k) ? T(0) : -a0;
  out.y = is_cdir(g, i, j, k, cD) ? T(0) : -a1;
  reinterpret_cast<T2*>(r_s)[t] = out;
}

template <typename T, typename M, bool NT>
__global__ __launch_bounds__(kBlock) void k_line_residual_zs(Geom g, const M* A_all,
                                                             const T* D_all, const T* x_all,
                                                             T* r_all, const int* mask,
                                                             const int* list) {
  using T2 = typename V2<T>::type;
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  // slab order: the colours' work differs (24, 18, 6, 0 blocks for column colours 0-3),
  // so every XCD takes the same share of each colour
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int col, tile;
  if (!slab_tile(g, blockIdx.x % kXcds, (blockIdx.x / kXcds) * (kBlock / kTile) + wave, col,
                 tile))
    return;
  const int place = tile * kTile + (threadIdx.x & 63);
  if (place >= g.cnt[col]) return;
  const int t = g.off[col] + place;
  int i, j, k;
  colour_decode_in(g, col, place, i, j, k);
  const size_t Np = g.off[8];
  const M* A = A_all + (size_t)s * kPlanes * Np;
  const T* D = D_all ? D_all + (size_t)s * 4 * Np : nullptr;
  const T* x = x_all + (size_t)s * 2 * Np;
  T* r = r_all + (size_t)s * 2 * Np;
  switch (col & 3) {
    case 0: line_residual_upper<T, M, NT, 0>(g, t, col, i, j, k, A, D, x, r); break;
    case 1: line_residual_upper<T, M, NT, 1>(g, t, col, i, j, k, A, D, x, r); break;
    case 2: line_residual_upper<T, M, NT, 2>(g, t, col, i, j, k, A, D, x, r); break;
    default: {
      T2 z;
      z.x = 0;
      z.y = 0;
      reinterpret_cast<T2*>(r)[t] = z;
    }
  }
}

template <typename T, typename M>
void launch_line_residual_zs_m(const Geom& g, const M* A, const T* D, const T* x, T* r, int S,
                               const int* mask, const int* list, hipStream_t st) {
  dim3 grid(slab_blocks(g), S);
  const bool nt = (double)S * kPlanes * g.off[8] * sizeof(M) > kLineCachedBytes;
  auto kern = nt ? k_line_residual_zs<T, M, true> : k_line_residual_zs<T, M, false>;
  hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, st, g, A, D, x, r, mask, list);
}

template <typename T>
void launch_line_residual_zs(const Geom& g, const T* A, const T* x, T* r, int S, const int* mask,
                             const int* list, hipStream_t st) {
  launch_line_residual_zs_m<T, T>(g, A, nullptr, x, r, S, mask, list, st);
}

void launch_line_residual_zs_f16(const Geom& g, const _Float16* A, const float* D, const float* x,
                                 float* r, int S, const int* mask, const int* list,
                                 hipStream_t st) {
  launch_line_residual_zs_m<float, _Float16>(g, A, D, x, r, S, mask, list, st);
}

#define EDF_LINE_INST(T)                                                                        \
  template void launch_line_factor<T>(const Geom&, const T*, T*, int, const int*, hipStream_t);  \
  template void launch_line_smooth<T>(const Geom&, int, const T*, const T*, const T*, T*, int,   \
                                      const int*, const int*, hipStream_t, hipEvent_t,           \
                                      hipEvent_t, bool, int);                                    \
  template bool line_cols_valid<T>(const Geom&, int);                                            \
  template void launch_line_residual_zs<T>(const Geom&, const T*, const T*, T*, int,            \
                                           const int*, const int*, hipStream_t);
EDF_LINE_INST(double)
EDF_LINE_INST(float)

}  // namespace edf
