// Internal declarations shared by the HIP kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace edf {

constexpr int kBlock = 256;        // threads per workgroup of the streaming kernels
constexpr int kPlanes = 108;       // 27 neighbours x 2 equations x 2 unknowns
constexpr int kDiag = 13;          // neighbour index of the vertex itself
constexpr int kMaxCoarse = 2048;   // largest coarsest-grid system (unknowns)

// Geometry of one grid level.  Stencil arrays of a level are indexed by a
// colour-major vertex position t: the 8 colours (i%2, j%2, k%2) one after the
// other, each colour's vertices in (i/2, j/2, k/2) lexicographic order, and each
// colour starting at a multiple of kTile.  Positions are grouped in tiles of kTile
// (one wavefront); a stencil array with P values per vertex is stored as
// [tile][P][kTile], so one wavefront streams one contiguous block.
// Vectors are in natural order v = i + nx (j + ny k).
constexpr int kTile = 64;
struct Geom {
  int nx, ny, nz, N;
  int off[9];        // colour offsets (multiples of kTile); off[8] = Np, the padded size
  int cnt[8];        // vertices per colour
  int mx[8], my[8];  // colour sub-grid extents in x and y
  int pi0, pi1, pj0, pj1;  // vertex index range of the salt patch on k = 0 (empty if pi0 > pi1)
  double hx, hy, hz;
};

// Physical constants and the scaling of one level (passed by value).
struct Phys {
  double rho0, drho, mu, g, Dm;
  double dt;       // time step (kernels given a per-sample dt array override it)
  double s_row;    // dt / (rho0 phi_mean hx hy hz): scale of the finite-volume rows
  double row_c;    // 1 / (rho0 phi_mean hx hy hz), so that s_row = dt * row_c
  double p_unit;   // rho0 max(g,1) lz: pressure unit of the scaled unknowns
};

struct FieldParams {
  double lx, ly, lz, phi_mean, K_mean;
  int model, n_xi;
};

// Per-sample scalars of BiCGStab (device resident).
struct KrylovScalars {
  double rho, rho_old, alpha, omega, beta;
  double bb, rr, tol2, rv, ts, tt, ss;
  double hh;      // (r^, r^) of the shadow residual
  int it, state;  // state: 0 running, 1 converged, 2 breakdown with no restart left
  int restart;    // 1: the next iteration restarts with r^ = p = r (set by the update)
  int restarts;   // restarts so far
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// kernel launchers (fv_kernels.hip)
// ---------------------------------------------------------------------------
void launch_coefficients(const Geom& g, const FieldParams& fp, const double* xi, int S,
                         double* phi, double* K, hipStream_t st);
// bad[s] |= 1 when some hexahedron of sample s would get phi outside (0, 1) or a K that
// is not finite and positive (nothing is written)
void launch_check_coefficients(const Geom& g, const FieldParams& fp, const double* xi, int S,
                               int* bad, hipStream_t st);
// dts: per-sample time steps [S] in device memory, or nullptr for ph.dt
void launch_defect(const Geom& g, const Phys& ph, const double* dts, const double* phi,
                   const double* K, const double* u, const double* u_old, double* F, int S,
                   const int* mask, hipStream_t st);
// FP64 mass balance of a (sub-)step: acc[s][0..5] += (salt storage change, its absolute
// sum, liquid storage change, its absolute sum, dt x salt rows at the c-Dirichlet
// vertices, dt x liquid rows at the pinned vertices) for the samples in mask; part is
// scratch [S][balance_blocks(g)][8]
int balance_blocks(const Geom& g);
void launch_balance(const Geom& g, const Phys& ph, const double* dts, const double* phi,
                    const double* K, const double* u, const double* u_old, double* part,
                    double* acc, int S, const int* mask, hipStream_t st);
void launch_assemble(const Geom& g, const Phys& ph, const double* dts, const double* phi,
                     const double* K, const double* u, double* A64, float* A32, int S,
                     const int* mask, hipStream_t st, bool frozen);
void launch_c_range(const Geom& g, const double* u, double* part, double* out, int S,
                    const int* mask, hipStream_t st);
void launch_block_inverse_f64(const Geom& g, const double* A, double* Dinv, int S,
                              const int* mask, hipStream_t st);
void launch_block_inverse_f32(const Geom& g, const float* A, float* Dinv, int S,
                              const int* mask, hipStream_t st);
void launch_inject(const Geom& gf, const Geom& gc, const double* uf, double* uc, int S,
                   const int* mask, hipStream_t st);
void launch_stencil_to_natural(const Geom& g, const double* A, double* out, hipStream_t st);

// ---------------------------------------------------------------------------
// multigrid and stencil kernels (mg_kernels.hip), T = double or float
// ---------------------------------------------------------------------------
// The V-cycle launches take (S, mask, list): grid row y works on sample list[y] (or y when
// list is null) for y < S, and returns at once when mask is set and mask[sample] is 0.
// A list of the active samples keeps the launch from dispatching workgroups of finished
// samples (70k one-wave workgroups cost about 14 us to dispatch even when they all
// return at once).

// Colour of the neighbour at offset (dx, dy, dz) of a vertex of colour col: an odd
// offset along an axis flips that axis's parity bit.
__host__ __device__ constexpr int nbr_colour(int col, int dx, int dy, int dz) {
  return col ^ ((dx != 0) | ((dy != 0) << 1) | ((dz != 0) << 2));
}

// Whether the first forward sweep from x = 0 needs the neighbour of colour col at offset
// (dx, dy, dz): only the colours already swept (below col) hold non-zero values; the
// vertex itself and the colours above col are still zero and contribute nothing.
__host__ __device__ constexpr bool zero_start_reads(int col, int dx, int dy, int dz) {
  return nbr_colour(col, dx, dy, dz) < col;
}

// Number of 2x2 stencil blocks that sweep reads per vertex of colour col (0 for colour
// 0, all 26 off-diagonal blocks for colour 7, 13 on average).
__host__ __device__ constexpr int zero_start_blocks(int col) {
  int n = 0;
  for (int o = 0; o < 27; ++o)
    if (zero_start_reads(col, o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1)) ++n;
  return n;
}

// Vertical-line block Gauss-Seidel (line_kernels.hip): columns (i, j) in 4 colours
// cc = (i % 2) + 2 (j % 2); the neighbour column at (dx, dy) has colour cc with the parity
// bit of every odd component flipped.
constexpr int kLineFactors = 8;  // per vertex: M^{-1} of the column's block LU, then C
constexpr int kLineVals = 10;    // per (row, column) of a line sweep in LDS: e (2), G (4), C (4)
__host__ __device__ constexpr int line_column_colour(int cc, int dx, int dy) {
  return cc ^ ((dx != 0) | ((dy != 0) << 1));
}
// the first line sweep from x = 0 of column colour cc reads the neighbour column (dx, dy)
// only when its colour is below cc (the columns already swept)
__host__ __device__ constexpr bool line_zero_start_reads(int cc, int dx, int dy) {
  return (dx != 0 || dy != 0) && line_column_colour(cc, dx, dy) < cc;
}
// stencil blocks that sweep reads per vertex besides the column's own (3 per column)
__host__ __device__ constexpr int line_zero_start_blocks(int cc) {
  int n = 0;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx)
      if (line_zero_start_reads(cc, dx, dy)) n += 3;
  return n;
}
// the factors F [S][Np x 8] of every column's block tridiagonal part (diagonal, above,
// below blocks of A), computed in FP64 and stored in T
template <typename T>
void launch_line_factor(const Geom& g, const T* A, T* F, int S, const int* mask, hipStream_t st);
// one line sweep of column colour cc; zero_start: the level's first forward sweep from x = 0;
// cols: columns per workgroup (8, 16 or 32; an invalid choice falls back to 16), the tile
// shape the autotuner picks per level
template <typename T>
void launch_line_smooth(const Geom& g, int cc, const T* A, const T* F, const T* b, T* x, int S,
                        const int* mask, const int* list, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1, bool zero_start, int cols = 16);
// The same three for an FP16-stored finest level of the FP32 V-cycle: the matrix is
// D^{-1} A (identity diagonal blocks) and b holds D^{-1} b; the factors (FP32) are those of
// the scaled columns, and the residual is unscaled with the FP32 diagonal blocks D
void launch_line_factor_f16(const Geom& g, const _Float16* A, float* F, int S, const int* mask,
                            hipStream_t st);
void launch_line_smooth_f16(const Geom& g, int cc, const _Float16* A, const float* F,
                            const float* b, float* x, int S, const int* mask, const int* list,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, bool zero_start,
                            int cols);
void launch_line_residual_zs_f16(const Geom& g, const _Float16* A, const float* D, const float* x,
                                 float* r, int S, const int* mask, const int* list,
                                 hipStream_t st);
// LDS of one k_line_sweep workgroup at most (the column walk takes deeper grids)
constexpr size_t kLineLdsMax = 64 * 1024;
// whether cols columns per workgroup is a tile shape k_line_sweep offers for this grid
template <typename T>
bool line_cols_valid(const Geom& g, int cols);
// r = b - A x after a single forward line sweep from x = 0 (blocks towards the columns of
// the colours swept later only; b is not read)
template <typename T>
void launch_line_residual_zs(const Geom& g, const T* A, const T* x, T* r, int S, const int* mask,
                             const int* list, hipStream_t st);

// one block Gauss-Seidel sweep of one colour; zero_start: the first forward sweep of a
// level whose x is zero on entry (reads only the colours already swept, writes x)
template <typename T>
void launch_smooth(const Geom& g, int colour, const T* A, const T* Dinv, const T* b, T* x, int S,
                   const int* mask, const int* list, hipStream_t st, hipEvent_t ev0 = nullptr,
                   hipEvent_t ev1 = nullptr, bool zero_start = false);
// r = b - A x, zero in Dirichlet rows; zero_sweep: x is the result of a single forward
// sweep from x = 0, whose residual needs only the blocks towards the colours not yet swept
// when each vertex was updated (b is not read)
template <typename T>
void launch_residual(const Geom& g, const T* A, const T* b, const T* x, T* r, int S,
                     const int* mask, const int* list, hipStream_t st, bool zero_sweep = false);
// bc = R rf (full weighting, coarse row scaling); with Dc (the coarse block inverses) the
// first forward sweep from zero of colour 0 into xc (x = Dc b on colour 0, the other
// colours untouched), else xc, when not null, cleared
template <typename T>
void launch_restrict(const Geom& gf, const Geom& gc, const T* rf, T* bc, T* xc, const T* Dc,
                     int S, const int* mask, const int* list, hipStream_t st);
template <typename T>
void launch_prolong(const Geom& gf, const Geom& gc, const T* xc, T* xf, int S, const int* mask,
                    const int* list, hipStream_t st);
template <typename T>
void launch_fill(T* x, size_t per_sample, int S, const int* mask, T value, hipStream_t st);
// FP16 finest level (EDF_PREC_MIXED_F16): from the FP32 matrix A32, the block-scaled
// A16 = D^{-1} A (FP16, unit diagonal blocks) and the diagonal blocks D32 (FP32)
void launch_scale_f16(const Geom& g, const float* A32, _Float16* A16, float* D32, int S,
                      const int* mask, hipStream_t st);
// block Gauss-Seidel with A16: x_v = bh_v - sum_{o != diag} A16_vo x_{v+o}, bh = D^{-1} b
void launch_smooth_f16(const Geom& g, int colour, const _Float16* A16, const float* bh, float* x,
                       int S, const int* mask, const int* list, hipStream_t st, hipEvent_t ev0,
                       hipEvent_t ev1, bool zero_start = false);
// r = b - A x = D (bh - A16 x), zero in Dirichlet rows
void launch_residual_f16(const Geom& g, const _Float16* A16, const float* D32, const float* bh,
                         const float* x, float* r, int S, const int* mask, const int* list,
                         hipStream_t st, bool zero_sweep = false);
// entry: bh = D^{-1} b, FP64 natural [N][2] -> FP32 colour-major [Np][2]
// (x, when not null: the zero-start sweep of colour 0, x = bh there)
void launch_to_colour_scaled(const Geom& g, const double* in, const float* D32, float* out,
                             float* x, int S, const int* mask, const int* list, hipStream_t st);
// finest-level V-cycle entry and exit: FP64 natural [N][2] <-> T colour-major [Np][2]
// (D, when not null: the zero-start sweep of colour 0 into x, x = D b there)
template <typename T>
void launch_to_colour(const Geom& g, const double* in, T* out, const T* D, T* x, int S,
                      const int* mask, const int* list, hipStream_t st);
template <typename T>
void launch_from_colour(const Geom& g, const T* in, double* out, int S, const int* mask,
                        const int* list, hipStream_t st);
void launch_coarse_dense(const Geom& g, const double* A, double* M, int S, const int* mask,
                         hipStream_t st);
void launch_gauss_jordan(int n, double* M, int* piv, int* status, int S, const int* mask,
                         hipStream_t st);

// The bottom of a V-cycle run by one workgroup per sample: levels 0..n-2 of this
// struct are smoothed, level n-1 is solved with the dense inverse.  Array pointers
// are the all-sample bases of the respective level.  The kernel reads the struct from
// device memory (indexing a by-value kernel argument with the runtime level number
// would copy it to per-lane scratch).
constexpr int kMaxFused = 6;
constexpr int kFuseMaxN = 4096;  // levels with at most this many vertices are fused
template <typename T>
struct FusedLevels {
  int n, nc, nu1, nu2;
  // lds_off[k] >= 0: level k's x, b and r are kept in LDS at element lds_off[k] (x, then
  // b at + 2 Np, r at + 4 Np) instead of in x/b/r; only the first level's b is read from
  // and its x written back to device memory.  All levels or none are in LDS.
  int lds_off[kMaxFused];
  // line_lds >= 0: the levels with line factors LF[k] are swept by vertical lines (as the
  // levels swept by their own launches), with the per-(row, column) values of a sweep in
  // LDS at element line_lds; the others (LF[k] null) by points
  int line_lds;
  Geom g[kMaxFused];
  const T* A[kMaxFused];
  const T* D[kMaxFused];
  const T* LF[kMaxFused];
  T* x[kMaxFused];
  T* b[kMaxFused];
  T* r[kMaxFused];
  const double* Minv;
};
// lds_bytes: dynamic LDS of the launch (the levels' vectors when they are kept there, and
// the line sweeps' values)
template <typename T>
void launch_vcycle_bottom(const FusedLevels<T>* F_dev, size_t lds_bytes, int S, const int* mask,
                          const int* list, hipStream_t st);
// LDS a workgroup of the fused bottom may take for the levels' vectors (0 when the device
// does not allow more than the static part)
template <typename T>
size_t vcycle_bottom_lds_limit();

// ---------------------------------------------------------------------------
// Krylov / Newton kernels (krylov_kernels.hip), FP64 vectors of n = 2N per sample
// ---------------------------------------------------------------------------
int reduce_blocks(size_t n);
// The operator y = J~ x of the outer Krylov method: the assembled FP64 stencil A, or, with
// A null, the matrix-free product at state u with the coefficients phi, K and the per-sample
// time steps dts (or ph.dt) (launch_jx)
struct JacOp {
  const double* A = nullptr;
  Phys ph{};
  const double* dts = nullptr;
  const double* phi = nullptr;
  const double* K = nullptr;
  const double* u = nullptr;
};
// matrix-free y = J~ x (fv_kernels.hip); mode 0: plain, 1: with the dot (d, y) into part,
// 2: with (d, y) and (y, y); grid rows = rows (list[row] or row is the sample); returns the
// number of partial sums per sample
int launch_jx(const Geom& g, const Phys& ph, const double* dts, const double* phi, const double* K,
              const double* u, const double* x, double* y, const double* d, double* part, int mode,
              int S, const int* mask, const int* list, int rows, hipStream_t st);
// the partial sums per sample that launch_jx writes on grid g
int jx_blocks(const Geom& g);
void launch_spmv(const Geom& g, const JacOp& J, const double* x, double* y, int S,
                 const int* mask, hipStream_t st);
// BiCGStab phases; `part` is scratch [S][nb][4], `ks` the per-sample scalars.
void launch_bicg_init(size_t n, const double* b, double* x, double* r, double* rh, double* p,
                      double* v, double* part, KrylovScalars* ks, const double* rtol, int* active,
                      int S, const int* mask, hipStream_t st);
// The iteration's launches run grid row y over sample sl.idx[y] for y < sl.n (all S samples
// when sl.idx is null); mask still gates every sample, and the per-sample reductions that
// follow run over all S.
struct SampleList {
  const int* idx = nullptr;
  int n = 0;
  int rows(int S) const { return idx ? n : S; }
};
// p = r + beta (p - omega v); on a restart (ks.restart) p = r and the shadow residual r^ = r
void launch_bicg_p(size_t n, const double* r, const double* v, double* p, double* rh,
                   const KrylovScalars* ks, int S, const int* mask, SampleList sl, hipStream_t st);
void launch_bicg_alpha(const Geom& g, const JacOp& J, const double* ph, double* v, const double* rh,
                       double* part, KrylovScalars* ks, int S, const int* mask, SampleList sl,
                       hipStream_t st);
void launch_bicg_s(size_t n, const double* r, const double* v, double* s, double* part,
                   KrylovScalars* ks, int S, const int* mask, SampleList sl, hipStream_t st);
void launch_bicg_omega(const Geom& g, const JacOp& J, const double* sh, const double* s, double* t,
                       double* part, KrylovScalars* ks, int S, const int* mask, SampleList sl,
                       hipStream_t st);
void launch_bicg_update(size_t n, const double* ph, const double* sh, const double* s,
                        const double* t, const double* rh, double* x, double* r, double* part,
                        KrylovScalars* ks, int* active, int S, const int* mask, SampleList sl,
                        hipStream_t st);
// Newton helpers
void launch_sq_norm(size_t n, const double* x, double* part, double* out, int S, const int* mask,
                    hipStream_t st);
void launch_axpy_state(size_t N, const double* u, const double* d, const double* lam, double p_unit,
                       double* out, int S, const int* mask, hipStream_t st);
void launch_masked_copy(size_t n, const double* a, double* b, int S, const int* mask,
                        hipStream_t st);
// A launch over the samples of several groups whose levels share one grid and one
// allocation (slots of the groups side by side): its list is built on the device from the
// groups' own lists, segment q contributing off_q + src_q[j] (j < n_q; src_q null: j) at
// dst[at_q + j]
constexpr int kMaxListSegs = 8;
struct ListSeg {
  const int* src;
  int n, off, at;
};
struct ListSegs {
  ListSeg seg[kMaxListSegs];
  int nseg;
};
void launch_concat_lists(const ListSegs& L, int total, int* dst, hipStream_t st);
// out = 2 u - u_prev for the masked samples
void launch_extrapolate(size_t n, const double* u, const double* u_prev, double* out, int S,
                        const int* mask, hipStream_t st);
void launch_gather_common(const Geom& gf, int cx, int cy, int cz, const double* u, double* out,
                          int S, hipStream_t st);
// chunked form of launch_moments (pass 0: mean and exceedance, pass 1: variance), the
// fields of samples s0 .. s0 + n - 1 in f [n][Nc]; bitwise the unchunked sums
void launch_moments_chunk(int pass, int Nc, int s0, int n, const double* f, const double* w,
                          double thr, double* mean, double* var, double* exc, hipStream_t st);
// w[s] = 0 where flag[s], then w /= sum(w) (sample order); *sum_out = the sum
void launch_normalise_weights(int S, double* w, const int* flag, double* sum_out, hipStream_t st);
void launch_moments(int Nc, int S, const double* f, const double* w, double thr, double* mean,
                    double* var, double* exc, hipStream_t st);

}  // namespace edf
