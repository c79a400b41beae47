// Finite-volume kernels of the Elder box: coefficient fields, the nonlinear
// defect and its Jacobian as a 27-point stencil of 2x2 blocks.
//
// Discretisation (vertex-centred finite volumes, Section 2.3 of the paper, model
// of Section 2.1): each vertex owns the union of the octants of its adjacent
// hexahedra.  Inside a hexahedron, every edge v_a -> v_b = v_a + e_d carries one
// sub-control-volume face: the quarter of the hex mid-plane normal to d next to
// the edge, with area (product of the other two h)/4 and one integration point at
// its centre.  At that point c, d_d p and d_d c come from trilinear interpolation
// over the 8 hex corners, the Darcy flux is Q = -(K_e/mu)(d_d p - rho(c) g_d) A,
// the liquid flux rho(c) Q and the salt flux rho(c_up) c_up Q - rho(c) phi_e D_m d_d c A
// with the upstream vertex c_up = c(v_a) if Q >= 0 else c(v_b).  Storage uses the
// lumped porous volume m_v = sum_e phi_e V_e / 8 and implicit Euler.
//
// Every vertex gathers the 24 faces it touches (each face is evaluated once from
// each of its two vertices), so no atomics are needed and results are
// deterministic.  All loops over hexes, faces and corners are unrolled with
// compile-time offsets: the 3x3x3 neighbourhood lives in registers.
#include <cmath>

#include "fv_common.h"

namespace edf {

// ---------------------------------------------------------------------------
// coefficient fields, one thread per hexahedron (Section 2.2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void field_value(const Geom& g, const FieldParams& fp, const double* q,
                                            int i, int j, int k, double& phi_out, double& K_out) {
  const double x = (i + 0.5) * g.hx, y = (j + 0.5) * g.hy, z = (k + 0.5) * g.hz;
  const double pm = fp.phi_mean;
  const double px = M_PI * x / fp.lx, py = M_PI * y / fp.ly, pz = M_PI * z / fp.lz;
  double phi = pm, logK_extra = 0.0;
  bool kc = true;
  switch (fp.model) {
    case 0:
      kc = false;
      break;
    case 1:
      phi = pm * (1.0 + 0.2 * q[0] * cos(px) * cos(py));
      break;
    case 2:
      phi = pm * (1.0 + 0.2 * q[0] * cos(px) * cos(py) + 0.2 * q[1] * sin(px) * sin(py));
      logK_extra = 0.5 * q[2] * cos(pz) + 0.5 * q[3] * sin(px) * cos(pz);
      break;
    default: {
      const double sx = sin(px), sy = sin(py), sz = sin(pz);
      phi = pm + 0.01 * (q[0] * sx + q[1] * sy + q[2] * sz + q[0] * sx * sy + q[1] * sx * sz);
    }
  }
  double K = fp.K_mean;
  if (kc) {  // Kozeny-Carman, normalised to K(phi_mean) = K_mean
    const double r = phi / pm, w = (1.0 - pm) / (1.0 - phi);
    K = fp.K_mean * r * r * r * w * w;
    if (logK_extra != 0.0) K = exp(log(K) + logK_extra);
  }
  phi_out = phi;
  K_out = K;
}

// phi_all/K_all null: only check that phi lies in (0, 1) and K is finite and positive,
// setting bad[s] for a sample with a hexahedron outside
__global__ __launch_bounds__(kBlock) void k_coefficients(Geom g, FieldParams fp, const double* xi,
                                                         double* phi_all, double* K_all,
                                                         int* bad) {
  const int s = blockIdx.y;
  const int cx = g.nx - 1, cy = g.ny - 1, cz = g.nz - 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cx * cy * cz) return;
  const int i = e % cx, j = (e / cx) % cy, k = e / (cx * cy);
  const double* q = xi + (size_t)s * (fp.n_xi > 0 ? fp.n_xi : 1);
  double phi, K;
  field_value(g, fp, q, i, j, k, phi, K);
  if (bad) {
    if (!(phi > 0.0 && phi < 1.0) || !(K > 0.0 && K < INFINITY)) atomicOr(bad + s, 1);
    return;
  }
  const size_t cells = (size_t)cx * cy * cz;
  phi_all[(size_t)s * cells + e] = phi;
  K_all[(size_t)s * cells + e] = K;
}

void launch_coefficients(const Geom& g, const FieldParams& fp, const double* xi, int S,
                         double* phi, double* K, hipStream_t st) {
  const int cells = (g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  dim3 grid(ceil_div(cells, kBlock), S);
  hipLaunchKernelGGL(k_coefficients, grid, dim3(kBlock), 0, st, g, fp, xi, phi, K, (int*)nullptr);
}

void launch_check_coefficients(const Geom& g, const FieldParams& fp, const double* xi, int S,
                               int* bad, hipStream_t st) {
  const int cells = (g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  dim3 grid(ceil_div(cells, kBlock), S);
  hipLaunchKernelGGL(k_coefficients, grid, dim3(kBlock), 0, st, g, fp, xi, (double*)nullptr,
                     (double*)nullptr, bad);
}

// ---------------------------------------------------------------------------
// one sub-control-volume face seen from vertex v, v = corner (AX,AY,AZ) of the hex
// ---------------------------------------------------------------------------
struct FaceGeo {
  double ih[3];    // 1/h per direction
  double area[3];  // face area per normal direction
};

template <int AX, int AY, int AZ, int D>
struct FaceT {
  static constexpr int SB0 = D == 0 ? 0 : AX;  // start corner of the edge through v
  static constexpr int SB1 = D == 1 ? 0 : AY;
  static constexpr int SB2 = D == 2 ? 0 : AZ;
  static constexpr int VD = D == 0 ? AX : (D == 1 ? AY : AZ);  // 0: v is the start
  static constexpr int NA = nb_index(SB0 - AX, SB1 - AY, SB2 - AZ);
  static constexpr int NB = nb_index(SB0 + (D == 0) - AX, SB1 + (D == 1) - AY, SB2 + (D == 2) - AZ);
  // trilinear weight of corner w at the integration point, and its d/dt_D
  static __device__ __forceinline__ double N(int w) {
    const int wx = w & 1, wy = (w >> 1) & 1, wz = w >> 2;
    const double gx = D == 0 ? 0.5 : (wx == SB0 ? 0.75 : 0.25);
    const double gy = D == 1 ? 0.5 : (wy == SB1 ? 0.75 : 0.25);
    const double gz = D == 2 ? 0.5 : (wz == SB2 ? 0.75 : 0.25);
    return gx * gy * gz;
  }
  static __device__ __forceinline__ double dN(int w) {
    const int wx = w & 1, wy = (w >> 1) & 1, wz = w >> 2;
    const double gx = wx == SB0 ? 0.75 : 0.25;
    const double gy = wy == SB1 ? 0.75 : 0.25;
    const double gz = wz == SB2 ? 0.75 : 0.25;
    const int wd = D == 0 ? wx : (D == 1 ? wy : wz);
    const double t = D == 0 ? gy * gz : (D == 1 ? gx * gz : gx * gy);
    return wd ? t : -t;
  }
  static __device__ __forceinline__ int nb(int w) {
    return nb_index((w & 1) - AX, ((w >> 1) & 1) - AY, (w >> 2) - AZ);
  }
};

template <int AX, int AY, int AZ, int D>
__device__ __forceinline__ void face_residual(const double* P, const double* C, double phi, double K,
                                              const Phys& ph, const FaceGeo& fg, double& Fl,
                                              double& Fs) {
  using F = FaceT<AX, AY, AZ, D>;
  double cf = 0.0, dp = 0.0, dc = 0.0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    cf += F::N(w) * C[F::nb(w)];
    dp += F::dN(w) * P[F::nb(w)];
    dc += F::dN(w) * C[F::nb(w)];
  }
  dp *= fg.ih[D];
  dc *= fg.ih[D];
  const double area = fg.area[D];
  const double gD = D == 2 ? ph.g : 0.0;
  const double rf = ph.rho0 + ph.drho * cf;
  const double Q = -(K / ph.mu) * (dp - rf * gD) * area;
  const double cup = Q >= 0.0 ? C[F::NA] : C[F::NB];
  const double fl = rf * Q;
  const double fs = (ph.rho0 + ph.drho * cup) * cup * Q - rf * phi * ph.Dm * dc * area;
  if (F::VD == 0) {
    Fl += fl;
    Fs += fs;
  } else {
    Fl -= fl;
    Fs -= fs;
  }
}

template <int AX, int AY, int AZ>
__device__ __forceinline__ void hex_residual(const Geom& g, int i, int j, int k, const double* phi,
                                             const double* K, const double* P, const double* C,
                                             const Phys& ph, const FaceGeo& fg, double& Fl,
                                             double& Fs, double& msum) {
  const int hi = i - AX, hj = j - AY, hk = k - AZ;
  if (hi < 0 || hj < 0 || hk < 0 || hi > g.nx - 2 || hj > g.ny - 2 || hk > g.nz - 2) return;
  const size_t e = hi + (size_t)(g.nx - 1) * (hj + (size_t)(g.ny - 1) * hk);
  const double pe = phi[e], Ke = K[e];
  msum += pe;
  face_residual<AX, AY, AZ, 0>(P, C, pe, Ke, ph, fg, Fl, Fs);
  face_residual<AX, AY, AZ, 1>(P, C, pe, Ke, ph, fg, Fl, Fs);
  face_residual<AX, AY, AZ, 2>(P, C, pe, Ke, ph, fg, Fl, Fs);
}

__device__ __forceinline__ void load_neighbourhood(const Geom& g, const double2* u, int i, int j,
                                                   int k, double* P, double* C) {
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int ii = clampi(i + dx, 0, g.nx - 1), jj = clampi(j + dy, 0, g.ny - 1),
                  kk = clampi(k + dz, 0, g.nz - 1);
        const double2 w = u[ii + (size_t)g.nx * (jj + (size_t)g.ny * kk)];
        P[nb_index(dx, dy, dz)] = w.x;
        C[nb_index(dx, dy, dz)] = w.y;
      }
}

__device__ __forceinline__ FaceGeo face_geo(const Geom& g) {
  FaceGeo fg;
  fg.ih[0] = 1.0 / g.hx;
  fg.ih[1] = 1.0 / g.hy;
  fg.ih[2] = 1.0 / g.hz;
  fg.area[0] = g.hy * g.hz * 0.25;
  fg.area[1] = g.hx * g.hz * 0.25;
  fg.area[2] = g.hx * g.hy * 0.25;
  return fg;
}

// ---------------------------------------------------------------------------
// scaled defect F~(u; u_old), one thread per vertex (natural order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ Phys sample_phys(const Phys& ph, const double* dts, int s) {
  Phys p = ph;
  if (dts) {
    p.dt = dts[s];
    p.s_row = p.dt * ph.row_c;
  }
  return p;
}

// Finite-volume rows of vertex (i, j, k) before Dirichlet rows (R9 of the reading):
// Fl, Fs = storage change over dt + outgoing face fluxes [kg/s]; m = the vertex's
// porous volume m_v.  P, C: the 3x3x3 neighbourhood of the current state.
__device__ __forceinline__ void fv_rows(const Geom& g, const Phys& ph, const double* phi,
                                        const double* K, const double* P, const double* C,
                                        double co, int i, int j, int k, double& Fl, double& Fs,
                                        double& m) {
  const FaceGeo fg = face_geo(g);
  double msum = 0.0;
  Fl = 0.0;
  Fs = 0.0;
  hex_residual<0, 0, 0>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  hex_residual<1, 0, 0>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  hex_residual<0, 1, 0>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  hex_residual<1, 1, 0>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  hex_residual<0, 0, 1>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  hex_residual<1, 0, 1>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  hex_residual<0, 1, 1>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  hex_residual<1, 1, 1>(g, i, j, k, phi, K, P, C, ph, fg, Fl, Fs, msum);
  m = msum * (g.hx * g.hy * g.hz * 0.125);
  const double c = C[kDiag];
  const double rc = ph.rho0 + ph.drho * c, rco = ph.rho0 + ph.drho * co;
  Fl += m * (rc - rco) / ph.dt;
  Fs += m * (rc * c - rco * co) / ph.dt;
}

__global__ __launch_bounds__(kBlock) void k_defect(Geom g, Phys ph0, const double* dts,
                                                   const double* phi_all, const double* K_all,
                                                   const double* u_all, const double* uo_all,
                                                   double* F_all, const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const Phys ph = sample_phys(ph0, dts, s);
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.N) return;
  const int i = v % g.nx, j = (v / g.nx) % g.ny, k = v / (g.nx * g.ny);
  const size_t cells = (size_t)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  const double* phi = phi_all + s * cells;
  const double* K = K_all + s * cells;
  const double2* u = reinterpret_cast<const double2*>(u_all) + (size_t)s * g.N;
  const double2* uo = reinterpret_cast<const double2*>(uo_all) + (size_t)s * g.N;
  double P[27], C[27];
  load_neighbourhood(g, u, i, j, k, P, C);
  double Fl, Fs, m;
  fv_rows(g, ph, phi, K, P, C, uo[v].y, i, j, k, Fl, Fs, m);
  double2 out;
  out.x = is_pin(g, i, j, k) ? P[kDiag] / ph.p_unit : ph.s_row * Fl;
  double cD;
  out.y = is_cdir(g, i, j, k, cD) ? C[kDiag] - cD : ph.s_row * Fs;
  reinterpret_cast<double2*>(F_all)[(size_t)s * g.N + v] = out;
}

void launch_defect(const Geom& g, const Phys& ph, const double* dts, const double* phi,
                   const double* K, const double* u, const double* u_old, double* F, int S,
                   const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(g.N, kBlock), S);
  hipLaunchKernelGGL(k_defect, grid, dim3(kBlock), 0, st, g, ph, dts, phi, K, u, u_old, F, mask);
}

// ---------------------------------------------------------------------------
// Matrix-free Jacobian product y~ = J~ x~: the directional derivative of the scaled
// defect at state u in the direction (p_unit x~_p, x~_c), with the upwind choice frozen
// at u (the same operator as the assembled exact Jacobian, k_assemble<false>).  Per face,
// with the trilinear weights of its integration point:
//   dQ = -(K/mu) A (d_d(dp) - (rho1 - rho0) dc_f g_d),
//   liquid  d(rho(c_f) Q) = (rho1 - rho0) dc_f Q + rho(c_f) dQ,
//   salt    d(rho(c_up) c_up Q) - d(rho(c_f) phi D_m d_d c) A
//         = (rho0 + 2 (rho1 - rho0) c_up) dc_up Q + rho(c_up) c_up dQ
//           - ((rho1 - rho0) dc_f phi D_m d_d c + rho(c_f) phi D_m d_d(dc)) A,
// plus the storage derivatives; Dirichlet rows are identity rows.
//
// Every face is linearised once, by the hexahedron that holds it (12 per hexahedron).  A
// workgroup takes a tile of kHexT x kHexT hexahedron columns and walks a segment of
// layers upwards; per layer each thread evaluates its hexahedron's faces direction by
// direction (sums and differences along the direction over the 4 edges, then the
// bilinear weights 3/4 and 1/4 across it) and adds each face's fluxes to the edge's start
// corner and subtracts them from its end corner.  The corners in the layer's lower plane
// are then complete (the hexahedron below carried its upper ones up), go to LDS, and the
// thread of each of the tile's inner kHexV x kHexV vertex columns sums the 4 hexahedra
// around its vertex and finishes the rows.  Neighbouring tiles overlap by one hexahedron
// column.
// ---------------------------------------------------------------------------
// the linearised fluxes of a face of direction D from the values at its integration
// point: c, and the D-derivatives of p and c (not yet divided by h_D), of the state and of
// the direction (t*); c and the direction's c at the edge's start (cA, xA) and end (cB, xB)
template <int D>
__device__ __forceinline__ void face_flux(double cf, double dp, double dc, double tcf, double tdp,
                                          double tdc, double cA, double cB, double xA, double xB,
                                          double phi, double kmu, const Phys& ph,
                                          const FaceGeo& fg, double& yl, double& ys) {
  const double ih = fg.ih[D];
  dp *= ih;
  dc *= ih;
  tdp *= ih;
  tdc *= ih;
  const double area = fg.area[D];
  const double gD = D == 2 ? ph.g : 0.0;
  const double rf = ph.rho0 + ph.drho * cf;
  const double ka = kmu * area;
  const double Q = -ka * (dp - rf * gD);
  const double tQ = -ka * (tdp - ph.drho * tcf * gD);
  const bool up_start = Q >= 0.0;
  const double cup = up_start ? cA : cB;
  const double tcup = up_start ? xA : xB;
  const double ru = ph.rho0 + ph.drho * cup;
  const double diff = phi * ph.Dm * area;
  yl = ph.drho * tcf * Q + rf * tQ;
  ys = (ph.rho0 + 2.0 * ph.drho * cup) * tcup * Q + ru * cup * tQ -
       (ph.drho * tcf * dc + rf * tdc) * diff;
}

// corner index of the point at position t along direction D and (a, b) along the other
// two directions in increasing order
template <int D>
__host__ __device__ constexpr int ecorner(int t, int a, int b) {
  return D == 0 ? t + 2 * a + 4 * b : (D == 1 ? a + 2 * t + 4 * b : a + 2 * b + 4 * t);
}

// the 4 faces of direction D of a hexahedron with corner values P, C, XP, XC: fluxes
// added to (al, as) at each edge's start corner and subtracted at its end corner
template <int D>
__device__ __forceinline__ void hex_direction(const double* P, const double* C, const double* XP,
                                              const double* XC, double pe, double kmu,
                                              const Phys& ph, const FaceGeo& fg, double (&al)[8],
                                              double (&as)[8]) {
  // per edge e = a + 2 b: sums and differences along D
  double sc[4], dc[4], dp[4], sx[4], dxc[4], dxp[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int w0 = ecorner<D>(0, e & 1, e >> 1), w1 = ecorner<D>(1, e & 1, e >> 1);
    sc[e] = C[w1] + C[w0];
    dc[e] = C[w1] - C[w0];
    dp[e] = P[w1] - P[w0];
    sx[e] = XC[w1] + XC[w0];
    dxc[e] = XC[w1] - XC[w0];
    dxp[e] = XP[w1] - XP[w0];
  }
  // weights across D: 3/4 for the face's own edge, 1/4 for the other, per coordinate,
  // first along a, then along b; the mean along D halves the sums
  double tc[4], tdc[4], tdp[4], tx[4], tdxc[4], tdxp[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int o = e ^ 1;
    tc[e] = 0.375 * sc[e] + 0.125 * sc[o];
    tdc[e] = 0.75 * dc[e] + 0.25 * dc[o];
    tdp[e] = 0.75 * dp[e] + 0.25 * dp[o];
    tx[e] = 0.375 * sx[e] + 0.125 * sx[o];
    tdxc[e] = 0.75 * dxc[e] + 0.25 * dxc[o];
    tdxp[e] = 0.75 * dxp[e] + 0.25 * dxp[o];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int o = e ^ 2;
    const int w0 = ecorner<D>(0, e & 1, e >> 1), w1 = ecorner<D>(1, e & 1, e >> 1);
    double yl, ys;
    face_flux<D>(0.75 * tc[e] + 0.25 * tc[o], 0.75 * tdp[e] + 0.25 * tdp[o],
                 0.75 * tdc[e] + 0.25 * tdc[o], 0.75 * tx[e] + 0.25 * tx[o],
                 0.75 * tdxp[e] + 0.25 * tdxp[o], 0.75 * tdxc[e] + 0.25 * tdxc[o], C[w0], C[w1],
                 XC[w0], XC[w1], pe, kmu, ph, fg, yl, ys);
    al[w0] += yl;
    as[w0] += ys;
    al[w1] -= yl;
    as[w1] -= ys;
  }
}

// the state and the direction (pressure in physical units) at the corners w0 ... w0 + 3
// of the hexahedron column's plane k
__device__ __forceinline__ void hex_plane(const Geom& g, const double2* u, const double2* x,
                                          int hi, int hj, int k, double p_unit, int w0, double* P,
                                          double* C, double* XP, double* XC) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int v = hi + (w & 1) + g.nx * (hj + (w >> 1) + g.ny * k);
    const double2 a = u[v], b = x[v];
    P[w0 + w] = a.x;
    C[w0 + w] = a.y;
    XP[w0 + w] = p_unit * b.x;
    XC[w0 + w] = b.y;
  }
}

// the finished rows of vertex (i, j, k) from the sums of its faces' fluxes (Yl, Ys) and of
// the porosity of the hexahedra around it: storage derivatives, Dirichlet identity rows,
// the product written to *yv and the dots accumulated; xv, c, dv: the direction, the
// state's c and (MODE != 0) the dot vector at the vertex
template <int MODE>
__device__ __forceinline__ void vertex_rows(const Geom& g, const Phys& ph, int i, int j, int k,
                                            double inv_dt, double2 xv, double c, double2 dv,
                                            double Yl, double Ys, double msum, double2* yv,
                                            double (&acc)[2]) {
  const double m = msum * (g.hx * g.hy * g.hz * 0.125);
  Yl += m * ph.drho * xv.y * inv_dt;
  Ys += m * (ph.rho0 + 2.0 * ph.drho * c) * xv.y * inv_dt;
  double cD;
  const double r0 = is_pin(g, i, j, k) ? xv.x : ph.s_row * Yl;
  const double r1 = is_cdir(g, i, j, k, cD) ? xv.y : ph.s_row * Ys;
  *yv = make_double2(r0, r1);
  if (MODE != 0) {
    acc[0] += dv.x * r0 + dv.y * r1;
    if (MODE == 2) acc[1] += r0 * r0 + r1 * r1;
  }
}

constexpr int kHexT = 16;         // hexahedron columns per tile side
constexpr int kHexV = kHexT - 1;  // vertex columns finished per tile side
static_assert(kHexT * kHexT == kBlock, "one hexahedron column per thread");

// MODE as k_spmv: 0 plain, 1 with the dot (d, y), 2 with (d, y) and (y, y).  Workgroup b
// of a sample row takes tile b % (ntx nty) (hexahedron columns from 15 tx - 1 and
// 15 ty - 1; thread t the column (t % 16, t / 16) in it) and the segment b / (ntx nty) of
// nseg equal segments of the nz vertices.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_jx(Geom g, Phys ph0, const double* dts,
                                               const double* phi_all, const double* K_all,
                                               const double* u_all, const double* x_all,
                                               double* y_all, const double* d_all, double* part,
                                               const int* mask, const int* list, int nseg, int ntx,
                                               int nty) {
  __shared__ double2 ex[2][4][kBlock];  // per layer parity: the corners' rows of each thread
  __shared__ double exm[2][kBlock];     // and its porosity sum
  const int s = list ? list[blockIdx.y] : blockIdx.y;
  if (mask && !mask[s]) return;
  const Phys ph = sample_phys(ph0, dts, s);
  const int tiles = ntx * nty;
  const int seg = blockIdx.x / tiles, tile = blockIdx.x - seg * tiles;
  const int ty = tile / ntx, tx = tile - ty * ntx;
  const int tid = threadIdx.x, ta = tid % kHexT, tb = tid / kHexT;
  const int hi = tx * kHexV - 1 + ta, hj = ty * kHexV - 1 + tb;  // hexahedron column
  const bool hex = hi >= 0 && hi <= g.nx - 2 && hj >= 0 && hj <= g.ny - 2;
  // the vertex column (hi, hj) is finished here when its 4 hexahedron columns are in the tile
  const bool vert = ta >= 1 && tb >= 1 && hi < g.nx && hj < g.ny;
  const double inv_mu = 1.0 / ph.mu, inv_dt = 1.0 / ph.dt;
  const int k0 = (seg * g.nz) / nseg, k1 = ((seg + 1) * g.nz) / nseg;  // vertices [k0, k1)
  const int cells = (g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  const double* phi = phi_all + (size_t)s * cells;
  const double* K = K_all + (size_t)s * cells;
  const double2* u = reinterpret_cast<const double2*>(u_all) + (size_t)s * g.N;
  const double2* x = reinterpret_cast<const double2*>(x_all) + (size_t)s * g.N;
  double2* y = reinterpret_cast<double2*>(y_all) + (size_t)s * g.N;
  const double2* d = MODE ? reinterpret_cast<const double2*>(d_all) + (size_t)s * g.N : nullptr;
  const FaceGeo fg = face_geo(g);
  const int L0 = k0 > 0 ? k0 - 1 : 0, L1 = k1 - 1 < g.nz - 2 ? k1 - 1 : g.nz - 2;
  double P[8], C[8], XP[8], XC[8];
  if (hex) hex_plane(g, u, x, hi, hj, L0, ph.p_unit, 0, P, C, XP, XC);
  // the upper corners' rows of the hexahedron below and its porosity
  double cl[4] = {0.0, 0.0, 0.0, 0.0}, cs[4] = {0.0, 0.0, 0.0, 0.0}, cm = 0.0;
  double acc[2] = {0.0, 0.0};
  // the rows of vertex (hi, hj, k) from the 4 hexahedron columns around it (this thread's
  // corner 0, its -x neighbour's corner 1, -y: corner 2, -x -y: corner 3), then finished
  auto finish = [&](int k) {
    const int p = k & 1;
    const double2 r0 = ex[p][0][tid], r1 = ex[p][1][tid - 1], r2 = ex[p][2][tid - kHexT],
                  r3 = ex[p][3][tid - kHexT - 1];
    const double ms =
        exm[p][tid] + exm[p][tid - 1] + exm[p][tid - kHexT] + exm[p][tid - kHexT - 1];
    const int v = hi + g.nx * (hj + g.ny * k);
    const double2 xv = x[v], dv = MODE ? d[v] : make_double2(0.0, 0.0);
    vertex_rows<MODE>(g, ph, hi, hj, k, inv_dt, xv, u[v].y, dv, r0.x + r1.x + r2.x + r3.x,
                      r0.y + r1.y + r2.y + r3.y, ms, y + v, acc);
  };
#pragma unroll 1
  for (int L = L0; L <= L1; ++L) {
    double al[8], as[8], pe = 0.0;
#pragma unroll
    for (int w = 0; w < 8; ++w) al[w] = as[w] = 0.0;
    if (hex) {
      const int e = hi + (g.nx - 1) * (hj + (g.ny - 1) * L);
      pe = phi[e];
      const double kmu = K[e] * inv_mu;
      hex_plane(g, u, x, hi, hj, L + 1, ph.p_unit, 4, P, C, XP, XC);
      hex_direction<0>(P, C, XP, XC, pe, kmu, ph, fg, al, as);
      hex_direction<1>(P, C, XP, XC, pe, kmu, ph, fg, al, as);
      hex_direction<2>(P, C, XP, XC, pe, kmu, ph, fg, al, as);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        P[w] = P[w + 4];
        C[w] = C[w + 4];
        XP[w] = XP[w + 4];
        XC[w] = XC[w + 4];
      }
    }
    const int p = L & 1;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      ex[p][w][tid] = make_double2(cl[w] + al[w], cs[w] + as[w]);
      cl[w] = al[w + 4];
      cs[w] = as[w + 4];
    }
    exm[p][tid] = cm + pe;
    cm = pe;
    __syncthreads();
    if (vert && L >= k0) finish(L);
  }
  // the top plane has only the hexahedra below it
  if (k1 == g.nz) {
    const int p = (g.nz - 1) & 1;
#pragma unroll
    for (int w = 0; w < 4; ++w) ex[p][w][tid] = make_double2(cl[w], cs[w]);
    exm[p][tid] = cm;
    __syncthreads();
    if (vert) finish(g.nz - 1);
  }
  if (MODE == 1) {
    double a1[1] = {acc[0]};
    block_partial<1>(a1, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
  } else if (MODE == 2) {
    block_partial<2>(acc, part + ((size_t)s * gridDim.x + blockIdx.x) * 4);
  }
}

// vertices per column segment: short enough that a few active samples still give the
// device many workgroups, long enough that the layer evaluated twice (below each
// segment's first vertex) stays a small part of the work
constexpr int kJxSegment = 8;

int jx_blocks(const Geom& g) {
  return ceil_div(g.nx, kHexV) * ceil_div(g.ny, kHexV) * ceil_div(g.nz, kJxSegment);
}

int launch_jx(const Geom& g, const Phys& ph, const double* dts, const double* phi, const double* K,
              const double* u, const double* x, double* y, const double* d, double* part, int mode,
              int S, const int* mask, const int* list, int rows, hipStream_t st) {
  const int nseg = ceil_div(g.nz, kJxSegment);
  const int ntx = ceil_div(g.nx, kHexV), nty = ceil_div(g.ny, kHexV);
  const int nb = jx_blocks(g);
  dim3 grid(nb, rows);
  if (mode == 0)
    hipLaunchKernelGGL(k_jx<0>, grid, dim3(kBlock), 0, st, g, ph, dts, phi, K, u, x, y, d, part,
                       mask, list, nseg, ntx, nty);
  else if (mode == 1)
    hipLaunchKernelGGL(k_jx<1>, grid, dim3(kBlock), 0, st, g, ph, dts, phi, K, u, x, y, d, part,
                       mask, list, nseg, ntx, nty);
  else
    hipLaunchKernelGGL(k_jx<2>, grid, dim3(kBlock), 0, st, g, ph, dts, phi, K, u, x, y, d, part,
                       mask, list, nseg, ntx, nty);
  (void)S;
  return nb;
}

// ---------------------------------------------------------------------------
// Global mass balance of one (sub-)step in FP64 (eqs. e_cont_eq and e_tran_eq summed
// over all control volumes).  Interior face fluxes cancel in pairs and the no-flow
// faces carry none, so the storage change of the box equals dt times the rows of the
// vertices whose equation is replaced by a Dirichlet condition: the salt rows of the
// c-Dirichlet vertices and the liquid rows of the pinned vertices.  Per vertex and
// sample: [0] salt storage change m_v (rho c - rho_old c_old), [1] its absolute value,
// [2] liquid storage change m_v (rho - rho_old), [3] its absolute value, [4] dt x the
// salt row at a c-Dirichlet vertex, [5] dt x the liquid row at a pinned vertex (kg).
// Block totals go to part[s][b][0..7]; k_balance_add adds the samples' sums to
// acc[s][0..7] in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_balance(Geom g, Phys ph0, const double* dts,
                                                    const double* phi_all, const double* K_all,
                                                    const double* u_all, const double* uo_all,
                                                    double* part, const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const Phys ph = sample_phys(ph0, dts, s);
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (v < g.N) {
    const int i = v % g.nx, j = (v / g.nx) % g.ny, k = v / (g.nx * g.ny);
    const size_t cells = (size_t)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
    const double* phi = phi_all + s * cells;
    const double* K = K_all + s * cells;
    const double2* u = reinterpret_cast<const double2*>(u_all) + (size_t)s * g.N;
    const double2* uo = reinterpret_cast<const double2*>(uo_all) + (size_t)s * g.N;
    double cD;
    const bool cdir = is_cdir(g, i, j, k, cD), pin = is_pin(g, i, j, k);
    const double c = u[v].y, co = uo[v].y;
    double m;
    if (cdir || pin) {
      double P[27], C[27], Fl, Fs;
      load_neighbourhood(g, u, i, j, k, P, C);
      fv_rows(g, ph, phi, K, P, C, co, i, j, k, Fl, Fs, m);
      if (cdir) a[4] = ph.dt * Fs;
      if (pin) a[5] = ph.dt * Fl;
    } else {
      double msum = 0.0;
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int hi = i - (h & 1), hj = j - ((h >> 1) & 1), hk = k - (h >> 2);
        if (hi < 0 || hj < 0 || hk < 0 || hi > g.nx - 2 || hj > g.ny - 2 || hk > g.nz - 2) continue;
        msum += phi[hi + (size_t)(g.nx - 1) * (hj + (size_t)(g.ny - 1) * hk)];
      }
      m = msum * (g.hx * g.hy * g.hz * 0.125);
    }
    const double rc = ph.rho0 + ph.drho * c, rco = ph.rho0 + ph.drho * co;
    a[0] = m * (rc * c - rco * co);
    a[1] = fabs(a[0]);
    a[2] = m * (rc - rco);
    a[3] = fabs(a[2]);
  }
  block_partial<6>(a, part + ((size_t)s * gridDim.x + blockIdx.x) * 8);
}

__global__ __launch_bounds__(64) void k_balance_add(int nb, const double* part, double* acc,
                                                    const int* mask) {
  const int s = blockIdx.x;
  if (mask && !mask[s]) return;
  const int lane = threadIdx.x;
  double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = lane; b < nb; b += 64)
#pragma unroll
    for (int e = 0; e < 6; ++e) q[e] += part[((size_t)s * nb + b) * 8 + e];
#pragma unroll
  for (int e = 0; e < 6; ++e)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q[e] += __shfl_down(q[e], off, 64);
  if (lane == 0)
#pragma unroll
    for (int e = 0; e < 6; ++e) acc[(size_t)s * 8 + e] += q[e];
}

int balance_blocks(const Geom& g) { return ceil_div(g.N, kBlock); }

void launch_balance(const Geom& g, const Phys& ph, const double* dts, const double* phi,
                    const double* K, const double* u, const double* u_old, double* part,
                    double* acc, int S, const int* mask, hipStream_t st) {
  const int nb = balance_blocks(g);
  hipLaunchKernelGGL(k_balance, dim3(nb, S), dim3(kBlock), 0, st, g, ph, dts, phi, K, u, u_old,
                     part, mask);
  hipLaunchKernelGGL(k_balance_add, dim3(S), dim3(64), 0, st, nb, part, acc, mask);
}

// ---------------------------------------------------------------------------
// Jacobian rows: derivatives of one equation row EQ of vertex v with respect to
// (p, c) at its 27 neighbours, upwind choice frozen.
// ---------------------------------------------------------------------------
template <int EQ, bool FROZEN, int AX, int AY, int AZ, int D>
__device__ __forceinline__ void face_jacobian(const double* P, const double* C, double phi,
                                              double K, const Phys& ph, const FaceGeo& fg,
                                              double* Ap, double* Ac) {
  using F = FaceT<AX, AY, AZ, D>;
  double cf = 0.0, dp = 0.0, dc = 0.0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    cf += F::N(w) * C[F::nb(w)];
    dp += F::dN(w) * P[F::nb(w)];
    dc += F::dN(w) * C[F::nb(w)];
  }
  const double ih = fg.ih[D];
  dp *= ih;
  dc *= ih;
  const double area = fg.area[D];
  const double gD = D == 2 ? ph.g : 0.0;
  const double rf = ph.rho0 + ph.drho * cf;
  const double kmu = K / ph.mu * area;
  const double Q = -kmu * (dp - rf * gD);
  const bool up_start = Q >= 0.0;
  const double cup = up_start ? C[F::NA] : C[F::NB];
  const double ru = ph.rho0 + ph.drho * cup;
  const double sgn = F::VD == 0 ? 1.0 : -1.0;
  const double dup = (ph.rho0 + 2.0 * ph.drho * cup) * Q;  // d(rho(c) c Q)/dc_up
  const double diff = phi * ph.Dm * area;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    const double Nw = F::N(w);
    const double dNw = F::dN(w) * ih;
    const double dQdp = -kmu * dNw;
    const double dQdc = kmu * ph.drho * gD * Nw;
    double dpw, dcw;
    if (EQ == 0) {
      dpw = rf * dQdp;
      dcw = ph.drho * Nw * Q + rf * dQdc;
    } else {
      dpw = ru * cup * dQdp;
      dcw = (FROZEN ? 0.0 : ru * cup * dQdc) - ph.drho * Nw * diff * dc - rf * diff * dNw;
      if (F::nb(w) == F::NA && up_start) dcw += dup;
      if (F::nb(w) == F::NB && !up_start) dcw += dup;
    }
    Ap[F::nb(w)] += sgn * dpw;
    Ac[F::nb(w)] += sgn * dcw;
  }
}

template <int EQ, bool FROZEN, int AX, int AY, int AZ>
__device__ __forceinline__ void hex_jacobian(const Geom& g, int i, int j, int k, const double* phi,
                                             const double* K, const double* P, const double* C,
                                             const Phys& ph, const FaceGeo& fg, double* Ap,
                                             double* Ac, double& msum) {
  const int hi = i - AX, hj = j - AY, hk = k - AZ;
  if (hi < 0 || hj < 0 || hk < 0 || hi > g.nx - 2 || hj > g.ny - 2 || hk > g.nz - 2) return;
  const size_t e = hi + (size_t)(g.nx - 1) * (hj + (size_t)(g.ny - 1) * hk);
  const double pe = phi[e], Ke = K[e];
  msum += pe;
  face_jacobian<EQ, FROZEN, AX, AY, AZ, 0>(P, C, pe, Ke, ph, fg, Ap, Ac);
  face_jacobian<EQ, FROZEN, AX, AY, AZ, 1>(P, C, pe, Ke, ph, fg, Ap, Ac);
  face_jacobian<EQ, FROZEN, AX, AY, AZ, 2>(P, C, pe, Ke, ph, fg, Ap, Ac);
}

template <int EQ, bool FROZEN>
__device__ __forceinline__ void assemble_row(const Geom& g, const Phys& ph, const double* phi,
                                             const double* K, const double* P, const double* C,
                                             int i, int j, int k, size_t s0, int t,
                                             double* A64, float* A32) {
  double Ap[27], Ac[27];
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    Ap[o] = 0.0;
    Ac[o] = 0.0;
  }
  const FaceGeo fg = face_geo(g);
  double msum = 0.0;
  hex_jacobian<EQ, FROZEN, 0, 0, 0>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  hex_jacobian<EQ, FROZEN, 1, 0, 0>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  hex_jacobian<EQ, FROZEN, 0, 1, 0>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  hex_jacobian<EQ, FROZEN, 1, 1, 0>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  hex_jacobian<EQ, FROZEN, 0, 0, 1>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  hex_jacobian<EQ, FROZEN, 1, 0, 1>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  hex_jacobian<EQ, FROZEN, 0, 1, 1>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  hex_jacobian<EQ, FROZEN, 1, 1, 1>(g, i, j, k, phi, K, P, C, ph, fg, Ap, Ac, msum);
  const double m = msum * (g.hx * g.hy * g.hz * 0.125);
  const double c = C[kDiag];
  if (EQ == 0)
    Ac[kDiag] += m * ph.drho / ph.dt;
  else
    Ac[kDiag] += m * (ph.rho0 + 2.0 * ph.drho * c) / ph.dt;
  double cD;
  const bool dir = EQ == 0 ? is_pin(g, i, j, k) : is_cdir(g, i, j, k, cD);
  const double sp = ph.s_row * ph.p_unit, sc = ph.s_row;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    double ap = sp * Ap[o], ac = sc * Ac[o];
    if (dir) {
      ap = (o == kDiag && EQ == 0) ? 1.0 : 0.0;
      ac = (o == kDiag && EQ == 1) ? 1.0 : 0.0;
    }
    const int pl = o * 4 + EQ * 2;  // (row EQ, column p) and (row EQ, column c)
    if (A64) {
      double* a = A64 + s0 + sidx<double>(t, 0, kPlanes);
      a[soff<double>(pl)] = ap;
      a[soff<double>(pl + 1)] = ac;
    }
    if (A32) {
      float* a = A32 + s0 + sidx<float>(t, 0, kPlanes);
      a[soff<float>(pl)] = (float)ap;
      a[soff<float>(pl + 1)] = (float)ac;
    }
  }
}

// FROZEN = true assembles the matrix of the multigrid preconditioner: the salt rows
// are linearised at a frozen Darcy flux (the derivative of Q with respect to c through
// the buoyancy term is dropped).  With it, inflow of brine at c_up = 1 into a vertex at
// c = 0 would make the salt block lose diagonal dominance, and point smoothers diverge;
// in the full system the pressure response cancels most of that feedback.  The Krylov
// method always multiplies with the exact Jacobian (FROZEN = false).
template <bool FROZEN>
__global__ __launch_bounds__(kBlock) void k_assemble(Geom g, Phys ph0, const double* dts,
                                                     const double* phi_all, const double* K_all,
                                                     const double* u_all, double* A64, float* A32,
                                                     const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const Phys ph = sample_phys(ph0, dts, s);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t >= g.off[8] || !colour_decode(g, t, i, j, k)) return;
  const size_t cells = (size_t)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  const double* phi = phi_all + s * cells;
  const double* K = K_all + s * cells;
  const double2* u = reinterpret_cast<const double2*>(u_all) + (size_t)s * g.N;
  double P[27], C[27];
  load_neighbourhood(g, u, i, j, k, P, C);
  const size_t s0 = (size_t)s * kPlanes * g.off[8];
  if (blockIdx.z == 0)
    assemble_row<0, FROZEN>(g, ph, phi, K, P, C, i, j, k, s0, t, A64, A32);
  else
    assemble_row<1, FROZEN>(g, ph, phi, K, P, C, i, j, k, s0, t, A64, A32);
}

void launch_assemble(const Geom& g, const Phys& ph, const double* dts, const double* phi,
                     const double* K, const double* u, double* A64, float* A32, int S,
                     const int* mask, hipStream_t st, bool frozen) {
  dim3 grid(ceil_div(g.off[8], kBlock), S, 2);
  if (frozen)
    hipLaunchKernelGGL(k_assemble<true>, grid, dim3(kBlock), 0, st, g, ph, dts, phi, K, u, A64,
                       A32, mask);
  else
    hipLaunchKernelGGL(k_assemble<false>, grid, dim3(kBlock), 0, st, g, ph, dts, phi, K, u, A64,
                       A32, mask);
}

// ---------------------------------------------------------------------------
// inverses of the 2x2 diagonal blocks, Dinv[s][Np x 4] (colour-major, packed)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_block_inverse(Geom g, const T* A, T* Dinv,
                                                          const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t >= g.off[8] || !colour_decode(g, t, i, j, k)) return;
  const size_t Np = g.off[8];
  const T* a = A + (size_t)s * kPlanes * Np + sidx<T>(t, 0, kPlanes);
  const double a00 = a[soff<T>(kDiag * 4)], a01 = a[soff<T>(kDiag * 4 + 1)],
               a10 = a[soff<T>(kDiag * 4 + 2)], a11 = a[soff<T>(kDiag * 4 + 3)];
  const double det = a00 * a11 - a01 * a10;
  const double id = det != 0.0 ? 1.0 / det : 0.0;
  T* d = Dinv + (size_t)s * 4 * Np + sidx<T>(t, 0, 4);
  d[soff<T>(0)] = (T)(a11 * id);
  d[soff<T>(1)] = (T)(-a01 * id);
  d[soff<T>(2)] = (T)(-a10 * id);
  d[soff<T>(3)] = (T)(a00 * id);
}

void launch_block_inverse_f64(const Geom& g, const double* A, double* Dinv, int S,
                              const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(g.off[8], kBlock), S);
  hipLaunchKernelGGL(k_block_inverse<double>, grid, dim3(kBlock), 0, st, g, A, Dinv, mask);
}
void launch_block_inverse_f32(const Geom& g, const float* A, float* Dinv, int S,
                              const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(g.off[8], kBlock), S);
  hipLaunchKernelGGL(k_block_inverse<float>, grid, dim3(kBlock), 0, st, g, A, Dinv, mask);
}

// ---------------------------------------------------------------------------
// state injection to the next coarser grid: u_c(I,J,K) = u_f(2I,2J,2K)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_inject(Geom gf, Geom gc, const double* uf, double* uc,
                                                   const int* mask) {
  const int s = blockIdx.y;
  if (mask && !mask[s]) return;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= gc.N) return;
  const int I = v % gc.nx, J = (v / gc.nx) % gc.ny, K = v / (gc.nx * gc.ny);
  const size_t vf = 2 * I + (size_t)gf.nx * (2 * J + (size_t)gf.ny * 2 * K);
  reinterpret_cast<double2*>(uc)[(size_t)s * gc.N + v] =
      reinterpret_cast<const double2*>(uf)[(size_t)s * gf.N + vf];
}

void launch_inject(const Geom& gf, const Geom& gc, const double* uf, double* uc, int S,
                   const int* mask, hipStream_t st) {
  dim3 grid(ceil_div(gc.N, kBlock), S);
  hipLaunchKernelGGL(k_inject, grid, dim3(kBlock), 0, st, gf, gc, uf, uc, mask);
}

// stencil of one sample, colour-major -> natural vertex order (inspection only)
__global__ __launch_bounds__(kBlock) void k_stencil_to_natural(Geom g, const double* A,
                                                               double* out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.N) return;
  const int i = v % g.nx, j = (v / g.nx) % g.ny, k = v / (g.nx * g.ny);
  const int t = colour_encode(g, i, j, k);
  for (int p = 0; p < kPlanes; ++p) out[(size_t)p * g.N + v] = A[sidx<double>(t, p, kPlanes)];
}

void launch_stencil_to_natural(const Geom& g, const double* A, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_stencil_to_natural, dim3(ceil_div(g.N, kBlock)), dim3(kBlock), 0, st, g, A,
                     out);
}

}  // namespace edf
