// Device helpers shared by the kernel files: index maps and boundary sets.
#pragma once

#include "edf_internal.h"

namespace edf {

// neighbour index of offset (dx, dy, dz) in {-1,0,1}^3
__host__ __device__ constexpr int nb_index(int dx, int dy, int dz) {
  return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
}

__device__ __forceinline__ int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

// Layout of per-vertex coefficient arrays (stencils: P = 108, block inverses: P = 4):
// colour-major positions in tiles of kTile; inside a tile the P values of a position
// are packed W at a time into 16-byte lane vectors (W = 2 doubles or 4 floats), so
// one load per lane fetches W coefficients and a wave's load is 1 KiB contiguous.
template <typename T>
constexpr int kPack = sizeof(T) == 2 ? 4 : 16 / (int)sizeof(T);  // FP16: one 2x2 block

// index of value p (of P per vertex) at colour-major position t
template <typename T>
__host__ __device__ __forceinline__ size_t sidx(int t, int p, int P) {
  constexpr int W = kPack<T>;
  return ((size_t)(t / kTile) * (P / W) + p / W) * (kTile * W) + (size_t)(t % kTile) * W + p % W;
}

// offset of value p from value 0 of the same position
template <typename T>
__host__ __device__ __forceinline__ size_t soff(int p) {
  constexpr int W = kPack<T>;
  return (size_t)(p / W) * (kTile * W) + p % W;
}

// the 2x2 block (a00, a01, a10, a11) stored at values p..p+3 (p a multiple of 4).  NT:
// streaming (non-temporal) loads for coefficients read once per sweep, which should not
// evict the vectors; plain loads for the small coarse levels, which may stay cached from
// one sweep to the next.  FP16 blocks are returned in FP32.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef _Float16 nt_h4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Block2 {
  T a00, a01, a10, a11;
};
template <bool NT, typename V>
__device__ __forceinline__ V load_vec(const V* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT = true>
__device__ __forceinline__ Block2<double> load_block(const double* base, int p) {
  const nt_d2 u = load_vec<NT>(reinterpret_cast<const nt_d2*>(base + soff<double>(p)));
  const nt_d2 w = load_vec<NT>(reinterpret_cast<const nt_d2*>(base + soff<double>(p + 2)));
  return {u.x, u.y, w.x, w.y};
}
template <bool NT = true>
__device__ __forceinline__ Block2<float> load_block(const float* base, int p) {
  const nt_f4 u = load_vec<NT>(reinterpret_cast<const nt_f4*>(base + soff<float>(p)));
  return {u.x, u.y, u.z, u.w};
}
template <bool NT = true>
__device__ __forceinline__ Block2<float> load_block(const _Float16* base, int p) {
  const nt_h4 u = load_vec<NT>(reinterpret_cast<const nt_h4*>(base + soff<_Float16>(p)));
  return {(float)u.x, (float)u.y, (float)u.z, (float)u.w};
}

// two-component vector of T (one vertex's (p, c) pair)
template <typename T>
struct V2;
template <>
struct V2<double> {
  using type = double2;
};
template <>
struct V2<float> {
  using type = float2;
};

// colour-major position t -> vertex (i, j, k); false for padding positions
__device__ __forceinline__ bool colour_decode(const Geom& g, int t, int& i, int& j, int& k) {
  int col = 0;
#pragma unroll
  for (int c = 1; c < 8; ++c) col += (t >= g.off[c]) ? 1 : 0;
  const int s = t - g.off[col];
  if (s >= g.cnt[col]) return false;
  const int mx = g.mx[col], my = g.my[col];
  const int a = s % mx;
  const int r = s / mx;
  const int b = r % my;
  const int c = r / my;
  i = 2 * a + (col & 1);
  j = 2 * b + ((col >> 1) & 1);
  k = 2 * c + (col >> 2);
  return true;
}

// position inside colour `col` -> vertex (i, j, k)
__device__ __forceinline__ void colour_decode_in(const Geom& g, int col, int s, int& i, int& j,
                                                 int& k) {
  const int mx = g.mx[col], my = g.my[col];
  const int a = s % mx;
  const int r = s / mx;
  i = 2 * a + (col & 1);
  j = 2 * (r % my) + ((col >> 1) & 1);
  k = 2 * (r / my) + (col >> 2);
}

// vertex (i, j, k) -> colour-major position
__device__ __forceinline__ int colour_encode(const Geom& g, int i, int j, int k) {
  const int col = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
  return g.off[col] + (i >> 1) + g.mx[col] * ((j >> 1) + g.my[col] * (k >> 1));
}

// colour of position t for a wave of 64 consecutive positions that starts at a multiple
// of 64: colours start at multiples of 64, so the wave lies in one colour, which is
// returned as a scalar
__device__ __forceinline__ int wave_colour(const Geom& g, int t) {
  int col = 0;
#pragma unroll
  for (int c = 1; c < 8; ++c) col += (t >= g.off[c]) ? 1 : 0;
  return __builtin_amdgcn_readfirstlane(col);
}

// colour_decode for such a wave, also giving the (scalar) colour
__device__ __forceinline__ bool colour_decode_wave(const Geom& g, int t, int& col, int& i, int& j,
                                                   int& k) {
  col = wave_colour(g, t);
  const int s = t - g.off[col];
  if (s >= g.cnt[col]) return false;
  colour_decode_in(g, col, s, i, j, k);
  return true;
}

// colour_encode where the colour differs between the lanes of a wave: the colour's
// start, row length and plane size are picked by selects among scalars instead of
// per-lane reads of the grid description
__device__ __forceinline__ int colour_encode_sel(const Geom& g, int i, int j, int k) {
  const bool bx = i & 1, by = j & 1, bz = k & 1;
  const int o0 = bx ? g.off[1] : g.off[0], o1 = bx ? g.off[3] : g.off[2];
  const int o2 = bx ? g.off[5] : g.off[4], o3 = bx ? g.off[7] : g.off[6];
  const int o = bz ? (by ? o3 : o2) : (by ? o1 : o0);
  const int mx = bx ? g.mx[1] : g.mx[0], my = by ? g.my[2] : g.my[0];
  return o + (i >> 1) + mx * ((j >> 1) + my * (k >> 1));
}

// Neighbour values for the vertices of one colour.  Colour c = px + 2 py + 4 pz holds
// the vertices with those coordinate parities; its row length g.mx[c] depends on px only
// and its rows per plane g.my[c] on py only.  The colour of neighbour (dx, dy, dz) is the
// same for every vertex of a colour, so once the colour is known for the whole wave the
// neighbour colour's start, size, row length and plane size are scalars, and the
// neighbour's place in its colour is one of four per-vertex bases (one per parity flip in
// x and y) plus a scalar.  A neighbour outside the grid carries a zero stencil block; its
// place is clamped into the neighbour colour's range (never empty: every dimension has at
// least 2 vertices), so it reads some valid value of that colour.
struct NbrMap {
  int px, py, pz;
  int base[4];  // a + mx(px ^ fx) (b + my(py ^ fy) c) for the flips fx + 2 fy
};

__device__ __forceinline__ NbrMap nbr_map(const Geom& g, int col, int i, int j, int k) {
  NbrMap m;
  m.px = col & 1;
  m.py = (col >> 1) & 1;
  m.pz = col >> 2;
  const int a = i >> 1, b = j >> 1, c = k >> 1;
#pragma unroll
  for (int f = 0; f < 4; ++f)
    m.base[f] = a + g.mx[m.px ^ (f & 1)] * (b + g.my[2 * (m.py ^ (f >> 1))] * c);
  return m;
}

// place of neighbour (dx, dy, dz) in its colour cn (a scalar for the wave): inside the
// grid, colour_encode(i + dx, j + dy, k + dz) = g.off[cn] + place.  A place below 0 wraps
// to a large unsigned value and is clamped like one beyond the colour's end.
__device__ __forceinline__ unsigned nbr_place(const Geom& g, const NbrMap& m, int dx, int dy,
                                              int dz, int& cn) {
  const int qx = m.px ^ (dx & 1), qy = m.py ^ (dy & 1), qz = m.pz ^ (dz & 1);
  cn = qx + 2 * qy + 4 * qz;
  const int shift =
      ((m.px + dx) >> 1) + g.mx[qx] * (((m.py + dy) >> 1) + g.my[2 * qy] * ((m.pz + dz) >> 1));
  return min((unsigned)(m.base[(dx & 1) + 2 * (dy & 1)] + shift), (unsigned)(g.cnt[cn] - 1));
}

// the value of neighbour (dx, dy, dz) in a colour-major vector of V: the colour's start
// offsets the (scalar) base pointer, the place is a 32-bit unsigned byte offset
template <typename V>
__device__ __forceinline__ V load_nbr(const V* x, const Geom& g, const NbrMap& m, int dx, int dy,
                                      int dz) {
  int cn;
  const unsigned u = nbr_place(g, m, dx, dy, dz, cn);
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(x + g.off[cn]) +
                                     u * (unsigned)sizeof(V));
}

// XCD-aware tile order.  The workgroups of a launch go to the device's 8 XCDs in turn
// (linear workgroup id bx + by gx modulo 8), and each XCD has its own L2.  Workgroup bx of
// grid row by takes a tile such that each XCD works through one contiguous range of the
// row's gx tiles (a bijection of [0, gx)): the tiles of neighbouring grid rows, which
// gather the same neighbour values, then share one L2 instead of fetching those values
// into several.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int bx, int by, int gx) {
  const int c0 = (int)(((long long)by * gx) % kXcds);  // the XCD of the row's first workgroup
  const int xcd = (c0 + bx) % kXcds;
  int start = 0;  // tiles of the XCDs before this one
  for (int x = 0; x < xcd; ++x) {
    const int f = (x - c0 + kXcds) % kXcds;  // first workgroup of the row on XCD x
    start += f < gx ? (gx - 1 - f) / kXcds + 1 : 0;
  }
  return start + (bx - (xcd - c0 + kXcds) % kXcds) / kXcds;
}

// Slab order of a level's 64-position tiles for kernels whose work differs by colour.
// Each colour's tiles are cut into kXcds slabs (positions run through k/2 slowest, so
// slab x of every colour covers about the same depth range); XCD x takes slab x of every
// colour, which gives every XCD the same mix of colours and keeps its neighbour gathers
// in its own depth range.  With gridDim.x a multiple of kXcds, workgroup bx runs on XCD
// bx % kXcds whatever its grid row.  Tile e of slab x -> (colour, tile within the colour);
// false past the slab's end.
__host__ __device__ __forceinline__ int slab_tiles(const Geom& g, int c, int x) {
  const int T = (g.off[c + 1] - g.off[c]) / kTile;
  return ((x + 1) * T) / kXcds - (x * T) / kXcds;
}
__device__ __forceinline__ bool slab_tile(const Geom& g, int x, int e, int& col, int& tile) {
  for (int c = 0; c < 8; ++c) {
    const int n = slab_tiles(g, c, x);
    if (e < n) {
      col = c;
      tile = (x * ((g.off[c + 1] - g.off[c]) / kTile)) / kXcds + e;
      return true;
    }
    e -= n;
  }
  return false;
}
// workgroups of kBlock threads along x for a launch in slab order
inline int slab_blocks(const Geom& g) {
  int most = 0;
  for (int x = 0; x < kXcds; ++x) {
    int n = 0;
    for (int c = 0; c < 8; ++c) n += slab_tiles(g, c, x);
    most = n > most ? n : most;
  }
  return kXcds * ceil_div(most, kBlock / kTile);
}

// Vertical lines (z-columns) of the line smoother: the blocks of a column's tridiagonal
// part and the colour-major position of its vertex at height k.  Column q of column
// colour cc is (i, j) = (2 (q % mx) + (cc & 1), 2 (q / mx) + (cc >> 1)), mx = g.mx[cc]; its
// vertex at height k has vertex colour cc + 4 (k & 1) and place q + mx my (k >> 1) there.
constexpr int kLineL = 4;   // nb_index(0, 0, -1): the vertex above (smaller depth)
constexpr int kLineU = 22;  // nb_index(0, 0, +1): the vertex below
__device__ __forceinline__ int line_pos(const Geom& g, int cc, int q, int k) {
  return g.off[cc + 4 * (k & 1)] + q + g.mx[cc] * g.my[cc] * (k >> 1);
}

// salt Dirichlet vertex (closed top patch: c = 1; bottom: c = 0)
__device__ __forceinline__ bool is_cdir(const Geom& g, int i, int j, int k, double& value) {
  if (k == g.nz - 1) { value = 0.0; return true; }
  if (k == 0 && i >= g.pi0 && i <= g.pi1 && j >= g.pj0 && j <= g.pj1) { value = 1.0; return true; }
  return false;
}

// pressure-pinned vertex (the four top corners)
__device__ __forceinline__ bool is_pin(const Geom& g, int i, int j, int k) {
  return k == 0 && (i == 0 || i == g.nx - 1) && (j == 0 || j == g.ny - 1);
}

// Sums Q per-lane values over a workgroup of kBlock lanes and writes the Q block totals
// to part[0..Q-1] (wave shuffles, then the waves' sums in a fixed order: deterministic).
template <int Q>
__device__ __forceinline__ void block_partial(double (&v)[Q], double* part) {
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

}  // namespace edf
