// HIP kernels (gfx950) for the k+1 shifted SPD solves of the BURA method
// (Section 2.2, eq. (16)): matrix-free 5/7-point stencils of the scaled operator
// A + s I (Section 1.4, eq. (10); Section 5.3), weighted-Jacobi smoothing,
// full-weighting restriction, multilinear prolongation, an in-LDS V-cycle for
// the coarse levels, the PCG vector updates with FP64 block reductions, the
// FP64 residual of the refinement loop and the FP64 combine of eq. (16).
//
// Every launch processes a batch of independent systems: blockIdx.z (stencil
// launches) or blockIdx.y (flat kernels) selects the system; a system whose `active` flag
// is 0 is skipped by whole blocks.  Reductions are deterministic: each block
// writes one FP64 partial per system and a per-system kernel adds the partials
// in a fixed order, so a system's result does not depend on what else is in
// the batch.
#include "bura_internal.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace bura {

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------

// Tile coordinates of a stencil workgroup: (x tile, y tile, system), in launch
// order.  Workgroups are dealt to the 8 XCDs round-robin, so vertically
// adjacent tiles sit on different L2s and their common halo rows are fetched
// twice; those second fetches hit the on-package last-level cache.  Renumbering
// the workgroups so that an XCD takes contiguous tiles removed them but made
// every stencil kernel slower (it concentrates each XCD on one address range),
// so launch order is kept.
struct Tile {
  int x, y, z;
};

__device__ __forceinline__ Tile block_tile() {
  Tile r;
  r.x = blockIdx.x;
  r.y = blockIdx.y;
  r.z = blockIdx.z;
  return r;
}

template <int DIM>
__device__ __forceinline__ void tile_ijk(const Tile& tl, int n, int& i, int& j, int& k) {
  i = tl.x * kTileX + threadIdx.x;
  const int ytiles = (n + kTileY - 1) / kTileY;
  int by = tl.y;
  if (DIM == 3) {
    k = by / ytiles;
    by -= k * ytiles;
  } else {
    k = 0;
  }
  j = by * kTileY + threadIdx.y;
}

// 3D launches that march along z (the stencil product, the smoothing sweeps
// and the FP64 residual): a workgroup of march_x(n) x (256 / march_x(n))
// threads owns that
// block of columns over kMarchZ consecutive planes, and each thread carries
// its column's values at planes k-1, k, k+1 in registers from one plane to the
// next, so the points above and below are not loaded again (a
// one-point-per-thread launch reads them from the last-level caches).
constexpr int kMarchZ = 8;
// rows per thread of the marching kernels that write per-block partials (the
// rows above and below a thread's interior rows come from its own registers;
// a workgroup covers march_x(n) x ((256 / march_x(n)) kMarchRows) columns)
// (4 since the workgroups are up to 256 columns wide and so only a few rows
// high: 255^3 mixed went from 35.8 ms with 2 rows to 34.5 ms; 8 rows gained
// another 0.5 % but halves the workgroups of small grids)
constexpr int kMarchRows = 4;

struct Column {
  int i, j, k0, k1;   // the thread's first column (i, j) (rows j .. j + rows - 1) and its planes [k0, k1)
};

__device__ __forceinline__ Column march_column(const Tile& tl, int n, int rows) {
  Column c;
  // the workgroup's shape is chosen per grid (march_x on the host)
  const int my = blockDim.y;
  const int yt = (n + my * rows - 1) / (my * rows);
  const int kc = tl.y / yt;
  c.i = tl.x * blockDim.x + threadIdx.x;
  c.j = ((tl.y - kc * yt) * my + threadIdx.y) * rows;
  c.k0 = kc * kMarchZ;
  c.k1 = min(c.k0 + kMarchZ, n);
  return c;
}

// A thread's R rows in a marching kernel: row r is j0 + r; rows at or beyond n
// are not computed (their loads read row n - 1).  Offsets of the rows and of
// the halo rows j0 - 1 and j0 + R within a plane.
template <int R>
struct Rows {
  long long col[R];   // in-plane offset of row r (clamped)
  bool valid[R];
  bool has_d, has_u;  // rows j0 - 1 and j0 + R inside the grid
  long long col_d, col_u;
  int il, ir;         // x-neighbour offsets (0 at the boundary)
  __device__ __forceinline__ Rows(int i, int j0, int n) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      valid[r] = j0 + r < n;
      col[r] = (long long)min(j0 + r, n - 1) * n + i;
    }
    has_d = j0 > 0;
    has_u = j0 + R < n;
    col_d = (long long)(has_d ? j0 - 1 : j0) * n + i;
    col_u = (long long)(has_u ? j0 + R : n - 1) * n + i;
    il = i > 0 ? -1 : 0;
    ir = i < n - 1 ? 1 : 0;
  }
  // the row-below / row-above neighbours of row r from the rows' centre values
  // and the halo values (0 outside the grid)
  template <typename T>
  __device__ __forceinline__ T down(int r, const T* centre, T halo_d) const {
    return r == 0 ? (has_d ? halo_d : T(0)) : centre[r - 1];
  }
  template <typename T>
  __device__ __forceinline__ T up(int r, const T* centre, T halo_u) const {
    return r == R - 1 ? (has_u ? halo_u : T(0)) : (valid[r + 1] ? centre[r + 1] : T(0));
  }
};

// FP64 block sum; the result is valid in thread 0 only.  Fixed order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[16];   // one value per wave, up to 1024 threads
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0) {
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
    for (int w = 0; w < nw; ++w) r += sh[w];
  }
  return r;
}

// Stencil launches: the block's (x, y) tile index; flat launches: blockIdx.x.
__device__ __forceinline__ void write_partial(double* partial, int sys, double v, int blk, int nblk) {
  const double s = block_sum(v);
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if (tid == 0) partial[(size_t)sys * nblk + blk] = s;
}

__device__ __forceinline__ void write_partial_tile(const Tile& tl, double* partial, int sys, double v) {
  write_partial(partial, sys, v, tl.y * gridDim.x + tl.x, gridDim.x * gridDim.y);
}

__device__ __forceinline__ void write_partial_flat(double* partial, int sys, double v) {
  write_partial(partial, sys, v, blockIdx.x, gridDim.x);
}

__device__ void apply_op(int op, double tot, const SysState& S, int sys, double tol, int max_iter);

// The last block of `sys` (after every block has written its partial) sums
// the partials in the same fixed order as k_scalars and applies fin.op.
__device__ __forceinline__ void finish(const Fin& fin, const double* partial, int sys, int blk_count) {
  if (fin.op < 0) return;
  __shared__ int s_last;
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int nthr = blockDim.x * blockDim.y;
  if (tid == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(fin.cnt + sys, 1u);
    s_last = prev == (unsigned)(blk_count - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double v = 0.0;
  for (int b = tid; b < blk_count; b += nthr) v += partial[(size_t)sys * blk_count + b];
  const double tot = block_sum(v);
  if (tid == 0) {
    atomicExch(fin.cnt + sys, 0u);
    apply_op(fin.op, tot, fin.st, sys, fin.tol, fin.max_iter);
  }
}

// Profiling: the first block of each system adds that system's algorithmic
// bytes for the whole launch (each vector element read or written once) to a
// per-kernel-class counter -- one atomic per system per launch.
// Stencil launches: grid (x tiles, y tiles, system); element-wise launches:
// grid (chunks, system); the coarse solve: one block per system.
enum CountKind { COUNT_TILE, COUNT_FLAT, COUNT_ONE };

template <CountKind K>
__device__ __forceinline__ void count_bytes(unsigned long long* ctr, unsigned long long b) {
  if (ctr == nullptr || threadIdx.x != 0 || threadIdx.y != 0) return;
  const bool first = K == COUNT_ONE ? true : (K == COUNT_FLAT ? blockIdx.x == 0 : (blockIdx.x == 0 && blockIdx.y == 0));
  if (first) atomicAdd(ctr, b);
}

// stencil launches: the workgroup holding tile (0, 0) of the system counts
__device__ __forceinline__ void count_bytes_tile(const Tile& tl, unsigned long long* ctr, unsigned long long b) {
  if (ctr == nullptr || threadIdx.x != 0 || threadIdx.y != 0) return;
  if (tl.x == 0 && tl.y == 0) atomicAdd(ctr, b);
}


// (A_l + s I) x at interior point (i,j,k), flux form sum_f w_f (x_c - x_nb) + s x_c.
// Also returns the diagonal through *dg when dg != nullptr.
template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T apply_pt(const LevelDev<T>& L, const T* __restrict__ x, int i, int j, int k,
                                      long long p, T s, T* dg) {
  const int n = L.n;
  const long long nn = (long long)n * n;
  // neighbour loads are unconditional (a boundary neighbour reads the centre
  // instead) so that they are all in flight together; the value is selected after
  const T xc = x[p];
  const T xl0 = x[i > 0 ? p - 1 : p], xr0 = x[i < n - 1 ? p + 1 : p];
  const T xd0 = x[j > 0 ? p - n : p], xu0 = x[j < n - 1 ? p + n : p];
  T xb0 = T(0), xf0 = T(0);
  if (DIM == 3) {
    xb0 = x[k > 0 ? p - nn : p];
    xf0 = x[k < n - 1 ? p + nn : p];
  }
  const T xl = i > 0 ? xl0 : T(0), xr = i < n - 1 ? xr0 : T(0);
  const T xd = j > 0 ? xd0 : T(0), xu = j < n - 1 ? xu0 : T(0);
  const T xb = DIM == 3 && k > 0 ? xb0 : T(0), xf = DIM == 3 && k < n - 1 ? xf0 : T(0);
  if (!VAR) {
    const T w = L.wc;
    T sum = (xc - xl) + (xc - xr) + (xc - xd) + (xc - xu);
    if (DIM == 3) sum += (xc - xb) + (xc - xf);
    if (dg) *dg = w * T(2 * DIM) + s;
    return w * sum + s * xc;
  } else {
    const long long fx = ((long long)k * n + j) * (n + 1) + i;
    const T wl = L.wf0[fx], wr = L.wf0[fx + 1];
    const long long fy = ((long long)k * (n + 1) + j) * n + i;
    const T wd = L.wf1[fy], wu = L.wf1[fy + n];
    T acc = wl * (xc - xl) + wr * (xc - xr) + wd * (xc - xd) + wu * (xc - xu);
    T d = wl + wr + wd + wu;
    if (DIM == 3) {
      const long long fz = ((long long)k * n + j) * n + i;
      const T wb = L.wf2[fz], wf = L.wf2[fz + nn];
      acc += wb * (xc - xb) + wf * (xc - xf);
      d += wb + wf;
    }
    if (dg) *dg = d + s;
    return acc + s * xc;
  }
}

template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T diag_pt(const LevelDev<T>& L, int i, int j, int k, T s) {
  if (!VAR) return L.wc * T(2 * DIM) + s;
  const int n = L.n;
  const long long fx = ((long long)k * n + j) * (n + 1) + i;
  const long long fy = ((long long)k * (n + 1) + j) * n + i;
  T d = L.wf0[fx] + L.wf0[fx + 1] + L.wf1[fy] + L.wf1[fy + n];
  if (DIM == 3) {
    const long long fz = ((long long)k * n + j) * n + i;
    d += L.wf2[fz] + L.wf2[fz + (long long)n * n];
  }
  return d + s;
}

// apply_pt for DIM = 3 from values already loaded: the centre, its in-plane
// neighbours l, r, d, u and the points below (b) and above (f), each 0 outside
// the grid.  Same arithmetic and order as apply_pt.
template <typename T, bool VAR>
__device__ __forceinline__ T apply_col3(const LevelDev<T>& L, int i, int j, int k, long long p, T xc, T xl, T xr,
                                        T xd, T xu, T xb, T xf, T s, T* dg) {
  if (!VAR) {
    T sum = (xc - xl) + (xc - xr) + (xc - xd) + (xc - xu);
    sum += (xc - xb) + (xc - xf);
    if (dg) *dg = L.wc * T(6) + s;
    return L.wc * sum + s * xc;
  }
  const int n = L.n;
  const long long fx = ((long long)k * n + j) * (n + 1) + i;
  const long long fy = ((long long)k * (n + 1) + j) * n + i;
  const T wl = L.wf0[fx], wr = L.wf0[fx + 1], wd = L.wf1[fy], wu = L.wf1[fy + n];
  const T wb = L.wf2[p], wf = L.wf2[p + (long long)n * n];
  T acc = wl * (xc - xl) + wr * (xc - xr) + wd * (xc - xd) + wu * (xc - xu);
  T d = wl + wr + wd + wu;
  acc += wb * (xc - xb) + wf * (xc - xf);
  d += wb + wf;
  if (dg) *dg = d + s;
  return acc + s * xc;
}

// In-plane neighbour offsets of a column (0 where the neighbour is outside the
// grid: the load then reads the centre and the value is replaced by 0).
struct PlaneNb {
  int l, r, d, u;
};

__device__ __forceinline__ PlaneNb plane_nb(int i, int j, int n) {
  PlaneNb o;
  o.l = i > 0 ? -1 : 0;
  o.r = i < n - 1 ? 1 : 0;
  o.d = j > 0 ? -n : 0;
  o.u = j < n - 1 ? n : 0;
  return o;
}

// --------------------------------------------------------------------------
// smoother: x_out = x_in + omega D^-1 (b - (A+s) x_in)   (x_in = 0 if ZERO)
// DOT: partial = b . x_out  (r.z when this is the last sweep of z = M r)
// --------------------------------------------------------------------------
template <typename T, int DIM, bool VAR, bool ZERO, bool DOT>
__global__ __launch_bounds__(kBlock) void k_jacobi(LevelDev<T> L, const T* __restrict__ b,
                                                   const T* __restrict__ xin, T* __restrict__ xout,
                                                   const T* __restrict__ shift, const int* __restrict__ active,
                                                   T omega, double* __restrict__ partial,
                                                   unsigned long long* __restrict__ ctr, Fin fin) {
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  int i, j, k;
  tile_ijk<DIM>(tl, L.n, i, j, k);
  const bool ok = i < L.n && j < L.n;
  const long long off = (long long)sys * L.N;
  const long long p = ((long long)k * L.n + j) * L.n + i;
  const T s = shift[sys];
  // b and x_out, plus x_in unless the guess is zero; faces once per launch
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * sizeof(T) * ((ZERO ? 2 : 3) + (VAR && sys == 0 ? DIM : 0)));
  double dot = 0.0;
  if (ok) {
    const T bv = b[off + p];
    T xn;
    if (ZERO) {
      xn = omega * bv / diag_pt<T, DIM, VAR>(L, i, j, k, s);
    } else {
      T dg;
      const T ax = apply_pt<T, DIM, VAR>(L, xin + off, i, j, k, p, s, &dg);
      xn = xin[off + p] + omega * (bv - ax) / dg;
    }
    xout[off + p] = xn;
    if (DOT) dot = (double)bv * (double)xn;
  }
  if (DOT) {
    write_partial_tile(tl, partial, sys, dot);
    finish(fin, partial, sys, gridDim.x * gridDim.y);
  }
}

// k_jacobi in 3D, marching along z (one workgroup per kMarchZ planes,
// kMarchRows rows per thread).
template <typename T, bool VAR, bool ZERO, bool DOT>
__global__ __launch_bounds__(kBlock) void k_jacobi3(LevelDev<T> L, const T* __restrict__ b,
                                                    const T* __restrict__ xin, T* __restrict__ xout,
                                                    const T* __restrict__ shift, const int* __restrict__ active,
                                                    T omega, double* __restrict__ partial,
                                                    unsigned long long* __restrict__ ctr, Fin fin) {
  constexpr int R = kMarchRows;
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * sizeof(T) * ((ZERO ? 2 : 3) + (VAR && sys == 0 ? 3 : 0)));
  const int n = L.n;
  const Column c = march_column(tl, n, R);
  double dot = 0.0;
  if (c.i < n && c.j < n) {
    const long long off = (long long)sys * L.N, nn = (long long)n * n;
    const Rows<R> w(c.i, c.j, n);
    const T s = shift[sys];
    const T* bs = b + off;
    T* xo = xout + off;
    if (ZERO) {
      for (int k = c.k0; k < c.k1; ++k) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!w.valid[r]) continue;
          const long long p = k * nn + w.col[r];
          const T bv = bs[p];
          const T xn = omega * bv / diag_pt<T, 3, VAR>(L, c.i, c.j + r, k, s);
          xo[p] = xn;
          if (DOT) dot += (double)bv * (double)xn;
        }
      }
    } else {
      const T* xs = xin + off;
      T below[R], centre[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long long p0 = c.k0 * nn + w.col[r];
        const T xb0 = xs[c.k0 > 0 ? p0 - nn : p0];
        below[r] = c.k0 > 0 ? xb0 : T(0);
        centre[r] = xs[p0];
      }
      for (int k = c.k0; k < c.k1; ++k) {
        const long long pk = k * nn;
        // every load of the plane first, then the arithmetic (loading the next
        // plane one step ahead measured slower)
        T xa[R], xl[R], xr[R], bv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const long long p = pk + w.col[r];
          xa[r] = xs[k + 1 < n ? p + nn : p];
          xl[r] = xs[p + w.il];
          xr[r] = xs[p + w.ir];
          bv[r] = bs[p];
        }
        const T hd = xs[pk + w.col_d], hu = xs[pk + w.col_u];
        T above[R];
#pragma unroll
        for (int r = 0; r < R; ++r) above[r] = k + 1 < n ? xa[r] : T(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!w.valid[r]) continue;
          const long long p = pk + w.col[r];
          T dg;
          const T ax = apply_col3<T, VAR>(L, c.i, c.j + r, k, p, centre[r], w.il ? xl[r] : T(0),
                                          w.ir ? xr[r] : T(0), w.down(r, centre, hd), w.up(r, centre, hu),
                                          below[r], above[r], s, &dg);
          const T xn = centre[r] + omega * (bv[r] - ax) / dg;
          xo[p] = xn;
          if (DOT) dot += (double)bv[r] * (double)xn;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          below[r] = centre[r];
          centre[r] = above[r];
        }
      }
    }
  }
  if (DOT) {
    write_partial_tile(tl, partial, sys, dot);
    finish(fin, partial, sys, gridDim.x * gridDim.y);
  }
}

// The first pre-smoothing sweep of the fine level (from x = 0) with the PCG
// residual update folded in: b = b_old - alpha q is written to bout with its
// squared norm into partial, and x_out = omega D^-1 b.  The sweep reads no
// neighbour of b, so the update needs no second pass.
template <typename T, int DIM, bool VAR>
__global__ __launch_bounds__(kBlock) void k_jacobi0_rup(LevelDev<T> L, const T* __restrict__ bold,
                                                        const T* __restrict__ q, const double* __restrict__ alpha,
                                                        T* __restrict__ bout, T* __restrict__ xout,
                                                        const T* __restrict__ shift, const int* __restrict__ active,
                                                        T omega, double* __restrict__ partial,
                                                        unsigned long long* __restrict__ ctr, Fin fin) {
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  const int n = L.n;
  // 2D: one point; 3D: kMarchRows rows over kMarchZ planes
  constexpr int R = DIM == 3 ? kMarchRows : 1;
  int i, j, k0, k1;
  if (DIM == 3) {
    const Column c = march_column(tl, n, R);
    i = c.i;
    j = c.j;
    k0 = c.k0;
    k1 = c.k1;
  } else {
    tile_ijk<DIM>(tl, n, i, j, k0);
    k1 = k0 + 1;
  }
  const long long off = (long long)sys * L.N;
  const T s = shift[sys];
  const T a = (T)alpha[sys];
  // b_old and q read, b and x_out written; faces once per launch
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * sizeof(T) * (4 + (VAR && sys == 0 ? DIM : 0)));
  double rr = 0.0;
  if (i < n) {
    for (int k = k0; k < k1; ++k) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (j + r >= n) continue;
        const long long p = ((long long)k * n + j + r) * n + i;
        const T bv = bold[off + p] - a * q[off + p];
        bout[off + p] = bv;
        xout[off + p] = omega * bv / diag_pt<T, DIM, VAR>(L, i, j + r, k, s);
        rr += (double)bv * (double)bv;
      }
    }
  }
  write_partial_tile(tl, partial, sys, rr);
  finish(fin, partial, sys, gridDim.x * gridDim.y);
}

// 3D first fine sweep with the PCG residual update, forming q = (A + s) p
// itself from p while marching along z (as k_jacobi3 forms (A + s) x):
// b = b_old - alpha q to bout with |b|^2 into partial, x_out = omega D^-1 b.
// The stencil product then stores no q (one vector pass less per iteration).
template <typename T, bool VAR>
__global__ __launch_bounds__(kBlock) void k_jacobi0_rup3p(LevelDev<T> L, const T* __restrict__ bold,
                                                          const T* __restrict__ pv, const double* __restrict__ alpha,
                                                          T* __restrict__ bout, T* __restrict__ xout,
                                                          const T* __restrict__ shift, const int* __restrict__ active,
                                                          T omega, double* __restrict__ partial,
                                                          unsigned long long* __restrict__ ctr, Fin fin) {
  constexpr int R = kMarchRows;
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  // b_old and p read, b and x_out written; faces once per launch
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * sizeof(T) * (4 + (VAR && sys == 0 ? 3 : 0)));
  const int n = L.n;
  const Column c = march_column(tl, n, R);
  double rr = 0.0;
  if (c.i < n && c.j < n) {
    const long long off = (long long)sys * L.N, nn = (long long)n * n;
    const Rows<R> w(c.i, c.j, n);
    const T s = shift[sys];
    const T a = (T)alpha[sys];
    const T* ps = pv + off;
    const T* bs = bold + off;
    T below[R], centre[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long p0 = c.k0 * nn + w.col[r];
      const T pb0 = ps[c.k0 > 0 ? p0 - nn : p0];
      below[r] = c.k0 > 0 ? pb0 : T(0);
      centre[r] = ps[p0];
    }
    for (int k = c.k0; k < c.k1; ++k) {
      const long long pk = k * nn;
      T pa[R], pl[R], pr[R], bv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long long p = pk + w.col[r];
        pa[r] = ps[k + 1 < n ? p + nn : p];
        pl[r] = ps[p + w.il];
        pr[r] = ps[p + w.ir];
        bv[r] = bs[p];
      }
      const T hd = ps[pk + w.col_d], hu = ps[pk + w.col_u];
      T above[R];
#pragma unroll
      for (int r = 0; r < R; ++r) above[r] = k + 1 < n ? pa[r] : T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!w.valid[r]) continue;
        const long long p = pk + w.col[r];
        T dg;
        const T ap = apply_col3<T, VAR>(L, c.i, c.j + r, k, p, centre[r], w.il ? pl[r] : T(0), w.ir ? pr[r] : T(0),
                                        w.down(r, centre, hd), w.up(r, centre, hu), below[r], above[r], s, &dg);
        const T bn = bv[r] - a * ap;
        bout[off + p] = bn;
        xout[off + p] = omega * bn / dg;
        rr += (double)bn * (double)bn;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        below[r] = centre[r];
        centre[r] = above[r];
      }
    }
  }
  write_partial_tile(tl, partial, sys, rr);
  finish(fin, partial, sys, gridDim.x * gridDim.y);
}

// --------------------------------------------------------------------------
// b_c = R (b - (A+s) x): full weighting of the fine residual (weights
// (1/4, 1/2, 1/4) per axis), fine node 2I+1 under coarse node I (0-based).
// --------------------------------------------------------------------------
template <typename T, int DIM, bool VAR>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelDev<T> Lf, LevelDev<T> Lc, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ bc,
                                                     const T* __restrict__ shift, const int* __restrict__ active,
                                                     unsigned long long* __restrict__ ctr) {
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  // per coarse point: b and x on its 2^dim fine points, b_c written
  count_bytes_tile(tl, ctr, (unsigned long long)Lc.N * sizeof(T) * (2 * (1 << DIM) + 1 + (VAR && sys == 0 ? DIM * (1 << DIM) : 0)));
  int I, J, K;
  tile_ijk<DIM>(tl, Lc.n, I, J, K);
  if (I >= Lc.n || J >= Lc.n) return;
  const int nf = Lf.n;
  const T s = shift[sys];
  const T* bs = b + (long long)sys * Lf.N;
  const T* xs = x + (long long)sys * Lf.N;
  const T wt[3] = {T(0.25), T(0.5), T(0.25)};
  T acc = T(0);
  const int kmin = DIM == 3 ? -1 : 0, kmax = DIM == 3 ? 1 : 0;
  for (int dk = kmin; dk <= kmax; ++dk) {
    const int fk = DIM == 3 ? 2 * K + 1 + dk : 0;
    const T wk = DIM == 3 ? wt[dk + 1] : T(1);
    for (int dj = -1; dj <= 1; ++dj) {
      const int fj = 2 * J + 1 + dj;
      for (int di = -1; di <= 1; ++di) {
        const int fi = 2 * I + 1 + di;
        const long long p = ((long long)fk * nf + fj) * nf + fi;
        const T r = bs[p] - apply_pt<T, DIM, VAR>(Lf, xs, fi, fj, fk, p, s, nullptr);
        acc += wk * wt[dj + 1] * wt[di + 1] * r;
      }
    }
  }
  bc[(long long)sys * Lc.N + ((long long)K * Lc.n + J) * Lc.n + I] = acc;
}

// --------------------------------------------------------------------------
// x_f += P x_c  (multilinear interpolation, P = 2^dim R^T)
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int axis_parents(int f, int nc, int* ci, T* w) {
  if (f & 1) {
    ci[0] = (f - 1) >> 1;
    w[0] = T(1);
    return 1;
  }
  int cnt = 0;
  const int c0 = (f >> 1) - 1, c1 = f >> 1;
  if (c0 >= 0) { ci[cnt] = c0; w[cnt] = T(0.5); ++cnt; }
  if (c1 < nc) { ci[cnt] = c1; w[cnt] = T(0.5); ++cnt; }
  return cnt;
}

template <typename T, int DIM>
__device__ __forceinline__ T interp_pt(const T* __restrict__ xc, int nc, int fi, int fj, int fk) {
  int ci[2], cj[2], ck[2];
  T wi[2], wj[2], wk[2];
  const int ni = axis_parents<T>(fi, nc, ci, wi);
  const int nj = axis_parents<T>(fj, nc, cj, wj);
  int nk = 1;
  ck[0] = 0;
  wk[0] = T(1);
  if (DIM == 3) nk = axis_parents<T>(fk, nc, ck, wk);
  T v = T(0);
  for (int c = 0; c < nk; ++c)
    for (int b = 0; b < nj; ++b)
      for (int a = 0; a < ni; ++a)
        v += wk[c] * wj[b] * wi[a] * xc[((long long)ck[c] * nc + cj[b]) * nc + ci[a]];
  return v;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong(LevelDev<T> Lc, LevelDev<T> Lf, const T* __restrict__ xc,
                                                    T* __restrict__ xf, const int* __restrict__ active,
                                                    unsigned long long* __restrict__ ctr) {
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  // x_f read and written; x_c read once (1/2^dim per fine point)
  count_bytes_tile(tl, ctr, (unsigned long long)Lf.N * sizeof(T) * 2 + (unsigned long long)Lc.N * sizeof(T));
  int i, j, k;
  tile_ijk<DIM>(tl, Lf.n, i, j, k);
  if (i >= Lf.n || j >= Lf.n) return;
  const long long p = ((long long)k * Lf.n + j) * Lf.n + i;
  xf[(long long)sys * Lf.N + p] += interp_pt<T, DIM>(xc + (long long)sys * Lc.N, Lc.n, i, j, k);
}

// --------------------------------------------------------------------------
// 3D transfer operators marching along z (grids of 2^L - 1 points: n_f = 2 n_c + 1)
// --------------------------------------------------------------------------
// The two coarse parents of fine index f on one axis and their weights: odd f
// lies on coarse point (f - 1) / 2 (weight 1, second weight 0); even f halfway
// between f/2 - 1 and f/2 (weight 1/2 each, 0 for a parent outside the grid,
// whose index is clamped).
template <typename T>
__device__ __forceinline__ void axis_pair(int f, int nc, int& a, int& b, T& wa, T& wb) {
  if (f & 1) {
    a = b = f >> 1;
    wa = T(1);
    wb = T(0);
  } else {
    a = (f >> 1) - 1;
    b = f >> 1;
    wa = a >= 0 ? T(0.5) : T(0);
    wb = b < nc ? T(0.5) : T(0);
    a = max(a, 0);
    b = min(b, nc - 1);
  }
}

// x_f += P x_c: one thread per fine column (i, j) over kMarchZ fine planes.  The
// in-plane interpolant of each coarse plane is formed once and kept for the
// two or three fine planes that use it.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong3(LevelDev<T> Lc, LevelDev<T> Lf, const T* __restrict__ xc,
                                                     T* __restrict__ xf, const int* __restrict__ active,
                                                     unsigned long long* __restrict__ ctr) {
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)Lf.N * sizeof(T) * 2 + (unsigned long long)Lc.N * sizeof(T));
  const int nf = Lf.n, nc = Lc.n;
  const Column c = march_column(tl, nf, 1);
  if (c.i >= nf || c.j >= nf) return;
  int ia, ib, ja, jb;
  T wia, wib, wja, wjb;
  axis_pair<T>(c.i, nc, ia, ib, wia, wib);
  axis_pair<T>(c.j, nc, ja, jb, wja, wjb);
  const T* xcs = xc + (long long)sys * Lc.N;
  const long long ncc = (long long)nc * nc;
  const long long oaa = (long long)ja * nc + ia, oab = (long long)ja * nc + ib;
  const long long oba = (long long)jb * nc + ia, obb = (long long)jb * nc + ib;
  // the in-plane interpolant on coarse plane K (0 off the grid)
  auto plane = [&](int K) -> T {
    const long long base = (long long)min(max(K, 0), nc - 1) * ncc;
    const T v00 = xcs[base + oaa], v01 = xcs[base + oab], v10 = xcs[base + oba], v11 = xcs[base + obb];
    const T v = wja * (wia * v00 + wib * v01) + wjb * (wia * v10 + wib * v11);
    return (K >= 0 && K < nc) ? v : T(0);
  };
  // fine plane k: odd k lies on coarse plane (k - 1) / 2, even k halfway between
  // k/2 - 1 and k/2; (vlo, vhi) hold coarse planes Kc and Kc + 1
  int Kc = (c.k0 >> 1) - 1;
  T vlo = plane(Kc), vhi = plane(Kc + 1);
  T* xfs = xf + (long long)sys * Lf.N;
  const long long nnf = (long long)nf * nf, col = (long long)c.j * nf + c.i;
  for (int k = c.k0; k < c.k1; ++k) {
    const int klo = (k >> 1) - 1 + (k & 1);
    if (Kc < klo) {
      vlo = vhi;
      ++Kc;
      vhi = plane(Kc + 1);
    }
    const T v = (k & 1) ? vlo : T(0.5) * (vlo + vhi);
    const long long p = k * nnf + col;
    xfs[p] += v;
  }
}

// b_c = R (b - (A+s) x) in 3D.  A workgroup owns kRcx x kRcy coarse columns over
// kMarchZ coarse planes, i.e. the (2 kRcx + 1) x (2 kRcy + 1) fine columns under
// them.  Plane by plane, each fine point's residual is formed once and put in
// LDS; each coarse column then takes the weighted 3 x 3 sum of its plane, and
// the weighted sums of fine planes 2K, 2K+1, 2K+2 give coarse plane K (plane
// 2K+2 is shared with coarse plane K+1).  Every thread keeps x of its fine
// points at the plane below and at the current one in registers; the current
// plane also goes to an LDS tile with a one-point ring (loaded by the first
// threads), from which the in-plane neighbours are read, so a point costs two
// loads per plane (x above, b) instead of six, and the kernel holds far fewer
// registers (FP32: 98 VGPRs instead of 146, 4 waves per SIMD instead of 3).
constexpr int kRcx = 32, kRcy = 8;
constexpr int kRfx = 2 * kRcx + 1, kRfy = 2 * kRcy + 1, kRfn = kRfx * kRfy;
constexpr int kRhx = kRfx + 2, kRhy = kRfy + 2, kRhn = kRhx * kRhy;   // with the ring
constexpr int kRring = 2 * kRhx + 2 * (kRhy - 2);

static_assert(kRcx * kRcy == 256, "one coarse column per thread");
static_assert(kRring <= 256, "one ring point per thread at most");

template <typename T, bool VAR>
__global__ __launch_bounds__(256) void k_restrict3(LevelDev<T> Lf, LevelDev<T> Lc, const T* __restrict__ b,
                                                   const T* __restrict__ x, T* __restrict__ bc,
                                                   const T* __restrict__ shift, const int* __restrict__ active,
                                                   unsigned long long* __restrict__ ctr) {
  constexpr int PER = (kRfn + 255) / 256;
  __shared__ T rb[kRfn];
  __shared__ T xt[kRhn];
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)Lc.N * sizeof(T) * (2 * 8 + 1 + (VAR && sys == 0 ? 3 * 8 : 0)));
  const int nf = Lf.n, nc = Lc.n;
  const int yt = (nc + kRcy - 1) / kRcy;
  const int kc = tl.y / yt;
  const int I0 = tl.x * kRcx, J0 = (tl.y - kc * yt) * kRcy;
  const int K0 = kc * kMarchZ, K1 = min(K0 + kMarchZ, nc);
  const int tid = threadIdx.x;
  const T s = shift[sys];
  const T* bs = b + (long long)sys * Lf.N;
  const T* xs = x + (long long)sys * Lf.N;
  const long long nnf = (long long)nf * nf;
  int fk = 2 * K0;
  T xm[PER], xc0[PER];   // x at the fine plane below and at the current one, per owned fine point
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + 256 * u;
    const int fy = q / kRfx, fx = q - fy * kRfx;
    const int fi = 2 * I0 + fx, fj = 2 * J0 + fy;
    xm[u] = T(0);
    xc0[u] = T(0);
    if (q < kRfn && fi < nf && fj < nf) {
      const long long p = fk * nnf + (long long)fj * nf + fi;
      const T xb = xs[fk > 0 ? p - nnf : p];
      xm[u] = fk > 0 ? xb : T(0);
      xc0[u] = xs[p];
    }
  }
  // this thread's ring point (tid < kRring): its place in the tile and its
  // in-plane offset (-1 when outside the grid: it holds 0)
  int ring_h = -1;
  long long ring_off = -1;
  if (tid < kRring) {
    int hx, hy;
    if (tid < kRhx) {
      hx = tid;
      hy = 0;
    } else if (tid < 2 * kRhx) {
      hx = tid - kRhx;
      hy = kRhy - 1;
    } else {
      const int t2 = tid - 2 * kRhx;
      hx = (t2 & 1) ? kRhx - 1 : 0;
      hy = 1 + (t2 >> 1);
    }
    ring_h = hy * kRhx + hx;
    const int fi = 2 * I0 - 1 + hx, fj = 2 * J0 - 1 + hy;
    if (fi >= 0 && fi < nf && fj >= 0 && fj < nf) ring_off = (long long)fj * nf + fi;
  }
  const int ci = tid % kRcx, cj = tid / kRcx;
  // the residual on fine plane fk (into LDS), then this coarse column's
  // weighted in-plane sum of it; advances fk and the registers
  auto rplane = [&]() -> T {
    // x of plane fk into the tile (0 off the grid), x above and b loaded
    T xa[PER], bv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = tid + 256 * u;
      const int fy = q / kRfx, fx = q - fy * kRfx;
      const int fi = 2 * I0 + fx, fj = 2 * J0 + fy;
      const bool in = q < kRfn && fi < nf && fj < nf;
      const long long p = fk * nnf + (in ? (long long)fj * nf + fi : 0LL);
      xa[u] = xs[fk + 1 < nf ? p + nnf : p];
      bv[u] = bs[p];
      if (q < kRfn) xt[(fy + 1) * kRhx + fx + 1] = xc0[u];
    }
    if (ring_h >= 0) xt[ring_h] = ring_off >= 0 ? xs[fk * nnf + ring_off] : T(0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = tid + 256 * u;
      const int fy = q / kRfx, fx = q - fy * kRfx;
      const int fi = 2 * I0 + fx, fj = 2 * J0 + fy;
      if (q < kRfn) {
        T r = T(0);
        if (fi < nf && fj < nf) {
          const long long p = fk * nnf + (long long)fj * nf + fi;
          const int h = (fy + 1) * kRhx + fx + 1;
          const T above = fk + 1 < nf ? xa[u] : T(0);
          r = bv[u] - apply_col3<T, VAR>(Lf, fi, fj, fk, p, xc0[u], xt[h - 1], xt[h + 1], xt[h - kRhx], xt[h + kRhx],
                                         xm[u], above, s, nullptr);
          xm[u] = xc0[u];
          xc0[u] = above;
        }
        rb[q] = r;
      }
    }
    __syncthreads();
    const T wt[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int di = q % 3, dj = q / 3;
      acc += wt[dj] * wt[di] * rb[(2 * cj + dj) * kRfx + 2 * ci + di];
    }
    // (the next plane writes rb only after its first barrier, which every
    // thread reaches after this sum)
    ++fk;
    return acc;
  };
  const bool mine = I0 + ci < nc && J0 + cj < nc;
  T* bcs = bc + (long long)sys * Lc.N + ((long long)(J0 + cj) * nc + (I0 + ci));
  const long long ncc = (long long)nc * nc;
  T rlo = rplane();   // fine plane 2 K0
  for (int K = K0; K < K1; ++K) {
    const T rmid = rplane();   // 2K + 1
    const T rhi = rplane();    // 2K + 2
    if (mine) bcs[K * ncc] = T(0.25) * rlo + T(0.5) * rmid + T(0.25) * rhi;
    rlo = rhi;
  }
}

// --------------------------------------------------------------------------
// coarse solve: `cycles` V-cycles on the levels in H, one workgroup per system,
// all vectors in LDS.  Symmetric (nu Jacobi sweeps before and after), so the
// composite is an SPD preconditioner component.
// --------------------------------------------------------------------------
// weight i of a half-cycle (selected without indexing the array, which would
// put the by-value argument in scratch memory)
template <typename T>
__device__ __forceinline__ T sweep_w(const Sweeps<T>& sw, int i) {
  return i == 0 ? sw.w[0] : (i == 1 ? sw.w[1] : sw.w[2]);
}

// (i, j, k) of point p of an n^DIM grid held in LDS: the quotients by n
// through a float reciprocal instead of an integer division.  Exact: p +
// 0.5 lies at least 0.5/n from every multiple of n, and for the LDS levels
// (p < 2^15) the float rounding error of (p + 0.5) * (1/n) stays below 1e-5.
template <int DIM>
__device__ __forceinline__ void ijk_of(int p, int n, float rn, int& i, int& j, int& k) {
  const int q = (int)(((float)p + 0.5f) * rn);
  i = p - q * n;
  if (DIM == 3) {
    k = (int)(((float)q + 0.5f) * rn);
    j = q - k * n;
  } else {
    j = q;
    k = 0;
  }
}

// omega for every sweep, or (per != nullptr) the half-cycle weights, reversed
// for post-smoothing
template <typename T, int DIM, bool VAR>
__device__ void lds_smooth(const LevelDev<T>& L, T* X, const T* B, T* Tm, T s, T omega, int sweeps,
                           const Sweeps<T>* per = nullptr, bool reverse = false) {
  const int n = L.n;
  const float rn = 1.0f / (float)n;
  const int nthr = blockDim.x;
  for (int sw = 0; sw < sweeps; ++sw) {
    const T om = per ? sweep_w(*per, reverse ? sweeps - 1 - sw : sw) : omega;
    for (int p = threadIdx.x; p < L.N; p += nthr) {
      int i, j, k;
      ijk_of<DIM>(p, n, rn, i, j, k);
      T dg;
      const T ax = apply_pt<T, DIM, VAR>(L, X, i, j, k, p, s, &dg);
      Tm[p] = X[p] + om * (B[p] - ax) / dg;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < L.N; p += nthr) X[p] = Tm[p];
    __syncthreads();
  }
}

template <typename T, int DIM, bool VAR>
__global__ __launch_bounds__(1024) void k_coarse(LdsHierarchy<T> H, const T* __restrict__ b, T* __restrict__ x,
                                                const T* __restrict__ shift, const int* __restrict__ active,
                                                unsigned long long* __restrict__ ctr) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int sys = blockIdx.x;
  if (!active[sys]) return;
  count_bytes<COUNT_ONE>(ctr, 2ULL * H.lev[0].N * sizeof(T));
  const T s = shift[sys];
  const int nthr = blockDim.x;
  const LevelDev<T>& L0 = H.lev[0];
  T* X0 = sm + H.off[0];
  T* B0 = X0 + L0.N;
  for (int p = threadIdx.x; p < L0.N; p += nthr) {
    B0[p] = b[(long long)sys * L0.N + p];
    X0[p] = T(0);
  }
  __syncthreads();
  for (int cyc = 0; cyc < H.cycles; ++cyc) {
    for (int l = 0; l + 1 < H.nlev; ++l) {
      const LevelDev<T>& Lf = H.lev[l];
      const LevelDev<T>& Lc = H.lev[l + 1];
      T* X = sm + H.off[l];
      T* B = X + Lf.N;
      T* Tm = B + Lf.N;
      lds_smooth<T, DIM, VAR>(Lf, X, B, Tm, s, H.omega, H.nu, &H.pre, false);
      // residual on the fine level into Tm, then full weighting into B_c
      const float rf = 1.0f / (float)Lf.n, rc = 1.0f / (float)Lc.n;
      for (int p = threadIdx.x; p < Lf.N; p += nthr) {
        int i, j, k;
        ijk_of<DIM>(p, Lf.n, rf, i, j, k);
        Tm[p] = B[p] - apply_pt<T, DIM, VAR>(Lf, X, i, j, k, p, s, nullptr);
      }
      __syncthreads();
      T* Xc = sm + H.off[l + 1];
      T* Bc = Xc + Lc.N;
      const T wt[3] = {T(0.25), T(0.5), T(0.25)};
      for (int p = threadIdx.x; p < Lc.N; p += nthr) {
        int I, J, K;
        ijk_of<DIM>(p, Lc.n, rc, I, J, K);
        T acc = T(0);
        for (int dk = (DIM == 3 ? -1 : 0); dk <= (DIM == 3 ? 1 : 0); ++dk) {
          const int fk = DIM == 3 ? 2 * K + 1 + dk : 0;
          const T wk = DIM == 3 ? wt[dk + 1] : T(1);
          for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di)
              acc += wk * wt[dj + 1] * wt[di + 1] * Tm[((long long)fk * Lf.n + 2 * J + 1 + dj) * Lf.n + 2 * I + 1 + di];
        }
        Bc[p] = acc;
        Xc[p] = T(0);
      }
      __syncthreads();
    }
    {  // bottom level
      const int l = H.nlev - 1;
      const LevelDev<T>& Lb = H.lev[l];
      T* X = sm + H.off[l];
      T* B = X + Lb.N;
      T* Tm = B + Lb.N;
      if (Lb.N == 1) {
        if (threadIdx.x == 0) X[0] = B[0] / diag_pt<T, DIM, VAR>(Lb, 0, 0, 0, s);
        __syncthreads();
      } else {
        lds_smooth<T, DIM, VAR>(Lb, X, B, Tm, s, H.omega, H.bottom_sweeps);
      }
    }
    for (int l = H.nlev - 2; l >= 0; --l) {
      const LevelDev<T>& Lf = H.lev[l];
      const LevelDev<T>& Lc = H.lev[l + 1];
      T* X = sm + H.off[l];
      T* B = X + Lf.N;
      T* Tm = B + Lf.N;
      const T* Xc = sm + H.off[l + 1];
      const float rf = 1.0f / (float)Lf.n;
      for (int p = threadIdx.x; p < Lf.N; p += nthr) {
        int i, j, k;
        ijk_of<DIM>(p, Lf.n, rf, i, j, k);
        X[p] += interp_pt<T, DIM>(Xc, Lc.n, i, j, k);
      }
      __syncthreads();
      lds_smooth<T, DIM, VAR>(Lf, X, B, Tm, s, H.omega, H.nu, &H.pre, true);
    }
  }
  for (int p = threadIdx.x; p < L0.N; p += nthr) x[(long long)sys * L0.N + p] = X0[p];
}

// --------------------------------------------------------------------------
// Fused multigrid level kernels with LDS-staged halo tiles (2D).
//
// k_down: from b on level l, nu Jacobi sweeps starting at x = 0, the residual
// r = b - (A+s) x and its full weighting onto level l+1 -- one pass over b,
// writing x (owned points) and b_c.  A block owns a CX x CY tile of coarse
// points, i.e. fine points [2 I0, 2 I0 + 2 CX) per axis (the last tile also
// the final fine point), and stages b on that range widened by nu on each
// side plus one on the right; sweep m is valid on the range shrunk by m-1,
// the residual on the range shrunk by nu = exactly the points the weighting
// needs.  Points outside the grid hold 0 (Dirichlet) and are never updated.
//
// k_up: x = x_in + P x_c on an OX x OY tile widened by nu, nu Jacobi sweeps
// (valid region shrinking by one per sweep), x written on the tile, and the
// block partial of b.x when this is the finest level (r.z for the PCG).
// --------------------------------------------------------------------------
template <typename T, bool VAR>
__device__ __forceinline__ T lds_apply2(const T* __restrict__ X, int q, int RX, const LevelDev<T>& L, int gi, int gj,
                                        T s, T* dg) {
  const T xc = X[q];
  const T xl = X[q - 1], xr = X[q + 1], xd = X[q - RX], xu = X[q + RX];
  if (!VAR) {
    const T w = L.wc;
    if (dg) *dg = w * T(4) + s;
    return w * ((xc - xl) + (xc - xr) + (xc - xd) + (xc - xu)) + s * xc;
  }
  const int n = L.n;
  const long long fx = (long long)gj * (n + 1) + gi;
  const long long fy = (long long)gj * n + gi;
  const T wl = L.wf0[fx], wr = L.wf0[fx + 1], wd = L.wf1[fy], wu = L.wf1[fy + n];
  if (dg) *dg = wl + wr + wd + wu + s;
  return wl * (xc - xl) + wr * (xc - xr) + wd * (xc - xd) + wu * (xc - xu) + s * xc;
}

// Face weights of the LDS region points a thread owns in the fused 2D kernels
// (points tid + 256 u, u < PER), held in registers.  Constant coefficients:
// empty.  Points off the grid hold the weights of the nearest grid point
// (clamped; never used in a sweep).
template <typename T, bool VAR, int PER>
struct RegionFaces {
  T wl[VAR ? PER : 1], wr[VAR ? PER : 1], wd[VAR ? PER : 1], wu[VAR ? PER : 1];
  __device__ __forceinline__ void load(const LevelDev<T>& L, int tid, int RX, int RN, int gx0, int gy0) {
    if (!VAR) return;
    const int n = L.n;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = min(tid + 256 * u, RN - 1);
      const int ry = q / RX, rx = q - ry * RX;
      const int ci = min(max(gx0 + rx, 0), n - 1), cj = min(max(gy0 + ry, 0), n - 1);
      const int fx = cj * (n + 1) + ci;   // 2D faces: fewer than 2^31
      const int fy = cj * n + ci;
      wl[u] = L.wf0[fx];
      wr[u] = L.wf0[fx + 1];
      wd[u] = L.wf1[fy];
      wu[u] = L.wf1[fy + n];
    }
  }
  // D = sum of the faces + s (same order as diag_pt)
  __device__ __forceinline__ T diag(int u, T s) const { return wl[u] + wr[u] + wd[u] + wu[u] + s; }
  // (A + s) x at region point q from LDS values X (row length RX); same
  // arithmetic and order as lds_apply2; *dg = D when dg != nullptr
  __device__ __forceinline__ T apply(int u, const T* X, int q, int RX, T s, T* dg) const {
    const T xc = X[q];
    const T xl = X[q - 1], xr = X[q + 1], xd = X[q - RX], xu = X[q + RX];
    if (dg) *dg = wl[u] + wr[u] + wd[u] + wu[u] + s;
    return wl[u] * (xc - xl) + wr[u] * (xc - xr) + wd[u] * (xc - xd) + wu[u] * (xc - xu) + s * xc;
  }
};

// The fine-level vectors the 2D stencil product and fused level kernels write
// (p_new, q, x; the pre-smoothed iterate and the updated residual; z) are
// stored with the nontemporal hint: each is read again only by a later
// kernel, after more than the last-level cache has streamed through, so
// keeping them out of the caches leaves room for the halo re-reads (measured:
// 2 % faster per solve, the down kernel 5 %).

// Tile shapes of the 2D kernels, one row per launch-shape variant (variant 0
// is the default; a plan may time the others at creation and keep the
// fastest): coarse points per block of the down kernel, fine points per block
// of the up kernel, rows per thread and threads along x (of 256) of the
// stencil product.  The stencil product's default is 128 columns wide: each
// row of a tile then spans 8 cache lines of 128 bytes (FP64) plus one line of
// halo on each side, against 4 plus 2 at 64 columns, which took 3.5 % off its
// time at 1023^2 (256 columns, two rows per thread, was slower: less reuse
// along y).  The down kernel's default region is 133 fine columns wide for
// the same reason (7 % faster than 69 columns); the up kernel stays at 64
// fine columns, where it is faster than at 128.
// Variants 3 and 4 of the stencil product and of the down and up kernels are
// k_spmv_r2 / k_down2r / k_up2r (whole rows, levels of up to 1023 points per
// axis; a larger level runs variant 0 in their place, and the tuner skips
// them there): segments of 128 fine rows (variant 3) or 32 (variant 4, more
// workgroups for launches of few systems; 1023^2 with 30 systems: stencil
// product 121 -> 109 us in FP32 and 229 -> 214 us in FP64, the FP32 up
// kernel 108 -> 92 us, where 128-row segments were slower than the tiles).
constexpr int kDownTile[kTileVariants][2] = {{64, 6}, {32, 8}, {64, 8}, {64, 6}, {64, 6}};
constexpr int kUpTile[kTileVariants][2] = {{64, 16}, {64, 8}, {64, 24}, {64, 16}, {64, 16}};
constexpr int kSpmvTile[kTileVariants][2] = {{4, 128}, {2, 64}, {8, 128}, {4, 128}, {4, 128}};
constexpr int kRowsSeg = 128, kShortRowsSeg = 32;   // fine rows per workgroup
// The marching kernels keep the global loads of the next kRowLead rows in
// flight in a ring of registers: slot s serves steps s, s + kRowLead, ...,
// is used at the start of its step and is refilled after the step's
// barriers with the row kRowLead steps ahead (the barriers keep the compiler
// from issuing the new load before the old value is used, so the slot stays
// one register and no register copy has to wait on a load).  The loop over
// steps is unrolled by kRowLead so that every slot index is a constant.  A
// load used in the step that issued it (or copied at its end) makes the wave
// wait there for every load in flight: one memory round trip per row.
constexpr int kRowLead = 3;
// the lead of the 3D marching kernels, in planes (a plane's loads are
// several points per thread)
constexpr int kPlaneLead = 2;
// A copy of a value the register allocator cannot merge with its source:
// the ring slot the source came from is free after it, so the refill load
// can go into the same register and no copy at the loop's end waits on it.
// A vector (one system's, or the face weights every system shares) as a
// buffer resource: loads and stores at this lane's byte offset voff (a vector
// register, fixed for the whole march) plus a byte offset soff that is the
// same for the whole workgroup (a scalar register, the row).  Addressing a
// row then costs no per-lane arithmetic, where a 64-bit pointer costs a
// 64-bit add per access.  Every access is in range (rows are clamped), so
// the bounds of the resource never apply.
constexpr int kBufWord3 = 0x00020000;   // resource word 3: 32-bit data format
template <typename T>
struct RowBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ RowBuf(const T* base, long long count)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, (int)(count * (long long)sizeof(T)), kBufWord3)) {}
  __device__ __forceinline__ T ld(unsigned voff, unsigned soff) const {
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  // NT: the nontemporal hint (the value is read again only by a later kernel)
  template <bool NT>
  __device__ __forceinline__ void st(T v, unsigned voff, unsigned soff) const {
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, NT ? 2 : 0);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(unsigned __attribute__((ext_vector_type(2))), v), r,
                                            voff, soff, NT ? 2 : 0);
  }
};

// Runs step(t, slot) for t = t0 .. t1 with slot = (t - t0) mod kRowLead as a
// compile-time constant: whole groups of kRowLead steps in a loop without
// exits (an exit inside the group makes the compiler peel the loop, and the
// waits of the loop then serve the peeled path too), then the remainder.
template <int LEAD, typename Step, int... S>
__device__ __forceinline__ void ring_march_impl(int t0, int t1, Step& step, std::integer_sequence<int, S...>) {
  int tb = t0;
  for (; tb + LEAD - 1 <= t1; tb += LEAD) (step(tb + S, std::integral_constant<int, S>{}), ...);
  const int rem = t1 - tb + 1;
  ((S < rem ? (step(tb + S, std::integral_constant<int, S>{}), 0) : 0), ...);
}
template <int LEAD = kRowLead, typename Step>
__device__ __forceinline__ void ring_march(int t0, int t1, Step step) {
  ring_march_impl<LEAD>(t0, t1, step, std::make_integer_sequence<int, LEAD>{});
}
// the lead of the fused row kernels: in FP64 with variable coefficients
// three rows of loads do not fit the registers a 1024-thread workgroup
// leaves (they spilled to scratch memory), so those keep two, and one with
// three sweeps
template <typename T, bool VAR, int NU>
constexpr int row_lead() { return sizeof(T) == 8 && VAR ? (NU >= 3 ? 1 : 2) : kRowLead; }
// the up kernel holds twice the sweeps' rows (it forms the pre-smoothed
// iterate again): FP64 with variable coefficients keeps one row of lead
template <typename T, bool VAR, int NU>
constexpr int up_row_lead() { return sizeof(T) == 8 && VAR ? 1 : kRowLead; }
// Before a marching loop starts its ring: every load of the set-up has
// arrived.  The waits inside the loop must suit both the first step and the
// steady state; with set-up loads still in flight they are computed for the
// shorter history before the first step and wait for far more than the
// steady state needs, on every step.
__device__ __forceinline__ void ring_prologue_wait() { __builtin_amdgcn_s_waitcnt(0); }
template <typename T>
__device__ __forceinline__ T ring_take(T v) {
  T o;
  if constexpr (sizeof(T) == 4) asm("v_mov_b32 %0, %1" : "=v"(o) : "v"(v));
  else asm("v_mov_b64 %0, %1" : "=v"(o) : "v"(v));
  return o;
}
constexpr int kRowsMaxN = 1023;
constexpr int kRowsMinN = 255;   // smallest level the row kernels are the default on
// A row kernel's workgroup: its system and row segment, from a launch grid of
// (1, segments, systems): the segments of a system run next to each other.
// Systems first, (systems, segments), so that workgroups running at the same
// time share a segment's face weights in the L2, made the FP64 residual 1 %
// faster but the FP32 row kernels 1 - 2 % slower (511^2, 2048 systems).
struct RowTile {
  int sys, seg, nseg;
};
__device__ __forceinline__ RowTile row_tile() {
  RowTile r;
  r.sys = blockIdx.z;
  r.seg = blockIdx.y;
  r.nseg = gridDim.y;
  return r;
}
static inline dim3 rows_grid(int nseg, int nsys) { return dim3(1, nseg, nsys); }
// profiling: the workgroup of segment 0 of each system counts its bytes
__device__ __forceinline__ void count_bytes_row(const RowTile& rt, unsigned long long* ctr, unsigned long long b) {
  if (ctr == nullptr || threadIdx.x != 0 || rt.seg != 0) return;
  atomicAdd(ctr, b);
}
// whether the stencil product / down / up kernel of a level of n points per
// axis runs k_spmv_r2 / k_down2r / k_up2r in variant tv, and their threads
// per workgroup (one per column and at least one past the grid, in waves)
static inline bool down_rows(int dim, int n, int tv) {
  const int v = tile_variant(tv);
  return dim == 2 && (v == kRowsVariant || v == kShortRowsVariant) && n <= kRowsMaxN;
}
static inline bool up_rows(int dim, int n, int tv) { return down_rows(dim, n, tv); }
static inline bool spmv_rows(int dim, int n, int tv) { return down_rows(dim, n, tv); }
static inline int rows_threads(int n) { return ((n + 1 + 63) / 64) * 64; }
// fine rows per workgroup of a row variant (the down kernel: half as many coarse rows)
static inline int rows_seg(int tv) { return tile_variant(tv) == kShortRowsVariant ? kShortRowsSeg : kRowsSeg; }

// Reciprocal of a Jacobi diagonal, formed once per point and kernel: the sweeps
// multiply by it.  FP32: the hardware reciprocal (within 1 ulp); FP64: IEEE
// division.  A damped Jacobi sweep with D^-1 off by an ulp is the same
// symmetric smoother up to rounding, and the value is the same for a point in
// every launch shape.
__device__ __forceinline__ float jacobi_recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double jacobi_recip(double d) { return 1.0 / d; }

// The fused 2D level kernels are bound by instruction issue (FP32 moves half
// the bytes of FP64 per point with the same instructions), so their sweeps are
// branch-free: every thread updates all of its region points, points off the
// grid carry a zero inverse diagonal and stay exactly 0 (b = 0 there), and the
// LDS array is padded so that the neighbours of every lane's point, the
// unused lanes of the last row of threads included, are inside it (the pads
// hold zeros, everything else finite values).  A sweep's values are exact on
// the range it is valid on (shrinking by one point per sweep) and finite
// garbage outside it, which no valid point reads.  Per-point branches had
// kept one exec mask per point and phase alive, which spilled the scalar
// registers into vector lanes (about 600 lane moves per wave).

// RUP: the right-hand side is first advanced by the PCG step, b = b_old -
// alpha (A + s) p (read from b, written to bout on the owned points, |b|^2 into
// partial), so the vector update of the PCG iteration costs no pass of its
// own.  The product (A + s) p is formed here from p (pv), staged on the region
// widened by one point, with the stencil product's arithmetic: that kernel
// then only dots it with p and stores no q, one vector pass less per
// iteration.  bout must not be b: neighbouring blocks still read b_old in
// their halos.
// (occupancy: for FP32 constant coefficients the compiler is asked for 5
// waves per SIMD; left alone it takes a few registers more and one wave
// less.  Variable coefficients (4 face weights per region point in
// registers) and FP64 spill registers under such a request -- the 64 x 8
// variable-coefficient tile at 4 waves ran at half the speed it has at 3 --
// and are left to the compiler.)
template <typename T, bool VAR, int NU, bool RUP, int CX, int CY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !VAR ? 5 : 1))) void k_down2(
    LevelDev<T> Lf, LevelDev<T> Lc, const T* __restrict__ b,
                                               T* __restrict__ xout, T* __restrict__ bc,
                                               const T* __restrict__ shift, const int* __restrict__ active,
                                               Sweeps<T> om, unsigned long long* __restrict__ ctr,
                                               const T* __restrict__ pv, const double* __restrict__ alpha,
                                               T* __restrict__ bout, double* __restrict__ partial, Fin fin) {
  constexpr int RX = 2 * CX + 2 * NU + 1, RY = 2 * CY + 2 * NU + 1, RN = RX * RY;
  // RUP: p on the region widened by one point per side (row length PX),
  // staged in the same LDS array before it takes the iterate
  constexpr int PX = RX + 2, PY = RY + 2, PN = PX * PY;
  constexpr int PER = (RN + 255) / 256, PPER = RUP ? (PN + 255) / 256 : 1;
  // LDS: a zero pad of PAD values before the data, the data at PAD + q, and
  // room after it for the farthest neighbour any lane reads (lanes q >= RN of
  // the last row of threads included); the p layout (row length PX) reaches
  // further than the iterate layout
  constexpr int PAD = (RUP ? PX : RX) + 1;
  constexpr int QMAX = PER * 256 - 1;
  constexpr int PQMAX = RUP ? ((QMAX / RX) + 1) * PX + RX : 0;
  constexpr int HI = (QMAX + RX) > (PQMAX + PX) ? (QMAX + RX) : (PQMAX + PX);
  constexpr int DATA = PER * 256 > (RUP ? PPER * 256 : 0) ? PER * 256 : PPER * 256;
  constexpr int LN = PAD + (HI + 1 > DATA ? HI + 1 : DATA);
  // One LDS array: p (RUP), then the iterate, then the residual.  Thread tid
  // owns region points tid + 256 u (u < PER) throughout and keeps their b,
  // x and 1/D in registers; a sweep reads its neighbours from LDS, and its
  // results are written back after a barrier (a second barrier before the
  // next reads).
  __shared__ T sx[LN];
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)Lf.N * sizeof(T) * (RUP ? 4 : 2) +
                                   (unsigned long long)Lc.N * sizeof(T) +
                                   (VAR && sys == 0 ? (unsigned long long)Lf.N * sizeof(T) * 2 : 0ULL));
  const T am = RUP ? (T)alpha[sys] : T(0);
  const int nf = Lf.n, nc = Lc.n;
  const int I0 = tl.x * CX, J0 = tl.y * CY;
  const int gx0 = 2 * I0 - NU, gy0 = 2 * J0 - NU;
  const T sh = shift[sys];
  const T dcon = Lf.wc * T(4) + sh;   // the diagonal for constant coefficients
  const T rcon = jacobi_recip(dcon);
  const long long off = (long long)sys * Lf.N;
  const T* __restrict__ bs = b + off;
  const int tid = threadIdx.x;
  // the pads: zeros (the data range is written below before it is read)
  for (int i = tid; i < PAD; i += 256) sx[i] = T(0);
  for (int i = PAD + DATA + tid; i < LN; i += 256) sx[i] = T(0);
  // per point: whether it is on the grid (bit u of `in`); its grid index,
  // clamped into the grid for the loads, is recomputed where needed (held in
  // registers it cost occupancy)
  unsigned in = 0u;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + 256 * u;
    const int ry = q / RX, rx = q - ry * RX;
    const int gi = gx0 + rx, gj = gy0 + ry;
    const bool on = q < RN && gi >= 0 && gi < nf && gj >= 0 && gj < nf;
    in |= (on ? 1u : 0u) << u;
  }
  auto gidx = [&](int u) {
    const int q = tid + 256 * u;
    const int ry = q / RX, rx = q - ry * RX;
    return min(max(gy0 + ry, 0), nf - 1) * nf + min(max(gx0 + rx, 0), nf - 1);
  };
  // variable coefficients: the four face weights of each of this thread's
  // region points, loaded once for every sweep and the residual
  RegionFaces<T, VAR, PER> fw;
  fw.load(Lf, tid, RX, RN, gx0, gy0);
  // stage b and the first sweep from x = 0: x1 = omega b / D.  All loads of a
  // thread are issued before any is used, so a wave keeps them all in flight.
  T bl[PER];
  if (RUP) {
    // p first, into LDS (0 off the grid); b is loaded after the barrier, so
    // the two sets of loads do not hold registers at the same time
    const T* __restrict__ ps = pv + off;
    T pl[PPER];
#pragma unroll
    for (int u = 0; u < PPER; ++u) {
      const int q = tid + 256 * u;
      const int py = q / PX, px = q - py * PX;
      const int gi = gx0 - 1 + px, gj = gy0 - 1 + py;
      pl[u] = ps[min(max(gj, 0), nf - 1) * nf + min(max(gi, 0), nf - 1)];
    }
#pragma unroll
    for (int u = 0; u < PPER; ++u) {
      const int q = tid + 256 * u;
      const int py = q / PX, px = q - py * PX;
      const int gi = gx0 - 1 + px, gj = gy0 - 1 + py;
      const bool on = q < PN && gi >= 0 && gi < nf && gj >= 0 && gj < nf;
      sx[PAD + q] = on ? pl[u] : T(0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) bl[u] = bs[gidx(u)];
  // 1/D per point (0 off the grid): held for variable coefficients, a select
  // of the one constant value otherwise
  T bv[PER], xv[PER], rdv[VAR ? PER : 1];
  auto rd = [&](int u) { return VAR ? rdv[VAR ? u : 0] : (((in >> u) & 1u) ? rcon : T(0)); };
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + 256 * u;
    const bool on = (in >> u) & 1u;
    T bn = bl[u];
    if (RUP) {
      const int ry = q / RX, rx = q - ry * RX;
      const int pq = PAD + (ry + 1) * PX + (rx + 1);
      const T ap = VAR ? fw.apply(u, sx, pq, PX, sh, nullptr) : lds_apply2<T, false>(sx, pq, PX, Lf, 0, 0, sh, nullptr);
      bn = bl[u] - am * ap;
    }
    bv[u] = on ? bn : T(0);
    if (VAR) rdv[VAR ? u : 0] = on ? jacobi_recip(fw.diag(u, sh)) : T(0);
    xv[u] = sweep_w(om, 0) * bv[u] * rd(u);
  }
  if (RUP) __syncthreads();   // every read of p done before sx takes the iterate
#pragma unroll
  for (int u = 0; u < PER; ++u) sx[PAD + tid + 256 * u] = xv[u];
  __syncthreads();
#pragma unroll
  for (int m = 1; m < NU; ++m) {   // sweep m+1, exact on the range shrunk by m
    const T wm = sweep_w(om, m);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = PAD + tid + 256 * u;
      const T ax = VAR ? fw.apply(u, sx, q, RX, sh, nullptr) : lds_apply2<T, false>(sx, q, RX, Lf, 0, 0, sh, nullptr);
      xv[u] = xv[u] + wm * (bv[u] - ax) * rd(u);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) sx[PAD + tid + 256 * u] = xv[u];
    __syncthreads();
  }
  // owned fine points: [2 I0, 2 I0 + 2 CX) per axis, extended to the grid end on the last tile
  {
    const int hx = (I0 + CX >= nc) ? nf : 2 * (I0 + CX);
    const int hy = (J0 + CY >= nc) ? nf : 2 * (J0 + CY);
    T* __restrict__ xs = xout + off;
    T* __restrict__ bo = RUP ? bout + off : nullptr;
    double rr = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = tid + 256 * u;
      const int ry = q / RX, rx = q - ry * RX;
      const int gi = gx0 + rx, gj = gy0 + ry;
      const bool own = ((in >> u) & 1u) && gi >= 2 * I0 && gi < hx && gj >= 2 * J0 && gj < hy;
      if (own) {
        const int g = gj * nf + gi;
        __builtin_nontemporal_store(xv[u], &xs[g]);
        if (RUP) __builtin_nontemporal_store(bv[u], &bo[g]);
      }
      if (RUP) rr += own ? (double)bv[u] * (double)bv[u] : 0.0;
    }
    if (RUP) {
      write_partial_tile(tl, partial, sys, rr);
      finish(fin, partial, sys, gridDim.x * gridDim.y);
    }
  }
  // residual b - (A + s) x, exact on the range shrunk by NU (fine points
  // 2 I0 .. 2 I0 + 2 CX, all on the grid: the weighting below reads no other),
  // formed from the final iterate in sx and then written over it
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = PAD + tid + 256 * u;
    xv[u] = bv[u] - (VAR ? fw.apply(u, sx, q, RX, sh, nullptr) : lds_apply2<T, false>(sx, q, RX, Lf, 0, 0, sh, nullptr));
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) sx[PAD + tid + 256 * u] = xv[u];
  __syncthreads();
  // full weighting: coarse (I, J) <- fine 2I+1 +- 1
  T* __restrict__ bcs = bc + (long long)sys * Lc.N;
  for (int q2 = tid; q2 < CX * CY; q2 += 256) {
    const int I = I0 + (q2 % CX), J = J0 + (q2 / CX);
    if (I < nc && J < nc) {
      const int cx = 2 * I + 1 - gx0, cy = 2 * J + 1 - gy0;
      const T* R = sx + PAD + cy * RX + cx;
      const T v = T(0.25) * R[0] + T(0.125) * (R[-1] + R[1] + R[-RX] + R[RX]) +
                  T(0.0625) * (R[-RX - 1] + R[-RX + 1] + R[RX - 1] + R[RX + 1]);
      bcs[J * nc + I] = v;
    }
  }
}

template <typename T, bool VAR, int NU, bool DOT, int OX, int OY>
__global__ __launch_bounds__(256) void k_up2(LevelDev<T> Lc, LevelDev<T> Lf, const T* __restrict__ xc,
                                             const T* __restrict__ xin, const T* __restrict__ b, T* __restrict__ xout,
                                             const T* __restrict__ shift, const int* __restrict__ active, Sweeps<T> om,
                                             double* __restrict__ partial, unsigned long long* __restrict__ ctr,
                                             Fin fin) {
  constexpr int RX = OX + 2 * NU, RY = OY + 2 * NU, RN = RX * RY;
  // FP64 constant coefficients: each sweep updates only the points it is
  // exact on (the range shrinking by one per sweep) behind a per-point test.
  // Branch-free, every point in every sweep, this kernel held 114 VGPRs (4
  // waves per SIMD) against 66 (7) and ran 25 % slower at 1023^2; in FP32 and
  // with variable coefficients the branch-free form is the faster one.
  constexpr bool GUARD = sizeof(T) == 8 && !VAR;
  // coarse values under the region, zero-padded: coarse index c at cx0 + (c - c0)
  constexpr int CRX = RX / 2 + 3, CRY = RY / 2 + 3, CRN = CRX * CRY;
  constexpr int PER = (RN + 255) / 256, CPER = (CRN + 255) / 256;
  // the iterate at PAD + q, zero pads around it (branch-free sweeps, as in k_down2)
  constexpr int PAD = RX + 1;
  constexpr int LN = PAD + PER * 256 + RX + 1;
  __shared__ T sx[LN];
  __shared__ T sc[CRN];
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)Lf.N * sizeof(T) * 3 + (unsigned long long)Lc.N * sizeof(T) +
                                   (VAR && sys == 0 ? (unsigned long long)Lf.N * sizeof(T) * 2 : 0ULL));
  const int nf = Lf.n, nc = Lc.n;
  const int ox0 = tl.x * OX, oy0 = tl.y * OY;
  const int gx0 = ox0 - NU, gy0 = oy0 - NU;
  // smallest coarse index any region point interpolates from (floor division)
  const int cx0 = ((gx0 >= 0) ? gx0 / 2 : -((-gx0 + 1) / 2)) - 1;
  const int cy0 = ((gy0 >= 0) ? gy0 / 2 : -((-gy0 + 1) / 2)) - 1;
  const T sh = shift[sys];
  const T rcon = jacobi_recip(Lf.wc * T(4) + sh);
  const long long off = (long long)sys * Lf.N;
  const T* __restrict__ xcs = xc + (long long)sys * Lc.N;
  const T* __restrict__ bs = b + off;
  const T* __restrict__ xis = xin + off;
  const int tid = threadIdx.x;
  for (int i = tid; i < PAD; i += 256) sx[i] = T(0);
  for (int i = PAD + PER * 256 + tid; i < LN; i += 256) sx[i] = T(0);
  unsigned in = 0u;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + 256 * u;
    const int ry = q / RX, rx = q - ry * RX;
    const int gi = gx0 + rx, gj = gy0 + ry;
    const bool on = q < RN && gi >= 0 && gi < nf && gj >= 0 && gj < nf;
    in |= (on ? 1u : 0u) << u;
  }
  auto gidx = [&](int u) {
    const int q = tid + 256 * u;
    const int ry = q / RX, rx = q - ry * RX;
    return min(max(gy0 + ry, 0), nf - 1) * nf + min(max(gx0 + rx, 0), nf - 1);
  };
  RegionFaces<T, VAR, PER> fw;
  fw.load(Lf, tid, RX, RN, gx0, gy0);
  // every global load of the staging phase is issued up front (clamped
  // addresses, selected afterwards): the coarse tile, then b and x_in
  T cl[CPER], bl[PER], xl[PER];
#pragma unroll
  for (int u = 0; u < CPER; ++u) {
    const int q = tid + 256 * u;
    const int cy = q / CRX, cx = q - cy * CRX;
    cl[u] = xcs[min(max(cy0 + cy, 0), nc - 1) * nc + min(max(cx0 + cx, 0), nc - 1)];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int g = gidx(u);
    bl[u] = bs[g];
    xl[u] = xis[g];
  }
#pragma unroll
  for (int u = 0; u < CPER; ++u) {
    const int q = tid + 256 * u;
    if (q < CRN) {
      const int cy = q / CRX, cx = q - cy * CRX;
      const int I = cx0 + cx, J = cy0 + cy;
      sc[q] = (I >= 0 && I < nc && J >= 0 && J < nc) ? cl[u] : T(0);
    }
  }
  __syncthreads();
  T bv[PER], xv[PER], rdv[VAR ? PER : 1];
  auto rd = [&](int u) { return VAR ? rdv[VAR ? u : 0] : (((in >> u) & 1u) ? rcon : T(0)); };
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    // lanes past the region interpolate at its last point (in range of sc)
    const int q = min(tid + 256 * u, RN - 1);
    const int ry = q / RX, rx = q - ry * RX;
    const int gi = gx0 + rx, gj = gy0 + ry;
    const bool on = (in >> u) & 1u;
    // multilinear interpolation from the zero-padded coarse tile
    const int ia = (gi & 1) ? (gi - 1) / 2 : gi / 2 - 1;
    const int ja = (gj & 1) ? (gj - 1) / 2 : gj / 2 - 1;
    const T* C = sc + (ja - cy0) * CRX + (ia - cx0);
    T v;
    if (gi & 1) {
      v = (gj & 1) ? C[0] : T(0.5) * (C[0] + C[CRX]);
    } else {
      v = (gj & 1) ? T(0.5) * (C[0] + C[1]) : T(0.25) * (C[0] + C[1] + C[CRX] + C[CRX + 1]);
    }
    bv[u] = on ? bl[u] : T(0);
    xv[u] = on ? xl[u] + v : T(0);
    if (VAR) rdv[VAR ? u : 0] = on ? jacobi_recip(fw.diag(u, sh)) : T(0);
    sx[PAD + tid + 256 * u] = xv[u];
  }
  __syncthreads();
#pragma unroll
  for (int m = 1; m <= NU; ++m) {   // post-smoothing: the pre-smoothing weights reversed
    const T wm = sweep_w(om, NU - m);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = PAD + tid + 256 * u;
      if (GUARD) {   // only the points the sweep is exact on
        const int qq = tid + 256 * u;
        const int ry = qq / RX, rx = qq - ry * RX;
        if (((in >> u) & 1u) && rx >= m && rx < RX - m && ry >= m && ry < RY - m)
          xv[u] = xv[u] + wm * (bv[u] - lds_apply2<T, false>(sx, q, RX, Lf, 0, 0, sh, nullptr)) * rcon;
        continue;
      }
      const T ax = VAR ? fw.apply(u, sx, q, RX, sh, nullptr) : lds_apply2<T, false>(sx, q, RX, Lf, 0, 0, sh, nullptr);
      xv[u] = xv[u] + wm * (bv[u] - ax) * rd(u);
    }
    if (m < NU) {   // the last sweep's values are written out from registers
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PER; ++u) sx[PAD + tid + 256 * u] = xv[u];
      __syncthreads();
    }
  }
  double dot = 0.0;
  T* __restrict__ xs = xout + off;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + 256 * u;
    const int ry = q / RX, rx = q - ry * RX;
    const bool own = ((in >> u) & 1u) && rx >= NU && rx < NU + OX && ry >= NU && ry < NU + OY;
    if (own) __builtin_nontemporal_store(xv[u], &xs[(gy0 + ry) * nf + gx0 + rx]);
    if (DOT) dot += own ? (double)bv[u] * (double)xv[u] : 0.0;
  }
  if (DOT) {
    write_partial_tile(tl, partial, sys, dot);
    finish(fin, partial, sys, gridDim.x * gridDim.y);
  }
}

// --------------------------------------------------------------------------
// k_down2r: the down kernel of k_down2 (same inputs and outputs, the same
// arithmetic per point except the order of the full weighting's sum)
// marching along y over whole grid rows.  A workgroup has one
// thread per grid column (blockDim.x >= n + 1, a multiple of 64) and owns the
// fine rows of ky coarse rows (a launch parameter); it walks up its rows with the stages
// lagging one row behind each other, as the 3D kernels walk up their planes:
// at step t row t of b (RUP: b_old - alpha (A + s) p, p of rows t - 1 .. t + 1)
// enters, the first sweep is formed on it pointwise, sweep m + 1 on row t - m,
// the residual on row t - NU, and the full weighting of coarse row K once the
// residual of fine row 2K + 2 is there.  The newest row of every stage goes
// into LDS for the left/right neighbours; the rows below and above stay in
// registers.  A workgroup starts NU rows below its first owned row (warm-up),
// so every row it writes is exact.  There is no halo across columns and none
// along y beyond the warm-up rows, where the tiles of k_down2 fetch 1.4 - 1.8
// times their points (halo rows and columns, partial cache lines) and sweep
// that many.  Columns past the grid and rows outside it carry a zero
// right-hand side and a zero inverse diagonal, so they stay exactly 0; the
// LDS rows have a zero pad on each side.  Two barriers per row.  With xout
// == nullptr the pre-smoothed iterate is not stored (the level's up kernel
// is k_up2r, which forms it again).
// --------------------------------------------------------------------------
template <typename T, bool VAR, int NU, bool RUP>
__global__ __launch_bounds__(1024) void k_down2r(LevelDev<T> Lf, LevelDev<T> Lc, const T* __restrict__ b,
                                                 T* __restrict__ xout, T* __restrict__ bc,
                                                 const T* __restrict__ shift, const int* __restrict__ active,
                                                 Sweeps<T> om, unsigned long long* __restrict__ ctr,
                                                 const T* __restrict__ pv, const double* __restrict__ alpha,
                                                 T* __restrict__ bout, double* __restrict__ partial, Fin fin,
                                                 int ky) {
  constexpr int LW = 1024 + 2;   // an LDS row: pad, up to 1024 columns, pad
  __shared__ T sx[NU][LW];       // newest row of each sweep's output
  __shared__ T sr[LW];           // residual row
  __shared__ T sp[RUP ? LW : 1]; // p of the row being updated (RUP)
  const RowTile rt = row_tile();
  const int sys = rt.sys;
  constexpr int LEAD = row_lead<T, VAR, NU>();
  if (!active[sys]) return;
  // xout == nullptr: the pre-smoothed iterate is not stored (the level's up
  // kernel is k_up2r, which forms it again)
  const bool keepx = xout != nullptr;
  count_bytes_row(rt, ctr, (unsigned long long)Lf.N * sizeof(T) * ((RUP ? 3 : 1) + (keepx ? 1 : 0)) +
                                   (unsigned long long)Lc.N * sizeof(T) +
                                   (VAR && sys == 0 ? (unsigned long long)Lf.N * sizeof(T) * 2 : 0ULL));
  const int nf = Lf.n, nc = Lc.n;
  const int K0 = rt.seg * ky, K1 = min(K0 + ky, nc);
  const int f1 = K1 == nc ? nf : 2 * K1;   // owned fine rows [2 K0, f1) (the last segment: the top one too)
  const int i = threadIdx.x;               // this thread's column
  const int NT = blockDim.x;
  const bool col_on = i < nf;
  const int ic = min(i, nf - 1);           // clamped column for the loads
  const unsigned cb = (unsigned)ic * (unsigned)sizeof(T), ib = (unsigned)i * (unsigned)sizeof(T);
  const unsigned rowb = (unsigned)nf * (unsigned)sizeof(T);   // bytes per grid row
  const T sh = shift[sys];
  const T rcon = jacobi_recip(Lf.wc * T(4) + sh);
  const T am = RUP ? (T)alpha[sys] : T(0);
  const long long off = (long long)sys * Lf.N;
  const T* __restrict__ bs = b + off;
  const T* __restrict__ ps = RUP ? pv + off : nullptr;
  T* __restrict__ xs = keepx ? xout + off : nullptr;
  T* __restrict__ bo = RUP ? bout + off : nullptr;
  const RowBuf<T> bsb(bs, Lf.N), psb(RUP ? ps : bs, Lf.N), xsb(xs, Lf.N), bob(RUP ? bo : xs, Lf.N);
  const RowBuf<T> w0b(VAR ? Lf.wf0 : bs, VAR ? (long long)(nf + 1) * nf : 1), w1b(VAR ? Lf.wf1 : bs, VAR ? (long long)(nf + 1) * nf : 1);
  const int q = 1 + i;   // this column in an LDS row
  // the pads (columns -1 and NT) stay 0; every other entry is written before it is read
  if (i < 2) {
    const int pq = i == 0 ? 0 : NT + 1;
#pragma unroll
    for (int m = 0; m < NU; ++m) sx[m][pq] = T(0);
    sr[pq] = T(0);
    if (RUP) sp[pq] = T(0);
  }
  auto row_on = [&](int r) { return col_on && r >= 0 && r < nf; };
  auto crow = [&](int r) { return min(max(r, 0), nf - 1); };
  // 1 on the grid, 0 off it, applied to a row's loads when they are used
  auto on_f = [&](int r) { return row_on(r) ? T(1) : T(0); };
  // face weights of row r at this column (clamped row: finite off the grid,
  // where no sweep uses them) and the inverse diagonal of row r
  struct Faces { T l, r, d, u; };
  auto load_faces = [&](int r) {
    Faces f{T(0), T(0), T(0), T(0)};
    if (VAR) {
      const unsigned rr = (unsigned)crow(r);
      const unsigned o0 = rr * (unsigned)(nf + 1) * (unsigned)sizeof(T), o1 = rr * rowb;
      f.l = w0b.ld(cb, o0);
      f.r = w0b.ld(cb + (unsigned)sizeof(T), o0);
      f.d = w1b.ld(cb, o1);
      f.u = w1b.ld(cb, o1 + rowb);
    }
    return f;
  };
  auto rdiag = [&](const Faces& f, int r) {
    if (!VAR) return row_on(r) ? rcon : T(0);
    return row_on(r) ? jacobi_recip(f.l + f.r + f.d + f.u + sh) : T(0);
  };
  // (A + s) x at this column of a row with faces f, centre xc, left/right from
  // the LDS row X, below xd and above xu (the arithmetic and order of k_down2)
  auto apply = [&](const Faces& f, const T* X, T xc, T xd, T xu) {
    const T xl = X[q - 1], xr = X[q + 1];
    if (!VAR) return Lf.wc * ((xc - xl) + (xc - xr) + (xc - xd) + (xc - xu)) + sh * xc;
    return f.l * (xc - xl) + f.r * (xc - xr) + f.d * (xc - xd) + f.u * (xc - xu) + sh * xc;
  };
  // one damped Jacobi update x + w (b - (A + s) x) / diag written as
  // x + w ((b + the neighbours' face-weighted sum) / diag - x): diag holds
  // every face weight and the shift, so the two agree in exact arithmetic, and
  // this form takes 6 instead of 12 vector operations per point (the residual
  // keeps the difference form)
  auto relax = [&](const Faces& f, const T* X, T xc, T xd, T xu, T bb, T w, T r) {
    const T xl = X[q - 1], xr = X[q + 1];
    const T nb = VAR ? bb + f.l * xl + f.r * xr + f.d * xd + f.u * xu : bb + Lf.wc * ((xl + xr) + (xd + xu));
    return xc + w * (r * nb - xc);
  };
  const int t0 = 2 * K0 - NU, t1 = 2 * K1 + NU;
  // registers: bh[d] = b of row t - d; xh[m][0], xh[m][1] = sweep m+1's output
  // at its newest row of the previous step and the one below; fw[d], rd[d] =
  // faces and inverse diagonal of row t - d
  T bh[NU + 1], xh[NU][2], rd[NU + 1];
  Faces fw[NU + 1];
#pragma unroll
  for (int d = 0; d <= NU; ++d) {
    bh[d] = T(0);
    rd[d] = T(0);
    fw[d] = load_faces(t0 - 1 - d);
  }
#pragma unroll
  for (int m = 0; m < NU; ++m) xh[m][0] = xh[m][1] = T(0);
  // p of rows t - 1, t, t + 1 (RUP; 0 outside the grid) during step t, p(t)
  // also in sp; before the first step they hold rows t0 - 1 and t0
  T pm = T(0), pc = T(0), pa = T(0);
  if (RUP) {
    pc = ps[(long long)crow(t0 - 1) * nf + ic] * on_f(t0 - 1);
    pa = ps[(long long)crow(t0) * nf + ic] * on_f(t0);
    sp[q] = pa;
  }
  // the coarse column of this thread (threads I < nc) and its weighted
  // in-row sums of the residual on fine rows 2K and 2K + 1
  const bool restricts = i < nc;
  T s_lo = T(0), s_mid = T(0);
  const RowBuf<T> bcb(bc + (long long)sys * Lc.N, Lc.N);
  const unsigned cbc = (unsigned)min(i, nc - 1) * (unsigned)sizeof(T);   // this lane's coarse column
  double rr = 0.0;
  ring_prologue_wait();
  __syncthreads();
  // the ring of row loads (see kRowLead): slot s of step t holds b and the
  // faces of row t and p of row t + 1, as loaded (clamped rows, unmasked)
  T rb[LEAD], rp[LEAD];
  Faces rf[LEAD];
#pragma unroll
  for (int s = 0; s < LEAD; ++s) {
    rb[s] = bsb.ld(cb, (unsigned)crow(t0 + s) * rowb);
    rf[s] = load_faces(t0 + s);
    rp[s] = RUP ? psb.ld(cb, (unsigned)crow(t0 + 1 + s) * rowb) : T(0);
  }
  ring_march<LEAD>(t0, t1, [&](int t, auto slot) {
    constexpr int s = decltype(slot)::value;
#pragma unroll
    for (int d = NU; d > 0; --d) {
      bh[d] = bh[d - 1];
      fw[d] = fw[d - 1];
      rd[d] = rd[d - 1];
    }
    if (VAR) fw[0] = Faces{ring_take(rf[s].l), ring_take(rf[s].r), ring_take(rf[s].d), ring_take(rf[s].u)};
    rd[0] = rdiag(fw[0], t);
    if (RUP) {
      pm = pc;
      pc = pa;
      pa = rp[s] * on_f(t + 1);
    }
    T bn = rb[s];
    if (RUP) bn = bn - am * apply(fw[0], sp, pc, pm, pa);
    bh[0] = row_on(t) ? bn : T(0);
    if (RUP && t >= 2 * K0 && t < f1 && col_on) {
      bob.template st<true>(bh[0], ib, (unsigned)t * rowb);
      rr += (double)bh[0] * (double)bh[0];
    }
    // sweep 1 on row t from x = 0; sweep m + 1 on row t - m from sweep m's
    // output (centre row in sx[m - 1], below in xh, above just formed)
    T xn[NU];
    xn[0] = sweep_w(om, 0) * bh[0] * rd[0];
#pragma unroll
    for (int m = 1; m < NU; ++m) {
      xn[m] = relax(fw[m], sx[m - 1], xh[m - 1][0], xh[m - 1][1], xn[m - 1], bh[m], sweep_w(om, m), rd[m]);
    }
    // the residual on row t - NU
    const T res = bh[NU] - apply(fw[NU], sx[NU - 1], xh[NU - 1][0], xh[NU - 1][1], xn[NU - 1]);
    // the pre-smoothed iterate: sweep NU's newest row t - NU + 1
    const int gx = t - NU + 1;
    if (keepx && gx >= 2 * K0 && gx < f1 && col_on) xsb.template st<true>(xn[NU - 1], ib, (unsigned)gx * rowb);
    __syncthreads();   // every read of this step's LDS rows is done
#pragma unroll
    for (int m = 0; m < NU; ++m) sx[m][q] = xn[m];
    sr[q] = res;
    if (RUP) sp[q] = pa;   // p(t + 1), the centre row of the next step
    __syncthreads();
    // refill the slot with the rows LEAD steps ahead
    rb[s] = bsb.ld(cb, (unsigned)crow(t + LEAD) * rowb);
    rf[s] = load_faces(t + LEAD);
    if (RUP) rp[s] = psb.ld(cb, (unsigned)crow(t + 1 + LEAD) * rowb);
    // full weighting: this coarse column's in-row sum of fine row f = t - NU,
    // and coarse row K = f/2 - 1 once f = 2K + 2 (weights 1/4, 1/2, 1/4 along y)
    const int f = t - NU;
    if (restricts && f >= 2 * K0) {
      const T* R = sr + 1 + 2 * i;   // fine columns 2I .. 2I + 2
      const T acc = T(0.25) * R[0] + T(0.5) * R[1] + T(0.25) * R[2];
      const bool odd = f & 1;
      if (!odd && f != 2 * K0) {
        const int K = f / 2 - 1;
        bcb.template st<false>(T(0.25) * s_lo + T(0.5) * s_mid + T(0.25) * acc, cbc, (unsigned)K * (unsigned)nc * (unsigned)sizeof(T));
      }
      // selects, not stores in two branches: the compiler would merge those
      // into one store through a pointer and keep both sums in scratch memory
      s_mid = odd ? acc : s_mid;
      s_lo = odd ? s_lo : acc;
    }
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      xh[m][1] = xh[m][0];
      xh[m][0] = xn[m];
    }
  });
  if (RUP) {
    write_partial(partial, sys, rr, rt.seg, rt.nseg);
    finish(fin, partial, sys, rt.nseg);
  }
}

// k_up2r: the up kernel of k_up2 (same output; its sweeps in the form of
// k_down2r's relax, equal in exact arithmetic)
// marching along y over whole grid rows, as k_down2r, without reading the
// pre-smoothed iterate: it forms it again from b, as the down kernel did
// (NU sweeps from zero, the same weights and order), so the down kernel of
// the level need not store it (8 bytes per point in FP32 less for the pair,
// 30 -> 22).  2 NU stages lag one row behind each other: at step t row t of
// b enters, pre-sweep k + 1 runs on row t - k (k < NU; the first one
// pointwise), the last of them adds P x_c, and post-sweep m on row
// t - NU + 1 - m (the pre-smoothing weights reversed); post-sweep NU's row
// t - 2 NU + 1 is written on the owned rows [rows s, rows (s + 1)) of
// segment s (rows: a launch parameter), with b.x when this is the finest
// level.  Each thread reads the coarse values under its column (the coarse
// columns left and right of it) from the two coarse rows that bracket the row
// where P x_c is added.  xin is not read.
// (FP32, up to two sweeps: at most 80 VGPRs, six waves per SIMD, three
// 512-thread workgroups per CU)
template <typename T, bool VAR, int NU, bool DOT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && NU <= 2 ? 6 : 1))) void k_up2r(LevelDev<T> Lc, LevelDev<T> Lf, const T* __restrict__ xc,
                                               const T* __restrict__ xin, const T* __restrict__ b,
                                               T* __restrict__ xout, const T* __restrict__ shift,
                                               const int* __restrict__ active, Sweeps<T> om,
                                               double* __restrict__ partial, unsigned long long* __restrict__ ctr,
                                               Fin fin, int rows) {
  (void)xin;
  constexpr int LW = 1024 + 2;
  constexpr int NS = 2 * NU;   // stages: NU pre-sweeps (the last one adds P x_c), NU post-sweeps
  __shared__ T sx[NS - 1][LW];   // newest row of stages 0 .. NS - 2 (the next stage's left/right neighbours)
  const RowTile rt = row_tile();
  const int sys = rt.sys;
  constexpr int LEAD = up_row_lead<T, VAR, NU>();
  if (!active[sys]) return;
  count_bytes_row(rt, ctr, (unsigned long long)Lf.N * sizeof(T) * 2 + (unsigned long long)Lc.N * sizeof(T) +
                                   (VAR && sys == 0 ? (unsigned long long)Lf.N * sizeof(T) * 2 : 0ULL));
  const int nf = Lf.n, nc = Lc.n;
  const int y0 = rt.seg * rows, y1 = min(y0 + rows, nf);   // owned fine rows
  const int i = threadIdx.x;
  const int NT = blockDim.x;
  const bool col_on = i < nf;
  const int ic = min(i, nf - 1);
  const T sh = shift[sys];
  const T rcon = jacobi_recip(Lf.wc * T(4) + sh);
  const long long off = (long long)sys * Lf.N;
  const T* __restrict__ xcs = xc + (long long)sys * Lc.N;
  const T* __restrict__ bs = b + off;
  T* __restrict__ xs = xout + off;
  const unsigned cb = (unsigned)ic * (unsigned)sizeof(T), ib = (unsigned)i * (unsigned)sizeof(T);
  const unsigned rowb = (unsigned)nf * (unsigned)sizeof(T);   // bytes per grid row
  const RowBuf<T> xcb(xcs, Lc.N), bsb(bs, Lf.N), xsb(xs, Lf.N);
  const RowBuf<T> w0b(VAR ? Lf.wf0 : bs, VAR ? (long long)(nf + 1) * nf : 1), w1b(VAR ? Lf.wf1 : bs, VAR ? (long long)(nf + 1) * nf : 1);
  const int q = 1 + i;
  if (i < 2) {
    const int pq = i == 0 ? 0 : NT + 1;
#pragma unroll
    for (int k = 0; k < NS - 1; ++k) sx[k][pq] = T(0);
  }
  auto row_on = [&](int r) { return col_on && r >= 0 && r < nf; };
  auto crow = [&](int r) { return min(max(r, 0), nf - 1); };
  struct Faces { T l, r, d, u; };
  auto load_faces = [&](int r) {
    Faces f{T(0), T(0), T(0), T(0)};
    if (VAR) {
      const int rr = crow(r);
      const unsigned o0 = (unsigned)rr * (unsigned)(nf + 1) * (unsigned)sizeof(T), o1 = (unsigned)rr * rowb;
      f.l = w0b.ld(cb, o0);
      f.r = w0b.ld(cb + (unsigned)sizeof(T), o0);
      f.d = w1b.ld(cb, o1);
      f.u = w1b.ld(cb, o1 + rowb);
    }
    return f;
  };
  auto rdiag = [&](const Faces& f, int r) {
    if (!VAR) return row_on(r) ? rcon : T(0);
    return row_on(r) ? jacobi_recip(f.l + f.r + f.d + f.u + sh) : T(0);
  };
  // the damped Jacobi update in the form of k_down2r's relax
  auto relax = [&](const Faces& f, const T* X, T xc_, T xd, T xu, T bb, T w, T r) {
    const T xl = X[q - 1], xr = X[q + 1];
    const T nb = VAR ? bb + f.l * xl + f.r * xr + f.d * xd + f.u * xu : bb + Lf.wc * ((xl + xr) + (xd + xu));
    return xc_ + w * (r * nb - xc_);
  };
  // the coarse columns of this fine column: ia (and ia + 1 for an even column)
  const int ia = (i & 1) ? (i - 1) / 2 : i / 2 - 1;
  const bool ia0_on = ia >= 0 && ia < nc, ia1_on = ia + 1 >= 0 && ia + 1 < nc;
  const unsigned ca0 = (unsigned)min(max(ia, 0), nc - 1) * (unsigned)sizeof(T),
                 ca1 = (unsigned)min(max(ia + 1, 0), nc - 1) * (unsigned)sizeof(T);
  // coarse row K at columns ia, ia + 1 as loaded (clamped, unmasked) and the
  // masks that make them 0 outside the coarse grid
  auto load_c = [&](int K, T& c0, T& c1) {
    const int Kc_ = min(max(K, 0), nc - 1);
    const unsigned ko = (unsigned)Kc_ * (unsigned)nc * (unsigned)sizeof(T);
    c0 = xcb.ld(ca0, ko);
    c1 = xcb.ld(ca1, ko);
  };
  auto mask_c = [&](int K, T& c0, T& c1) {
    const bool kin = K >= 0 && K < nc;
    c0 = kin && ia0_on ? c0 : T(0);
    c1 = kin && ia1_on ? c1 : T(0);
  };
  // lowest coarse row of fine row t (odd t lies on it, even t halfway to the next)
  auto klo = [](int t) { return (t >> 1) - 1 + (t & 1); };
  const int t0 = y0 - (NS - 1), t1 = y1 + NS - 2;
  // registers: bh[d], fw[d], rd[d] = b, faces and inverse diagonal of row
  // t - d; xh[k][0], xh[k][1] = stage k's output at its newest row of the
  // previous step and the one below
  T bh[NS], xh[NS - 1][2], rd[NS];
  Faces fw[NS];
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    bh[d] = T(0);
    rd[d] = T(0);
    fw[d] = load_faces(t0 - 1 - d);
  }
#pragma unroll
  for (int k = 0; k < NS - 1; ++k) xh[k][0] = xh[k][1] = T(0);
  double dot = 0.0;
  ring_prologue_wait();
  __syncthreads();
  // the ring of row loads (see kRowLead): slot s of step t holds b and the
  // faces of row t and the coarse rows klo(r), klo(r) + 1 at columns ia,
  // ia + 1 for the row r = t - NU + 1 where P x_c is added, as loaded
  // (clamped, unmasked); a coarse row serves four fine steps and is loaded
  // for each (the repeats hit the cache)
  T rb[LEAD], rl0[LEAD], rl1[LEAD], rh0[LEAD], rh1[LEAD];
  Faces rf[LEAD];
  auto fill = [&](int t, int s) {
    rb[s] = bsb.ld(cb, (unsigned)crow(t) * rowb);
    rf[s] = load_faces(t);
    const int r = t - (NU - 1);
    load_c(klo(r), rl0[s], rl1[s]);
    load_c(klo(r) + 1, rh0[s], rh1[s]);
  };
#pragma unroll
  for (int s = 0; s < LEAD; ++s) fill(t0 + s, s);
  ring_march<LEAD>(t0, t1, [&](int t, auto slot) {
    constexpr int s = decltype(slot)::value;
#pragma unroll
    for (int d = NS - 1; d > 0; --d) {
      bh[d] = bh[d - 1];
      fw[d] = fw[d - 1];
      rd[d] = rd[d - 1];
    }
    if (VAR) fw[0] = Faces{ring_take(rf[s].l), ring_take(rf[s].r), ring_take(rf[s].d), ring_take(rf[s].u)};
    rd[0] = rdiag(fw[0], t);
    bh[0] = row_on(t) ? rb[s] : T(0);
    // P x_c on row r = t - NU + 1 (multilinear, the expressions of k_up2)
    const int r = t - (NU - 1);
    T lo0 = rl0[s], lo1 = rl1[s], hi0 = rh0[s], hi1 = rh1[s];
    mask_c(klo(r), lo0, lo1);
    mask_c(klo(r) + 1, hi0, hi1);
    // without a branch on the column's parity (odd and even columns share a
    // wave): an odd column counts its one coarse column twice, which the
    // weights 1/2 and 1/4 undo exactly
    const bool odd_col = i & 1;
    const T sl = lo0 + (odd_col ? lo0 : lo1), sh_ = hi0 + (odd_col ? hi0 : hi1);
    const T v = (r & 1) ? T(0.5) * sl : T(0.25) * (sl + sh_);
    // stage k on row t - k from stage k - 1's output (centre row in
    // sx[k - 1], below in xh, above just formed); the pre-sweeps are those
    // of the down kernel (zero start, the first one pointwise)
    T xn[NS];
    xn[0] = sweep_w(om, 0) * bh[0] * rd[0];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (k > 0) {
        const T w = k < NU ? sweep_w(om, k) : sweep_w(om, NS - 1 - k);
        xn[k] = relax(fw[k], sx[k - 1], xh[k - 1][0], xh[k - 1][1], xn[k - 1], bh[k], w, rd[k]);
      }
      if (k == NU - 1) xn[k] = row_on(r) ? xn[k] + v : T(0);   // x_pre + P x_c
    }
    const int g = t - (NS - 1);
    if (g >= y0 && g < y1 && col_on) {
      xsb.template st<true>(xn[NS - 1], ib, (unsigned)g * rowb);
      if (DOT) dot += (double)bh[NS - 1] * (double)xn[NS - 1];
    }
    __syncthreads();   // every read of this step's LDS rows is done
#pragma unroll
    for (int k = 0; k < NS - 1; ++k) sx[k][q] = xn[k];
    __syncthreads();
    fill(t + LEAD, s);   // refill the slot with row t + LEAD
#pragma unroll
    for (int k = 0; k < NS - 1; ++k) {
      xh[k][1] = xh[k][0];
      xh[k][0] = xn[k];
    }
  });
  if (DOT) {
    write_partial(partial, sys, dot, rt.seg, rt.nseg);
    finish(fin, partial, sys, rt.nseg);
  }
}

// --------------------------------------------------------------------------
// Fused 3D level kernels (constant coefficients), marching along z.  The 2D
// fused kernels stage a tile with a halo and run every sweep on it in LDS; in
// 3D a halo in z would cost about as much as the tile, so a workgroup owns an
// xy tile (with its halo) and walks up the planes with the stages lagging one
// plane behind each other.  At step t plane t enters; the first sweep (from
// x = 0 in the down kernel, the interpolated correction in the up kernel) is
// formed on it pointwise, and sweep m on plane t - m + 1 (down) or t - m (up).
// The newest plane of every stage goes into LDS for its in-plane neighbours;
// the planes above and below stay in registers.  A workgroup starts NU planes
// below its own (warm-up), so every plane it writes is exact; two barriers per
// plane.  Points off the grid (also planes below 0 and above n - 1) carry a
// zero right-hand side and a zero inverse diagonal, so they stay exactly 0,
// and the sweeps are branch-free as in the 2D kernels.
//
// k_down3: b (or, RUP, b_old - alpha (A + s) p formed on the fly, as in
// k_down2), NU sweeps from zero, the residual b - (A + s) x and its full
// weighting (the weights and order of k_restrict3); writes the pre-smoothed
// iterate on the owned fine planes and kD3Kz coarse planes of the coarse
// right-hand side.  One coarse column per thread.
// k_up3: x = x_in + P x_c (trilinear, as k_prolong3 along z), NU sweeps (the
// pre-smoothing weights reversed); writes the result on kU3Fz owned fine
// planes (and b.x when it is the finest level).
// --------------------------------------------------------------------------
constexpr int kD3Cx = 32, kD3Cy = 8, kD3Kz = 16;   // coarse columns and planes per workgroup (down)
constexpr int kU3Ox = 64, kU3Oy = 16, kU3Fz = 32;  // fine columns and planes per workgroup (up)
// 512 threads per workgroup: half the region points per thread of a
// 256-thread workgroup, so every sweep's planes fit in about 100 registers
// (FP32; 4 waves per SIMD instead of 2)
constexpr int kF3Threads = 512;
static_assert(kD3Cx * kD3Cy <= kF3Threads, "one coarse column per thread");

// (A + s) x at region point PAD + q from the in-plane values in LDS (row
// length RX) and the values below (xb) and above (xf): constant
// coefficients, the arithmetic and order of apply_col3
template <typename T>
__device__ __forceinline__ T lds_apply3(const T* X, int q, int RX, T xb, T xf, T w, T s) {
  const T xc = X[q];
  T sum = (xc - X[q - 1]) + (xc - X[q + 1]) + (xc - X[q - RX]) + (xc - X[q + RX]);
  sum += (xc - xb) + (xc - xf);
  return w * sum + s * xc;
}

// one damped Jacobi update at region point PAD + q (constant coefficients;
// xc = X[q], held in a register by the caller): x + w_m ((b + w times the
// six neighbours) r - x) with r the inverse diagonal (0 off the grid), equal
// to x + w_m (b - (A + s) x) r in exact arithmetic; 8 vector operations per
// point against 17
template <typename T>
__device__ __forceinline__ T lds_relax3(const T* X, int q, int RX, T xc, T xb, T xf, T w, T bb, T wm, T r) {
  T sum = (X[q - 1] + X[q + 1]) + (X[q - RX] + X[q + RX]);
  sum += xb + xf;
  return xc + wm * ((bb + w * sum) * r - xc);
}

template <typename T, int NU, bool RUP>
__global__ __launch_bounds__(kF3Threads) void k_down3(LevelDev<T> Lf, LevelDev<T> Lc, const T* __restrict__ b,
                                               T* __restrict__ xout, T* __restrict__ bc,
                                               const T* __restrict__ shift, const int* __restrict__ active,
                                               Sweeps<T> om, unsigned long long* __restrict__ ctr,
                                               const T* __restrict__ pv, const double* __restrict__ alpha,
                                               T* __restrict__ bout, double* __restrict__ partial, Fin fin) {
  constexpr int CX = kD3Cx, CY = kD3Cy;
  // the region: the owned fine columns with a halo of NU + 1; p (RUP) on
  // the region widened by one point, in a layout of its own
  constexpr int RX = 2 * CX + 2 * NU + 1, RY = 2 * CY + 2 * NU + 1, RN = RX * RY;
  constexpr int PX = RX + 2, PY = RY + 2, PN = PX * PY;
  constexpr int PER = (RN + kF3Threads - 1) / kF3Threads, PPER = RUP ? (PN + kF3Threads - 1) / kF3Threads : 1;
  constexpr int PAD = RX + 1, LX = PAD + PER * kF3Threads + RX + 1;
  constexpr int PADP = PX + 1, LP = RUP ? PADP + PPER * kF3Threads + PX + 1 : 1;
  __shared__ T sx[NU][LX];         // newest plane of each sweep's output
  __shared__ T sr[LX];             // residual plane
  __shared__ T sp[RUP ? 3 : 1][LP];   // p of planes z in slot z mod 3 (RUP): below, centre, above
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)Lf.N * sizeof(T) * (RUP ? 4 : 2) +
                                   (unsigned long long)Lc.N * sizeof(T));
  const int nf = Lf.n, nc = Lc.n;
  const int yt = (nc + CY - 1) / CY;
  const int kseg = tl.y / yt;
  const int I0 = tl.x * CX, J0 = (tl.y - kseg * yt) * CY;
  const int K0 = kseg * kD3Kz, K1 = min(K0 + kD3Kz, nc);
  const int fz1 = K1 == nc ? nf : 2 * K1;   // owned fine planes [2 K0, fz1) (the last segment: the top one too)
  const int gx0 = 2 * I0 - NU, gy0 = 2 * J0 - NU;
  const long long nn = (long long)nf * nf, off = (long long)sys * Lf.N;
  const T sh = shift[sys], w = Lf.wc;
  const T rcon = jacobi_recip(w * T(6) + sh);
  const T am = RUP ? (T)alpha[sys] : T(0);
  const int tid = threadIdx.x;
  // zero planes: the pads stay 0, the rest is written before a valid point reads it
  for (int i = tid; i < LX; i += kF3Threads) {
#pragma unroll
    for (int m = 0; m < NU; ++m) sx[m][i] = T(0);
    sr[i] = T(0);
  }
  if (RUP)
    for (int i = tid; i < LP; i += kF3Threads) sp[0][i] = sp[1][i] = sp[2][i] = T(0);
  __syncthreads();
  // region point u of this thread: on the grid in-plane (bit u of `in`),
  // owned (bit u of `own`), its in-plane offset clamped into the grid
  const int hx = (I0 + CX >= nc) ? nf : 2 * (I0 + CX);
  const int hy = (J0 + CY >= nc) ? nf : 2 * (J0 + CY);
  unsigned in = 0u, own = 0u;
  int col[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + kF3Threads * u;
    const int ry = q / RX, rx = q - ry * RX;
    const int gi = gx0 + rx, gj = gy0 + ry;
    const bool on = q < RN && gi >= 0 && gi < nf && gj >= 0 && gj < nf;
    in |= (on ? 1u : 0u) << u;
    own |= ((on && gi >= 2 * I0 && gi < hx && gj >= 2 * J0 && gj < hy) ? 1u : 0u) << u;
    col[u] = min(max(gj, 0), nf - 1) * nf + min(max(gi, 0), nf - 1);
  }
  const T* __restrict__ bs = b + off;
  const T* __restrict__ ps = RUP ? pv + off : nullptr;
  // p-layout point u of this thread: on the grid (bit u of `pin`), its clamped in-plane offset
  unsigned pin = 0u;
  int pcol[PPER];
#pragma unroll
  for (int u = 0; u < PPER; ++u) {
    const int q = tid + kF3Threads * u;
    const int py = q / PX, px = q - py * PX;
    const int gi = gx0 - 1 + px, gj = gy0 - 1 + py;
    pin |= ((RUP && q < PN && gi >= 0 && gi < nf && gj >= 0 && gj < nf) ? 1u : 0u) << u;
    pcol[u] = min(max(gj, 0), nf - 1) * nf + min(max(gi, 0), nf - 1);
  }
  // a plane z of p at this thread's p-layout points (0 off the grid)
  auto load_p = [&](int z, T* dst) {
    const bool zin = z >= 0 && z < nf;
    const long long base = (long long)min(max(z, 0), nf - 1) * nn;
#pragma unroll
    for (int u = 0; u < PPER; ++u) {
      const T v = ps[base + pcol[u]];
      dst[u] = (zin && ((pin >> u) & 1u)) ? v : T(0);
    }
  };
  auto slot = [](int z) { return ((z % 3) + 3) % 3; };
  // planes t0 .. t1 enter: the first written residual (fine plane 2 K0)
  // depends on the first sweep down to plane 2 K0 - NU; the last is the
  // residual of fine plane 2 K1
  const int t0 = 2 * K0 - NU, t1 = 2 * K1 + NU;
  // registers: bh[d] = b of plane t - d; xh[m][0], xh[m][1] = sweep m+1's
  // output at its newest plane of the previous step and the one below
  T bh[NU + 1][PER], xh[NU][2][PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
#pragma unroll
    for (int d = 0; d <= NU; ++d) bh[d][u] = T(0);
#pragma unroll
    for (int m = 0; m < NU; ++m) xh[m][0][u] = xh[m][1][u] = T(0);
  }
  if (RUP) {
    for (int z = t0 - 1; z <= t0 + 1; ++z) {
      T pl[PPER];
      load_p(z, pl);
#pragma unroll
      for (int u = 0; u < PPER; ++u) sp[slot(z)][PADP + tid + kF3Threads * u] = pl[u];
    }
  }
  // the coarse column of this thread: its centre fine point in the region and
  // the weighted in-plane sums of the residual on fine planes 2K and 2K + 1
  const bool restricts = tid < CX * CY;   // whole waves
  const int ci = tid % CX, cj = restricts ? tid / CX : 0;
  const bool mine = restricts && I0 + ci < nc && J0 + cj < nc;
  const int rcq = PAD + (2 * cj + NU) * RX + (2 * ci + NU);   // fine (2I, 2J) of its 3 x 3 block
  T s_lo = T(0), s_mid = T(0);
  const long long ncc = (long long)nc * nc;
  T* __restrict__ bcs = bc + (long long)sys * Lc.N + ((long long)(J0 + cj) * nc + (I0 + ci));
  T* __restrict__ xs = xout + off;
  T* __restrict__ bo = RUP ? bout + off : nullptr;
  double rr = 0.0;
  ring_prologue_wait();
  __syncthreads();
  // the ring of plane loads (see kRowLead; kPlaneLead planes ahead): slot s
  // of step t holds b of plane t and p of plane t + 2 (RUP), as loaded
  // (clamped planes, unmasked)
  T rbv[kPlaneLead][PER], rpv[kPlaneLead][RUP ? PPER : 1];
  auto fill = [&](int t, int s) {
    const long long bb = (long long)min(max(t, 0), nf - 1) * nn;
#pragma unroll
    for (int u = 0; u < PER; ++u) rbv[s][u] = bs[bb + col[u]];
    if (RUP) {
      const long long pb = (long long)min(max(t + 2, 0), nf - 1) * nn;
#pragma unroll
      for (int u = 0; u < PPER; ++u) rpv[s][u] = ps[pb + pcol[u]];
    }
  };
#pragma unroll
  for (int s = 0; s < kPlaneLead; ++s) fill(t0 + s, s);
  ring_march<kPlaneLead>(t0, t1, [&](int t, auto sl) {
    constexpr int s = decltype(sl)::value;
    const long long base = (long long)min(max(t, 0), nf - 1) * nn;
    // in-grid mask of plane g for point u (0 off the grid, above and below it)
    auto on_at = [&](int g, int u) { return g >= 0 && g < nf && ((in >> u) & 1u); };
#pragma unroll
    for (int d = NU; d > 0; --d)
#pragma unroll
      for (int u = 0; u < PER; ++u) bh[d][u] = bh[d - 1][u];
    const bool wr_t = RUP && t >= 2 * K0 && t < fz1;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      T bn = rbv[s][u];
      if (RUP) {
        const int q = tid + kF3Threads * u;
        const int ry = q / RX, rx = q - ry * RX;
        const int pq = PADP + (ry + 1) * PX + (rx + 1);
        bn = bn - am * lds_apply3<T>(sp[slot(t)], pq, PX, sp[slot(t - 1)][pq], sp[slot(t + 1)][pq], w, sh);
      }
      bh[0][u] = on_at(t, u) ? bn : T(0);
      if (wr_t && ((own >> u) & 1u)) {
        __builtin_nontemporal_store(bh[0][u], &bo[base + col[u]]);
        rr += (double)bh[0][u] * (double)bh[0][u];
      }
    }
    // sweep 1 on plane t from x = 0; sweep m + 1 on plane t - m from sweep
    // m's output (centre plane in sx[m - 1], below in xh, above just formed)
    T xn[NU][PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) xn[0][u] = sweep_w(om, 0) * bh[0][u] * (on_at(t, u) ? rcon : T(0));
#pragma unroll
    for (int m = 1; m < NU; ++m) {
      const T wm = sweep_w(om, m);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int q = PAD + tid + kF3Threads * u;
        xn[m][u] = lds_relax3<T>(sx[m - 1], q, RX, xh[m - 1][0][u], xh[m - 1][1][u], xn[m - 1][u], w, bh[m][u], wm,
                                 on_at(t - m, u) ? rcon : T(0));
      }
    }
    // the residual on plane t - NU
    T res[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = PAD + tid + kF3Threads * u;
      res[u] = bh[NU][u] - lds_apply3<T>(sx[NU - 1], q, RX, xh[NU - 1][1][u], xn[NU - 1][u], w, sh);
    }
    // the pre-smoothed iterate: sweep NU's newest plane t - NU + 1
    const int gx = t - NU + 1;
    if (gx >= 2 * K0 && gx < fz1) {
      const long long bx = (long long)gx * nn;
#pragma unroll
      for (int u = 0; u < PER; ++u)
        if ((own >> u) & 1u) __builtin_nontemporal_store(xn[NU - 1][u], &xs[bx + col[u]]);
    }
    __syncthreads();   // every read of this step's LDS planes is done
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = PAD + tid + kF3Threads * u;
#pragma unroll
      for (int m = 0; m < NU; ++m) sx[m][q] = xn[m][u];
      sr[q] = res[u];
    }
    if (RUP) {   // p(t + 2) takes the slot of p(t - 1) (0 off the grid)
      const bool zin = t + 2 >= 0 && t + 2 < nf;
#pragma unroll
      for (int u = 0; u < PPER; ++u)
        sp[slot(t + 2)][PADP + tid + kF3Threads * u] = (zin && ((pin >> u) & 1u)) ? rpv[s][u] : T(0);
    }
    __syncthreads();
    fill(t + kPlaneLead, s);   // refill the slot with the planes kPlaneLead steps ahead
    // full weighting: this coarse column's in-plane sum of fine plane f = t - NU,
    // and coarse plane K = f/2 - 1 once f = 2K + 2 (weights 1/4, 1/2, 1/4 along z)
    const int f = t - NU;
    if (restricts && f >= 2 * K0) {
      const T wt[3] = {T(0.25), T(0.5), T(0.25)};
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int di = q % 3, dj = q / 3;
        acc += wt[dj] * wt[di] * sr[rcq + dj * RX + di];
      }
      const bool odd = f & 1;
      if (!odd && f != 2 * K0) {
        const int K = f / 2 - 1;
        if (mine) bcs[K * ncc] = T(0.25) * s_lo + T(0.5) * s_mid + T(0.25) * acc;
      }
      // selects, not stores in two branches (see k_down2r)
      s_mid = odd ? acc : s_mid;
      s_lo = odd ? s_lo : acc;
    }
    // shift the registers one plane up
#pragma unroll
    for (int u = 0; u < PER; ++u) {
#pragma unroll
      for (int m = 0; m < NU; ++m) {
        xh[m][1][u] = xh[m][0][u];
        xh[m][0][u] = xn[m][u];
      }
    }
  });
  if (RUP) {
    write_partial_tile(tl, partial, sys, rr);
    finish(fin, partial, sys, gridDim.x * gridDim.y);
  }
}

template <typename T, int NU, bool DOT>
__global__ __launch_bounds__(kF3Threads) void k_up3(LevelDev<T> Lc, LevelDev<T> Lf, const T* __restrict__ xc,
                                             const T* __restrict__ xin, const T* __restrict__ b, T* __restrict__ xout,
                                             const T* __restrict__ shift, const int* __restrict__ active, Sweeps<T> om,
                                             double* __restrict__ partial, unsigned long long* __restrict__ ctr,
                                             Fin fin) {
  constexpr int OX = kU3Ox, OY = kU3Oy;
  constexpr int RX = OX + 2 * NU, RY = OY + 2 * NU, RN = RX * RY;
  constexpr int PER = (RN + kF3Threads - 1) / kF3Threads;
  constexpr int PAD = RX + 1, LX = PAD + PER * kF3Threads + RX + 1;
  // the coarse columns under the region, zero-padded: coarse index c at cx0 + (c - c0)
  constexpr int CRX = RX / 2 + 3, CRY = RY / 2 + 3, CRN = CRX * CRY;
  constexpr int CPER = (CRN + kF3Threads - 1) / kF3Threads;
  __shared__ T sx[NU][LX];   // newest plane of the correction and of sweeps 1 .. NU-1
  __shared__ T sc[CRN];      // one coarse plane under the region
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)Lf.N * sizeof(T) * 3 + (unsigned long long)Lc.N * sizeof(T));
  const int nf = Lf.n, nc = Lc.n;
  const int yt = (nf + OY - 1) / OY;
  const int zseg = tl.y / yt;
  const int ox0 = tl.x * OX, oy0 = (tl.y - zseg * yt) * OY;
  const int z0 = zseg * kU3Fz, z1 = min(z0 + kU3Fz, nf);
  const int gx0 = ox0 - NU, gy0 = oy0 - NU;
  const int cx0 = ((gx0 >= 0) ? gx0 / 2 : -((-gx0 + 1) / 2)) - 1;
  const int cy0 = ((gy0 >= 0) ? gy0 / 2 : -((-gy0 + 1) / 2)) - 1;
  const long long nn = (long long)nf * nf, off = (long long)sys * Lf.N, ncc = (long long)nc * nc;
  const T sh = shift[sys], w = Lf.wc;
  const T rcon = jacobi_recip(w * T(6) + sh);
  const int tid = threadIdx.x;
  // zero planes: the pads stay 0, the rest is written before a valid point reads it
  for (int i = tid; i < LX; i += kF3Threads) {
#pragma unroll
    for (int m = 0; m < NU; ++m) sx[m][i] = T(0);
  }
  unsigned in = 0u, own = 0u;
  int col[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + kF3Threads * u;
    const int ry = q / RX, rx = q - ry * RX;
    const int gi = gx0 + rx, gj = gy0 + ry;
    const bool on = q < RN && gi >= 0 && gi < nf && gj >= 0 && gj < nf;
    in |= (on ? 1u : 0u) << u;
    own |= ((on && rx >= NU && rx < NU + OX && ry >= NU && ry < NU + OY) ? 1u : 0u) << u;
    col[u] = min(max(gj, 0), nf - 1) * nf + min(max(gi, 0), nf - 1);
  }
  const T* __restrict__ xcs = xc + (long long)sys * Lc.N;
  const T* __restrict__ bs = b + off;
  const T* __restrict__ xis = xin + off;
  // coarse plane K under the region into sc (0 off the grid)
  auto stage = [&](int K) {
    const long long cb = (long long)min(max(K, 0), nc - 1) * ncc;
    T cl[CPER];
#pragma unroll
    for (int u = 0; u < CPER; ++u) {
      const int q = tid + kF3Threads * u;
      const int cy = q / CRX, cx = q - cy * CRX;
      cl[u] = xcs[cb + (long long)min(max(cy0 + cy, 0), nc - 1) * nc + min(max(cx0 + cx, 0), nc - 1)];
    }
#pragma unroll
    for (int u = 0; u < CPER; ++u) {
      const int q = tid + kF3Threads * u;
      if (q < CRN) {
        const int cy = q / CRX, cx = q - cy * CRX;
        const int I = cx0 + cx, J = cy0 + cy;
        sc[q] = (K >= 0 && K < nc && I >= 0 && I < nc && J >= 0 && J < nc) ? cl[u] : T(0);
      }
    }
  };
  // the in-plane interpolant of the staged coarse plane at region point u
  // (lanes past the region interpolate at its last point, in range of sc)
  auto interp = [&](int u) -> T {
    const int q = min(tid + kF3Threads * u, RN - 1);
    const int ry = q / RX, rx = q - ry * RX;
    const int gi = gx0 + rx, gj = gy0 + ry;
    const int ia = (gi & 1) ? (gi - 1) / 2 : gi / 2 - 1;
    const int ja = (gj & 1) ? (gj - 1) / 2 : gj / 2 - 1;
    const T* C = sc + (ja - cy0) * CRX + (ia - cx0);
    if (gi & 1) return (gj & 1) ? C[0] : T(0.5) * (C[0] + C[CRX]);
    return (gj & 1) ? T(0.5) * (C[0] + C[1]) : T(0.25) * (C[0] + C[1] + C[CRX] + C[CRX + 1]);
  };
  // lowest coarse plane of fine plane t (odd t lies on it, even t halfway to the next)
  auto klo = [](int t) { return (t >> 1) - 1 + (t & 1); };
  // planes t0 .. t1 enter: the owned plane z0 needs the correction down to z0 - NU
  const int t0 = z0 - NU, t1 = z1 + NU - 1;
  // vlo, vhi: the in-plane interpolants of coarse planes Kc and Kc + 1
  int Kc = klo(t0);
  T vlo[PER], vhi[PER];
  stage(Kc);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) vlo[u] = interp(u);
  __syncthreads();
  stage(Kc + 1);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) vhi[u] = interp(u);
  // registers: bh[d] = b of plane t - d; xh[m][0], xh[m][1] = stage m's
  // output (m = 0: the corrected x) at its newest plane of the previous step and
  // the one below
  T bh[NU + 1][PER], xh[NU][2][PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
#pragma unroll
    for (int d = 0; d <= NU; ++d) bh[d][u] = T(0);
#pragma unroll
    for (int m = 0; m < NU; ++m) xh[m][0][u] = xh[m][1][u] = T(0);
  }
  T* __restrict__ xs = xout + off;
  double dot = 0.0;
  ring_prologue_wait();
  __syncthreads();
  // the ring of plane loads (see kRowLead; kPlaneLead planes ahead): slot s
  // of step t holds x_in and b of plane t and the coarse plane klo(t + 1) + 1
  // under the region (staged at step t when klo(t + 1) > klo(t)), as loaded
  // (clamped, unmasked)
  T rxv[kPlaneLead][PER], rbv[kPlaneLead][PER], rcv[kPlaneLead][CPER];
  auto fill = [&](int t, int s) {
    const long long bb = (long long)min(max(t, 0), nf - 1) * nn;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      rxv[s][u] = xis[bb + col[u]];
      rbv[s][u] = bs[bb + col[u]];
    }
    const long long cb = (long long)min(max(klo(t + 1) + 1, 0), nc - 1) * ncc;
#pragma unroll
    for (int u = 0; u < CPER; ++u) {
      const int q = tid + kF3Threads * u;
      const int cy = q / CRX, cx = q - cy * CRX;
      rcv[s][u] = xcs[cb + (long long)min(max(cy0 + cy, 0), nc - 1) * nc + min(max(cx0 + cx, 0), nc - 1)];
    }
  };
#pragma unroll
  for (int s = 0; s < kPlaneLead; ++s) fill(t0 + s, s);
  ring_march<kPlaneLead>(t0, t1, [&](int t, auto sl) {
    constexpr int s = decltype(sl)::value;
    auto on_at = [&](int g, int u) { return g >= 0 && g < nf && ((in >> u) & 1u); };
    if (klo(t) > Kc) {   // sc holds coarse plane Kc + 2 (staged in the previous step)
      ++Kc;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        vlo[u] = vhi[u];
        vhi[u] = interp(u);
      }
    }
#pragma unroll
    for (int d = NU; d > 0; --d)
#pragma unroll
      for (int u = 0; u < PER; ++u) bh[d][u] = bh[d - 1][u];
    // stage 0 on plane t: x_in + P x_c; stage m on plane t - m
    T xn[NU + 1][PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const bool on = on_at(t, u);
      bh[0][u] = on ? rbv[s][u] : T(0);
      const T v = (t & 1) ? vlo[u] : T(0.5) * (vlo[u] + vhi[u]);
      xn[0][u] = on ? rxv[s][u] + v : T(0);
    }
#pragma unroll
    for (int m = 1; m <= NU; ++m) {
      const T wm = sweep_w(om, NU - m);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int q = PAD + tid + kF3Threads * u;
        xn[m][u] = lds_relax3<T>(sx[m - 1], q, RX, xh[m - 1][0][u], xh[m - 1][1][u], xn[m - 1][u], w, bh[m][u], wm,
                                 on_at(t - m, u) ? rcon : T(0));
      }
    }
    const int g = t - NU;
    if (g >= z0 && g < z1) {
      const long long bx = (long long)g * nn;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const bool o = (own >> u) & 1u;
        if (o) __builtin_nontemporal_store(xn[NU][u], &xs[bx + col[u]]);
        if (DOT) dot += o ? (double)bh[NU][u] * (double)xn[NU][u] : 0.0;
      }
    }
    __syncthreads();   // every read of this step's LDS planes is done
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = PAD + tid + kF3Threads * u;
#pragma unroll
      for (int m = 0; m < NU; ++m) sx[m][q] = xn[m][u];
    }
    if (klo(t + 1) > Kc) {   // coarse plane Kc + 2 into sc (0 off the grid)
      const int K = Kc + 2;
#pragma unroll
      for (int u = 0; u < CPER; ++u) {
        const int q = tid + kF3Threads * u;
        if (q < CRN) {
          const int cy = q / CRX, cx = q - cy * CRX;
          const int I = cx0 + cx, J = cy0 + cy;
          sc[q] = (K >= 0 && K < nc && I >= 0 && I < nc && J >= 0 && J < nc) ? rcv[s][u] : T(0);
        }
      }
    }
    __syncthreads();
    fill(t + kPlaneLead, s);   // refill the slot with the planes kPlaneLead steps ahead
#pragma unroll
    for (int u = 0; u < PER; ++u)
#pragma unroll
      for (int m = 0; m < NU; ++m) {
        xh[m][1][u] = xh[m][0][u];
        xh[m][0][u] = xn[m][u];
      }
  });
  if (DOT) {
    write_partial_tile(tl, partial, sys, dot);
    finish(fin, partial, sys, gridDim.x * gridDim.y);
  }
}

// --------------------------------------------------------------------------
// PCG pieces
// --------------------------------------------------------------------------
// p_new = z + beta p_old and q = (A+s) p_new in one pass (p_new formed at the
// stencil points on the fly); p_old and p_new are different buffers.
// XUP: also x += alpha_prev p_old, the iterate update of the previous PCG
// iteration, deferred to this pass which reads p_old anyway.  alpha == 0 marks
// "nothing pending" (first iteration); p_old is then not used.
//
// 3D version, marching along z with kMarchRows rows per thread: p_new =
// z + beta p_old is formed once per point; the rows' values below and at the
// point stay in registers.
template <typename T, bool VAR, bool XUP, bool WQ>
__global__ __launch_bounds__(kBlock) void k_spmv_p3(LevelDev<T> L, const T* __restrict__ z, const T* __restrict__ pold,
                                                    T* __restrict__ pnew, T* __restrict__ q,
                                                    const double* __restrict__ beta, const T* __restrict__ shift,
                                                    const int* __restrict__ active, double* __restrict__ partial,
                                                    unsigned long long* __restrict__ ctr, Fin fin,
                                                    T* __restrict__ x, const double* __restrict__ alpha) {
  constexpr int R = kMarchRows;
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  const T bt = (T)beta[sys];
  const T ap = XUP ? (T)alpha[sys] : T(0);
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * sizeof(T) *
                                ((bt == T(0) ? 3 : 4) - (WQ ? 0 : 1) + (XUP && ap != T(0) ? 2 : 0) +
                                 (VAR && sys == 0 ? 3 : 0)));
  const int n = L.n;
  const Column c = march_column(tl, n, R);
  double dot = 0.0;
  if (c.i < n && c.j < n) {
    const long long off = (long long)sys * L.N, nn = (long long)n * n;
    const Rows<R> w(c.i, c.j, n);
    const T* zs = z + off;
    // beta = 0 (first iteration): p_old may hold anything, so read z in its place
    const T* pe = bt == T(0) ? zs : pold + off;
    const T s = shift[sys];
    T below[R], centre[R], pold_c[R];   // pold_c: p_old at the point (alpha != 0 => beta != 0)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long p0 = c.k0 * nn + w.col[r];
      const long long pb = c.k0 > 0 ? p0 - nn : p0;
      const T zb = zs[pb], eb = pe[pb], zc = zs[p0], ec = pe[p0];
      below[r] = c.k0 > 0 ? zb + bt * eb : T(0);
      centre[r] = zc + bt * ec;
      pold_c[r] = ec;
    }
    for (int k = c.k0; k < c.k1; ++k) {
      const long long pk = k * nn;
      // every load of the plane first, then the arithmetic
      T za[R], ea[R], zl[R], el[R], zr[R], er[R], xv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long long p = pk + w.col[r];
        const long long pa = k + 1 < n ? p + nn : p;
        za[r] = zs[pa];
        ea[r] = pe[pa];
        zl[r] = zs[p + w.il];
        el[r] = pe[p + w.il];
        zr[r] = zs[p + w.ir];
        er[r] = pe[p + w.ir];
        xv[r] = XUP ? x[off + p] : T(0);
      }
      const T zd = zs[pk + w.col_d], ed = pe[pk + w.col_d], zu = zs[pk + w.col_u], eu = pe[pk + w.col_u];
      const T hd = zd + bt * ed, hu = zu + bt * eu;
      T above[R];
#pragma unroll
      for (int r = 0; r < R; ++r) above[r] = k + 1 < n ? za[r] + bt * ea[r] : T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!w.valid[r]) continue;
        const long long p = pk + w.col[r];
        const T lv = w.il ? zl[r] + bt * el[r] : T(0), rv = w.ir ? zr[r] + bt * er[r] : T(0);
        const T qv = apply_col3<T, VAR>(L, c.i, c.j + r, k, p, centre[r], lv, rv, w.down(r, centre, hd),
                                        w.up(r, centre, hu), below[r], above[r], s, nullptr);
        pnew[off + p] = centre[r];
        if (WQ) q[off + p] = qv;
        if (XUP && ap != T(0)) x[off + p] = xv[r] + ap * pold_c[r];
        dot += (double)centre[r] * (double)qv;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        below[r] = centre[r];
        centre[r] = above[r];
        pold_c[r] = ea[r];
      }
    }
  }
  write_partial_tile(tl, partial, sys, dot);
  finish(fin, partial, sys, gridDim.x * gridDim.y);
}

// 2D version: each thread owns R consecutive rows of one column (a workgroup
// of TX x (256 / TX) threads covers TX x (256 / TX) R points), so the column's p_new values are formed
// once and reused by the rows above and below; only the left/right neighbours
// are extra loads.
template <typename T, bool VAR, bool XUP, bool WQ, int R, int TX>
__global__ __launch_bounds__(kBlock) void k_spmv_p2(LevelDev<T> L, const T* __restrict__ z, const T* __restrict__ pold,
                                                    T* __restrict__ pnew, T* __restrict__ q,
                                                    const double* __restrict__ beta, const T* __restrict__ shift,
                                                    const int* __restrict__ active, double* __restrict__ partial,
                                                    unsigned long long* __restrict__ ctr, Fin fin,
                                                    T* __restrict__ x, const double* __restrict__ alpha) {
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active[sys]) return;
  const T bt = (T)beta[sys];
  const T ap = XUP ? (T)alpha[sys] : T(0);
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * sizeof(T) *
                                ((bt == T(0) ? 3 : 4) - (WQ ? 0 : 1) + (XUP && ap != T(0) ? 2 : 0) +
                                 (VAR && sys == 0 ? 2 : 0)));
  const int n = L.n;
  const int i = tl.x * TX + threadIdx.x;
  const int j0 = (tl.y * (kBlock / TX) + threadIdx.y) * R;
  const long long off = (long long)sys * L.N;
  double dot = 0.0;
  if (i < n && j0 < n) {
    const T* zs = z + off;
    // beta = 0 (first iteration): p_old may hold anything, so read z in its place
    const T* pe = bt == T(0) ? zs : pold + off;
    const T s = shift[sys];
    const int il = i > 0 ? i - 1 : i, ir = i < n - 1 ? i + 1 : i;
    // every load first (clamped rows/columns), then the arithmetic
    T zc[R + 2], pc[R + 2], zl[R], pl[R], zr[R], pr[R], xv[R];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
      const int jj = min(max(j0 - 1 + r, 0), n - 1);
      const long long g = (long long)jj * n + i;
      zc[r] = zs[g];
      pc[r] = pe[g];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long row = (long long)min(j0 + r, n - 1) * n;
      zl[r] = zs[row + il];
      pl[r] = pe[row + il];
      zr[r] = zs[row + ir];
      pr[r] = pe[row + ir];
      if (XUP) xv[r] = x[off + row + i];
    }
    T v[R + 2];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
      const int jj = j0 - 1 + r;
      v[r] = (jj >= 0 && jj < n) ? zc[r] + bt * pc[r] : T(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = j0 + r;
      if (j < n) {
        const T c = v[r + 1], dn = v[r], up = v[r + 2];
        const T lv = i > 0 ? zl[r] + bt * pl[r] : T(0);
        const T rv = i < n - 1 ? zr[r] + bt * pr[r] : T(0);
        T qv;
        if (!VAR) {
          qv = L.wc * ((c - lv) + (c - rv) + (c - dn) + (c - up)) + s * c;
        } else {
          const long long fx = (long long)j * (n + 1) + i;
          const long long fy = (long long)j * n + i;
          qv = L.wf0[fx] * (c - lv) + L.wf0[fx + 1] * (c - rv) + L.wf1[fy] * (c - dn) + L.wf1[fy + n] * (c - up) +
               s * c;
        }
        const long long g = off + (long long)j * n + i;
        __builtin_nontemporal_store(c, &pnew[g]);
        if (WQ) __builtin_nontemporal_store(qv, &q[g]);
        // the deferred update uses p_old = pc (pe is p_old whenever alpha != 0)
        if (XUP && ap != T(0)) __builtin_nontemporal_store(xv[r] + ap * pc[r + 1], &x[g]);
        dot += (double)c * (double)qv;
      }
    }
  }
  write_partial_tile(tl, partial, sys, dot);
  finish(fin, partial, sys, gridDim.x * gridDim.y);
}

// Row-marching version of k_spmv_p2 (launch-shape variant 3): one thread per
// grid column, a workgroup walks `rows` rows (a launch parameter); p_new of the rows below, at
// and above the current one stays in registers and the current row's p_new
// is in LDS for the left/right neighbours, so z and p_old are read once per
// point (plus one row above and below a segment).  Same values per point as
// k_spmv_p2; two barriers per row.

template <typename T, bool VAR, bool XUP, bool WQ>
__global__ __launch_bounds__(1024) void k_spmv_r2(LevelDev<T> L, const T* __restrict__ z, const T* __restrict__ pold,
                                                  T* __restrict__ pnew, T* __restrict__ q,
                                                  const double* __restrict__ beta, const T* __restrict__ shift,
                                                  const int* __restrict__ active, double* __restrict__ partial,
                                                  unsigned long long* __restrict__ ctr, Fin fin,
                                                  T* __restrict__ x, const double* __restrict__ alpha, int rows) {
  constexpr int LW = 1024 + 2;
  __shared__ T sp[LW];   // p_new of the current row, zero pads at columns -1 and blockDim.x
  const RowTile rt = row_tile();
  const int sys = rt.sys;
  if (!active[sys]) return;
  const T bt = (T)beta[sys];
  const T ap = XUP ? (T)alpha[sys] : T(0);
  count_bytes_row(rt, ctr, (unsigned long long)L.N * sizeof(T) *
                                ((bt == T(0) ? 3 : 4) - (WQ ? 0 : 1) + (XUP && ap != T(0) ? 2 : 0) +
                                 (VAR && sys == 0 ? 2 : 0)));
  const int n = L.n;
  const int i = threadIdx.x, NT = blockDim.x;
  const int j0 = rt.seg * rows, j1 = min(j0 + rows, n);
  const bool col_on = i < n;
  const int ic = min(i, n - 1);
  const int qi = 1 + i;
  const long long off = (long long)sys * L.N;
  const T* __restrict__ zs = z + off;
  // beta = 0 (first iteration): p_old may hold anything, so read z in its place
  const T* __restrict__ pe = bt == T(0) ? zs : pold + off;
  const unsigned cb = (unsigned)ic * (unsigned)sizeof(T), ib = (unsigned)i * (unsigned)sizeof(T);
  const unsigned rowb = (unsigned)n * (unsigned)sizeof(T);   // bytes per grid row
  const RowBuf<T> zsb(zs, L.N), peb(pe, L.N), xb(XUP ? x + off : zs, L.N), pnb(pnew + off, L.N), qb(WQ ? q + off : pnew + off, L.N);
  const RowBuf<T> w0b(VAR ? L.wf0 : zs, VAR ? (long long)(n + 1) * n : 1), w1b(VAR ? L.wf1 : zs, VAR ? (long long)(n + 1) * n : 1);
  const T s_ = shift[sys];
  if (i < 2) sp[i == 0 ? 0 : NT + 1] = T(0);
  auto crow = [&](int r) { return min(max(r, 0), n - 1); };
  // 1 on the grid, 0 off it: a factor rather than a select (a select lets the
  // compiler move a load into a branch and wait there for every load in flight)
  auto on_f = [&](int r) { return (col_on && r >= 0 && r < n) ? T(1) : T(0); };
  // p_new below and at row j0 (dn, c) and p_old at row j0 (pc)
  T dn, c, pc;
  {
    const int rb = crow(j0 - 1) * n + ic, rc = j0 * n + ic;
    const T zb = zs[rb], eb = pe[rb], zc = zs[rc], ec = pe[rc];
    dn = (zb + bt * eb) * on_f(j0 - 1);
    c = (zc + bt * ec) * on_f(j0);
    pc = ec;
  }
  sp[qi] = c;
  double dot = 0.0;
  ring_prologue_wait();
  __syncthreads();
  auto walk = [&](auto upd_c) {
    constexpr bool UPD = XUP && decltype(upd_c)::value;
    // the ring of row loads (see kRowLead): slot s of step j holds z and
    // p_old of row j + 1 and x and the faces of row j, as loaded (clamped
    // rows, unmasked)
    T rz[kRowLead], re[kRowLead], rx[kRowLead], rfl[kRowLead], rfr[kRowLead], rfd[kRowLead], rfu[kRowLead];
    auto fill = [&](int j, int s) {
      const unsigned ra = (unsigned)crow(j + 1) * rowb, rw = (unsigned)crow(j) * rowb;
      rz[s] = zsb.ld(cb, ra);
      re[s] = peb.ld(cb, ra);
      rx[s] = UPD ? xb.ld(cb, rw) : T(0);
      if (VAR) {
        const unsigned fx = (unsigned)crow(j) * (unsigned)(n + 1) * (unsigned)sizeof(T);
        rfl[s] = w0b.ld(cb, fx);
        rfr[s] = w0b.ld(cb + (unsigned)sizeof(T), fx);
        rfd[s] = w1b.ld(cb, rw);
        rfu[s] = w1b.ld(cb, rw + rowb);
      }
    };
#pragma unroll
    for (int s = 0; s < kRowLead; ++s) fill(j0 + s, s);
    ring_march(j0, j1 - 1, [&](int j, auto slot) {
      constexpr int s = decltype(slot)::value;
      const int row = j * n;   // 2D grids: fewer than 2^31 points
      const T up = (rz[s] + bt * re[s]) * on_f(j + 1);
      const T lv = sp[qi - 1], rv = sp[qi + 1];
      T qv;
      if (!VAR) qv = L.wc * ((c - lv) + (c - rv) + (c - dn) + (c - up)) + s_ * c;
      else qv = rfl[s] * (c - lv) + rfr[s] * (c - rv) + rfd[s] * (c - dn) + rfu[s] * (c - up) + s_ * c;
      if (col_on) {
        const unsigned g = (unsigned)row * (unsigned)sizeof(T);
        pnb.template st<true>(c, ib, g);
        if (WQ) qb.template st<true>(qv, ib, g);
        // the deferred update uses p_old = pc (pe is p_old whenever alpha != 0)
        if (UPD) xb.template st<true>(rx[s] + ap * pc, ib, g);
        dot += (double)c * (double)qv;
      }
      const T pn = ring_take(re[s]);   // p_old of row j + 1, the next step's pc
      __syncthreads();   // every read of this row's p_new is done
      sp[qi] = up;
      __syncthreads();
      fill(j + kRowLead, s);
      dn = c;
      c = up;
      pc = pn;
    });
  };
  if (XUP && ap != T(0)) walk(std::true_type{});
  else walk(std::false_type{});
  write_partial(partial, sys, dot, rt.seg, rt.nseg);
  finish(fin, partial, sys, rt.nseg);
}

// --------------------------------------------------------------------------
constexpr int kFlatItems = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_update_xr(long long N, T* __restrict__ x, T* __restrict__ r,
                                                   const T* __restrict__ pv, const T* __restrict__ q,
                                                   const double* __restrict__ alpha, const int* __restrict__ active,
                                                   double* __restrict__ partial, unsigned long long* __restrict__ ctr,
                                                   Fin fin) {
  const int sys = blockIdx.y;
  if (!active[sys]) return;
  count_bytes<COUNT_FLAT>(ctr, (unsigned long long)N * sizeof(T) * 6);
  const T a = (T)alpha[sys];
  const long long off = (long long)sys * N;
  const long long base = (long long)blockIdx.x * 256 * kFlatItems + threadIdx.x;
  double rr = 0.0;
  // all loads first (clamped index), then the updates and stores
  T xv[kFlatItems], pl[kFlatItems], rl[kFlatItems], ql[kFlatItems];
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) {
    const long long p = min(base + (long long)it * 256, N - 1);
    xv[it] = x[off + p];
    pl[it] = pv[off + p];
    rl[it] = r[off + p];
    ql[it] = q[off + p];
  }
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) {
    const long long p = base + (long long)it * 256;
    if (p < N) {
      x[off + p] = xv[it] + a * pl[it];
      const T rv = rl[it] - a * ql[it];
      r[off + p] = rv;
      rr += (double)rv * (double)rv;
    }
  }
  write_partial_flat(partial, sys, rr);
  finish(fin, partial, sys, gridDim.x);
}

// The deferred update of the last PCG iteration: x += alpha p_last, with
// p_last in pa when the system's iteration count is even and in pb otherwise
// (iteration c reads p_old from pa for even c and writes p_new to the other).
template <typename T>
__global__ __launch_bounds__(256) void k_finish_x(long long N, T* __restrict__ x, const T* __restrict__ pa,
                                                  const T* __restrict__ pb, const double* __restrict__ alpha,
                                                  const int* __restrict__ iters, unsigned long long* __restrict__ ctr) {
  const int sys = blockIdx.y;
  const int it = iters[sys];
  const T a = (T)alpha[sys];
  if (it <= 0 || a == T(0)) return;
  count_bytes<COUNT_FLAT>(ctr, (unsigned long long)N * sizeof(T) * 3);
  const T* pl = ((it - 1) & 1) ? pa : pb;
  const long long off = (long long)sys * N;
  const long long base = (long long)blockIdx.x * 256 * kFlatItems + threadIdx.x;
  T xv[kFlatItems], pv[kFlatItems];
#pragma unroll
  for (int k = 0; k < kFlatItems; ++k) {
    const long long p = min(base + (long long)k * 256, N - 1);
    xv[k] = x[off + p];
    pv[k] = pl[off + p];
  }
#pragma unroll
  for (int k = 0; k < kFlatItems; ++k) {
    const long long p = base + (long long)k * 256;
    if (p < N) x[off + p] = xv[k] + a * pv[k];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_update_p(long long N, T* __restrict__ pv, const T* __restrict__ z,
                                                  const double* __restrict__ beta, const int* __restrict__ active,
                                                  unsigned long long* __restrict__ ctr) {
  const int sys = blockIdx.y;
  if (!active[sys]) return;
  const T bt = (T)beta[sys];
  count_bytes<COUNT_FLAT>(ctr, (unsigned long long)N * sizeof(T) * (bt == T(0) ? 2 : 3));
  const long long off = (long long)sys * N;
  const long long base = (long long)blockIdx.x * 256 * kFlatItems + threadIdx.x;
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) {
    const long long p = base + (long long)it * 256;
    if (p < N) pv[off + p] = bt == T(0) ? z[off + p] : z[off + p] + bt * pv[off + p];
  }
}

// r = (T) f[rhs of system], x = 0, partial = ||r||^2 (FP64 from the FP64 input).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_rhs(long long N, const double* __restrict__ f, T* __restrict__ r,
                                                  T* __restrict__ x, int nrhs,
                                                  const int* __restrict__ active, double* __restrict__ partial) {
  const int sys = blockIdx.y;
  if (!active[sys]) return;
  const int rhs = sys % nrhs;
  const long long off = (long long)sys * N;
  const long long base = (long long)blockIdx.x * 256 * kFlatItems + threadIdx.x;
  double ff = 0.0;
  double fl[kFlatItems];
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) fl[it] = f[(long long)rhs * N + min(base + (long long)it * 256, N - 1)];
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) {
    const long long p = base + (long long)it * 256;
    if (p < N) {
      const double fv = fl[it];
      r[off + p] = (T)fv;
      x[off + p] = T(0);
      ff += fv * fv;
    }
  }
  write_partial_flat(partial, sys, ff);
}

// --------------------------------------------------------------------------
// FP64 refinement residual: r32 = f - (A + s) x64, e = 0, partial = ||r||^2
// --------------------------------------------------------------------------
// k_residual64 in 2D with the stencil product's layout: R rows per thread over
// TX columns, the column's values of the rows above and below from the
// thread's own registers, every load issued before the arithmetic (a
// one-point-per-thread launch reads each x value from the caches five times)
constexpr int kRes2Rows = 4, kRes2Cols = 128;
template <bool VAR>
__global__ __launch_bounds__(kBlock) void k_residual64_2(LevelDev<double> L, const double* __restrict__ f,
                                                         const double* __restrict__ x64, float* __restrict__ e,
                                                         float* __restrict__ r32, const double* __restrict__ shift,
                                                         const int* __restrict__ active64, int nrhs,
                                                         double* __restrict__ partial,
                                                         unsigned long long* __restrict__ ctr) {
  constexpr int R = kRes2Rows, TX = kRes2Cols;
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active64[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * (8 + 8 + 4 + 4 + (VAR && sys == 0 ? 16 : 0)));
  const int n = L.n;
  const int i = tl.x * TX + threadIdx.x;
  const int j0 = (tl.y * (kBlock / TX) + threadIdx.y) * R;
  double rr = 0.0;
  if (i < n && j0 < n) {
    const long long off = (long long)sys * L.N;
    const double* __restrict__ xs = x64 + off;
    const double* __restrict__ fs = f + (long long)(sys % nrhs) * L.N;
    const double s = shift[sys];
    const int il = i > 0 ? i - 1 : i, ir = i < n - 1 ? i + 1 : i;
    double xc[R + 2], xl[R], xr[R], fv[R];
    double wl[VAR ? R : 1], wr[VAR ? R : 1], wd[VAR ? R : 1], wu[VAR ? R : 1];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) xc[r] = xs[min(max(j0 - 1 + r, 0), n - 1) * n + i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int row = min(j0 + r, n - 1) * n;
      xl[r] = xs[row + il];
      xr[r] = xs[row + ir];
      fv[r] = fs[row + i];
      if (VAR) {
        const int jr = min(j0 + r, n - 1);
        const int fx = jr * (n + 1) + i, fy = jr * n + i;
        wl[VAR ? r : 0] = L.wf0[fx];
        wr[VAR ? r : 0] = L.wf0[fx + 1];
        wd[VAR ? r : 0] = L.wf1[fy];
        wu[VAR ? r : 0] = L.wf1[fy + n];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = j0 + r;
      if (j < n) {
        const double c = xc[r + 1];
        const double dn = j > 0 ? xc[r] : 0.0, up = j < n - 1 ? xc[r + 2] : 0.0;
        const double lv = i > 0 ? xl[r] : 0.0, rv = i < n - 1 ? xr[r] : 0.0;
        double ax;
        if (!VAR) {
          ax = L.wc * ((c - lv) + (c - rv) + (c - dn) + (c - up)) + s * c;
        } else {
          ax = wl[VAR ? r : 0] * (c - lv) + wr[VAR ? r : 0] * (c - rv) + wd[VAR ? r : 0] * (c - dn) +
               wu[VAR ? r : 0] * (c - up) + s * c;
        }
        const double rv64 = fv[r] - ax;
        const long long g = off + (long long)j * n + i;
        r32[g] = (float)rv64;
        e[g] = 0.0f;
        rr += rv64 * rv64;
      }
    }
  }
  write_partial_tile(tl, partial, sys, rr);
}

// Row-marching version of k_residual64_2 for wide launches: one thread per
// grid column, a workgroup walks kRes2rRows rows of one system with x64 of
// the rows below, at and above in registers and the current row in LDS, so
// x64 is read once per point (the 128 x 8 tiles read 1.25 - 1.5 times; 511^2,
// 2048 systems: 3290 -> 2890 us per launch).  Same values per point as
// k_residual64_2.
constexpr int kRes2rRows = 128;

// With UPD the kernel first applies the inner solve's correction, as
// k_x_from_e does (x64 += e, e taking the pending update e + alpha p when
// pa != nullptr), to every row it reads, and forms the residual of the
// updated iterate: one pass instead of two.  It writes the updated x64 and
// clears e on its own rows except the first and last one of its segment;
// those are the rows a neighbouring workgroup reads (with their old x64
// and e), and k_update_seg_rows updates and clears them after this kernel.
struct XUpdate {
  const float* pa;      // nullptr: e alone
  const float* pb;
  const double* alpha;
  const int* iters;
  int assign;           // x64 = e instead of x64 += e (x64 not read: the first update of a solve)
};
template <bool VAR, bool UPD>
__global__ __launch_bounds__(1024) void k_residual64_2r(LevelDev<double> L, const double* __restrict__ f,
                                                        double* __restrict__ x64, float* __restrict__ e,
                                                        float* __restrict__ r32, const double* __restrict__ shift,
                                                        const int* __restrict__ active64, int nrhs,
                                                        double* __restrict__ partial,
                                                        unsigned long long* __restrict__ ctr, XUpdate xu) {
  constexpr int LW = 1024 + 2;
  __shared__ double sx[LW];   // x64 of the current row, zero pads at columns -1 and blockDim.x
  const RowTile rt = row_tile();
  const int sys = rt.sys, seg = rt.seg;
  if (!active64[sys]) return;
  count_bytes_row(rt, ctr, (unsigned long long)L.N * (8 + 8 + 4 + 4 + (UPD ? 8 + 4 : 0) + (VAR && sys == 0 ? 16 : 0)));
  const int n = L.n;
  const int i = threadIdx.x, NT = blockDim.x;
  const int j0 = seg * kRes2rRows, j1 = min(j0 + kRes2rRows, n);
  const bool col_on = i < n;
  const int ic = min(i, n - 1), q = 1 + i;
  const long long off = (long long)sys * L.N;
  double* __restrict__ xs = x64 + off;
  const double* __restrict__ fs = f + (long long)(sys % nrhs) * L.N;
  const double sh = shift[sys];
  const unsigned cb = (unsigned)ic * 8u, rowb = (unsigned)n * 8u;
  const RowBuf<double> xsb(xs, L.N), fsb(fs, L.N);
  const RowBuf<double> w0b(VAR ? L.wf0 : xs, VAR ? (long long)(n + 1) * n : 1), w1b(VAR ? L.wf1 : xs, VAR ? (long long)(n + 1) * n : 1);
  const RowBuf<float> rb32(r32 + off, L.N), eb(e + off, L.N);
  // the pending update of the inner solve (UPD)
  const int its = UPD && xu.pa ? xu.iters[sys] : 0;
  const float a = UPD && xu.pa ? (float)xu.alpha[sys] : 0.0f;
  const bool pend = its > 0 && a != 0.0f;
  const float* pl = pend ? (((its - 1) & 1) ? xu.pa : xu.pb) + off : e + off;
  const RowBuf<float> plb(pl, L.N);
  if (i < 2) sx[i == 0 ? 0 : NT + 1] = 0.0;
  auto crow = [&](int r) { return min(max(r, 0), n - 1); };
  // 1 on the grid, 0 off it (a factor, not a select: see k_spmv_r2)
  auto on_f = [&](int r) { return (col_on && r >= 0 && r < n) ? 1.0 : 0.0; };
  // the iterate of a row from its loads (UPD: x64 + e, the arithmetic of k_x_from_e)
  auto xnew = [&](double xv, float ev, float pv) {
    if (!UPD) return xv;
    const float en = pend ? ev + a * pv : ev;
    return xv + (double)en;
  };
  const bool assign = UPD && xu.assign;
  auto ldrow = [&](int r) {
    const unsigned o = (unsigned)crow(r) * rowb, o4 = (unsigned)crow(r) * (unsigned)n * 4u;
    const double xv = assign ? 0.0 : xsb.ld(cb, o);
    const float ev = UPD ? eb.ld(cb / 2, o4) : 0.0f, pv = UPD && pend ? plb.ld(cb / 2, o4) : 0.0f;
    return xnew(xv, ev, pv) * on_f(r);
  };
  // x64 of rows j - 1, j, j + 1 during step j (dn, c, up); before the first
  // step c and up hold rows j0 - 1 and j0
  double dn = 0.0, c = ldrow(j0 - 1), up = ldrow(j0);
  sx[q] = up;
  double rr = 0.0;
  ring_prologue_wait();
  __syncthreads();
  // the ring of row loads (see kRowLead): slot s of step j holds x64 (UPD:
  // and e, p) of row j + 1 and f and the faces of row j, as loaded (clamped
  // rows, unmasked)
  double rx[kRowLead], rf[kRowLead], wl[kRowLead], wr[kRowLead], wd[kRowLead], wu[kRowLead];
  float re[kRowLead], rp[kRowLead];
  auto fill = [&](int j, int s) {
    const unsigned rw = (unsigned)crow(j) * rowb, ra = (unsigned)crow(j + 1) * rowb;
    rx[s] = assign ? 0.0 : xsb.ld(cb, ra);
    if (UPD) {
      re[s] = eb.ld(cb / 2, ra / 2);
      rp[s] = pend ? plb.ld(cb / 2, ra / 2) : 0.0f;
    }
    rf[s] = fsb.ld(cb, rw);
    if (VAR) {
      const unsigned fx = (unsigned)crow(j) * (unsigned)(n + 1) * 8u;
      wl[s] = w0b.ld(cb, fx);
      wr[s] = w0b.ld(cb + 8u, fx);
      wd[s] = w1b.ld(cb, rw);
      wu[s] = w1b.ld(cb, rw + rowb);
    }
  };
#pragma unroll
  for (int s = 0; s < kRowLead; ++s) fill(j0 + s, s);
  ring_march(j0, j1 - 1, [&](int j, auto slot) {
    constexpr int s = decltype(slot)::value;
    const int row = j * n;   // 2D grids: fewer than 2^31 points
    dn = c;
    c = up;
    up = xnew(rx[s], UPD ? re[s] : 0.0f, UPD ? rp[s] : 0.0f) * on_f(j + 1);
    const double lv = sx[q - 1], rv = sx[q + 1];
    double ax;
    if (!VAR) ax = L.wc * ((c - lv) + (c - rv) + (c - dn) + (c - up)) + sh * c;
    else ax = wl[s] * (c - lv) + wr[s] * (c - rv) + wd[s] * (c - dn) + wu[s] * (c - up) + sh * c;
    const double rv64 = rf[s] - ax;
    if (col_on) {
      const unsigned g = (unsigned)row * 4u, ib = (unsigned)i * 4u;
      rb32.template st<false>((float)rv64, ib, g);
      // UPD: the segment's first and last rows are left to k_update_seg_rows
      if (!UPD || (j != j0 && j != j1 - 1)) {
        eb.template st<false>(0.0f, ib, g);
        if (UPD) xsb.template st<false>(c, 2u * ib, 2u * g);
      }
      rr += rv64 * rv64;
    }
    __syncthreads();   // every read of row j's x64 is done
    sx[q] = up;
    __syncthreads();
    fill(j + kRowLead, s);
  });
  write_partial(partial, sys, rr, seg, rt.nseg);
}

// After k_residual64_2r<.., true>: x64 += e (with the pending update, as
// there) and e = 0 on the first and last row of every row segment.  One
// workgroup per system and such row, one thread per column.
__global__ __launch_bounds__(1024) void k_update_seg_rows(long long N, int n, double* __restrict__ x64,
                                                          float* __restrict__ e, const int* __restrict__ active64,
                                                          XUpdate xu) {
  const int sys = blockIdx.z;
  if (!active64[sys]) return;
  const int k = blockIdx.y;   // row 2 s or 2 s + 1 of segment s: its first or last row
  const int j0 = (k / 2) * kRes2rRows, j1 = min(j0 + kRes2rRows, n);
  const int j = (k & 1) ? j1 - 1 : j0;
  const int i = threadIdx.x;
  if (i >= n || ((k & 1) && j == j0)) return;   // a one-row segment: its row once
  const int its = xu.pa ? xu.iters[sys] : 0;
  const float a = xu.pa ? (float)xu.alpha[sys] : 0.0f;
  const bool pend = its > 0 && a != 0.0f;
  const long long g = (long long)sys * N + (long long)j * n + i;
  float en = e[g];
  if (pend) {
    const float* pl = ((its - 1) & 1) ? xu.pa : xu.pb;
    en = en + a * pl[g];
  }
  x64[g] = (xu.assign ? 0.0 : x64[g]) + (double)en;
  e[g] = 0.0f;
}

// the FP64 residual of a 2D batch of nsys systems walks whole rows when the
// other kernels do (levels of 255 - 1023 points, enough row segments)
static inline bool residual_rows(int dim, int n, long long nsys) {
  return dim == 2 && n >= kRowsMinN && n <= kRowsMaxN && nsys * ((n + kRes2rRows - 1) / kRes2rRows) >= kFillBlocks;
}

// k_residual64 in 3D, marching along z with kMarchRows rows per thread
template <bool VAR>
__global__ __launch_bounds__(kBlock) void k_residual64_3(LevelDev<double> L, const double* __restrict__ f,
                                                         const double* __restrict__ x64, float* __restrict__ e,
                                                         float* __restrict__ r32, const double* __restrict__ shift,
                                                         const int* __restrict__ active64, int nrhs,
                                                         double* __restrict__ partial,
                                                         unsigned long long* __restrict__ ctr) {
  constexpr int R = kMarchRows;
  const Tile tl = block_tile();
  const int sys = tl.z;
  if (!active64[sys]) return;
  count_bytes_tile(tl, ctr, (unsigned long long)L.N * (8 + 8 + 4 + 4 + (VAR && sys == 0 ? 8 * 3 : 0)));
  const int n = L.n;
  const Column c = march_column(tl, n, R);
  double rr = 0.0;
  if (c.i < n && c.j < n) {
    const long long off = (long long)sys * L.N, nn = (long long)n * n;
    const Rows<R> w(c.i, c.j, n);
    const double* xs = x64 + off;
    const double* fs = f + (long long)(sys % nrhs) * L.N;
    const double s = shift[sys];
    double below[R], centre[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long p0 = c.k0 * nn + w.col[r];
      const double xb0 = xs[c.k0 > 0 ? p0 - nn : p0];
      below[r] = c.k0 > 0 ? xb0 : 0.0;
      centre[r] = xs[p0];
    }
    for (int k = c.k0; k < c.k1; ++k) {
      const long long pk = k * nn;
      double xa[R], xl[R], xr[R], fv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long long p = pk + w.col[r];
        xa[r] = xs[k + 1 < n ? p + nn : p];
        xl[r] = xs[p + w.il];
        xr[r] = xs[p + w.ir];
        fv[r] = fs[p];
      }
      const double hd = xs[pk + w.col_d], hu = xs[pk + w.col_u];
      double above[R];
#pragma unroll
      for (int r = 0; r < R; ++r) above[r] = k + 1 < n ? xa[r] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!w.valid[r]) continue;
        const long long p = pk + w.col[r];
        const double ax = apply_col3<double, VAR>(L, c.i, c.j + r, k, p, centre[r], w.il ? xl[r] : 0.0,
                                                  w.ir ? xr[r] : 0.0, w.down(r, centre, hd), w.up(r, centre, hu),
                                                  below[r], above[r], s, nullptr);
        const double rv = fv[r] - ax;
        r32[off + p] = (float)rv;
        e[off + p] = 0.0f;
        rr += rv * rv;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        below[r] = centre[r];
        centre[r] = above[r];
      }
    }
  }
  write_partial_tile(tl, partial, sys, rr);
}

// first refinement step: x64 = 0 so r = f; partial = ||f||^2
// zero_x false: x64 is cleared only where f is 0 (a right-hand side that is
// 0 everywhere leaves its system inactive, and its x64 must read 0); the
// first x64 update of the refinement then assigns x64 = e instead of adding
__global__ __launch_bounds__(256) void k_first_residual(long long N, const double* __restrict__ f,
                                                        double* __restrict__ x64, float* __restrict__ e,
                                                        float* __restrict__ r32, int nrhs,
                                                        const int* __restrict__ active64,
                                                        double* __restrict__ partial, bool zero_x) {
  const int sys = blockIdx.y;
  if (!active64[sys]) return;
  const int rhs = sys % nrhs;
  const long long off = (long long)sys * N;
  const long long base = (long long)blockIdx.x * 256 * kFlatItems + threadIdx.x;
  double ff = 0.0;
  double fl[kFlatItems];
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) fl[it] = f[(long long)rhs * N + min(base + (long long)it * 256, N - 1)];
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) {
    const long long p = base + (long long)it * 256;
    if (p < N) {
      const double fv = fl[it];
      r32[off + p] = (float)fv;
      if (zero_x || fv == 0.0) x64[off + p] = 0.0;
      e[off + p] = 0.0f;
      ff += fv * fv;
    }
  }
  write_partial_flat(partial, sys, ff);
}

// x64 += e (final refinement update after the last inner solve)
// With pa != nullptr the inner solve's last deferred iterate update is
// applied here too (as k_finish_x would, in FP32 and the same expression):
// e + alpha p_last is formed in registers and never stored, one pass less.
__global__ __launch_bounds__(256) void k_x_from_e(long long N, const float* __restrict__ e, double* __restrict__ x64,
                                                  const int* __restrict__ active64, const float* __restrict__ pa,
                                                  const float* __restrict__ pb, const double* __restrict__ alpha,
                                                  const int* __restrict__ iters) {
  const int sys = blockIdx.y;
  if (!active64[sys]) return;
  const long long off = (long long)sys * N;
  const long long base = (long long)blockIdx.x * 256 * kFlatItems + threadIdx.x;
  const int its = pa ? iters[sys] : 0;
  const float a = pa ? (float)alpha[sys] : 0.0f;
  const bool pend = its > 0 && a != 0.0f;
  const float* pl = ((its - 1) & 1) ? pa : pb;
  double xl[kFlatItems];
  float el[kFlatItems], pv[kFlatItems];
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) {
    const long long p = min(base + (long long)it * 256, N - 1);
    xl[it] = x64[off + p];
    el[it] = e[off + p];
    pv[it] = pend ? pl[off + p] : 0.0f;
  }
#pragma unroll
  for (int it = 0; it < kFlatItems; ++it) {
    const long long p = base + (long long)it * 256;
    const float en = pend ? el[it] + a * pv[it] : el[it];
    if (p < N) x64[off + p] = xl[it] + (double)en;
  }
}

// u[r] = base_w base[r] + sum_j w_j x[j * stride + r], summed in the fixed order
// base, j = 0..nterms-1 (eq. (16); the base term serves the sequential forms).
// base may be u itself (each element is read before it is written).
// With pa != nullptr each system's last deferred iterate update is still
// pending and is applied here, as k_finish_x would (same expression), while x
// is read: x_j + alpha_j p_j, never stored (p = pa or pb by the parity of the
// system's iteration count).
__global__ __launch_bounds__(256) void k_combine(long long N, const double* x, const double* __restrict__ w,
                                                 int nterms, int stride, double* u, const double* base,
                                                 double base_w, unsigned long long* __restrict__ ctr, int wsys,
                                                 const double* __restrict__ pa, const double* __restrict__ pb,
                                                 const double* __restrict__ alpha, const int* __restrict__ iters) {
  const int r = blockIdx.y;
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  count_bytes<COUNT_FLAT>(ctr, (unsigned long long)N * 8ULL * (nterms * (pa ? 2 : 1) + 1 + (base ? 1 : 0)));
  if (p >= N) return;
  double acc = base ? base_w * base[(long long)r * N + p] : 0.0;
  for (int j = 0; j < nterms; ++j) {
    const long long sys = (long long)j * stride + r;
    const double wv = wsys ? w[sys] : w[j];
    // per-system weights: a zero weight marks an unused slot, whose x is not read
    if (wsys && wv == 0.0) continue;
    double xv = x[sys * N + p];
    if (pa) {
      const int it = iters[sys];
      const double a = alpha[sys];
      if (it > 0 && a != 0.0) xv = xv + a * (((it - 1) & 1) ? pa : pb)[sys * N + p];
    }
    acc += wv * xv;
  }
  u[(long long)r * N + p] = acc;
}

// Squared l2 norm of each row of u ([rows][N], FP64): per-block partials, then
// one block per row sums them in a fixed order (the result does not depend on
// which other rows share the launch).
__global__ __launch_bounds__(256) void k_row_norm2(const double* __restrict__ u, long long N,
                                                   double* __restrict__ partial) {
  const int r = blockIdx.y;
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  const double v = p < N ? u[(long long)r * N + p] : 0.0;
  write_partial(partial, r, v * v, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_row_sum(const double* __restrict__ partial, int nblk,
                                                 double* __restrict__ out) {
  const int r = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[(size_t)r * nblk + b];
  const double tot = block_sum(v);
  if (threadIdx.x == 0) out[r] = tot;
}

template <int DIM, bool VAR>
__global__ __launch_bounds__(kBlock) void k_apply64(LevelDev<double> L, const double* __restrict__ x,
                                                    double* __restrict__ y, double s) {
  const Tile tl = block_tile();
  const int v = tl.z;
  int i, j, k;
  tile_ijk<DIM>(tl, L.n, i, j, k);
  if (i >= L.n || j >= L.n) return;
  const long long off = (long long)v * L.N;
  const long long p = ((long long)k * L.n + j) * L.n + i;
  y[off + p] = apply_pt<double, DIM, VAR>(L, x + off, i, j, k, p, s, nullptr);
}

// --------------------------------------------------------------------------
// per-system scalar updates: one block per system sums the block partials in
// a fixed order, thread 0 advances that system's state.
// --------------------------------------------------------------------------
__device__ void apply_op(int op, double tot, const SysState& S, int sys, double tol, int max_iter) {
  switch (op) {
    case OP_INIT: {  // tot = ||b||^2 of the PCG right-hand side
      S.bnorm2[sys] = tot;
      S.iters[sys] = 0;
      S.relres[sys] = 1.0;
      S.beta[sys] = 0.0;
      S.alpha[sys] = 0.0;   // no deferred iterate update pending
      if (!(tot > 0.0)) {
        S.active[sys] = 0;
        if (!isfinite(tot)) S.flags[sys] |= 1;
        S.relres[sys] = 0.0;
      }
      break;
    }
    case OP_BETA: {  // tot = r.z
      if (S.iters[sys] == 0) {
        S.rho[sys] = tot;
        S.beta[sys] = 0.0;
      } else {
        S.beta[sys] = tot / S.rho[sys];
        S.rho[sys] = tot;
      }
      if (!isfinite(tot)) {
        S.flags[sys] |= 1;
        S.active[sys] = 0;
      }
      break;
    }
    case OP_ALPHA: {  // tot = p.q
      if (!(tot > 0.0) || !isfinite(tot)) {
        // p.q <= 0 only when the residual has vanished to rounding: stop here
        if (!isfinite(tot)) S.flags[sys] |= 1;
        S.active[sys] = 0;
        S.alpha[sys] = 0.0;
      } else {
        S.alpha[sys] = S.rho[sys] / tot;
      }
      break;
    }
    case OP_RESID: {  // tot = ||r||^2
      const int it = S.iters[sys] + 1;
      S.iters[sys] = it;
      S.total_iters[sys] += 1;
      const double rel = sqrt(tot / S.bnorm2[sys]);
      S.relres[sys] = rel;
      if (!isfinite(rel)) {
        S.flags[sys] |= 1;
        S.active[sys] = 0;
      } else if (rel <= (S.tol_inner ? S.tol_inner[sys] : S.tol_pcg ? S.tol_pcg[sys] : tol) || it >= max_iter) {
        S.active[sys] = 0;
      }
      break;
    }
    case OP_OUTER: {  // tot = ||f - (A+s) x64||^2 ; first call: x64 = 0 so tot = ||f||^2
      const int o = S.outer[sys];
      S.alpha[sys] = 0.0;   // the inner solve's deferred update has been applied (or is void)
      if (!isfinite(tot)) {
        S.flags[sys] |= 1;
        S.relres64[sys] = tot;
        S.active64[sys] = 0;
        S.active[sys] = 0;
        break;
      }
      if (o == 0) S.fnorm2[sys] = tot;
      const double fn = S.fnorm2[sys];
      const double rel = fn > 0.0 ? sqrt(tot / fn) : 0.0;
      S.relres64[sys] = rel;
      S.outer[sys] = o + 1;
      const double to = S.tol_outer ? S.tol_outer[sys] : tol;
      if (rel <= to || o >= max_iter) {
        S.active64[sys] = 0;
        S.active[sys] = 0;
      } else {
        S.active[sys] = 1;   // re-arm the inner solve on this residual
        S.bnorm2[sys] = tot;
        S.iters[sys] = 0;
        S.relres[sys] = 1.0;
        S.beta[sys] = 0.0;
        if (S.tol_inner) {
          // a step that can finish the system asks only for what is left
          const double want = 0.5 * to / rel;
          S.tol_inner[sys] = want > S.inner_floor ? want : S.inner_floor;
        }
      }
      break;
    }
  }
}

__global__ __launch_bounds__(256) void k_scalars(int op, const double* __restrict__ partial, int nblk, SysState S,
                                                 double tol, int max_iter) {
  const int sys = blockIdx.x;
  const bool inner = op != OP_OUTER;
  if (inner && !S.active[sys]) return;
  if (!inner && !S.active64[sys]) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[(size_t)sys * nblk + b];
  const double tot = block_sum(v);
  if (threadIdx.x != 0) return;
  apply_op(op, tot, S, sys, tol, max_iter);
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
// one point per thread (2D stencil kernels; 3D transfer operators)
static inline dim3 point_grid(int dim, int n, int nsys) {
  const int xt = (n + kTileX - 1) / kTileX;
  const int yt = (n + kTileY - 1) / kTileY;
  return dim3(xt, yt * (dim == 3 ? n : 1), nsys);
}

// 3D kernels marching along z: kMarchZ planes per workgroup, `rows` rows per thread
// Threads along x of a marching workgroup on a grid of n points per axis (the
// rest of the 256 along y).  Rows of n points are not aligned to 128-byte
// lines, so a wide row segment wastes a smaller share of its lines (255^3
// mixed: 64 -> 128 -> 256 columns took the solve from 39.9 to 37.4 to
// 36.5 ms); a narrow grid would leave most of a wide workgroup idle.
static inline int march_x(int n) { return n >= 192 ? 256 : (n >= 96 ? 128 : 64); }
static inline dim3 march_block(int n) { return dim3(march_x(n), kBlock / march_x(n)); }

static inline dim3 march_grid(int n, int nsys, int rows) {
  const int mx = march_x(n), my = kBlock / mx;
  const int xt = (n + mx - 1) / mx;
  const int yt = (n + my * rows - 1) / (my * rows);
  const int zt = (n + kMarchZ - 1) / kMarchZ;
  return dim3(xt, yt * zt, nsys);
}

// the smoothing sweeps, the stencil product and the FP64 residual (the kernels
// that write per-block partials outside the fused 2D path)
static inline dim3 stencil_grid(int dim, int n, int nsys) {
  return dim == 3 ? march_grid(n, nsys, kMarchRows) : point_grid(dim, n, nsys);
}
static inline dim3 stencil_block(int dim, int n) { return dim == 3 ? march_block(n) : dim3(kTileX, kTileY); }

int stencil_blocks(int dim, int n) {
  const dim3 g = stencil_grid(dim, n, 1);
  return (int)(g.x * g.y);
}

// the 2D stencil product: TX x ((256 / TX) R) points per workgroup
static inline dim3 spmv2_grid(int n, int nsys, int tv) {
  const int tx = kSpmvTile[tile_variant(tv)][1];
  const int rows = (kBlock / tx) * kSpmvTile[tile_variant(tv)][0];
  return dim3((n + tx - 1) / tx, (n + rows - 1) / rows, nsys);
}

int spmv_blocks(int dim, int n, int tv) {
  if (dim != 2) return stencil_blocks(dim, n);
  if (spmv_rows(dim, n, tv)) return (n + rows_seg(tv) - 1) / rows_seg(tv);
  const dim3 g = spmv2_grid(n, 1, tv);
  return (int)(g.x * g.y);
}

int flat_blocks(long long N) {
  const long long per = 256LL * kFlatItems;
  return (int)((N + per - 1) / per);
}

static inline dim3 flat_grid(long long N, int nsys) {
  const long long per = 256LL * kFlatItems;
  return dim3((unsigned)((N + per - 1) / per), nsys, 1);
}

// Calls f(std::integral_constant<int, v>) for the runtime variant tv.
template <typename F>
static inline void with_tile(int tv, F&& f) {
  static_assert(kTileVariants == 5, "one case per variant");
  switch (tile_variant(tv)) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
  }
}


bool tile_variant_distinct(int kind, int dim, int n, int tv) {
  (void)kind;
  const int v = tile_variant(tv);
  if (v != kRowsVariant && v != kShortRowsVariant) return true;
  return down_rows(dim, n, tv);
}

#define BURA_DISPATCH_DV(dim, var, KERNEL, ...)        \
  do {                                                 \
    if (dim == 2) {                                    \
      if (var) KERNEL(2, true, __VA_ARGS__);           \
      else KERNEL(2, false, __VA_ARGS__);              \
    } else {                                           \
      if (var) KERNEL(3, true, __VA_ARGS__);           \
      else KERNEL(3, false, __VA_ARGS__);              \
    }                                                  \
  } while (0)

template <typename T>
void Launch<T>::jacobi(int dim, bool var, const LevelDev<T>& L, const T* b, const T* xin, T* xout, const T* shift,
                       const int* active, T omega, bool zero_guess, double* partial, int nsys, hipStream_t st,
                       unsigned long long* ctr, Fin fin) {
  const dim3 g = stencil_grid(dim, L.n, nsys), blk = stencil_block(dim, L.n);
  const bool dot = partial != nullptr;
#define K_JAC(D, V, Z, DT)                                                                                      \
  do {                                                                                                          \
    if (D == 3)                                                                                                 \
      hipLaunchKernelGGL((k_jacobi3<T, V, Z, DT>), g, blk, 0, st, L, b, xin, xout, shift, active, omega, partial, \
                         ctr, fin);                                                                             \
    else                                                                                                        \
      hipLaunchKernelGGL((k_jacobi<T, 2, V, Z, DT>), g, blk, 0, st, L, b, xin, xout, shift, active, omega,       \
                         partial, ctr, fin);                                                                    \
  } while (0)
#define K_JAC4(D, V, dummy)                       \
  do {                                            \
    if (zero_guess) {                             \
      if (dot) K_JAC(D, V, true, true);           \
      else K_JAC(D, V, true, false);              \
    } else {                                      \
      if (dot) K_JAC(D, V, false, true);          \
      else K_JAC(D, V, false, false);             \
    }                                             \
  } while (0)
  BURA_DISPATCH_DV(dim, var, K_JAC4, 0);
#undef K_JAC4
#undef K_JAC
}

template <typename T>
void Launch<T>::jacobi_rup(int dim, bool var, const LevelDev<T>& L, const T* bold, const T* q, const double* alpha,
                           T* bout, T* xout, const T* shift, const int* active, T omega, double* partial, int nsys,
                           hipStream_t st, unsigned long long* ctr, Fin fin, const T* p) {
  const dim3 g = stencil_grid(dim, L.n, nsys), blk = stencil_block(dim, L.n);
  if (dim == 3 && !q) {   // q formed from p
    if (var)
      hipLaunchKernelGGL((k_jacobi0_rup3p<T, true>), g, blk, 0, st, L, bold, p, alpha, bout, xout, shift, active,
                         omega, partial, ctr, fin);
    else
      hipLaunchKernelGGL((k_jacobi0_rup3p<T, false>), g, blk, 0, st, L, bold, p, alpha, bout, xout, shift, active,
                         omega, partial, ctr, fin);
    return;
  }
#define K_JR(D, V, dummy)                                                                                         \
  hipLaunchKernelGGL((k_jacobi0_rup<T, D, V>), g, blk, 0, st, L, bold, q, alpha, bout, xout, shift, active, omega, \
                     partial, ctr, fin)
  BURA_DISPATCH_DV(dim, var, K_JR, 0);
#undef K_JR
}

template <typename T>
void Launch<T>::restrict_residual(int dim, bool var, const LevelDev<T>& Lf, const LevelDev<T>& Lc, const T* b,
                                  const T* x, T* bc, const T* shift, const int* active, int nsys, hipStream_t st,
                                  unsigned long long* ctr) {
  if (dim == 3) {
    const int nc = Lc.n;
    const dim3 g3((nc + kRcx - 1) / kRcx, ((nc + kRcy - 1) / kRcy) * ((nc + kMarchZ - 1) / kMarchZ), nsys);
    if (var) hipLaunchKernelGGL((k_restrict3<T, true>), g3, dim3(256), 0, st, Lf, Lc, b, x, bc, shift, active, ctr);
    else hipLaunchKernelGGL((k_restrict3<T, false>), g3, dim3(256), 0, st, Lf, Lc, b, x, bc, shift, active, ctr);
    return;
  }
  const dim3 g = point_grid(dim, Lc.n, nsys), blk(kTileX, kTileY);
#define K_RES(D, V, dummy) hipLaunchKernelGGL((k_restrict<T, D, V>), g, blk, 0, st, Lf, Lc, b, x, bc, shift, active, ctr)
  BURA_DISPATCH_DV(dim, var, K_RES, 0);
#undef K_RES
}

template <typename T>
void Launch<T>::prolong_add(int dim, const LevelDev<T>& Lc, const LevelDev<T>& Lf, const T* xc, T* xf,
                            const int* active, int nsys, hipStream_t st, unsigned long long* ctr) {
  if (dim == 2)
    hipLaunchKernelGGL((k_prolong<T, 2>), point_grid(2, Lf.n, nsys), dim3(kTileX, kTileY), 0, st, Lc, Lf, xc, xf,
                       active, ctr);
  else
    hipLaunchKernelGGL((k_prolong3<T>), march_grid(Lf.n, nsys, 1), march_block(Lf.n), 0, st, Lc, Lf, xc, xf,
                       active, ctr);
}

template <typename T>
void Launch<T>::coarse_solve(int dim, bool var, const LdsHierarchy<T>& H, const T* b, T* x, const T* shift,
                             const int* active, int nsys, size_t lds_bytes, hipStream_t st,
                             unsigned long long* ctr) {
  // 512 threads: the coarsest levels have few points per thread (63^2 has 8
  // at 512), and two workgroups per CU fit the LDS either way; against 1024
  // threads the 511^2 solve ran 0.8 % faster
  const dim3 g(nsys), blk(512);
#define K_CO(D, V, dummy) hipLaunchKernelGGL((k_coarse<T, D, V>), g, blk, lds_bytes, st, H, b, x, shift, active, ctr)
  BURA_DISPATCH_DV(dim, var, K_CO, 0);
#undef K_CO
}

template <typename T>
void Launch<T>::update_xr(const LevelDev<T>& L, int dim, T* x, T* r, const T* p, const T* q, const double* alpha,
                          const int* active, double* partial, int nsys, hipStream_t st, unsigned long long* ctr,
                          Fin fin) {
  (void)dim;
  hipLaunchKernelGGL((k_update_xr<T>), flat_grid(L.N, nsys), dim3(256), 0, st, L.N, x, r, p, q, alpha, active, partial,
                     ctr, fin);
}

template <typename T>
void Launch<T>::update_p(const LevelDev<T>& L, int dim, T* p, const T* z, const double* beta, const int* active,
                         int nsys, hipStream_t st, unsigned long long* ctr) {
  (void)dim;
  hipLaunchKernelGGL((k_update_p<T>), flat_grid(L.N, nsys), dim3(256), 0, st, L.N, p, z, beta, active, ctr);
}

template <typename T>
void Launch<T>::copy_rhs(const LevelDev<T>& L, int dim, const double* f, T* r, T* x, int nrhs, const int* active,
                         double* partial, int nsys, hipStream_t st) {
  (void)dim;
  // a batch is either all systems (sys = j * nrhs + r) or one pole (sys = r): rhs = sys % nrhs
  hipLaunchKernelGGL((k_copy_rhs<T>), flat_grid(L.N, nsys), dim3(256), 0, st, L.N, f, r, x, nrhs, active, partial);
}

template <typename T>
void Launch<T>::spmv_p(int dim, bool var, const LevelDev<T>& L, const T* z, const T* pold, T* pnew, T* q,
                       const double* beta, const T* shift, const int* active, double* partial, int nsys,
                       hipStream_t st, unsigned long long* ctr, Fin fin, T* x, const double* alpha, int tv) {
  const bool xup = x != nullptr;
  if (dim == 2 && spmv_rows(dim, L.n, tv)) {
    const int rows = rows_seg(tv);
    const dim3 g = rows_grid((L.n + rows - 1) / rows, nsys), blk(rows_threads(L.n));
#define K_SR(V, X_, Q_) \
  hipLaunchKernelGGL((k_spmv_r2<T, V, X_, Q_>), g, blk, 0, st, L, z, pold, pnew, q, beta, shift, active, partial, \
                     ctr, fin, x, alpha, rows)
    if (var) {
      if (!q) K_SR(true, true, false); else if (xup) K_SR(true, true, true); else K_SR(true, false, true);
    } else {
      if (!q) K_SR(false, true, false); else if (xup) K_SR(false, true, true); else K_SR(false, false, true);
    }
#undef K_SR
    return;
  }
  if (dim == 2) {
    const dim3 g2 = spmv2_grid(L.n, nsys, tv);
    with_tile(tv, [&](auto v) {
      constexpr int R = kSpmvTile[decltype(v)::value][0], TX = kSpmvTile[decltype(v)::value][1];
      const dim3 blk2(TX, kBlock / TX);
#define K_SP2(V, X_, Q_) \
  hipLaunchKernelGGL((k_spmv_p2<T, V, X_, Q_, R, TX>), g2, blk2, 0, st, L, z, pold, pnew, q, beta, shift, active, \
                     partial, ctr, fin, x, alpha)
      // q == nullptr: the product is only dotted with p (the fused down
      // kernel forms it again from p); that needs the deferred x update
      if (var) {
        if (!q) K_SP2(true, true, false); else if (xup) K_SP2(true, true, true); else K_SP2(true, false, true);
      } else {
        if (!q) K_SP2(false, true, false); else if (xup) K_SP2(false, true, true); else K_SP2(false, false, true);
      }
#undef K_SP2
    });
    return;
  }
  const dim3 g = march_grid(L.n, nsys, kMarchRows), blk = march_block(L.n);
#define K_SP3(V, X_, Q_)                                                                                          \
  hipLaunchKernelGGL((k_spmv_p3<T, V, X_, Q_>), g, blk, 0, st, L, z, pold, pnew, q, beta, shift, active, partial, \
                     ctr, fin, x, alpha)
  // q == nullptr: only p_new.q (the first fine sweep forms q from p_new)
  if (var) {
    if (!q) K_SP3(true, true, false); else if (xup) K_SP3(true, true, true); else K_SP3(true, false, true);
  } else {
    if (!q) K_SP3(false, true, false); else if (xup) K_SP3(false, true, true); else K_SP3(false, false, true);
  }
#undef K_SP3
}

template <typename T>
void Launch<T>::finish_x(long long N, T* x, const T* pa, const T* pb, const double* alpha, const int* iters,
                         int nsys, hipStream_t st, unsigned long long* ctr) {
  hipLaunchKernelGGL((k_finish_x<T>), flat_grid(N, nsys), dim3(256), 0, st, N, x, pa, pb, alpha, iters, ctr);
}

template <typename T>
bool Launch<T>::fused_down(int dim, bool var, int nu, const LevelDev<T>& Lf, const LevelDev<T>& Lc, const T* b,
                           T* xout, T* bc, const T* shift, const int* active, Sweeps<T> om, int nsys, hipStream_t st,
                           unsigned long long* ctr, const T* p, const double* alpha, T* bout, double* partial,
                           Fin fin, int tv, int tv_up) {
  const bool rup = bout != nullptr;
  if (dim == 3) {
    if (var || nu < 1 || nu > 2) return false;
    const dim3 g((Lc.n + kD3Cx - 1) / kD3Cx, ((Lc.n + kD3Cy - 1) / kD3Cy) * ((Lc.n + kD3Kz - 1) / kD3Kz), nsys);
#define K_D3(NU_, R_)                                                                                        \
  hipLaunchKernelGGL((k_down3<T, NU_, R_>), g, dim3(kF3Threads), 0, st, Lf, Lc, b, xout, bc, shift, active, om, ctr, \
                     p, alpha, bout, partial, fin)
    if (rup) {
      if (nu == 1) K_D3(1, true); else K_D3(2, true);
    } else {
      if (nu == 1) K_D3(1, false); else K_D3(2, false);
    }
#undef K_D3
    return true;
  }
  if (dim != 2 || nu < 1 || nu > 3) return false;
  if (down_rows(dim, Lf.n, tv)) {
    if (up_rows(dim, Lf.n, tv_up)) xout = nullptr;   // k_up2r forms the pre-smoothed iterate again
    const int ky = rows_seg(tv) / 2;
    const dim3 g = rows_grid((Lc.n + ky - 1) / ky, nsys), blk(rows_threads(Lf.n));
#define K_DR0(V, NU_, R_)                                                                                     \
  hipLaunchKernelGGL((k_down2r<T, V, NU_, R_>), g, blk, 0, st, Lf, Lc, b, xout, bc, shift, active, om, ctr, p, \
                     alpha, bout, partial, fin, ky)
#define K_DR(V, NU_) do { if (rup) K_DR0(V, NU_, true); else K_DR0(V, NU_, false); } while (0)
    if (var) {
      if (nu == 1) K_DR(true, 1); else if (nu == 2) K_DR(true, 2); else K_DR(true, 3);
    } else {
      if (nu == 1) K_DR(false, 1); else if (nu == 2) K_DR(false, 2); else K_DR(false, 3);
    }
#undef K_DR
#undef K_DR0
    return true;
  }
  with_tile(tv, [&](auto v) {
    constexpr int CX = kDownTile[decltype(v)::value][0], CY = kDownTile[decltype(v)::value][1];
    const dim3 g((Lc.n + CX - 1) / CX, (Lc.n + CY - 1) / CY, nsys), blk(256);
#define K_DN0(V, NU_, R_)                                                                                          \
  hipLaunchKernelGGL((k_down2<T, V, NU_, R_, CX, CY>), g, blk, 0, st, Lf, Lc, b, xout, bc, shift, active, om, ctr, \
                     p, alpha, bout, partial, fin)
#define K_DN(V, NU_) do { if (rup) K_DN0(V, NU_, true); else K_DN0(V, NU_, false); } while (0)
    if (var) {
      if (nu == 1) K_DN(true, 1); else if (nu == 2) K_DN(true, 2); else K_DN(true, 3);
    } else {
      if (nu == 1) K_DN(false, 1); else if (nu == 2) K_DN(false, 2); else K_DN(false, 3);
    }
#undef K_DN
#undef K_DN0
  });
  return true;
}

int down_blocks(int dim, int n, int tv) {
  const int nc = (n - 1) / 2;
  if (dim == 3)
    return ((nc + kD3Cx - 1) / kD3Cx) * ((nc + kD3Cy - 1) / kD3Cy) * ((nc + kD3Kz - 1) / kD3Kz);
  if (down_rows(dim, n, tv)) return (nc + rows_seg(tv) / 2 - 1) / (rows_seg(tv) / 2);
  const int cx = kDownTile[tile_variant(tv)][0], cy = kDownTile[tile_variant(tv)][1];
  return ((nc + cx - 1) / cx) * ((nc + cy - 1) / cy);
}

// The default shapes on a level of n points per axis when nsys systems share
// each launch.  The row-marching kernels (variant 3) fetch each point about
// once where the tiles fetch 1.3 - 1.8 times, but make one workgroup per
// system and segment of rows: on levels of at least kRowsMinN points per axis
// whose launches still make kFillBlocks of them they are the default (511^2,
// 2048 systems: stencil product 1286 -> 1105 us, down 1684 -> 1265, up 1351
// -> 811, the solve 107 -> 85 ms); with fewer systems (1023^2, 30 systems:
// 240 workgroups) or on small levels they are slower.  Otherwise the
// 64-column down tile (variant 0) fetches fewer halo lines but makes fewer
// workgroups than the 32 x 8 tile (variant 1): below about four per CU
// (one-system solves, coarse levels) variant 1 keeps more of the chip busy.

static inline bool rows_default(int dim, int n, long long nsys, int blocks) {
  return dim == 2 && n >= kRowsMinN && n <= kRowsMaxN && nsys * blocks >= kFillBlocks;
}

int default_down_tile(int dim, int n, long long nsys) {
  if (dim != 2) return 0;
  if (rows_default(dim, n, nsys, down_blocks(dim, n, kRowsVariant))) return kRowsVariant;
  return nsys * down_blocks(dim, n, 0) >= kFillBlocks ? 0 : 1;
}

int default_up_tile(int dim, int n, long long nsys) {
  return rows_default(dim, n, nsys, up_blocks(dim, n, kRowsVariant)) ? kRowsVariant : 0;
}

int default_spmv_tile(int dim, int n, long long nsys) {
  return rows_default(dim, n, nsys, spmv_blocks(dim, n, kRowsVariant)) ? kRowsVariant : 0;
}

template <typename T>
bool Launch<T>::fused_up(int dim, bool var, int nu, const LevelDev<T>& Lc, const LevelDev<T>& Lf, const T* xc,
                         const T* xin, const T* b, T* xout, const T* shift, const int* active, Sweeps<T> om,
                         double* partial, int nsys, hipStream_t st, unsigned long long* ctr, Fin fin, int tv) {
  const bool dot = partial != nullptr;
  if (dim == 3) {
    if (var || nu < 1 || nu > 2) return false;
    const dim3 g((Lf.n + kU3Ox - 1) / kU3Ox, ((Lf.n + kU3Oy - 1) / kU3Oy) * ((Lf.n + kU3Fz - 1) / kU3Fz), nsys);
#define K_U3(NU_, D_)                                                                                          \
  hipLaunchKernelGGL((k_up3<T, NU_, D_>), g, dim3(kF3Threads), 0, st, Lc, Lf, xc, xin, b, xout, shift, active, om, partial, \
                     ctr, fin)
    if (dot) {
      if (nu == 1) K_U3(1, true); else K_U3(2, true);
    } else {
      if (nu == 1) K_U3(1, false); else K_U3(2, false);
    }
#undef K_U3
    return true;
  }
  if (dim != 2 || nu < 1 || nu > 3) return false;
  if (up_rows(dim, Lf.n, tv)) {
    const int rows = rows_seg(tv);
    const dim3 g = rows_grid((Lf.n + rows - 1) / rows, nsys), blk(rows_threads(Lf.n));
#define K_UR0(V, NU_, D_)                                                                                        \
  hipLaunchKernelGGL((k_up2r<T, V, NU_, D_>), g, blk, 0, st, Lc, Lf, xc, xin, b, xout, shift, active, om, partial, \
                     ctr, fin, rows)
#define K_UR(V, NU_) do { if (dot) K_UR0(V, NU_, true); else K_UR0(V, NU_, false); } while (0)
    if (var) {
      if (nu == 1) K_UR(true, 1); else if (nu == 2) K_UR(true, 2); else K_UR(true, 3);
    } else {
      if (nu == 1) K_UR(false, 1); else if (nu == 2) K_UR(false, 2); else K_UR(false, 3);
    }
#undef K_UR
#undef K_UR0
    return true;
  }
  with_tile(tv, [&](auto v) {
    constexpr int OX = kUpTile[decltype(v)::value][0], OY = kUpTile[decltype(v)::value][1];
    const dim3 g((Lf.n + OX - 1) / OX, (Lf.n + OY - 1) / OY, nsys), blk(256);
#define K_UP(V, NU_, D_) \
  hipLaunchKernelGGL((k_up2<T, V, NU_, D_, OX, OY>), g, blk, 0, st, Lc, Lf, xc, xin, b, xout, shift, active, om,   \
                     partial, ctr, fin)
#define K_UPD(V, NU_) do { if (dot) K_UP(V, NU_, true); else K_UP(V, NU_, false); } while (0)
    if (var) {
      if (nu == 1) K_UPD(true, 1); else if (nu == 2) K_UPD(true, 2); else K_UPD(true, 3);
    } else {
      if (nu == 1) K_UPD(false, 1); else if (nu == 2) K_UPD(false, 2); else K_UPD(false, 3);
    }
#undef K_UPD
#undef K_UP
  });
  return true;
}

int up_blocks(int dim, int n, int tv) {
  if (dim == 3) return ((n + kU3Ox - 1) / kU3Ox) * ((n + kU3Oy - 1) / kU3Oy) * ((n + kU3Fz - 1) / kU3Fz);
  if (up_rows(dim, n, tv)) return (n + rows_seg(tv) - 1) / rows_seg(tv);
  const int ox = kUpTile[tile_variant(tv)][0], oy = kUpTile[tile_variant(tv)][1];
  return ((n + ox - 1) / ox) * ((n + oy - 1) / oy);
}

// the most blocks per system any reduction-writing launch shape can have
int max_partial_blocks(int dim, int n, long long N) {
  int m = std::max({stencil_blocks(dim, n), flat_blocks(N), residual_blocks(dim, n, 1)});
  for (int v = 0; v < kTileVariants; ++v)
    m = std::max({m, up_blocks(dim, n, v), down_blocks(dim, n, v), spmv_blocks(dim, n, v)});
  return m;
}

template struct Launch<float>;
template struct Launch<double>;

void launch_residual64(int dim, bool var, const LevelDev<double>& L, const double* f, const double* x64, float* e,
                       float* r32, const double* shift, const int* active64, double* partial, int nrhs, int nsys,
                       bool first, hipStream_t st, unsigned long long* ctr, bool zero_x) {
  if (first) {
    hipLaunchKernelGGL(k_first_residual, flat_grid(L.N, nsys), dim3(256), 0, st, L.N, f, const_cast<double*>(x64), e,
                       r32, nrhs, active64, partial, zero_x);
    return;
  }
  if (dim == 3) {
    const dim3 g = stencil_grid(dim, L.n, nsys), blk = stencil_block(dim, L.n);
    if (var)
      hipLaunchKernelGGL((k_residual64_3<true>), g, blk, 0, st, L, f, x64, e, r32, shift, active64, nrhs, partial, ctr);
    else
      hipLaunchKernelGGL((k_residual64_3<false>), g, blk, 0, st, L, f, x64, e, r32, shift, active64, nrhs, partial,
                         ctr);
  } else if (residual_rows(dim, L.n, nsys)) {
    const dim3 g = rows_grid((L.n + kRes2rRows - 1) / kRes2rRows, nsys), blk(rows_threads(L.n));
    double* x = const_cast<double*>(x64);   // not written without the update
    if (var)
      hipLaunchKernelGGL((k_residual64_2r<true, false>), g, blk, 0, st, L, f, x, e, r32, shift, active64, nrhs, partial,
                         ctr, XUpdate{});
    else
      hipLaunchKernelGGL((k_residual64_2r<false, false>), g, blk, 0, st, L, f, x, e, r32, shift, active64, nrhs,
                         partial, ctr, XUpdate{});
  } else {
    constexpr int rows_per_block = (kBlock / kRes2Cols) * kRes2Rows;
    const dim3 g2((L.n + kRes2Cols - 1) / kRes2Cols, (L.n + rows_per_block - 1) / rows_per_block, nsys);
    const dim3 b2(kRes2Cols, kBlock / kRes2Cols);
    if (var)
      hipLaunchKernelGGL((k_residual64_2<true>), g2, b2, 0, st, L, f, x64, e, r32, shift, active64, nrhs, partial, ctr);
    else
      hipLaunchKernelGGL((k_residual64_2<false>), g2, b2, 0, st, L, f, x64, e, r32, shift, active64, nrhs, partial,
                         ctr);
  }
}

bool residual_marches_rows(int dim, int n, long long nsys) { return residual_rows(dim, n, nsys); }

bool launch_update_residual64(int dim, bool var, const LevelDev<double>& L, const double* f, double* x64, float* e,
                              float* r32, const double* shift, const int* active64, double* partial, int nrhs,
                              int nsys, hipStream_t st, unsigned long long* ctr, const float* pa, const float* pb,
                              const double* alpha, const int* iters, bool assign) {
  if (!residual_rows(dim, L.n, nsys)) return false;
  const int nseg = (L.n + kRes2rRows - 1) / kRes2rRows;
  const dim3 g = rows_grid(nseg, nsys), blk(rows_threads(L.n));
  const XUpdate xu{pa, pb, alpha, iters, assign ? 1 : 0};
  if (var)
    hipLaunchKernelGGL((k_residual64_2r<true, true>), g, blk, 0, st, L, f, x64, e, r32, shift, active64, nrhs, partial,
                       ctr, xu);
  else
    hipLaunchKernelGGL((k_residual64_2r<false, true>), g, blk, 0, st, L, f, x64, e, r32, shift, active64, nrhs,
                       partial, ctr, xu);
  hipLaunchKernelGGL(k_update_seg_rows, dim3(1, 2 * nseg, nsys), blk, 0, st, L.N, L.n, x64, e, active64, xu);
  return true;
}

int residual_blocks(int dim, int n, long long nsys) {
  if (residual_rows(dim, n, nsys)) return (n + kRes2rRows - 1) / kRes2rRows;
  if (dim == 3) return stencil_blocks(dim, n);
  constexpr int rows_per_block = (kBlock / kRes2Cols) * kRes2Rows;
  return ((n + kRes2Cols - 1) / kRes2Cols) * ((n + rows_per_block - 1) / rows_per_block);
}

void launch_x_from_e(const LevelDev<double>& L, int dim, const float* e, double* x64, const int* active64, int nsys,
                     hipStream_t st, const float* pa, const float* pb, const double* alpha, const int* iters) {
  (void)dim;
  hipLaunchKernelGGL(k_x_from_e, flat_grid(L.N, nsys), dim3(256), 0, st, L.N, e, x64, active64, pa, pb, alpha,
                     iters);
}

void launch_combine(long long N, const double* x, const double* w, int nterms, int nrhs, int stride, double* u,
                    hipStream_t st, unsigned long long* ctr, const double* base, double base_w, bool w_per_system,
                    const double* pa, const double* pb, const double* alpha, const int* iters) {
  const dim3 g((unsigned)((N + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_combine, g, dim3(256), 0, st, N, x, w, nterms, stride, u, base, base_w, ctr,
                     w_per_system ? 1 : 0, pa, pb, alpha, iters);
}

void launch_row_norms(const double* u, long long N, int rows, double* partial, double* out, hipStream_t st) {
  const int nb = (int)((N + 255) / 256);
  hipLaunchKernelGGL(k_row_norm2, dim3(nb, rows), dim3(256), 0, st, u, N, partial);
  hipLaunchKernelGGL(k_row_sum, dim3(rows), dim3(256), 0, st, partial, nb, out);
}

void launch_apply64(int dim, bool var, const LevelDev<double>& L, const double* x, double* y, double shift, int nvec,
                    hipStream_t st) {
  const dim3 g = point_grid(dim, L.n, nvec), blk(kTileX, kTileY);
#define K_AP(D, V, dummy) hipLaunchKernelGGL((k_apply64<D, V>), g, blk, 0, st, L, x, y, shift)
  BURA_DISPATCH_DV(dim, var, K_AP, 0);
#undef K_AP
}

void launch_scalars(int op, const double* partial, int nblk, int nsys, SysState S, double tol, int max_iter,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_scalars, dim3(nsys), dim3(256), 0, st, op, partial, nblk, S, tol, max_iter);
}

// Terms of one right-hand-side slot of a slot plan (systems j R + slot,
// j < K): weights, shifts (FP64 and FP32), tolerances; resets the systems'
// counters and marks the used ones (j < nterms) in init.
__global__ void k_slot_terms(SlotTermsDev v, double* __restrict__ w, double* __restrict__ s64,
                             float* __restrict__ s32, double* __restrict__ tol, int* __restrict__ init,
                             int* __restrict__ total_iters, int* __restrict__ outer, int* __restrict__ flags,
                             int* __restrict__ active, int* __restrict__ active64) {
  const int j = threadIdx.x;
  if (j >= v.K) return;
  const long long sys = (long long)j * v.R + v.slot;
  const bool used = j < v.nterms;
  w[sys] = used ? v.w[j] : 0.0;
  s64[sys] = used ? v.s[j] : 0.0;
  if (s32) s32[sys] = used ? (float)v.s[j] : 0.0f;
  tol[sys] = v.tol;
  init[sys] = used ? 1 : 0;
  total_iters[sys] = 0;
  outer[sys] = 0;
  flags[sys] = 0;
  active[sys] = 0;
  active64[sys] = 0;
}

// active64 of the systems just initialised (their outer test ran on init)
__global__ void k_merge_init(int* __restrict__ init, int* __restrict__ active64, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (init[i]) {
    active64[i] = init[i];
    init[i] = 0;
  }
}

void launch_slot_terms(const SlotTermsDev& v, double* w, double* s64, float* s32, double* tol, int* init,
                       int* total_iters, int* outer, int* flags, int* active, int* active64, hipStream_t st) {
  hipLaunchKernelGGL(k_slot_terms, dim3(1), dim3(64), 0, st, v, w, s64, s32, tol, init, total_iters, outer, flags,
                     active, active64);
}

void launch_merge_init(int* init, int* active64, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_merge_init, dim3((n + 255) / 256), dim3(256), 0, st, init, active64, n);
}

__global__ void k_fill_int(int* __restrict__ p, long long n, int v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// flags of system j * R + r: 1 for r < nrhs, 0 otherwise
__global__ void k_slot_flags(int* __restrict__ p, int nterms, int R, int nrhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nterms * R) p[i] = (i % R) < nrhs ? 1 : 0;
}

void launch_slot_flags(int* p, int nterms, int R, int nrhs, hipStream_t st) {
  const int n = nterms * R;
  hipLaunchKernelGGL(k_slot_flags, dim3((n + 255) / 256), dim3(256), 0, st, p, nterms, R, nrhs);
}

void launch_fill_int(int* p, long long n, int v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

// Fill with zero bytes: 16-byte stores over the 16-byte-aligned body, single
// bytes for the unaligned head and tail.
__global__ void k_zero(unsigned char* p, size_t bytes) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t head = std::min<size_t>((16 - ((uintptr_t)p & 15)) & 15, bytes);
  const size_t words = (bytes - head) / 16;
  uint4* body = (uint4*)(p + head);
  for (size_t i = tid; i < words; i += stride) body[i] = make_uint4(0u, 0u, 0u, 0u);
  const size_t tail0 = head + words * 16;
  for (size_t i = tid; i < head + (bytes - tail0); i += stride) p[i < head ? i : tail0 + (i - head)] = 0;
}

// One read and one write of every byte: 16-byte vector accesses over the body,
// grid-stride over 2048 workgroups x 256 threads (8 per CU), bytes for the tail.
// One 16-byte word per thread and no loop: every wave has its load in flight
// at once.  On 2 GiB this reaches 6.1 TB/s; a grid-stride loop over 2048
// workgroups reached 4.7 TB/s (each wave then waits for one load at a time).
__global__ __launch_bounds__(256) void k_stream_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                     size_t words, unsigned char* __restrict__ dtail,
                                                     const unsigned char* __restrict__ stail, int tail) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) dst[i] = src[i];
  if (i < (size_t)tail) dtail[i] = stail[i];
}

void launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  const size_t words = bytes / 16;
  const int tail = (int)(bytes - words * 16);
  const size_t blocks = std::max<size_t>(1, (words + 255) / 256);
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st, (uint4*)dst, (const uint4*)src, words,
                     (unsigned char*)dst + words * 16, (const unsigned char*)src + words * 16, tail);
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  const size_t blocks = std::min<size_t>((bytes + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (unsigned char*)p, bytes);
}

}  // namespace bura
