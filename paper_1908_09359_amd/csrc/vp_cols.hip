// Column-wise boundaries for the vertical bonds (App. C's "similarly computed"
// read as 3-line networks between column boundary MPS): the vertical bond
// (y,x)-(y+1,x) is the horizontal bond (x,y)-(x,y+1) of the transposed lattice,
// site (y,x) -> (x,y) with legs (l,u,r,d) -> (u,l,d,r), the same state.  These
// kernels move tensors and configurations between the two lattices and join
// the transposed lattice's results to the row lattice's.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vp_kernels.hpp"

namespace vp {

namespace {

constexpr int CW = 256;

// T'_(x,y)[s][u][l][d][r] = T_(y,x)[s][l][u][r][d]; one work-group per site of
// the row lattice (offs / offs_t: each lattice's site offsets, dims: the row
// lattice's true leg dimensions).
__global__ void __launch_bounds__(CW) k_transpose_tensors(const double* __restrict__ T, double* __restrict__ Tt,
                                                          const int64_t* __restrict__ offs,
                                                          const int64_t* __restrict__ offs_t,
                                                          const int32_t* __restrict__ dims, int Ly, int Lx) {
  const int k = blockIdx.x;
  const int y = k / Lx, x = k - y * Lx;
  const int kt = x * Ly + y;
  const int dl = dims[4 * k], du = dims[4 * k + 1], dr = dims[4 * k + 2], dd = dims[4 * k + 3];
  const int n = dl * du * dr * dd;
  const double* src = T + offs[k];
  double* dst = Tt + offs_t[kt];
  for (int e = threadIdx.x; e < 2 * n; e += CW) {
    const int s = e / n;
    int r = e - s * n;  // ((l du + u) dr + rr) dd + d
    const int d = r % dd;
    r /= dd;
    const int rr = r % dr;
    r /= dr;
    const int u = r % du, l = r / du;
    dst[s * n + ((u * dl + l) * dd + d) * dr + rr] = src[e];
  }
}

// to_columns: t[c][x Ly + y] = s[c][y Lx + x]; otherwise the reverse.
__global__ void __launch_bounds__(CW) k_transpose_spins(const int8_t* __restrict__ s, int8_t* __restrict__ t,
                                                        int64_t n_chains, int Ly, int Lx, int to_columns) {
  const int N = Ly * Lx;
  const int64_t total = n_chains * N;
  for (int64_t i = blockIdx.x * (int64_t)CW + threadIdx.x; i < total; i += (int64_t)gridDim.x * CW) {
    const int64_t c = i / N;
    const int k = (int)(i - c * N);
    int j;
    if (to_columns) {
      const int y = k / Lx, x = k - y * Lx;
      j = x * Ly + y;
    } else {
      const int x = k / Ly, y = k - x * Ly;
      j = y * Lx + x;
    }
    t[c * N + j] = s[i];
  }
}

// Vertical ratios of the row lattice's pair order (after its Ly (Lx-1)
// horizontal pairs) from the transposed lattice's horizontal ratios.
__global__ void __launch_bounds__(CW) k_column_ratios(const double* __restrict__ rt, int npt, double* __restrict__ r,
                                                      int np, int n, int Ly, int Lx) {
  const int nv = (Ly - 1) * Lx, nh = Ly * (Lx - 1);
  const int64_t total = (int64_t)n * nv;
  for (int64_t i = blockIdx.x * (int64_t)CW + threadIdx.x; i < total; i += (int64_t)gridDim.x * CW) {
    const int64_t c = i / nv;
    const int v = (int)(i - c * nv), y = v / Lx, x = v - y * Lx;
    r[c * np + nh + v] = rt[c * npt + x * (Ly - 1) + y];
  }
}

// Knight bonds (y,x)-(y+2,x+1), y < Ly-2, x < Lx-1, of the row lattice's pair
// order (from base_r, row-major) from the transposed lattice's (x,y)-(x+1,y+2)
// bonds (from base_t, index x (Ly-2) + y).
__global__ void __launch_bounds__(CW) k_knight_ratios(const double* __restrict__ rt, int npt, int base_t,
                                                      double* __restrict__ r, int np, int base_r, int n, int Ly,
                                                      int Lx) {
  const int nk = (Ly - 2) * (Lx - 1);
  const int64_t total = (int64_t)n * nk;
  for (int64_t i = blockIdx.x * (int64_t)CW + threadIdx.x; i < total; i += (int64_t)gridDim.x * CW) {
    const int64_t c = i / nk;
    const int v = (int)(i - c * nk), y = v / (Lx - 1), x = v - y * (Lx - 1);
    r[c * np + base_r + v] = rt[c * npt + base_t + x * (Ly - 2) + y];
  }
}

__global__ void __launch_bounds__(CW) k_add_energy(double* __restrict__ e, int n_meas, int m,
                                                   const double* __restrict__ et, int n) {
  const int c = blockIdx.x * CW + threadIdx.x;
  if (c < n) e[(int64_t)c * n_meas + m] += et[c];
}

// out[c][0..1] (row stride `stride`) += the transposed lattice's (accepted, proposed)
__global__ void __launch_bounds__(CW) k_add_counts(const ChainMeta* __restrict__ b, int64_t* __restrict__ out,
                                                   int stride, int n) {
  const int c = blockIdx.x * CW + threadIdx.x;
  if (c < n) {
    out[(int64_t)stride * c] += b[c].accepted;
    out[(int64_t)stride * c + 1] += b[c].proposed;
  }
}

unsigned grid_of(int64_t n) {
  const int64_t b = (n + CW - 1) / CW;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

void launch_transpose_tensors(const double* T, double* Tt, const int64_t* offs, const int64_t* offs_t,
                              const int32_t* dims, int Ly, int Lx, hipStream_t s) {
  k_transpose_tensors<<<Ly * Lx, CW, 0, s>>>(T, Tt, offs, offs_t, dims, Ly, Lx);
}

void launch_transpose_spins(const int8_t* src, int8_t* dst, int n_chains, int Ly, int Lx, bool to_columns,
                            hipStream_t s) {
  if (n_chains <= 0) return;
  k_transpose_spins<<<grid_of((int64_t)n_chains * Ly * Lx), CW, 0, s>>>(src, dst, n_chains, Ly, Lx,
                                                                          to_columns ? 1 : 0);
}

void launch_column_ratios(const double* rt, int npt, double* r, int np, int n, int Ly, int Lx, hipStream_t s) {
  if (n <= 0 || Ly < 2) return;
  k_column_ratios<<<grid_of((int64_t)n * (Ly - 1) * Lx), CW, 0, s>>>(rt, npt, r, np, n, Ly, Lx);
}

void launch_knight_ratios(const double* rt, int npt, int base_t, double* r, int np, int base_r, int n, int Ly, int Lx,
                          hipStream_t s) {
  if (n <= 0 || Ly < 3 || Lx < 2) return;
  k_knight_ratios<<<grid_of((int64_t)n * (Ly - 2) * (Lx - 1)), CW, 0, s>>>(rt, npt, base_t, r, np, base_r, n, Ly, Lx);
}

void launch_add_energy(double* e, int n_meas, int m, const double* et, int n, hipStream_t s) {
  if (n <= 0) return;
  k_add_energy<<<(n + CW - 1) / CW, CW, 0, s>>>(e, n_meas, m, et, n);
}

void launch_add_counts(const ChainMeta* b, int64_t* out, int stride, int n, hipStream_t s) {
  if (n <= 0) return;
  k_add_counts<<<(n + CW - 1) / CW, CW, 0, s>>>(b, out, stride, n);
}

}  // namespace vp
