// Fused 3-line column step and 3-line defect tensor on the f32 / f64 16x16x4
// MFMA, for compile-time bond dimensions with D*D = 64 and D*Dc = 128
// (D = 8, Dc = 16).  Other shapes take the generic strided-GEMM path.
//
// Column step (App. B, the single-layer row network <D_{y+1}| M_y |U_{y-1}>):
//   Lout[b][r][e] = sum_{a,l,c,u,dd} Lin[a][l][c] A[a][u][b] t[l][u][r][dd] B[c][dd][e]
// computed per block of BB = Dc/4 upper-boundary indices b as three products
//   S1  X0[(l,c)][(u,bb)]  = sum_a      Lin[a][(l,c)]  A[a][(u,b0+bb)]
//   S2  X1[(c,bb)][(r,dd)] = sum_{l,u}  X0[(c,bb)][(l,u)] t[(l,u)][(r,dd)]
//   S3  Lout[(bb,r)][e]    = sum_{c,dd} X1[(bb,r)][(c,dd)] B[(c,dd)][e]
// The rows of Lin that a wave's S1 tiles need and the site-tensor columns of its
// S2 tile stay in registers for the whole step; X0 and X1 share one LDS buffer.
//
// Defect tensor (Sec. II.A Eq. (7), the environment of one site):
//   Out[l][u][r][dd] = sum_{a,b,c,e} Lp[a][l][c] A[a][u][b] Rn[b][r][e] B[c][dd][e]
// evaluated as sum_{c,b} P[l,c,u,b] Q[c,dd,b,r] with P = Lp.A (over a) and
// Q = B.Rn (over e), two lower-bond indices c at a time: D^4 Dc^2 + 2 D^2 Dc^3
// multiply-adds instead of the D^2 Dc^3 + D^3 Dc^3 + D^4 Dc^2 of contracting
// the legs one by one.
#pragma once

#include "vp_env4.hpp"

namespace vp {

template <int D, int C>
struct Env3Shape {
  static constexpr bool ok = D * D == 64 && D * C == 128;
  static constexpr int BB = C / 4, NBLK = 4;
  static constexpr int SA = C * D * C;   // one boundary-MPS site, staged in LDS
  // Row strides of the intermediates, chosen for the stores of the MFMA outputs:
  // the 16 lanes of a tile row write X0 at u P0 + bb (u, bb < 4) and X1 at
  // dd P1 + r (dd < 8, r < 2); P0 = 4 and P1 = 2 (mod 16) put them on distinct
  // banks (in float32 the next 16 lanes, four output rows on, land on the other
  // 16 banks).
  static constexpr int P0 = C * BB + 4;  // X0 rows (l,u), columns (c,bb)
  static constexpr int P1 = BB * D + 2;  // X1 rows (c,dd), columns (bb,r)
  static constexpr int SX = (D * D * P0 > C * D * P1) ? D * D * P0 : C * D * P1;
  static constexpr int SP = 2 * 256;     // split-K partial tiles of S3
  template <typename T>
  static constexpr size_t lds_bytes() { return sizeof(T) * (2 * SA + SX + SP); }
  // defect: A and Rn staged, P and Q of two lower-bond indices
  static constexpr int PQ = D * D + 1;
  template <typename T>
  static constexpr size_t defect_lds_bytes() { return sizeof(T) * (2 * SA + 2 * (2 * C) * PQ); }
};

template <typename T, int D, int C>
__device__ void env3_fused(T* __restrict__ Lout_p, const T* __restrict__ Lin_p, const T* __restrict__ A_p, S3 sA,
                           const T* __restrict__ t_p, S4 st, const T* __restrict__ B_p, S3 sB, char* lds) {
  auto* Lout = gmem(Lout_p);
  const auto* Lin = gmem(Lin_p);
  const auto* A = gmem(A_p);
  const auto* t = gmem(t_p);
  const auto* B = gmem(B_p);
  using Sh = Env3Shape<D, C>;
  static_assert(Sh::ok, "env3_fused: D*D = 64 and D*Dc = 128 only");
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  constexpr int BB = Sh::BB, P0 = Sh::P0, P1 = Sh::P1;
  T* As = reinterpret_cast<T*>(lds);
  T* Bs = As + Sh::SA;
  T* X = Bs + Sh::SA;
  T* Pp = X + Sh::SX;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q = lane >> 4, li = lane & 15;

  // registers: Lin rows (l,c) of S1 row tiles 2w and 2w+1, t columns of S2 tile w
  T lf[2][C / 4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int s = 0; s < C / 4; ++s) lf[mt][s] = Lin[(4 * s + q) * (D * C) + (2 * wave + mt) * 16 + li];
  T tf[D * D / 4];
  {
    const int j = 16 * wave + li, r = j / D, dd = j % D;
#pragma unroll
    for (int s = 0; s < D * D / 4; ++s) {
      const int k = 4 * s + q, l = k / D, u = k % D;
      tf[s] = t[l * st.l + u * st.u + r * st.r + dd * st.d];
    }
  }
  // boundary-MPS sites: A as [a][b-block][u][bb] (S1 columns contiguous), B as [c][dd][e]
  for (int e = tid; e < Sh::SA; e += WG) {
    const int p = e / (D * C), m = (e / C) % D, r = e % C;
    Bs[e] = B[p * sB.s0 + m * sB.s1 + r * sB.s2];
    const int rem = e % (D * C), blk = rem / (D * BB), u = (rem / BB) % D, b = blk * BB + rem % BB;
    As[e] = A[p * sA.s0 + u * sA.s1 + b * sA.s2];
  }
  __syncthreads();

  for (int blk = 0; blk < Sh::NBLK; ++blk) {
    const int b0 = blk * BB;
    {  // S1 -> X0 stored [(l,u)][(c,bb)]
      acc_t acc[2][2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < C / 4; ++s) {
        const int k = 4 * s + q;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const T b = As[k * (D * C) + b0 * D + nt * 16 + li];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) acc[mt][nt] = M::op(lf[mt][s], b, acc[mt][nt]);
        }
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = (2 * wave + mt) * 16 + M::row(lane, r), j = nt * 16 + li;
            const int l = i / C, c = i % C, u = j / BB, bb = j % BB;
            X[(l * D + u) * P0 + c * BB + bb] = acc[mt][nt][r];
          }
    }
    __syncthreads();
    // S2: rows (c,bb) in four tiles, columns (r,dd) of tile `wave`
    acc_t acc2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc2[mt] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < D * D / 4; ++s) {
      const int k = 4 * s + q;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc2[mt] = M::op(X[k * P0 + mt * 16 + li], tf[s], acc2[mt]);
    }
    __syncthreads();  // X0 consumed: X1 takes its place, stored [(c,dd)][(bb,r)]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = mt * 16 + M::row(lane, r), j = 16 * wave + li;
        const int c = i / BB, bb = i % BB, rr = j / D, dd = j % D;
        X[(c * D + dd) * P1 + bb * D + rr] = acc2[mt][r];
      }
    __syncthreads();
    {  // S3: row tile (wave & 1) of (bb,r), half (wave >> 1) of the (c,dd) sum
      constexpr int KH = C * D / 8;
      const int mt = wave & 1, kh = wave >> 1;
      acc_t a3 = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s2 = 0; s2 < KH; ++s2) {
        const int k = 4 * (kh * KH + s2) + q;
        a3 = M::op(X[k * P1 + mt * 16 + li], Bs[k * C + li], a3);
      }
      if (kh == 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) Pp[mt * 256 + M::row(lane, r) * 16 + li] = a3[r];
      __syncthreads();
      if (kh == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = mt * 16 + M::row(lane, r), bb = i / D, rr = i % D;
          Lout[((b0 + bb) * D + rr) * C + li] = a3[r] + Pp[mt * 256 + M::row(lane, r) * 16 + li];
        }
    }
  }
  __syncthreads();
}

// The optimal site of the variational boundary fit (App. B) for the same
// shapes: the 3-line network with its lower boundary site removed,
//   Mout[c][dd][e] = sum_{a,l,u,b,r} Lin[a][l][c] A[a][u][b] t[l][u][r][dd] Rn[b][r][e],
// as env3_fused's products S1 and S2 per block of BB upper-boundary indices b,
// then S3' Mout[(c,dd)][e] += sum_{bb,r} X1[(c,dd)][(bb,r)] Rn[(b0+bb,r)][e],
// accumulated over the blocks in registers (two row tiles per wavefront).
template <typename T, int D, int C>
__device__ void env3_center_fused(T* __restrict__ Mout_p, const T* __restrict__ Lin_p, const T* __restrict__ A_p,
                                  S3 sA, const T* __restrict__ t_p, S4 st, const T* __restrict__ Rn_p, char* lds) {
  auto* Mout = gmem(Mout_p);
  const auto* Lin = gmem(Lin_p);
  const auto* A = gmem(A_p);
  const auto* t = gmem(t_p);
  const auto* Rn = gmem(Rn_p);
  using Sh = Env3Shape<D, C>;
  static_assert(Sh::ok, "env3_center_fused: D*D = 64 and D*Dc = 128 only");
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  constexpr int BB = Sh::BB, P0 = Sh::P0, P1 = Sh::P1;
  T* As = reinterpret_cast<T*>(lds);
  T* Rs = As + Sh::SA;
  T* X = Rs + Sh::SA;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q = lane >> 4, li = lane & 15;

  T lf[2][C / 4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int s = 0; s < C / 4; ++s) lf[mt][s] = Lin[(4 * s + q) * (D * C) + (2 * wave + mt) * 16 + li];
  T tf[D * D / 4];
  {
    const int j = 16 * wave + li, r = j / D, dd = j % D;
#pragma unroll
    for (int s = 0; s < D * D / 4; ++s) {
      const int k = 4 * s + q, l = k / D, u = k % D;
      tf[s] = t[l * st.l + u * st.u + r * st.r + dd * st.d];
    }
  }
  // A as [a][b-block][u][bb] (S1 columns contiguous), Rn as [(b,r)][e]
  for (int e = tid; e < Sh::SA; e += WG) {
    const int p = e / (D * C);
    Rs[e] = Rn[e];
    const int rem = e % (D * C), blk = rem / (D * BB), u = (rem / BB) % D, b = blk * BB + rem % BB;
    As[e] = A[p * sA.s0 + u * sA.s1 + b * sA.s2];
  }
  __syncthreads();

  acc_t acc3[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) acc3[mt] = acc_t{0, 0, 0, 0};
  for (int blk = 0; blk < Sh::NBLK; ++blk) {
    const int b0 = blk * BB;
    {  // S1 -> X0 stored [(l,u)][(c,bb)]
      acc_t acc[2][2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < C / 4; ++s) {
        const int k = 4 * s + q;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const T b = As[k * (D * C) + b0 * D + nt * 16 + li];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) acc[mt][nt] = M::op(lf[mt][s], b, acc[mt][nt]);
        }
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = (2 * wave + mt) * 16 + M::row(lane, r), j = nt * 16 + li;
            const int l = i / C, c = i % C, u = j / BB, bb = j % BB;
            X[(l * D + u) * P0 + c * BB + bb] = acc[mt][nt][r];
          }
    }
    __syncthreads();
    // S2: rows (c,bb) in four tiles, columns (r,dd) of tile `wave`
    acc_t acc2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc2[mt] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < D * D / 4; ++s) {
      const int k = 4 * s + q;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc2[mt] = M::op(X[k * P0 + mt * 16 + li], tf[s], acc2[mt]);
    }
    __syncthreads();  // X0 consumed: X1 takes its place, stored [(c,dd)][(bb,r)]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = mt * 16 + M::row(lane, r), j = 16 * wave + li;
        const int c = i / BB, bb = i % BB, rr = j / D, dd = j % D;
        X[(c * D + dd) * P1 + bb * D + rr] = acc2[mt][r];
      }
    __syncthreads();
    // S3': row tiles 2w, 2w+1 of (c,dd), all e, the block's (bb,r) as the sum
#pragma unroll
    for (int s = 0; s < BB * D / 4; ++s) {
      const int k = 4 * s + q;
      const T b = Rs[(b0 * D + k) * C + li];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) acc3[mt] = M::op(X[((2 * wave + mt) * 16 + li) * P1 + k], b, acc3[mt]);
    }
    __syncthreads();  // X1 consumed before the next block's S1 stores
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) Mout[((2 * wave + mt) * 16 + M::row(lane, r)) * C + li] = acc3[mt][r];
  __syncthreads();
}

template <typename T, int D, int C>
__device__ void defect3_fused(T* __restrict__ Out_p, const T* __restrict__ Lp_p, const T* __restrict__ A_p, S3 sA,
                              const T* __restrict__ Rn_p, const T* __restrict__ B_p, S3 sB, char* lds) {
  auto* Out = gmem(Out_p);
  const auto* Lp = gmem(Lp_p);
  const auto* A = gmem(A_p);
  const auto* Rn = gmem(Rn_p);
  const auto* B = gmem(B_p);
  using Sh = Env3Shape<D, C>;
  static_assert(Sh::ok, "defect3_fused: D*D = 64 and D*Dc = 128 only");
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  constexpr int PQ = Sh::PQ;
  T* As = reinterpret_cast<T*>(lds);
  T* Rs = As + Sh::SA;          // Rn as [e][(b,r)]
  T* Pt = Rs + Sh::SA;          // [(cc,b)][(l,u)]
  T* Qt = Pt + 2 * C * PQ;      // [(cc,b)][(r,dd)]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q = lane >> 4, li = lane & 15;
  const int cc = li / D, lo = li % D;  // row (cc, l) of P and (cc, dd) of Q held by this lane

  for (int e = tid; e < Sh::SA; e += WG) {
    const int p = e / (D * C), m = (e / C) % D, r = e % C;
    As[e] = A[p * sA.s0 + m * sA.s1 + r * sA.s2];
    Rs[(e % C) * (C * D) + e / C] = Rn[e];
  }
  // A-operands of the P and Q products for one pair of lower-bond indices,
  // fetched one pair ahead
  T fp[C / 4], fq[C / 4], np[C / 4], nq[C / 4];
  auto fetch = [&](int c0, T* p, T* qv) {
#pragma unroll
    for (int s = 0; s < C / 4; ++s) {
      const int k = 4 * s + q;
      p[s] = Lp[(k * D + lo) * C + c0 + cc];
      qv[s] = B[(c0 + cc) * sB.s0 + lo * sB.s1 + k * sB.s2];
    }
  };
  fetch(0, fp, fq);
  acc_t acc[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) acc[mt] = acc_t{0, 0, 0, 0};
  __syncthreads();

  for (int c0 = 0; c0 < C; c0 += 2) {
    if (c0 + 2 < C) fetch(c0 + 2, np, nq);
    // P rows (cc,l), columns (u,b) of tiles 2w, 2w+1; Q rows (cc,dd), columns (b,r) of the same tiles
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int j = (2 * wave + nt) * 16 + li;
      acc_t ap = acc_t{0, 0, 0, 0}, aq = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < C / 4; ++s) {
        const int k = 4 * s + q;
        ap = M::op(fp[s], As[k * (D * C) + j], ap);
        aq = M::op(fq[s], Rs[k * (C * D) + j], aq);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = M::row(lane, r), c2 = i / D, o = i % D;
        const int pu = j / C, pb = j % C;  // P column (u, b)
        const int qb = j / D, qr = j % D;  // Q column (b, r)
        Pt[(c2 * C + pb) * PQ + o * D + pu] = ap[r];
        Qt[(c2 * C + qb) * PQ + qr * D + o] = aq[r];
      }
    }
    __syncthreads();
    // Out rows (l,u) in four tiles, columns (r,dd) of tile `wave`, sum over (cc,b)
#pragma unroll
    for (int s = 0; s < C / 2; ++s) {
      const int k = 4 * s + q;
      const T b = Qt[k * PQ + 16 * wave + li];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc[mt] = M::op(Pt[k * PQ + mt * 16 + li], b, acc[mt]);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < C / 4; ++s) {
      fp[s] = np[s];
      fq[s] = nq[s];
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) Out[(mt * 16 + M::row(lane, r)) * (D * D) + 16 * wave + li] = acc[mt][r];
  __syncthreads();
}

}  // namespace vp
