// Fused 2-row ("4-line") column step with bf16 operands, compile-time dimensions.
//
//   Lout[e][b][r1][r2] = sum Lin[c][a][l1][l2] A[a][u][b] t1[l1][u][r1][m]
//                             t2[l2][m][r2][dd] B[c][dd][e]
//
// Same contraction order as env4_fused (four pairwise products per block of BB
// upper-boundary indices and per lower-boundary index c, the last one
// accumulated across c in MFMA registers), but every operand lives in LDS as
// bf16 in the layout its MFMA consumes: k contiguous, rows of the contraction
// length rounded up to 8 (zero padded), so that each lane fetches its 8
// k-values of a 16x16x32 MFMA in one 16-byte read; k-groups past the
// contraction length are zero without a read.
// Products accumulate in f32; stage outputs are rounded to bf16 when stored
// for the next stage.  The first three products put the operand whose index
// runs fastest in the next stage's contraction (u, m, dd) on the MFMA's row
// side: a lane's four accumulator rows are then four consecutive elements of
// one destination row and go out in one 8-byte store (for D a multiple of 4).
// Row strides are 16-byte multiples chosen from measured LDS bank conflicts
// (64 banks of 4 bytes): a 16x16 operand tile's 16-byte reads are
// conflict-free over rows of 32 bytes (contraction length 16) and of 160
// bytes (length 64), and cost four cycles over 144-byte rows.
// Lin/Lout and the column tensors are in TS (float64 or float32) storage.
#pragma once
#include "vp_device.hpp"

namespace vp {

typedef __bf16 v8bf_e __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf_e __attribute__((ext_vector_type(4)));
typedef float v4f_e __attribute__((ext_vector_type(4)));

template <int D, int C>
struct Env4Bf {
  static constexpr int BB = (C % 4 == 0) ? C / 4 : ((C % 2 == 0) ? C / 2 : C);
  static constexpr int NBLK = C / BB;
  static constexpr int rup8(int x) { return (x + 7) / 8 * 8; }
  static constexpr int K1 = C, K2 = D * D, K3 = D * D, K4 = D;      // contraction lengths
  // row strides: Ls and AT unpadded, T1, T2 and X1 at 160 bytes for D = 8; X2
  // keeps 144-byte rows so that the step fits 40 KB (its reads pay the conflicts)
  static constexpr int P1 = rup8(K1), P2 = rup8(K2) + 16, P3 = rup8(K3) + 8, P4 = rup8(K4);
  static constexpr int PA = P1;                   // boundary tensor rows
  static constexpr int BS = D * P4 + 8;           // X3: stride of a block of D rows (bb, r1, .)
  static constexpr bool VEC = D % 4 == 0;         // four accumulator rows = four consecutive destination elements
  // X1 (read by S2 only) and X3 (written by S3) can share their buffer when no
  // zero padding is read (D a multiple of 8): at D = 8, C = 16 this keeps the
  // step under 40 KB of LDS, four work-groups per CU
  static constexpr bool ALIAS = D % 8 == 0;
  // operand arrays (bf16 elements); every array is a multiple of 8 elements long
  static constexpr int nAT = C * D * PA;          // [(b, u)][a]
  static constexpr int nLs = D * D * P1;          // [(l1, l2)][a]     (one lower-bond slice)
  static constexpr int nT1 = D * D * P2;          // [(r1, m)][(l1, u)]
  static constexpr int nT2 = D * D * P2;          // [(r2, dd)][(l2, m)]
  static constexpr int nBT = C * C * P4;          // [(c, e)][dd]
  static constexpr int nX1 = BB * D * P2;         // [(bb, l2)][(l1, u)]
  static constexpr int nX2 = BB * D * P3;         // [(bb, r1)][(l2, m)]
  static constexpr int nX3 = BB * D * BS;         // [(bb, r1)] blocks of [r2][dd]
  static constexpr int nX = ALIAS ? (nX1 > nX3 ? nX1 : nX3) + nX2 : nX1 + nX2 + nX3;  // the intermediates
  static constexpr int N4 = BB * D * D;           // output columns per block
  static constexpr int NT4 = (N4 + 15) / 16;
  static constexpr int T4W = (NT4 + 3) / 4;
  static constexpr size_t lds_bytes() {
    return 2 * (size_t)(nAT + nLs + nT1 + nT2 + nBT + nX);
  }
};

// 8 bf16 of a row from k0 on; zero past the contraction length K (rows are
// zero padded to a multiple of 8).
__device__ inline v8bf_e ld8(const __bf16* row, int k0, int K) {
  const v8bf_e z = {};
  return k0 < K ? *reinterpret_cast<const v8bf_e*>(row + k0) : z;
}

// 16x16 output tile of A (M x K, row stride PA) times B^T (N x K, row stride
// PB), both bf16 in LDS.
template <int K>
__device__ inline v4f_e bf_tile(const __bf16* A, int PA, const __bf16* B, int PB, int m0, int n0, int M, int N) {
  v4f_e acc = {0, 0, 0, 0};
  const int lane = threadIdx.x & 63;
  const int i = min(m0 + (lane & 15), M - 1), j = min(n0 + (lane & 15), N - 1), kq = (lane >> 4) * 8;
#pragma unroll
  for (int s = 0; s < (K + 31) / 32; ++s) {
    const v8bf_e a = ld8(A + i * PA, 32 * s + kq, K);
    const v8bf_e b = ld8(B + j * PB, 32 * s + kq, K);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// One stage over MT x NT output tiles: a wave's tiles t = wave + 4 w are all
// multiplied (tile(m0, n0) -> accumulator) before any is stored
// (store(m0, n0, acc)); a store into LDS could alias the operands, so storing
// each tile at once would hold back the next tile's reads.
template <int MT, int NT, typename FT, typename FS>
__device__ inline void bf_stage(FT tile, FS store) {
  constexpr int NTW = (MT * NT + 3) / 4;
  const int wave = threadIdx.x >> 6;
  v4f_e c[NTW];
#pragma unroll
  for (int w = 0; w < NTW; ++w) {
    const int t = min(wave + 4 * w, MT * NT - 1);  // a wave without a last tile repeats one, unstored
    c[w] = tile((t / NT) * 16, (t % NT) * 16);
  }
#pragma unroll
  for (int w = 0; w < NTW; ++w) {
    const int t = wave + 4 * w;
    if (t < MT * NT) store((t / NT) * 16, (t % NT) * 16, c[w]);
  }
}

template <int D, int C, typename TS>
__device__ void env4_bf16(TS* __restrict__ Lout_p, const TS* __restrict__ Lin_p, const TS* __restrict__ A_p, S3 sA,
                          const TS* __restrict__ t1_p, S4 s1, const TS* __restrict__ t2_p, S4 s2,
                          const TS* __restrict__ B_p, S3 sB, char* lds) {
  auto* Lout = gmem(Lout_p);
  const auto* Lin = gmem(Lin_p);
  const auto* A = gmem(A_p);
  const auto* t1 = gmem(t1_p);
  const auto* t2 = gmem(t2_p);
  const auto* B = gmem(B_p);
  using S = Env4Bf<D, C>;
  constexpr int BB = S::BB;
  __bf16* AT = reinterpret_cast<__bf16*>(lds);
  __bf16* Ls = AT + S::nAT;
  __bf16* T1 = Ls + S::nLs;
  __bf16* T2 = T1 + S::nT1;
  __bf16* BT = T2 + S::nT2;
  __bf16* X2 = BT + S::nBT;
  __bf16* X1 = X2 + S::nX2;
  __bf16* X3 = S::ALIAS ? X1 : X1 + S::nX1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const __bf16 zero = (__bf16)0.0f;

  // stage the column tensors once, transposed to k-contiguous rows; zero the
  // padding of every array (the intermediates' padding is never written later)
  for (int e = tid; e < S::nAT; e += WG) {
    const int row = e / S::PA, a = e - row * S::PA, b = row / D, u = row - b * D;  // row = (b, u)
    AT[e] = a < C ? (__bf16)(float)A[a * sA.s0 + u * sA.s1 + b * sA.s2] : zero;
  }
  for (int e = tid; e < S::nT1; e += WG) {
    const int row = e / S::P2, k = e - row * S::P2;  // row = (r1, m), k = (l1, u)
    const int r = row / D, m = row - r * D, l = k / D, u = k - l * D;
    T1[e] = k < D * D ? (__bf16)(float)t1[l * s1.l + u * s1.u + r * s1.r + m * s1.d] : zero;
  }
  for (int e = tid; e < S::nT2; e += WG) {
    const int row = e / S::P2, k = e - row * S::P2;  // row = (r2, dd), k = (l2, m)
    const int r = row / D, dd = row - r * D, l = k / D, m = k - l * D;
    T2[e] = k < D * D ? (__bf16)(float)t2[l * s2.l + m * s2.u + r * s2.r + dd * s2.d] : zero;
  }
  for (int e = tid; e < S::nBT; e += WG) {
    const int row = e / S::P4, dd = e - row * S::P4, c = row / C, ee = row - c * C;
    BT[e] = dd < D ? (__bf16)(float)B[c * sB.s0 + dd * sB.s1 + ee * sB.s2] : zero;
  }
  for (int e = tid; e < S::nX; e += WG) X2[e] = zero;
  for (int e = tid; e < S::nLs; e += WG) Ls[e] = zero;

  // lower-bond slices of Lin ([a][(l1,l2)], contiguous) are read coalesced one
  // slice ahead into registers, so their global-memory latency overlaps the
  // previous slice's products, and transposed into Ls when stored.  QUAD: a
  // thread holds four consecutive a of one row (l1,l2) and stores them in one
  // 8-byte write (single 2-byte writes of the transpose would put eight lanes
  // on each bank); each of its four reads is still coalesced across the row.
  constexpr int SL = C * D * D;
  constexpr bool QUAD = C % 4 == 0 && (C / 4) * D * D <= WG;
  constexpr int NPF = QUAD ? 4 : (SL + WG - 1) / WG;
  const int qrow = tid % (D * D), qa = 4 * (tid / (D * D));
  const bool qok = tid < (C / 4) * D * D;
  float pre[NPF];
  auto fetch = [&](int cs) {
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      if constexpr (QUAD) {
        pre[u] = qok ? (float)Lin[cs * SL + (qa + u) * (D * D) + qrow] : 0.0f;
      } else {
        const int e = tid + u * WG;
        pre[u] = e < SL ? (float)Lin[cs * SL + e] : 0.0f;
      }
    }
  };
  // slices in the order (block, slice); the next one is stored into Ls as soon
  // as S1 of the current one has read it, so a slice costs four barriers
  auto store = [&]() {
    if constexpr (QUAD) {
      if (qok) {
        const v4bf_e v = {(__bf16)pre[0], (__bf16)pre[1], (__bf16)pre[2], (__bf16)pre[3]};
        *reinterpret_cast<v4bf_e*>(Ls + qrow * S::P1 + qa) = v;  // 8-byte aligned: P1 % 8 == 0
      }
    } else {
#pragma unroll
      for (int u = 0; u < NPF; ++u) {
        const int e = tid + u * WG, a = e / (D * D), row = e - a * (D * D);  // row = (l1, l2)
        if (e < SL) Ls[row * S::P1 + a] = (__bf16)pre[u];
      }
    }
  };
  constexpr int NS = S::NBLK * C;
  fetch(0);
  __syncthreads();  // staging (and the zeroing of Ls) done
  store();
  if (NS > 1) fetch(1 % C);
  __syncthreads();
  for (int q = 0; q < S::NBLK; ++q) {
    const int b0 = q * BB;
    v4f_e acc[S::T4W];
#pragma unroll
    for (int w = 0; w < S::T4W; ++w) acc[w] = {0, 0, 0, 0};
    for (int cs = 0; cs < C; ++cs) {
      const int pos = q * C + cs;
      // S1: X1[(bb,l2)][(l1,u)] = sum_a AT[(b0+bb, u)][a] Ls[(l1,l2)][a]; M = BB D (rows (bb,u)), N = D^2
      bf_stage<(BB * D + 15) / 16, (D * D + 15) / 16>(
          [&](int m0, int n0) { return bf_tile<S::K1>(AT + b0 * D * S::PA, S::PA, Ls, S::P1, m0, n0, BB * D, D * D); },
          [&](int m0, int n0, const v4f_e& c4) {
            const int i = n0 + (lane & 15), j0 = m0 + 4 * (lane >> 4);  // column (l1, l2), rows (bb, u0 + r)
            if (i >= D * D) return;
            const int l1 = i / D, l2 = i - l1 * D;
            if constexpr (S::VEC) {
              if (j0 < BB * D) {
                const int bb = j0 / D, u0 = j0 - bb * D;
                const v4bf_e v = {(__bf16)c4[0], (__bf16)c4[1], (__bf16)c4[2], (__bf16)c4[3]};
                *reinterpret_cast<v4bf_e*>(X1 + (bb * D + l2) * S::P2 + l1 * D + u0) = v;
              }
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int j = j0 + r, bb = j / D, u = j - bb * D;
                if (j < BB * D) X1[(bb * D + l2) * S::P2 + l1 * D + u] = (__bf16)c4[r];
              }
            }
          });
      __syncthreads();
      if (pos + 1 < NS) {  // Ls is free: the next slice goes in
        store();
        if (pos + 2 < NS) fetch((pos + 2) % C);
      }
      // S2: X2[(bb,r1)][(l2,m)] = sum_{(l1,u)} T1[(r1,m)][(l1,u)] X1[(bb,l2)][(l1,u)]; M = D^2 (rows (r1,m)), N = BB D
      bf_stage<(D * D + 15) / 16, (BB * D + 15) / 16>(
          [&](int m0, int n0) { return bf_tile<S::K2>(T1, S::P2, X1, S::P2, m0, n0, D * D, BB * D); },
          [&](int m0, int n0, const v4f_e& c4) {
            const int n = n0 + (lane & 15), j0 = m0 + 4 * (lane >> 4);  // column (bb, l2), rows (r1, m0 + r)
            if (n >= BB * D) return;
            const int bb = n / D, l2 = n - bb * D;
            if constexpr (S::VEC) {
              if (j0 < D * D) {
                const int r1 = j0 / D, m = j0 - r1 * D;
                const v4bf_e v = {(__bf16)c4[0], (__bf16)c4[1], (__bf16)c4[2], (__bf16)c4[3]};
                *reinterpret_cast<v4bf_e*>(X2 + (bb * D + r1) * S::P3 + l2 * D + m) = v;
              }
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int j = j0 + r, r1 = j / D, m = j - r1 * D;
                if (j < D * D) X2[(bb * D + r1) * S::P3 + l2 * D + m] = (__bf16)c4[r];
              }
            }
          });
      __syncthreads();
      // S3: X3[(bb,r1)][r2][dd] = sum_{(l2,m)} T2[(r2,dd)][(l2,m)] X2[(bb,r1)][(l2,m)]; M = D^2 (rows (r2,dd)), N = BB D
      bf_stage<(D * D + 15) / 16, (BB * D + 15) / 16>(
          [&](int m0, int n0) { return bf_tile<S::K3>(T2, S::P2, X2, S::P3, m0, n0, D * D, BB * D); },
          [&](int m0, int n0, const v4f_e& c4) {
            const int n = n0 + (lane & 15), j0 = m0 + 4 * (lane >> 4);  // column (bb, r1), rows (r2, dd0 + r)
            if (n >= BB * D) return;
            if constexpr (S::VEC) {
              if (j0 < D * D) {
                const int r2 = j0 / D, dd = j0 - r2 * D;
                const v4bf_e v = {(__bf16)c4[0], (__bf16)c4[1], (__bf16)c4[2], (__bf16)c4[3]};
                *reinterpret_cast<v4bf_e*>(X3 + n * S::BS + r2 * S::P4 + dd) = v;
              }
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int j = j0 + r, r2 = j / D, dd = j - r2 * D;
                if (j < D * D) X3[n * S::BS + r2 * S::P4 + dd] = (__bf16)c4[r];
              }
            }
          });
      __syncthreads();
      // S4: acc[e][(bb,r1,r2)] += sum_dd BT[(cs, e)][dd] X3[(bb,r1)][r2][dd]; M = C, N = BB D^2
#pragma unroll
      for (int w = 0; w < S::T4W; ++w) {
        const int t = wave + 4 * w;
        if (t < S::NT4) {
          const int i = min(lane & 15, C - 1), j = min(t * 16 + (lane & 15), S::N4 - 1);
          const int kq = (lane >> 4) * 8, jb = j / D, r2 = j - jb * D;
#pragma unroll
          for (int s = 0; s < (S::K4 + 31) / 32; ++s) {
            const v8bf_e a = ld8(BT + (cs * C + i) * S::P4, 32 * s + kq, S::K4);
            const v8bf_e b = ld8(X3 + jb * S::BS + r2 * S::P4, 32 * s + kq, S::K4);
            acc[w] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[w], 0, 0, 0);
          }
        }
      }
      __syncthreads();  // X3 read: the next S1 may write X1
    }
    // write Lout[e][b0 + (bb, r1, r2)]
#pragma unroll
    for (int w = 0; w < S::T4W; ++w) {
      const int t = wave + 4 * w;
      if (t < S::NT4) {
        const int j = t * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = 4 * (lane >> 4) + r;
          if (e < C && j < S::N4) Lout[e * (C * D * D) + q * S::N4 + j] = (TS)acc[w][r];
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace vp
