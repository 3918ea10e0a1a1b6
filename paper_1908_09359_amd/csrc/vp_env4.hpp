// Fused 2-row ("4-line") column step on MFMA, compile-time dimensions.
//
//   Lout[e][b][r1][r2] = sum Lin[c][a][l1][l2] A[a][u][b] t1[l1][u][r1][m]
//                             t2[l2][m][r2][dd] B[c][dd][e]
//
// (environment layout: lower-boundary bond first).  The four pairwise
// contractions run slice by slice -- one block of BB upper-boundary indices b
// and one lower-boundary index c at a time -- so every intermediate stays in
// LDS; a block's output accumulates in MFMA registers across the c slices.  Inputs
// of arbitrary leg strides (mirrored or transposed views) are staged into LDS
// in canonical order once per step.  TC is the MFMA type (float: 16x16x4 f32,
// double: 16x16x4 f64), TB the storage type of the column tensors.
#pragma once
#include "vp_device.hpp"

namespace vp {

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v4d_t __attribute__((ext_vector_type(4)));

template <typename TC> struct Mfma;
template <> struct Mfma<float> {
  typedef v4f_t acc_t;
  __device__ static inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // lane l holds D[4 (l/16) + r][l % 16]
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
  typedef v4d_t acc_t;
  __device__ static inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // lane l holds D[(l/16) + 4 r][l % 16]
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// BBX > 0 overrides the b-block size (it must divide C).
template <int D, int C, int BBX = 0>
struct Env4Shape {
  static constexpr int BB = BBX > 0 ? BBX : ((C % 4 == 0) ? C / 4 : ((C % 2 == 0) ? C / 2 : C));  // b-block
  static constexpr int NBLK = C / BB;
  static constexpr int SA = C * D * C, ST = D * D * D * D;
  static constexpr int SL = C * D * D;            // one lower-bond slice of Lin
  // LDS rows are padded so that an MFMA operand read hits distinct banks: the
  // 16 lanes of one read pass for 8-byte words, the 32 lanes (two k-groups) of
  // one pass for 4-byte words.  Ls rows (one per a), X1 rows (l1,l2) of (u,bb),
  // X2 / X3 rows of D, the boundary tensor's rows (one per a) outside the Gram
  // step and its rows (a,u) in it.  E is the size of a working word.
  template <int E> static constexpr int lp() { return D * D + (E == 8 ? 4 : 16); }   // Ls
  template <int E> static constexpr int rs1() { return D * BB + (E == 8 ? 4 : 8); }  // X1
  template <int E> static constexpr int rs2() { return D + (E == 8 ? 1 : 2); }       // X2 / X3
  template <int E> static constexpr int arow() { return D * C + (E == 8 ? 0 : 16); } // A, per a
  static constexpr int AP = C + 4;                // Gram step: boundary tensor row stride
  template <int E> static constexpr int slp() { return C * lp<E>(); }
  template <int E> static constexpr int sx2() { return BB * D * D * rs2<E>(); }
  template <int E> static constexpr int sx13() {  // X1 and X3 share a buffer
    return D * D * rs1<E>() > sx2<E>() ? D * D * rs1<E>() : sx2<E>();
  }
  static constexpr int N4 = BB * D * D;           // S4 columns per block
  static constexpr int NT4 = (N4 + 15) / 16;      // S4 column tiles per block
  static constexpr int T4W = (NT4 + 3) / 4;       // S4 tiles per wave per block
  // Site tensors of S2 / S3 held in registers instead of LDS: when the D^2
  // output columns of those stages span exactly four 16-column tiles, wave w
  // always owns tile w, so its B operand is fixed for the whole step.
  template <bool GRAM = false, bool BF16 = false>
  static constexpr bool regt() { return !BF16 && (D * D + 15) / 16 == 4; }
  template <typename TC, typename TB, bool GRAM = false>
  static constexpr size_t lds_bytes() {
    constexpr int E = sizeof(TC);
    return sizeof(TB) * (GRAM ? C * D * AP : C * arow<sizeof(TB)>() + SA) +
           (regt<GRAM>() ? 0 : sizeof(TB) * (GRAM ? ST : 2 * ST)) + sizeof(TC) * (slp<E>() + sx13<E>() + sx2<E>());
  }
};

// One 16x16 output tile of a stage: acc += A(m0.., k) B(k, n0..) over K, with
// the operand fetchers given as lambdas (i, k) -> value and (k, j) -> value.
template <typename TC, int M, int N, int K, typename FA, typename FB>
__device__ inline typename Mfma<TC>::acc_t mfma_tile(int m0, int n0, FA fa, FB fb) {
  typename Mfma<TC>::acc_t acc = {0, 0, 0, 0};
  const int lane = threadIdx.x & 63;
  const int i = m0 + (lane & 15), j = n0 + (lane & 15), kq = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + kq;
    TC a = (i < M && k < K) ? fa(i, k) : TC(0);
    TC b = (j < N && k < K) ? fb(k, j) : TC(0);
    acc = Mfma<TC>::op(a, b, acc);
  }
  return acc;
}

typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));

// bf16 operands, f32 accumulation (16x16x32): lane l supplies A[l%16][8(l/16)..+7]
// and B[8(l/16)..+7][l%16]; the output layout is that of the f32 16x16x4.
template <int M, int N, int K, typename FA, typename FB>
__device__ inline v4f_t mfma_tile_bf16(int m0, int n0, FA fa, FB fb) {
  v4f_t acc = {0, 0, 0, 0};
  const int lane = threadIdx.x & 63;
  const int i = m0 + (lane & 15), j = n0 + (lane & 15), kq = (lane >> 4) * 8;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    v8bf_t a, b;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + kq + q;
      a[q] = (__bf16)((i < M && k < K) ? (float)fa(i, k) : 0.0f);
      b[q] = (__bf16)((j < N && k < K) ? (float)fb(k, j) : 0.0f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Accumulators of a stage: those of TC, or f32 (f32 output layout) with bf16 operands.
template <typename TC, bool BF16> struct Acc {
  typedef typename Mfma<TC>::acc_t type;
  __device__ static inline int row(int lane, int r) { return Mfma<TC>::row(lane, r); }
};
template <typename TC> struct Acc<TC, true> {
  typedef v4f_t type;
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Stage out[i][j] = sum_k A(i,k) B(k,j) into LDS (row-major, ld N), all waves.
// BF16: operands rounded to bf16, products accumulated in f32, stored as TC.
template <typename TC, int M, int N, int K, bool BF16 = false, typename FO, typename FA, typename FB>
__device__ inline void mfma_stage(TC* out, FO oidx, FA fa, FB fb) {
  constexpr int MT = (M + 15) / 16, NT = (N + 15) / 16, NTW = (MT * NT + 3) / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // a wave's tiles t = wave + 4 w accumulate side by side and are stored only
  // after all their operands are read (the stores could alias the operands in
  // LDS, so a store would hold back every later read)
  typename Acc<TC, BF16>::type acc[NTW];
#pragma unroll
  for (int w = 0; w < NTW; ++w) {
    const int t = min(wave + 4 * w, MT * NT - 1);  // a wave without a last tile repeats one, unstored
    const int m0 = (t / NT) * 16, n0 = (t % NT) * 16;
    if constexpr (BF16) acc[w] = mfma_tile_bf16<M, N, K>(m0, n0, fa, fb);
    else acc[w] = mfma_tile<TC, M, N, K>(m0, n0, fa, fb);
  }
#pragma unroll
  for (int w = 0; w < NTW; ++w) {
    const int t = wave + 4 * w;
    if (t < MT * NT) {
      const int m0 = (t / NT) * 16, n0 = (t % NT) * 16;
      const int j = n0 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + Acc<TC, BF16>::row(lane, r);
        if (i < M && j < N) out[oidx(i, j)] = (TC)acc[w][r];
      }
    }
  }
}

// A stage whose B operand sits in registers: N spans four 16-column tiles and
// wave w owns columns 16w..16w+15 of every row tile; f[s] holds
// B(4s + lane/16, 16w + lane%16).  The row tiles' accumulation chains are
// interleaved.
template <typename TC, int M, int N, int K, typename FO, typename FA>
__device__ inline void mfma_stage_regb(TC* out, FO oidx, FA fa, const TC (&f)[(K + 3) / 4]) {
  constexpr int MT = (M + 15) / 16, KS = (K + 3) / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kq = lane >> 4;
  typename Mfma<TC>::acc_t acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + kq;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int i = mt * 16 + (lane & 15);
      const TC a = (i < M && k < K) ? fa(i, k) : TC(0);
      acc[mt] = Mfma<TC>::op(a, f[s], acc[mt]);
    }
  }
  const int j = 16 * wave + (lane & 15);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = mt * 16 + Mfma<TC>::row(lane, r);
      if (i < M && j < N) out[oidx(i, j)] = acc[mt][r];
    }
}

// GRAM: t2 is the u<->d view of t1 and B is A (the Gram step of the boundary
// compression); each is then staged once.
// b-block of a fused step: the Gram step of the compression over float64
// tensors staged in LDS takes C/8 so that its LDS stays within two work-groups
// per CU.
template <typename TC, typename TB, int D, int C, bool GRAM>
constexpr int env4_bb() {
  return (GRAM && sizeof(TB) == 8 && C % 8 == 0 && (D * D + 15) / 16 != 4) ? C / 8 : 0;
}

// BBX > 0 takes that b-block size (a tile variant; it must divide C) instead of
// the default one.  The blocking partitions only the output columns, so every
// output element is summed in the same order for every BBX.
template <typename TC, typename TB, int D, int C, bool GRAM = false, bool BF16 = false, int BBX = 0>
__device__ void env4_fused(TC* __restrict__ Lout_p, const TC* __restrict__ Lin_p, const TB* __restrict__ A_p, S3 sA,
                           const TB* __restrict__ t1_p, S4 s1, const TB* __restrict__ t2_p, S4 s2,
                           const TB* __restrict__ B_p, S3 sB, char* lds) {
  auto* Lout = gmem(Lout_p);
  const auto* Lin = gmem(Lin_p);
  const auto* A = gmem(A_p);
  const auto* t1 = gmem(t1_p);
  const auto* t2 = gmem(t2_p);
  const auto* B = gmem(B_p);
  using Sh = Env4Shape<D, C, (BBX > 0 ? BBX : env4_bb<TC, TB, D, C, GRAM>())>;
  constexpr int BB = Sh::BB, NBLK = Sh::NBLK, N4 = Sh::N4, NT4 = Sh::NT4, T4W = Sh::T4W;
  constexpr bool REGT = Sh::template regt<GRAM, BF16>();
  constexpr int KS = (D * D + 3) / 4;
  constexpr int E = sizeof(TC);
  constexpr int LP = Sh::template lp<E>(), RS1 = Sh::template rs1<E>(), RS2 = Sh::template rs2<E>();
  constexpr int AP = Sh::AP, AR = Sh::template arow<sizeof(TB)>();
  TB* As = reinterpret_cast<TB*>(lds);
  TB* Bs = GRAM ? As : As + C * AR;
  TB* T1s = GRAM ? As + C * D * AP : Bs + Sh::SA;
  TB* T2s = GRAM ? T1s : T1s + Sh::ST;
  TC* Ls = reinterpret_cast<TC*>(REGT ? T1s : T2s + Sh::ST);
  TC* X1 = Ls + Sh::template slp<E>();  // X1 and X3
  TC* X2 = X1 + Sh::template sx13<E>();
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

  // this wave's B fragments of S2 (t1) and S3 (t2; for GRAM the u<->d view of
  // t1), read once from global memory
  TC f1[REGT ? KS : 1], f2[REGT ? KS : 1];
  if constexpr (REGT) {
    const int j = 16 * wave + (lane & 15), r = j / D, dq = j % D;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * s + (lane >> 4), l = k / D, u = k % D;
      const bool ok = j < D * D && k < D * D;
      f1[s] = ok ? (TC)t1[l * s1.l + u * s1.u + r * s1.r + dq * s1.d] : TC(0);
      f2[s] = ok ? (TC)t2[l * s2.l + u * s2.u + r * s2.r + dq * s2.d] : TC(0);
    }
  }

  // stage the column tensors: B as [c][dd][e]; A as [a][b-block][u][bb] (the
  // columns of S1 contiguous), or in the Gram step, where A is also B, as
  // [a][u][b] with rows padded to AP
  for (int e = tid; e < Sh::SA; e += WG) {
    const int p = e / (D * C), q = (e / C) % D, r = e % C;
    if constexpr (GRAM) {
      As[(p * D + q) * AP + r] = A[p * sA.s0 + q * sA.s1 + r * sA.s2];
    } else {
      Bs[e] = B[p * sB.s0 + q * sB.s1 + r * sB.s2];
      const int rem = e % (D * C), blk = rem / (D * BB), u = (rem / BB) % D, b = blk * BB + rem % BB;
      As[p * AR + rem] = A[p * sA.s0 + u * sA.s1 + b * sA.s2];
    }
  }
  if constexpr (!REGT)
    for (int e = tid; e < Sh::ST; e += WG) {
      const int l = e / (D * D * D), u = (e / (D * D)) % D, r = (e / D) % D, d = e % D;
      T1s[e] = t1[l * s1.l + u * s1.u + r * s1.r + d * s1.d];
      if (!GRAM) T2s[e] = t2[l * s2.l + u * s2.u + r * s2.r + d * s2.d];
    }

  // b-blocks outer, lower-bond slices inner: only one block's accumulators are
  // live.  Each slice of Lin is fetched one slice ahead into registers, so its
  // global-memory latency overlaps the previous slice's products.
  constexpr int NPF = (Sh::SL + WG - 1) / WG;
  TC pre[NPF];
  auto fetch = [&](int cs) {
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int e = tid + u * WG;
      pre[u] = e < Sh::SL ? Lin[cs * Sh::SL + e] : TC(0);
    }
  };
  // slices are taken in the order (block, slice); the next one is stored into
  // Ls as soon as S1 of the current one has read it, and the one after that is
  // then fetched, so a slice costs four barriers
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int e = tid + u * WG, a = e / (D * D);
      if (e < Sh::SL) Ls[a * LP + e - a * (D * D)] = pre[u];
    }
  };
  constexpr int NS = NBLK * C;
  fetch(0);
  __syncthreads();  // staging above done
  store();
  if (NS > 1) fetch(1 % C);
  __syncthreads();
  for (int q = 0; q < NBLK; ++q) {
    const int b0 = q * BB;
    typename Acc<TC, BF16>::type acc[T4W];
#pragma unroll
    for (int w = 0; w < T4W; ++w) acc[w] = {0, 0, 0, 0};
    for (int cs = 0; cs < C; ++cs) {
      const int pos = q * C + cs;
      // S1: X1[(l1,l2)][(u,bb)] = sum_a Ls[a][(l1,l2)] As[a][u][b0+bb]
      mfma_stage<TC, D * D, D * BB, C, BF16>(
          X1, [&](int i, int j) { return i * RS1 + j; }, [&](int i, int k) { return Ls[k * LP + i]; },
          [&](int k, int j) {
            if constexpr (GRAM) return (TC)As[(k * D + j / BB) * AP + b0 + j % BB];
            else return (TC)As[k * AR + q * (D * BB) + j];
          });
      __syncthreads();
      if (pos + 1 < NS) {  // Ls is free: the next slice goes in
        store();
        if (pos + 2 < NS) fetch((pos + 2) % C);
      }
      // rows (i, j / D) of X2 and X3 padded to RS2
      auto oidx23 = [&](int i, int j) { return (i * D + j / D) * RS2 + j % D; };
      // S2: X2[(l2,bb)][(r1,m)] = sum_{l1,u} X1[l1][l2][u][bb] T1s[(l1,u)][(r1,m)]
      auto fa2 = [&](int i, int k) { return X1[((k / D) * D + i / BB) * RS1 + (k % D) * BB + i % BB]; };
      if constexpr (REGT) mfma_stage_regb<TC, D * BB, D * D, D * D>(X2, oidx23, fa2, f1);
      else
        mfma_stage<TC, D * BB, D * D, D * D, BF16>(X2, oidx23, fa2,
                                                    [&](int k, int j) { return (TC)T1s[k * D * D + j]; });
      __syncthreads();
      // S3: X3[(bb,r1)][(r2,dd)] = sum_{l2,m} X2[l2][bb][r1][m] T2s[(l2,m)][(r2,dd)]
      auto fa3 = [&](int i, int k) { return X2[(((k / D) * BB + i / D) * D + i % D) * RS2 + k % D]; };
      if constexpr (REGT) mfma_stage_regb<TC, BB * D, D * D, D * D>(X1, oidx23, fa3, f2);
      else
        mfma_stage<TC, BB * D, D * D, D * D, BF16>(X1, oidx23, fa3, [&](int k, int j) {
          // GRAM: t2[l2][m][r2][dd] = t1[l2][dd][r2][m]
          return GRAM ? (TC)T1s[(k / D) * D * D * D + (j % D) * D * D + (j / D) * D + k % D]
                      : (TC)T2s[k * D * D + j];
        });
      __syncthreads();
      // S4: acc[e][(bb,r1,r2)] += sum_dd Bs[cs][dd][e] X3[(bb,r1,r2)][dd]
#pragma unroll
      for (int w = 0; w < T4W; ++w) {
        const int t = wave + 4 * w;
        if (t < NT4) {
          const int n0 = t * 16;
          if constexpr (BF16) {
            const int i = lane & 15, j = n0 + (lane & 15), kq = (lane >> 4) * 8;
            v8bf_t a, b;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int k = kq + q;
              a[q] = (__bf16)((i < C && k < D) ? (float)(GRAM ? Bs[(cs * D + k) * AP + i] : Bs[cs * D * C + k * C + i])
                                               : 0.0f);
              b[q] = (__bf16)((j < N4 && k < D) ? (float)X1[j * RS2 + k] : 0.0f);
            }
            acc[w] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[w], 0, 0, 0);
          } else {
            const int i = lane & 15, j = n0 + (lane & 15), kq = lane >> 4;
#pragma unroll
            for (int k0 = 0; k0 < D; k0 += 4) {
              const int k = k0 + kq;
              TC a = (i < C && k < D) ? (TC)(GRAM ? Bs[(cs * D + k) * AP + i] : Bs[cs * D * C + k * C + i]) : TC(0);
              TC b = (j < N4 && k < D) ? X1[j * RS2 + k] : TC(0);
              acc[w] = Mfma<TC>::op(a, b, acc[w]);
            }
          }
        }
      }
      __syncthreads();  // X3 read: the next S1 may write X1
    }
    // write Lout[e][b0 + (bb,r1,r2)]
#pragma unroll
    for (int w = 0; w < T4W; ++w) {
      const int t = wave + 4 * w;
      if (t < NT4) {
        const int j = t * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = Acc<TC, BF16>::row(lane, r);
          if (e < C && j < N4) Lout[e * (C * D * D) + q * N4 + j] = (TC)acc[w][r];
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace vp
