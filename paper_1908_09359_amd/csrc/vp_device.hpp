// Device-side building blocks of the VMC-PEPS hot path for gfx950.
//
// One work-group (256 threads, four 64-wide wavefronts) owns one Markov chain
// (or one fixed configuration) for the whole duration of a kernel and walks the
// columns of a row sequentially; every contraction of a column step is a
// work-group GEMM whose operands are addressed through 2-level strided views,
// so the tensor-network index permutations never need a separate transpose.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vp {

constexpr int WG = 256;

// Global-memory view of a pointer that addresses global memory.  Functions the
// compiler keeps out of line receive plain (generic) pointers; their accesses
// become flat instructions, which count on the LDS wait counter as well, so
// every LDS wait behind a flat load or store also waits for global memory.
// Accesses through this view are global instructions.
template <typename T>
__device__ inline __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// LDS-typed pointer to a work-group's shared memory.  A helper the compiler
// keeps out of line receives its LDS through such a parameter: converted to a
// plain pointer inside, the accesses are still LDS instructions (through a
// plain parameter they would be flat ones whenever the compiler cannot prove
// that every caller passes LDS).
typedef __attribute__((address_space(3))) char lds_char;
__device__ inline lds_char* as_lds(char* p) { return (lds_char*)p; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its
// definition: ten rounds of two 64x64->128 products, word permutation and key
// xor, with the Weyl increments added to the key between rounds.
// ---------------------------------------------------------------------------
struct U64x4 { uint64_t v[4]; };

__device__ __host__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t hi0 = __umul64hi(M0, c0), hi1 = __umul64hi(M1, c2);
#else
    uint64_t hi0 = (uint64_t)(((unsigned __int128)M0 * c0) >> 64);
    uint64_t hi1 = (uint64_t)(((unsigned __int128)M1 * c2) >> 64);
#endif
    uint64_t lo0 = M0 * c0, lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return U64x4{{c0, c1, c2, c3}};
}

__device__ __host__ inline double uniform53(uint64_t w) {
  return (double)(w >> 11) * (1.0 / 9007199254740992.0);
}

enum : uint64_t { TAG_INIT = 1, TAG_PERTURB = 2, TAG_SHUFFLE = 3, TAG_METRO = 4, TAG_SGD = 5, TAG_PLAQ = 6 };

// ---------------------------------------------------------------------------
// Strided 2-level views: element (i, j) of a matrix lives at
//   (i / n2i) * si1 + (i % n2i) * si2 + (j / n2j) * sj1 + (j % n2j) * sj2.
// ---------------------------------------------------------------------------
// The divisions use multiply-high by m = floor(2^32 / n2) + 1, exact for
// indices and divisors below 2^16 (the error term n (m n2 - 2^32) / 2^32 stays
// below 1/n2).
struct View {
  int n2i, n2j;
  int si1, si2, sj1, sj2;
  uint64_t mi, mj;
};

__host__ __device__ inline uint64_t div_magic(int d) { return (1ull << 32) / (uint64_t)d + 1; }
__host__ __device__ inline View view(int n2i, int si1, int si2, int n2j, int sj1, int sj2) {
  return View{n2i, n2j, si1, si2, sj1, sj2, div_magic(n2i), div_magic(n2j)};
}
__host__ __device__ inline View rowmajor(int ld) { return view(1, ld, 0, 1, 1, 0); }
__host__ __device__ inline View colmajor(int ld) { return view(1, 1, 0, 1, ld, 0); }

__device__ inline int vaddr(const View& v, int i, int j) {
  const int i1 = (int)(((uint64_t)(unsigned)i * v.mi) >> 32), i2 = i - i1 * v.n2i;
  const int j1 = (int)(((uint64_t)(unsigned)j * v.mj) >> 32), j2 = j - j1 * v.n2j;
  return i1 * v.si1 + i2 * v.si2 + j1 * v.sj1 + j2 * v.sj2;
}

// One LDS tile buffer shared by every GEMM instantiation of a kernel.
__device__ inline char* gemm_tiles() {
  __shared__ __attribute__((aligned(16))) char buf[2 * 16 * 65 * sizeof(double)];
  return buf;
}

typedef float v4f_g __attribute__((ext_vector_type(4)));
typedef double v4d_g __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA in the accumulation type; lane l holds output rows
// 4 (l/16) + r (f32) or (l/16) + 4 r (f64) of column l % 16.
__device__ inline v4f_g mfma4(float a, float b, v4f_g c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline v4d_g mfma4(double a, double b, v4d_g c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline int mfma4_row(float, int lane, int r) { return 4 * (lane >> 4) + r; }
__device__ inline int mfma4_row(double, int lane, int r) { return (lane >> 4) + 4 * r; }
template <typename T> struct Acc4;
template <> struct Acc4<float> { typedef v4f_g type; };
template <> struct Acc4<double> { typedef v4d_g type; };

// C(i,j) = alpha sum_k A(i,k) B(k,j) (+ C(i,j) when accumulate) for i < M,
// j < N, accumulated in TC on MFMA.
// 64x64 output blocks, K staged through LDS 16 at a time; each wave owns a
// 2x2 set of 16x16 tiles.  All threads of the work-group must call it; C is
// complete after the trailing barrier.
// tiles: LDS of GEMM_TILE_BYTES owned by the caller.
constexpr size_t GEMM_TILE_BYTES = 2 * 16 * 65 * sizeof(double);
typedef __bf16 v8bf_g __attribute__((ext_vector_type(8)));

// bf16 operands, f32 accumulation (C(i,j) as above, stored as TC): A and B are
// rounded to bf16 (round to nearest even) when staged, 32 k-values at a time,
// k-contiguous in LDS so that each lane fetches its 8 k-values of the
// 16x16x32 MFMA in one read; the output layout is that of the f32 16x16x4.
template <typename TC, typename TA, typename TB>
__device__ void wg_gemm_bf16(char* tiles, TC* __restrict__ C_p, View vc, const TA* __restrict__ A_p, View va,
                             const TB* __restrict__ B_p, View vb, int M, int N, int K, TC alpha,
                             bool accumulate) {
  auto* C = gmem(C_p);
  const auto* A = gmem(A_p);
  const auto* B = gmem(B_p);
  constexpr int BM = 64, BN = 64, BK = 32, LD = BK + 8;
  __bf16 (*As)[LD] = reinterpret_cast<__bf16 (*)[LD]>(tiles);
  __bf16 (*Bs)[LD] = reinterpret_cast<__bf16 (*)[LD]>(tiles + BM * LD * sizeof(__bf16));
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tr0 = (wave >> 1) * 32, tc0 = (wave & 1) * 32;
  const int kq = (lane >> 4) * 8, li = lane & 15;
  for (int m0 = 0; m0 < M; m0 += BM) {
    for (int n0 = 0; n0 < N; n0 += BN) {
      v4f_g acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = {0, 0, 0, 0};
      for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int e = 0; e < (BM * BK) / WG; ++e) {
          int idx = tid + e * WG;
          int mi = idx % BM, ki = idx / BM;
          int m = m0 + mi, k = k0 + ki;
          As[mi][ki] = (__bf16)((m < M && k < K) ? (float)A[vaddr(va, m, k)] : 0.0f);
        }
#pragma unroll
        for (int e = 0; e < (BN * BK) / WG; ++e) {
          int idx = tid + e * WG;
          int ni = idx % BN, ki = idx / BN;
          int n = n0 + ni, k = k0 + ki;
          Bs[ni][ki] = (__bf16)((n < N && k < K) ? (float)B[vaddr(vb, k, n)] : 0.0f);
        }
        __syncthreads();
        const v8bf_g a0 = *reinterpret_cast<const v8bf_g*>(&As[tr0 + li][kq]);
        const v8bf_g a1 = *reinterpret_cast<const v8bf_g*>(&As[tr0 + 16 + li][kq]);
        const v8bf_g b0 = *reinterpret_cast<const v8bf_g*>(&Bs[tc0 + li][kq]);
        const v8bf_g b1 = *reinterpret_cast<const v8bf_g*>(&Bs[tc0 + 16 + li][kq]);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int n = n0 + tc0 + 16 * b + li;
          if (n >= N) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = m0 + tr0 + 16 * a + 4 * (lane >> 4) + r;
            if (m < M) {
              auto* cp = C + vaddr(vc, m, n);
              *cp = accumulate ? *cp + alpha * (TC)acc[a][b][r] : alpha * (TC)acc[a][b][r];
            }
          }
        }
    }
  }
  __syncthreads();
}

template <typename TC, typename TA, typename TB>
__device__ void wg_gemm_t(char* tiles, TC* __restrict__ C_p, View vc, const TA* __restrict__ A_p, View va,
                          const TB* __restrict__ B_p, View vb, int M, int N, int K, TC alpha = TC(1),
                          bool accumulate = false) {
  auto* C = gmem(C_p);
  const auto* A = gmem(A_p);
  const auto* B = gmem(B_p);
  constexpr int BM = 64, BN = 64, BK = 16, NA = (BM * BK) / WG, NB = (BN * BK) / WG;
  TC (*As)[BM + 1] = reinterpret_cast<TC (*)[BM + 1]>(tiles);
  TC (*Bs)[BN + 1] = reinterpret_cast<TC (*)[BN + 1]>(tiles + BK * (BM + 1) * sizeof(TC));
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tr0 = (wave >> 1) * 32, tc0 = (wave & 1) * 32;  // this wave's 32x32 corner
  // the next K-chunk of both operands is read into registers while the current
  // one is multiplied
  TC pa[NA], pb[NB];
  auto fetch = [&](int m0, int n0, int k0) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + e * WG, mi = idx % BM, ki = idx / BM, m = m0 + mi, k = k0 + ki;
      pa[e] = (m < M && k < K) ? (TC)A[vaddr(va, m, k)] : TC(0);
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + e * WG, ni = idx % BN, ki = idx / BN, n = n0 + ni, k = k0 + ki;
      pb[e] = (n < N && k < K) ? (TC)B[vaddr(vb, k, n)] : TC(0);
    }
  };
  for (int m0 = 0; m0 < M; m0 += BM) {
    for (int n0 = 0; n0 < N; n0 += BN) {
      typename Acc4<TC>::type acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = {0, 0, 0, 0};
      fetch(m0, n0, 0);
      for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int e = 0; e < NA; ++e) {
          const int idx = tid + e * WG;
          As[idx / BM][idx % BM] = pa[e];
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
          const int idx = tid + e * WG;
          Bs[idx / BN][idx % BN] = pb[e];
        }
        __syncthreads();
        if (k0 + BK < K) fetch(m0, n0, k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          const int k = kk + (lane >> 4);
          TC a0 = As[k][tr0 + (lane & 15)], a1 = As[k][tr0 + 16 + (lane & 15)];
          TC b0 = Bs[k][tc0 + (lane & 15)], b1 = Bs[k][tc0 + 16 + (lane & 15)];
          acc[0][0] = mfma4(a0, b0, acc[0][0]);
          acc[0][1] = mfma4(a0, b1, acc[0][1]);
          acc[1][0] = mfma4(a1, b0, acc[1][0]);
          acc[1][1] = mfma4(a1, b1, acc[1][1]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int n = n0 + tc0 + 16 * b + (lane & 15);
          if (n >= N) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = m0 + tr0 + 16 * a + mfma4_row(TC(0), lane, r);
            if (m < M) {
              auto* cp = C + vaddr(vc, m, n);
              *cp = accumulate ? *cp + alpha * acc[a][b][r] : alpha * acc[a][b][r];
            }
          }
        }
    }
  }
  __syncthreads();
}

// The same with the kernel-wide static tile buffer.
template <typename TC, typename TA, typename TB>
__device__ void wg_gemm(TC* __restrict__ C, View vc, const TA* __restrict__ A, View va, const TB* __restrict__ B,
                        View vb, int M, int N, int K, TC alpha = TC(1), bool accumulate = false) {
  wg_gemm_t<TC>(gemm_tiles(), C, vc, A, va, B, vb, M, N, K, alpha, accumulate);
}

// Operand precision chosen at compile time: BF16 rounds both operands to bf16
// (f32 accumulation); otherwise the products are formed in TC.  tiles: LDS of
// GEMM_TILE_BYTES owned by the caller.
template <bool BF16, typename TC, typename TA, typename TB>
__device__ inline void wg_gemm_p(char* tiles, TC* __restrict__ C, View vc, const TA* __restrict__ A, View va,
                                 const TB* __restrict__ B, View vb, int M, int N, int K) {
  if constexpr (BF16) {
    wg_gemm_bf16<TC>(tiles, C, vc, A, va, B, vb, M, N, K, TC(1), false);
  } else {
    wg_gemm_t<TC>(tiles, C, vc, A, va, B, vb, M, N, K);
  }
}

// ---------------------------------------------------------------------------
// Work-group reductions (fixed order: per-thread partials, then a tree).
// ---------------------------------------------------------------------------
// Wavefront shuffle reduction, then the four wave partials through LDS in a
// fixed order (two barriers).
__device__ inline double wg_sum(double v) {
  __shared__ double red[WG / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

__device__ inline double wg_max(double v) {
  __shared__ double red[WG / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return r;
}

template <typename T>
__device__ inline void wg_copy(T* __restrict__ dst, const T* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += WG) dst[i] = src[i];
  __syncthreads();
}

template <typename T>
__device__ inline void wg_fill(T* dst, T v, int n) {
  for (int i = threadIdx.x; i < n; i += WG) dst[i] = v;
  __syncthreads();
}

// Scale x by an exact power of two so that max|x| lies in [1, 2); returns the
// exponent removed (0 for an all-zero tensor).  Exact in every precision.
template <typename T>
__device__ inline int wg_renorm(T* x_p, int n) {
  auto* x = gmem(x_p);
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += WG) m = fmax(m, fabs((double)x[i]));
  m = wg_max(m);
  if (!(m > 0.0) || !isfinite(m)) return 0;
  int e = ilogb(m);
  T f = (T)ldexp(1.0, -e);
  for (int i = threadIdx.x; i < n; i += WG) x[i] *= f;
  __syncthreads();
  return e;
}

template <typename T>
__device__ inline double wg_dot(const T* a_p, const T* b_p, int n) {
  const auto* a = gmem(a_p);
  const auto* b = gmem(b_p);
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += WG) s += (double)a[i] * (double)b[i];
  return wg_sum(s);
}

// ---------------------------------------------------------------------------
// Leg strides of the tensors a column step consumes.
// ---------------------------------------------------------------------------
struct S3 { int s0, s1, s2; };        // boundary-MPS site: left bond, physical, right bond
struct S4 { int l, u, r, d; };        // PEPS site

// 3-line left step (App. C): Lout[b][r][e] =
//   sum Lin[a][l][c] A[a][u][b] t[l][u][r][dd] B[c][dd][e].
// Lin/Lout are dense c x d x c; X0/X1 scratch of c*c*d*d elements.
template <typename T, bool BF16 = false>
__device__ void env3_step(T* Lout, const T* Lin, const T* A, S3 sA, const T* t, S4 st,
                          const T* B, S3 sB, T* X0, T* X1, int c, int d, char* tiles) {
  using TC = T;
  // X0[c'][b][l][u] = sum_a Lin[a][(l,c')] A[a][(u,b)]
  wg_gemm_p<BF16, TC>(tiles, X0, view(c, d, c * d * d, c, 1, d * d), Lin, view(c, c, 1, 1, d * c, 0),
             A, view(1, sA.s0, 0, c, sA.s1, sA.s2), d * c, d * c, c);
  // X1[b][r][c'][dd] = sum_{l,u} X0[(c',b)][(l,u)] t[(l,u)][(r,dd)]
  wg_gemm_p<BF16, TC>(tiles, X1, view(c, d, d * c * d, d, c * d, 1), X0, rowmajor(d * d),
             t, view(d, st.l, st.u, d, st.r, st.d), c * c, d * d, d * d);
  // Lout[(b,r)][e] = sum_{c',dd} X1[(b,r)][(c',dd)] B[(c',dd)][e]
  wg_gemm_p<BF16, TC>(tiles, Lout, rowmajor(c), X1, rowmajor(c * d), B, view(d, sB.s0, sB.s1, 1, sB.s2, 0),
             c * d, c, c * d);
}

// 4-line left step: Lout[b][r1][r2][e] = sum Lin[a][l1][l2][c] A[a][u][b]
//   t1[l1][u][r1][m] t2[l2][m][r2][dd] B[c][dd][e].
// X0/X1 scratch of d*d*d*c*c elements each.
template <typename TC, typename T, bool BF16 = false>
__device__ void env4_step(TC* Lout, const TC* Lin, const T* A, S3 sA, const T* t1, S4 s1,
                          const T* t2, S4 s2, const T* B, S3 sB, TC* X0, TC* X1, int c, int d, char* tiles) {
  // X0[(l2,c')][b][l1][u] = sum_a Lin[a][(l1,(l2,c'))] A[a][(u,b)]
  wg_gemm_p<BF16, TC>(tiles, X0, view(d * c, d, c * d * d, c, 1, d * d), Lin, view(d * c, d * c, 1, 1, d * d * c, 0),
             A, view(1, sA.s0, 0, c, sA.s1, sA.s2), d * d * c, d * c, c);
  // X1[(c',b)][r1][l2][m] = sum_{l1,u} X0[(l2,c',b)][(l1,u)] t1[(l1,u)][(r1,m)]
  wg_gemm_p<BF16, TC>(tiles, X1, view(c * c, d, d * d * d, d, d * d, 1), X0, rowmajor(d * d),
             t1, view(d, s1.l, s1.u, d, s1.r, s1.d), d * c * c, d * d, d * d);
  // X0[(b,r1)][r2][c'][dd] = sum_{l2,m} X1[(c',b,r1)][(l2,m)] t2[(l2,m)][(r2,dd)]
  wg_gemm_p<BF16, TC>(tiles, X0, view(c * d, d, d * d * c, d, c * d, 1), X1, rowmajor(d * d),
             t2, view(d, s2.l, s2.u, d, s2.r, s2.d), c * c * d, d * d, d * d);
  // Lout[(b,r1,r2)][e] = sum_{c',dd} X0[(b,r1,r2)][(c',dd)] B[(c',dd)][e]
  wg_gemm_p<BF16, TC>(tiles, Lout, rowmajor(c), X0, rowmajor(c * d), B, view(d, sB.s0, sB.s1, 1, sB.s2, 0),
             c * d * d, c, c * d);
}

// Defect tensor of one site in a 3-line network (Sec. II.A Eq. (7)):
//   Out[l][u][r][dd] = sum Lp[a][l][c] A[a][u][b] Rn[b][r][e] B[c][dd][e].
template <typename T>
__device__ void defect3(T* Out, const T* Lp, const T* A, S3 sA, const T* Rn, const T* B, S3 sB,
                        T* X0, T* X1, int c, int d, lds_char* tiles_l) {
  char* tiles = (char*)tiles_l;
  using TC = T;
  // X0[l][u][c'][b] = sum_a Lp[a][(l,c')] A[a][(u,b)]
  wg_gemm_t<TC>(tiles, X0, view(c, d * c * c, c, c, c * c, 1), Lp, view(c, c, 1, 1, d * c, 0),
             A, view(1, sA.s0, 0, c, sA.s1, sA.s2), d * c, d * c, c);
  // X1[(l,u)][r][c'][e] = sum_b X0[(l,u,c')][b] Rn[b][(r,e)]
  wg_gemm_t<TC>(tiles, X1, view(c, d * c * c, c, c, c * c, 1), X0, rowmajor(c), Rn, rowmajor(d * c),
             d * d * c, d * c, c);
  // Out[(l,u,r)][dd] = sum_{c',e} X1[(l,u,r)][(c',e)] B[(c',e)][dd]
  wg_gemm_t<TC>(tiles, Out, rowmajor(d), X1, rowmajor(c * c), B, view(c, sB.s0, sB.s2, 1, sB.s1, 0),
             d * d * d, d, c * c);
}

// Compression helper: Y[a][l][dd][k] = sum_{u,b,r} A[a][u][b] t[l][u][r][dd] Tin[b][r][k].
template <typename TC, typename T>
__device__ void compress_y(TC* Y, const T* A, S3 sA, const T* t, S4 st, const TC* Tin, TC* X0,
                           int c, int d, lds_char* tiles_l) {
  char* tiles = (char*)tiles_l;
  // X0[a][k][u][r] = sum_b A[(a,u)][b] Tin[b][(r,k)]
  wg_gemm_t<TC>(tiles, X0, view(d, c * d * d, d, c, 1, d * d), A, view(d, sA.s0, sA.s1, 1, sA.s2, 0),
             Tin, view(1, d * c, 0, c, c, 1), c * d, d * c, c);
  // Y[(a,k)][(l,dd)] = sum_{u,r} X0[(a,k)][(u,r)] t[(u,r)][(l,dd)]
  wg_gemm_t<TC>(tiles, Y, view(c, d * d * c, 1, d, d * c, c), X0, rowmajor(d * d),
             t, view(d, st.u, st.r, d, st.l, st.d), c * c, d * d, d * d);
}

}  // namespace vp
