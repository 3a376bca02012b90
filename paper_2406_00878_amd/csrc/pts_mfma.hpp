// Dense products on MFMA for gfx950, used by the network kernels of the learned iterate:
// float32 operands in memory, rounded to bfloat16 (nearest even) when staged into LDS,
// 16 x 16 x 16 bf16 MFMA tiles, float32 accumulation.
#pragma once
#include <hip/hip_runtime.h>

namespace pts_mm {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __builtin_bit_cast(unsigned, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

struct Gemm {
  const float* A;
  const float* B;
  float* C;
  int M, N, K;
  long sam, sak, bsa, sbk, sbn, bsb, scm, scn, bsc;
  float alpha, beta;
  int ksplit;       // K ranges per product; > 1 writes partial tiles to P
  float* P;         // [batch][ksplit][M][N] partials (ksplit > 1)
  const float* bias;  // optional epilogue (ksplit == 1): c += bias[m], then act = GELU(c)
  float* act;         // same layout as C
};

// GELU, tanh form: z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))
__device__ __forceinline__ float gelu(float z) {
  const float a = 0.7978845608028654f * (z + 0.044715f * z * z * z);
  const float t = 1.f - 2.f / (expf(2.f * a) + 1.f);  // tanh(a)
  return 0.5f * z * (1.f + t);
}

constexpr int BM = 64, BN = 64, BK = 32;  // BK: default K step (the template parameter of mm_tile)

// One 64 x 64 output tile (rows m0.., columns n0..) of product b, K range sp, computed by a
// 256-thread work-group (4 waves, 32 x 32 each). Staging follows the unit stride of each
// operand (coalesced loads for either layout), and the next K step is loaded into
// registers while the current one is multiplied.
template <int BKT = BK>
__device__ __forceinline__ void mm_tile(const Gemm& g, int m0, int n0, int b, int sp) {
  constexpr int BK = BKT;
  constexpr int kStage = BM * BK / 256;  // elements of A (and of B) each thread stages per K step
  __shared__ unsigned short As[BM][BK + 2];
  __shared__ unsigned short Bs[BK][BN + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float* A = g.A + (long)b * g.bsa;
  const float* B = g.B + (long)b * g.bsb;
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
  const int kbeg = sp * kchunk, kend = min(g.K, kbeg + kchunk);
  const bool a_mfast = g.sam == 1 && g.sak != 1;  // A contiguous along m
  const bool b_kfast = g.sbk == 1 && g.sbn != 1;  // B contiguous along k
  float4_t acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  float ra[kStage], rb[kStage];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int e = tid + r * 256;
      const int am = a_mfast ? e % BM : e / BK, ak = a_mfast ? e / BM : e % BK;
      const int gm = m0 + am, gk = k0 + ak;
      ra[r] = (gm < g.M && gk < kend) ? A[(long)gm * g.sam + (long)gk * g.sak] : 0.f;
      const int bk = b_kfast ? e % BK : e / BN, bn = b_kfast ? e / BK : e % BN;
      const int gk2 = k0 + bk, gn = n0 + bn;
      rb[r] = (gk2 < kend && gn < g.N) ? B[(long)gk2 * g.sbk + (long)gn * g.sbn] : 0.f;
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int e = tid + r * 256;
      const int am = a_mfast ? e % BM : e / BK, ak = a_mfast ? e / BM : e % BK;
      As[am][ak] = f2bf(ra[r]);
      const int bk = b_kfast ? e % BK : e / BN, bn = b_kfast ? e / BK : e % BN;
      Bs[bk][bn] = f2bf(rb[r]);
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int kq = kk + 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + 16 * i + (lane & 15);
        short4_t a;
        a[0] = (short)As[row][kq];
        a[1] = (short)As[row][kq + 1];
        a[2] = (short)As[row][kq + 2];
        a[3] = (short)As[row][kq + 3];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = wn + 16 * j + (lane & 15);
          short4_t bb;
          bb[0] = (short)Bs[kq][col];
          bb[1] = (short)Bs[kq + 1][col];
          bb[2] = (short)Bs[kq + 2][col];
          bb[3] = (short)Bs[kq + 3][col];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane l holds rows 4 (l / 16) + r, column l % 16 of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int gn = n0 + wn + 16 * j + (lane & 15);
        if (gm >= g.M || gn >= g.N) continue;
        if (g.ksplit > 1) {
          g.P[(((long)b * g.ksplit + sp) * g.M + gm) * g.N + gn] = acc[i][j][r];
        } else {
          const long off = (long)b * g.bsc + (long)gm * g.scm + (long)gn * g.scn;
          float* c = g.C + off;
          float val = g.alpha * acc[i][j][r] + (g.beta != 0.f ? g.beta * *c : 0.f);
          if (g.bias) {
            val += g.bias[gm];
            g.act[off] = gelu(val);
          }
          *c = val;
        }
      }
}


}  // namespace pts_mm
