// Complex GEMM engine on CDNA4 matrix cores (gfx950).
//
// Every dense contraction of the path is a complex GEMM: the metric and RHS
// pre-products of Algorithm 1 (T^k = X^k Y^{k H}), V^q = eta~ eta~^H of
// eqs. (7)-(8), the fragment pre-product T^k = X^k C^k of Algorithm 2 and the
// two contractions of eq. (19).  Complex products use four real MFMAs per
// 16x16 tile (re*re - im*im, re*im + im*re).  A 256-thread workgroup owns a
// 64x64 output tile: four waves in 2x2, each wave 2x2 MFMA tiles of 16x16.
// Operand tiles are staged through LDS as separate real and imaginary planes
// laid out [k][m] / [k][n], so the MFMA operand reads are 16 consecutive
// elements per k row.  The launch is persistent: blocks walk a global tile
// list that concatenates many descriptors (batched over k or q, or grouped
// over fragments of different sizes).
#include "kernels.hpp"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64;

// ---- precision traits ------------------------------------------------------
// FP64: LDS element double, v_mfma_f64_16x16x4 (K = 4 per MFMA), output
//       lane l register v holds row 4*v + l/16, column l%16.
// FP32: LDS element float, v_mfma_f32_16x16x4 (K = 4), output row
//       4*(l/16) + v, column l%16.
// BF16x3: LDS holds float; fragments are split at load into bf16 hi and lo,
//       v_mfma_f32_16x16x32_bf16 (K = 32, lane l holds k = 8*(l/16) .. +7),
//       output as FP32.
template <int P> struct Prec;
template <> struct Prec<0> { typedef double T; static constexpr int BK = 16; };
template <> struct Prec<1> { typedef float T; static constexpr int BK = 16; };
template <> struct Prec<2> { typedef float T; static constexpr int BK = 32; };

__device__ inline int isqrt_floor(long long x) {
  long long r = (long long)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return (int)r;
}

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <int P, bool A_KM, bool B_KN, bool A_CONJ, bool B_CONJ>
__global__ __launch_bounds__(256) void zgemm_kernel(const GemmDesc* __restrict__ descs, int ndesc,
                                                    long long total_tiles) {
  typedef typename Prec<P>::T T;
  constexpr int BK = Prec<P>::BK;
  constexpr int PAD = (sizeof(T) == 8) ? 1 : 1;
  constexpr int LDA_S = BM + PAD, LDB_S = BN + PAD;
  constexpr int NLOAD = (BM * BK) / 256;   // complex elements per thread per operand tile

  __shared__ T As_re[BK * LDA_S], As_im[BK * LDA_S];
  __shared__ T Bs_re[BK * LDB_S], Bs_im[BK * LDB_S];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  for (long long t = blockIdx.x; t < total_tiles; t += gridDim.x) {
    // ---- locate descriptor and tile ----
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (descs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const GemmDesc d = descs[lo];
    long long local = t - d.tile_begin;
    const int b = (int)(local / d.tiles_per_batch);
    int lt = (int)(local - (long long)b * d.tiles_per_batch);
    int tm, tn;
    if (d.herm) {
      tm = (isqrt_floor(8LL * lt + 1) - 1) / 2;
      tn = lt - tm * (tm + 1) / 2;
    } else {
      tm = lt / d.tiles_n;
      tn = lt - tm * d.tiles_n;
    }
    const int m0 = tm * BM, n0 = tn * BN;
    const cplx* Ab = d.A + (long long)b * d.sA_bat;
    const cplx* Bb = d.B + (long long)b * d.sB_bat;

    d4 acc_re[2][2], acc_im[2][2];
    f4 a32_re[2][2], a32_im[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc_re[i][j] = d4{0, 0, 0, 0};
        acc_im[i][j] = d4{0, 0, 0, 0};
        a32_re[i][j] = f4{0, 0, 0, 0};
        a32_im[i][j] = f4{0, 0, 0, 0};
      }

    for (int seg = 0; seg < d.nseg; ++seg) {
      const cplx* As = Ab + (long long)seg * d.sA_seg;
      const cplx* Bs = Bb + (long long)seg * d.sB_seg;
      const int Kcur = (seg == d.nseg - 1) ? d.Klast : d.Kseg;
      for (int k0 = 0; k0 < Kcur; k0 += BK) {
        cplx ra[NLOAD], rb[NLOAD];
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
          int idx = tid + 256 * i;
          int kk, mm;
          if (A_KM) { kk = idx / BM; mm = idx % BM; } else { mm = idx / BK; kk = idx % BK; }
          int gm = m0 + mm, gk = k0 + kk;
          cplx v = cmk(0.0, 0.0);
          if (gm < d.M && gk < Kcur)
            v = A_KM ? As[(long long)gk * d.lda + gm] : As[(long long)gm * d.lda + gk];
          if (A_CONJ) v.y = -v.y;
          ra[i] = v;
          int nn;
          if (B_KN) { kk = idx / BN; nn = idx % BN; } else { nn = idx / BK; kk = idx % BK; }
          int gn = n0 + nn;
          gk = k0 + kk;
          cplx w = cmk(0.0, 0.0);
          if (gn < d.N && gk < Kcur)
            w = B_KN ? Bs[(long long)gk * d.ldb + gn] : Bs[(long long)gn * d.ldb + gk];
          if (B_CONJ) w.y = -w.y;
          rb[i] = w;
        }
        __syncthreads();   // previous tile's reads are done
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
          int idx = tid + 256 * i;
          int kk, mm;
          if (A_KM) { kk = idx / BM; mm = idx % BM; } else { mm = idx / BK; kk = idx % BK; }
          As_re[kk * LDA_S + mm] = (T)ra[i].x;
          As_im[kk * LDA_S + mm] = (T)ra[i].y;
          int nn;
          if (B_KN) { kk = idx / BN; nn = idx % BN; } else { nn = idx / BK; kk = idx % BK; }
          Bs_re[kk * LDB_S + nn] = (T)rb[i].x;
          Bs_im[kk * LDB_S + nn] = (T)rb[i].y;
        }
        __syncthreads();

        if constexpr (P == 0 || P == 1) {
#pragma unroll
          for (int ks = 0; ks < BK; ks += 4) {
            const int kr = ks + (lane >> 4);
            T a_re[2], a_im[2], na_im[2], b_re[2], b_im[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              int mm = wm * 32 + i * 16 + (lane & 15);
              a_re[i] = As_re[kr * LDA_S + mm];
              a_im[i] = As_im[kr * LDA_S + mm];
              na_im[i] = -a_im[i];
              int nn = wn * 32 + i * 16 + (lane & 15);
              b_re[i] = Bs_re[kr * LDB_S + nn];
              b_im[i] = Bs_im[kr * LDB_S + nn];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 2; ++j) {
                if constexpr (P == 0) {
                  acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re[i], b_re[j], acc_re[i][j], 0, 0, 0);
                  acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(na_im[i], b_im[j], acc_re[i][j], 0, 0, 0);
                  acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re[i], b_im[j], acc_im[i][j], 0, 0, 0);
                  acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_im[i], b_re[j], acc_im[i][j], 0, 0, 0);
                } else {
                  a32_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_re[i], b_re[j], a32_re[i][j], 0, 0, 0);
                  a32_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(na_im[i], b_im[j], a32_re[i][j], 0, 0, 0);
                  a32_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_re[i], b_im[j], a32_im[i][j], 0, 0, 0);
                  a32_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_im[i], b_re[j], a32_im[i][j], 0, 0, 0);
                }
              }
          }
        } else {
          // bf16 x3: K = 32 per MFMA, lane holds 8 consecutive k of one row/column
          const int kb = (lane >> 4) * 8;
          bf8 ar_h[2], ar_l[2], ai_h[2], ai_l[2], nai_h[2], nai_l[2];
          bf8 br_h[2], br_l[2], bi_h[2], bi_l[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            int mm = wm * 32 + i * 16 + (lane & 15);
            int nn = wn * 32 + i * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              __bf16 h, l;
              split_bf16(As_re[(kb + e) * LDA_S + mm], h, l); ar_h[i][e] = h; ar_l[i][e] = l;
              float aim = As_im[(kb + e) * LDA_S + mm];
              split_bf16(aim, h, l); ai_h[i][e] = h; ai_l[i][e] = l;
              split_bf16(-aim, h, l); nai_h[i][e] = h; nai_l[i][e] = l;
              split_bf16(Bs_re[(kb + e) * LDB_S + nn], h, l); br_h[i][e] = h; br_l[i][e] = l;
              split_bf16(Bs_im[(kb + e) * LDB_S + nn], h, l); bi_h[i][e] = h; bi_l[i][e] = l;
            }
          }
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              f4 cr = a32_re[i][j], ci = a32_im[i][j];
              // re += ar*br - ai*bi  (each product as hi*hi + hi*lo + lo*hi)
              cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_l[i], br_h[j], cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h[i], br_l[j], cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai_l[i], bi_h[j], cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai_h[i], bi_l[j], cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h[i], br_h[j], cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai_h[i], bi_h[j], cr, 0, 0, 0);
              // im += ar*bi + ai*br
              ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_l[i], bi_h[j], ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h[i], bi_l[j], ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_l[i], br_h[j], ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_h[i], br_l[j], ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar_h[i], bi_h[j], ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai_h[i], br_h[j], ci, 0, 0, 0);
              a32_re[i][j] = cr;
              a32_im[i][j] = ci;
            }
        }
      }
      if constexpr (P != 0) {
        // FP64 accumulation across K segments (q blocks)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              acc_re[i][j][v] += (double)a32_re[i][j][v];
              acc_im[i][j][v] += (double)a32_im[i][j][v];
              a32_re[i][j][v] = 0.f;
              a32_im[i][j][v] = 0.f;
            }
      }
    }

    // ---- epilogue ----
    cplx* Cb = d.C + (long long)b * d.sC_bat;
    const bool mirror = d.herm && (tm != tn);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int r = (P == 0) ? (4 * v + (lane >> 4)) : (4 * (lane >> 4) + v);
          int c = lane & 15;
          int m = m0 + wm * 32 + i * 16 + r;
          int n = n0 + wn * 32 + j * 16 + c;
          if (m >= d.M || n >= d.N) continue;
          cplx val = cmk(acc_re[i][j][v], acc_im[i][j][v]);
          if (d.epi == 2) {
            const int nf = d.nf;
            const long long nf2 = (long long)nf * nf;
            const int s_ = n / nf, r_ = n - s_ * nf;
            Cb[(long long)m * nf2 + (long long)r_ * nf + s_] = val;
            if (mirror) {
              const int p_ = m / nf, q_ = m - p_ * nf;
              Cb[(long long)n * nf2 + (long long)q_ * nf + p_] = cconj(val);
            }
          } else {
            long long o = (long long)m * d.ldc + n;
            if (d.epi == 1) val = cadd(Cb[o], val);
            Cb[o] = val;
            if (mirror) {
              long long o2 = (long long)n * d.ldc + m;
              cplx v2 = cconj(cmk(acc_re[i][j][v], acc_im[i][j][v]));
              if (d.epi == 1) v2 = cadd(Cb[o2], v2);
              Cb[o2] = v2;
            }
          }
        }
  }
}

template <int P>
hipError_t launch_p(int flags, const GemmDesc* descs, int ndesc, long long total, int blocks,
                    hipStream_t s) {
  dim3 g(blocks), b(256);
  switch (flags & 15) {
#define CASE(F)                                                                                    \
  case F:                                                                                          \
    hipLaunchKernelGGL((zgemm_kernel<P, (F & 1) != 0, (F & 2) != 0, (F & 4) != 0, (F & 8) != 0>), \
                       g, b, 0, s, descs, ndesc, total);                                           \
    break;
    // layouts used by the path: A_KM|B_KN, B_CONJ, A_KM|B_KN|B_CONJ, B_KN (the
    // zeta route's Pi^+ eta), B_KN|B_CONJ (P^k X^{k H} of the exchange) and
    // A_KM|B_KN|A_CONJ (A^H A of the RPA determinant)
    CASE(2) CASE(3) CASE(7) CASE(8) CASE(10) CASE(11)
    default: return hipErrorInvalidValue;
#undef CASE
  }
  return hipGetLastError();
}

}  // namespace

long long gemm_plan(GemmDesc* d, int n) {
  long long acc = 0;
  for (int i = 0; i < n; ++i) {
    d[i].tiles_m = ceil_div(d[i].M, BM);
    d[i].tiles_n = ceil_div(d[i].N, BN);
    d[i].tiles_per_batch = d[i].herm ? d[i].tiles_m * (d[i].tiles_m + 1) / 2
                                     : d[i].tiles_m * d[i].tiles_n;
    if (d[i].Klast <= 0 || d[i].Klast > d[i].Kseg) d[i].Klast = d[i].Kseg;
    d[i].tile_begin = acc;
    acc += (long long)d[i].tiles_per_batch * d[i].batch;
  }
  return acc;
}

hipError_t gemm_launch(int prec, int flags, const GemmDesc* descs_dev, int ndesc,
                       long long total, int max_blocks, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  int blocks = (int)(total < max_blocks ? total : max_blocks);
  if (prec == 0) return launch_p<0>(flags, descs_dev, ndesc, total, blocks, s);
  if (prec == 1) return launch_p<1>(flags, descs_dev, ndesc, total, blocks, s);
  return launch_p<2>(flags, descs_dev, ndesc, total, blocks, s);
}
