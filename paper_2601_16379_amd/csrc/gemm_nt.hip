// Complex "NT" GEMM on CDNA4 matrix cores for the three large contractions
// of the path (V^q of eq. (7), U^q = R^q W^q and the fragment contraction of
// eq. (19)):
//
//   C[m][n] (+)= sum_{s < nseg} sum_{k} opA(A_s[m][k]) * opB(B_s[n][k])
//
// Both operands are k-contiguous rows (no transposes anywhere), stored in the
// format of the precision:
//   FP64    complex128 interleaved rows; v_mfma_f64_16x16x4;
//   FP32    two float planes (re, im), rows zero-padded to a multiple of 8;
//           v_mfma_f32_16x16x4.
// (bf16x3 operands use the kernel of gemm_x3.hip.)  A lane-local permutation
// of k (lane l of an MFMA step s takes k = K_l + s with K_l = (l/16) * steps)
// lets every lane read its operand fragment with 16-byte LDS loads; A and B
// use the same permutation, so the sum over k is unchanged.  In FP32 each K
// segment (one q, or one block of grid points) accumulates in FP32 and is
// added into FP64 registers, so sums over q are FP64.
//
// Workgroup: 256 threads, 64x64 output tile, four waves in 2x2, each wave
// 2x2 MFMA tiles of 16x16; persistent over a global tile list that
// concatenates descriptors (batches over q, or fragments of different sizes).
#include "kernels.hpp"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64;

__device__ inline int isqrt_floor(long long x) {
  long long r = (long long)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return (int)r;
}

template <int P> struct NtCfg;
// FP64: BK = 16, LDS planes re/im of doubles, row pitch 18 (16 + 2 pad)
template <> struct NtCfg<0> { static constexpr int BK = 16, PITCH = 18, PLANES = 2; typedef double T; };
// FP32: BK = 32, planes re/im of floats, pitch 36
template <> struct NtCfg<1> { static constexpr int BK = 32, PITCH = 36, PLANES = 2; typedef float T; };

// Stage one operand tile (64 rows x BK) from global memory into registers.
// Returns per-thread vectors; rows >= nrows or k >= kcur read as zero.
template <int P, bool CONJ>
__device__ inline void load_tile(const void* base, long long ld, long long plane, int row0, int nrows,
                                 int k0, int kcur, u4 (&r)[4]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = tid + 256 * i;
    u4 x = u4{0, 0, 0, 0};
    if constexpr (P == 0) {
      // 64 rows x 16 complex: v -> row v/16, k v%16 (one complex per vector)
      const int row = v >> 4, k = v & 15;
      if (row0 + row < nrows && k0 + k < kcur) {
        const cplx* p = (const cplx*)base + (long long)(row0 + row) * ld + k0 + k;
        x = *(const u4*)p;
        if (CONJ) {
          double im = -__builtin_bit_cast(double, (unsigned long long)x.z | ((unsigned long long)x.w << 32));
          unsigned long long b = __builtin_bit_cast(unsigned long long, im);
          x.z = (unsigned int)b;
          x.w = (unsigned int)(b >> 32);
        }
      }
    } else {
      // 2 planes x 64 rows x 8 chunks of 4 floats: v -> plane v/512, row, chunk
      const int pl = v >> 9, row = (v >> 3) & 63, c = v & 7;
      if (row0 + row < nrows && k0 + 4 * c < kcur) {
        const float* p = (const float*)base + pl * plane + (long long)(row0 + row) * ld + k0 + 4 * c;
        x = *(const u4*)p;
        if (CONJ && pl == 1) x = u4{x.x ^ 0x80000000u, x.y ^ 0x80000000u, x.z ^ 0x80000000u, x.w ^ 0x80000000u};
      }
    }
    r[i] = x;
  }
}

template <int P>
__device__ inline void store_tile(typename NtCfg<P>::T* s, const u4 (&r)[4]) {
  constexpr int PITCH = NtCfg<P>::PITCH;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = tid + 256 * i;
    if constexpr (P == 0) {
      const int row = v >> 4, k = v & 15;
      double* sd = (double*)s;
      sd[(0 * 64 + row) * PITCH + k] =
          __builtin_bit_cast(double, (unsigned long long)r[i].x | ((unsigned long long)r[i].y << 32));
      sd[(1 * 64 + row) * PITCH + k] =
          __builtin_bit_cast(double, (unsigned long long)r[i].z | ((unsigned long long)r[i].w << 32));
    } else {
      const int pl = v >> 9, row = (v >> 3) & 63, c = v & 7;
      *(u4*)((float*)s + (pl * 64 + row) * PITCH + 4 * c) = r[i];
    }
  }
}

// KIND only names the call site in profiles (0 generic, 1 V^q, 2 U^q,
// 3 fragment contraction); the code is the same.
template <int P, bool A_CONJ, bool B_CONJ, int KIND>
__global__ __launch_bounds__(256, 2) void zgemm_nt_kernel(const NtDesc* __restrict__ descs, int ndesc,
                                                       long long total_tiles) {
  typedef typename NtCfg<P>::T T;
  constexpr int BK = NtCfg<P>::BK, PITCH = NtCfg<P>::PITCH, PLANES = NtCfg<P>::PLANES;
  __shared__ __attribute__((aligned(16))) T sA[PLANES * 64 * PITCH];
  __shared__ __attribute__((aligned(16))) T sB[PLANES * 64 * PITCH];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15;     // row / column within a 16x16 MFMA tile
  const int lk = lane >> 4;     // k group of the lane

  // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs,
  // so iteration `it` of workgroup b maps to a tile such that each XCD walks
  // a contiguous range of the tile list (tiles that share operand rows then
  // share that XCD's L2).  gridDim.x is a multiple of 8.
  const long long t8 = (total_tiles + 7) / 8 * 8;
  const long long per = t8 / 8;
  for (long long it = blockIdx.x; it < t8; it += gridDim.x) {
    const long long t = (it % 8) * per + it / 8;
    if (t >= total_tiles) continue;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const NtDesc d = descs[lo];
    const long long local = t - d.tile_begin;
    const int b = (int)(local / d.tiles_per_batch);
    const int lt = (int)(local - (long long)b * d.tiles_per_batch);
    int tm, tn;
    if (d.herm) {
      tm = (isqrt_floor(8LL * lt + 1) - 1) / 2;
      tn = lt - tm * (tm + 1) / 2;
    } else {
      tm = lt / d.tiles_n;
      tn = lt - tm * d.tiles_n;
    }
    const int m0 = tm * TM, n0 = tn * TN;
    const size_t esz = (P == 0) ? sizeof(cplx) : sizeof(float);
    const char* Ab = (const char*)d.A + (long long)b * d.sA_bat * esz;
    const char* Bb = (const char*)d.B + (long long)b * d.sB_bat * esz;

    d4 acc_re[2][2], acc_im[2][2];
    f4 c_re[2][2], c_im[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc_re[i][j] = d4{0, 0, 0, 0};
        acc_im[i][j] = d4{0, 0, 0, 0};
        c_re[i][j] = f4{0, 0, 0, 0};
        c_im[i][j] = f4{0, 0, 0, 0};
      }

    for (int seg = 0; seg < d.nseg; ++seg) {
      const char* As = Ab + (long long)seg * d.sA_seg * esz;
      const char* Bs = Bb + (long long)seg * d.sB_seg * esz;
      const int kcur = (seg == d.nseg - 1) ? d.Klast : d.Kseg;
      u4 ra[4], rb[4];
      load_tile<P, A_CONJ>(As, d.lda, d.a_plane, m0, d.M, 0, kcur, ra);
      load_tile<P, B_CONJ>(Bs, d.ldb, d.b_plane, n0, d.N, 0, kcur, rb);
      for (int k0 = 0; k0 < kcur; k0 += BK) {
        __syncthreads();
        store_tile<P>(sA, ra);
        store_tile<P>(sB, rb);
        __syncthreads();
        if (k0 + BK < kcur) {   // prefetch the next k block while this one is multiplied
          load_tile<P, A_CONJ>(As, d.lda, d.a_plane, m0, d.M, k0 + BK, kcur, ra);
          load_tile<P, B_CONJ>(Bs, d.ldb, d.b_plane, n0, d.N, k0 + BK, kcur, rb);
        }
        if constexpr (P == 0) {
          // lane k-set: 4*lk + s, s = 0..3 (two 16-byte loads per plane)
          const double* a = (const double*)sA;
          const double* bb = (const double*)sB;
          double ar[2][4], ai[2][4], br[2][4], bi[2][4];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int ra_ = wm * 32 + i * 16 + lr, rb_ = wn * 32 + i * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              ar[i][s] = a[(0 * 64 + ra_) * PITCH + 4 * lk + s];
              ai[i][s] = a[(1 * 64 + ra_) * PITCH + 4 * lk + s];
              br[i][s] = bb[(0 * 64 + rb_) * PITCH + 4 * lk + s];
              bi[i][s] = bb[(1 * 64 + rb_) * PITCH + 4 * lk + s];
            }
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 2; ++j) {
                acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i][s], br[j][s], acc_re[i][j], 0, 0, 0);
                acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i][s], bi[j][s], acc_re[i][j], 0, 0, 0);
                acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i][s], bi[j][s], acc_im[i][j], 0, 0, 0);
                acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i][s], br[j][s], acc_im[i][j], 0, 0, 0);
              }
        } else {
          // lane k-set: 8*lk + s, s = 0..7
          const float* a = (const float*)sA;
          const float* bb = (const float*)sB;
#pragma unroll
          for (int half = 0; half < 2; ++half) {
            float ar[2][4], ai[2][4], br[2][4], bi[2][4];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              const int ra_ = wm * 32 + i * 16 + lr, rb_ = wn * 32 + i * 16 + lr;
              const f4 x0 = *(const f4*)&a[(0 * 64 + ra_) * PITCH + 8 * lk + 4 * half];
              const f4 x1 = *(const f4*)&a[(1 * 64 + ra_) * PITCH + 8 * lk + 4 * half];
              const f4 y0 = *(const f4*)&bb[(0 * 64 + rb_) * PITCH + 8 * lk + 4 * half];
              const f4 y1 = *(const f4*)&bb[(1 * 64 + rb_) * PITCH + 8 * lk + 4 * half];
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                ar[i][s] = x0[s];
                ai[i][s] = x1[s];
                br[i][s] = y0[s];
                bi[i][s] = y1[s];
              }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
              for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                  c_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i][s], br[j][s], c_re[i][j], 0, 0, 0);
                  c_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[i][s], bi[j][s], c_re[i][j], 0, 0, 0);
                  c_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i][s], bi[j][s], c_im[i][j], 0, 0, 0);
                  c_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i][s], br[j][s], c_im[i][j], 0, 0, 0);
                }
          }
        }
      }
      if constexpr (P != 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              acc_re[i][j][v] += (double)c_re[i][j][v];
              acc_im[i][j][v] += (double)c_im[i][j][v];
              c_re[i][j][v] = 0.f;
              c_im[i][j][v] = 0.f;
            }
      }
    }

    // ---- epilogue ----
    const bool mirror = (d.herm == 1) && (tm != tn);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = (P == 0) ? (4 * v + lk) : (4 * lk + v);
          const int m = m0 + wm * 32 + i * 16 + r;
          const int n = n0 + wn * 32 + j * 16 + lr;
          if (m >= d.M) continue;
          const double vr = acc_re[i][j][v], vi = acc_im[i][j][v];
          if (d.epi == 3) {
            // split store (format of P) with zero fill of the row padding
            if (n >= (d.npad ? d.npad : d.ldc)) continue;
            const bool in = n < d.N;
            const long long o = (long long)b * d.sC_bat + (long long)m * d.ldc + n;
            if constexpr (P == 1) {
              float* c = (float*)d.C;
              c[o] = in ? (float)vr : 0.f;
              c[d.c_plane + o] = in ? (float)vi : 0.f;
            }
            continue;
          }
          if (n >= d.N) continue;
          cplx* Cb = (cplx*)d.C + (long long)b * d.sC_bat;
          cplx val = cmk(vr, vi);
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
            const long long o = (long long)m * d.ldc + n;
            if (d.epi == 1) val = cadd(Cb[o], val);
            if (d.epi == 4) val = csub(Cb[o], val);
            Cb[o] = val;
            if (mirror) {
              const long long o2 = (long long)n * d.ldc + m;
              cplx v2 = cmk(vr, -vi);
              if (d.epi == 1) v2 = cadd(Cb[o2], v2);
              Cb[o2] = v2;
            }
          }
        }
  }
}

template <int P, int KIND>
hipError_t launch_nt(int conj, const NtDesc* descs, int ndesc, long long total, int blocks,
                     hipStream_t s) {
  dim3 g(blocks), b(256);
  switch (conj & 3) {
    case 0: hipLaunchKernelGGL((zgemm_nt_kernel<P, false, false, KIND>), g, b, 0, s, descs, ndesc, total); break;
    case 1: hipLaunchKernelGGL((zgemm_nt_kernel<P, true, false, KIND>), g, b, 0, s, descs, ndesc, total); break;
    case 2: hipLaunchKernelGGL((zgemm_nt_kernel<P, false, true, KIND>), g, b, 0, s, descs, ndesc, total); break;
    default: hipLaunchKernelGGL((zgemm_nt_kernel<P, true, true, KIND>), g, b, 0, s, descs, ndesc, total); break;
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_kind(int kind, int conj, const NtDesc* descs, int ndesc, long long total, int blocks,
                       hipStream_t s) {
  switch (kind) {
    case 1: return launch_nt<P, 1>(conj, descs, ndesc, total, blocks, s);
    case 2: return launch_nt<P, 2>(conj, descs, ndesc, total, blocks, s);
    case 3: return launch_nt<P, 3>(conj, descs, ndesc, total, blocks, s);
    default: return launch_nt<P, 0>(conj, descs, ndesc, total, blocks, s);
  }
}

}  // namespace

long long nt_plan(NtDesc* d, int n) {
  long long acc = 0;
  for (int i = 0; i < n; ++i) {
    d[i].tiles_m = ceil_div(d[i].M, TM);
    d[i].tiles_n = ceil_div(d[i].N, TN);
    d[i].tiles_per_batch = d[i].herm ? d[i].tiles_m * (d[i].tiles_m + 1) / 2
                                     : d[i].tiles_m * d[i].tiles_n;
    if (d[i].Klast <= 0 || d[i].Klast > d[i].Kseg) d[i].Klast = d[i].Kseg;
    d[i].tile_begin = acc;
    acc += (long long)d[i].tiles_per_batch * d[i].batch;
  }
  return acc;
}

hipError_t nt_launch(int prec, int conj, const NtDesc* descs_dev, int ndesc, long long total,
                     int max_blocks, hipStream_t s, int kind) {
  if (total <= 0) return hipSuccess;
  const long long t8 = (total + 7) / 8 * 8;
  max_blocks = max_blocks / 8 * 8;
  const int blocks = (int)(t8 < max_blocks ? t8 : max_blocks);
  // FP64 and FP32 operands; bf16 hi+lo operands go through x3_launch
  if (prec == 0) return launch_kind<0>(kind, conj, descs_dev, ndesc, total, blocks, s);
  if (prec == 1) return launch_kind<1>(kind, conj, descs_dev, ndesc, total, blocks, s);
  return hipErrorInvalidValue;
}
