// Large-tile complex "NT" GEMM for the FP32 mixed precision: 128x128 output
// tile per 512-thread workgroup, one K segment per launch (the bf16x3
// operands have their own kernel in gemm_x3.hip).
//
//   C[m][n] (+)= sum_k opA(A_seg[m][k]) opB(B_seg[n][k])
//
// The sums over segments (q of eq. (19), blocks of grid points of eq. (7))
// are made by launching once per segment and adding each FP32 partial into
// an FP64 output matrix (epi 1: the first segment stores, the later ones
// add), so every cross-segment sum is FP64 while the
// kernel keeps only FP32 accumulators; that frees the registers for a tile
// twice as large in each direction as the segmented kernel of gemm_nt.hip,
// which halves the operand traffic per flop.  Operand formats and the
// lane-local k permutation are those of gemm_nt.hip.  Eight waves in 4 x 2,
// each 32 x 64 (2 x 4 MFMA tiles of 16x16).  The template parameter P is the
// operand format (1 = two FP32 planes, the only one instantiated).
#include "kernels.hpp"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int BT = 128;     // tile edge
constexpr int NT = 512;     // threads

__device__ inline int isqrt_floor(long long x) {
  long long r = (long long)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return (int)r;
}
__device__ inline u4 neg_f32x4(u4 v) {
  return u4{v.x ^ 0x80000000u, v.y ^ 0x80000000u, v.z ^ 0x80000000u, v.w ^ 0x80000000u};
}

// BK = 64 k per stage: enough MFMA work per stage to cover the latency of
// the next stage's global loads (one workgroup per CU).
constexpr int BK = 64;
template <int P> struct BigCfg;
// per row: 64 floats (16 vectors of 4) + 4 pad
template <> struct BigCfg<1> { static constexpr int PITCH = 68, PLANES = 2, VPR = 16, EPV = 4; typedef float T; };
constexpr int NV = 8;   // 16-byte vectors per thread per operand stage (128 x 64 x 8 B / 16 B / 512)

// 128 rows x 64 k of one operand (all planes): 4096 16-byte vectors, 8 per thread
template <int P, bool CONJ>
__device__ inline void big_load(const void* base, long long ld, long long plane, int row0, int nrows,
                                int k0, int kcur, u4 (&r)[NV]) {
  typedef typename BigCfg<P>::T T;
  constexpr int VPR = BigCfg<P>::VPR, EPV = BigCfg<P>::EPV;
  constexpr int RSH = (VPR == 16) ? 4 : 3, PSH = RSH + 7;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int v = threadIdx.x + NT * i;
    const int pl = v >> PSH, row = (v >> RSH) & 127, c = v & (VPR - 1);
    u4 x = u4{0, 0, 0, 0};
    if (row0 + row < nrows && k0 + EPV * c < kcur) {
      x = *(const u4*)((const T*)base + pl * plane + (long long)(row0 + row) * ld + k0 + EPV * c);
      if constexpr (CONJ) {
        if (pl == 1) x = neg_f32x4(x);
      }
    }
    r[i] = x;
  }
}

template <int P>
__device__ inline void big_store(typename BigCfg<P>::T* s, const u4 (&r)[NV]) {
  constexpr int PITCH = BigCfg<P>::PITCH, VPR = BigCfg<P>::VPR, EPV = BigCfg<P>::EPV;
  constexpr int RSH = (VPR == 16) ? 4 : 3, PSH = RSH + 7;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int v = threadIdx.x + NT * i;
    const int pl = v >> PSH, row = (v >> RSH) & 127, c = v & (VPR - 1);
    *(u4*)(s + (pl * BT + row) * PITCH + EPV * c) = r[i];
  }
}

template <int P, bool A_CONJ, bool B_CONJ, int KIND>
__global__ __launch_bounds__(NT) void zgemm_big_kernel(const NtDesc* __restrict__ descs, int ndesc,
                                                        long long total_tiles, int seg) {
  typedef typename BigCfg<P>::T T;
  constexpr int PITCH = BigCfg<P>::PITCH, PLANES = BigCfg<P>::PLANES;
  __shared__ __attribute__((aligned(16))) T sA[PLANES * BT * PITCH];
  __shared__ __attribute__((aligned(16))) T sB[PLANES * BT * PITCH];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;   // 4 x 2 waves, each 32 x 64
  const int lr = lane & 15, lk = lane >> 4;

  const long long t8 = (total_tiles + 7) / 8 * 8;
  const long long per = t8 / 8;
  for (long long it = blockIdx.x; it < t8; it += gridDim.x) {
    const long long t = (it % 8) * per + it / 8;   // XCD-contiguous tile ranges
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
    const int m0 = tm * BT, n0 = tn * BT;
    const size_t esz = sizeof(T);
    // a triangular B (zero for k < n) contributes from k = n0 on
    const int kstart = d.ktri ? n0 : 0;
    const char* As = (const char*)d.A + ((long long)b * d.sA_bat + (long long)seg * d.sA_seg + kstart) * esz;
    const char* Bs = (const char*)d.B + ((long long)b * d.sB_bat + (long long)seg * d.sB_seg + kstart) * esz;
    const int kcur = ((seg == d.nseg - 1) ? d.Klast : d.Kseg) - kstart;

    f4 c_re[2][4], c_im[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c_re[i][j] = f4{0, 0, 0, 0};
        c_im[i][j] = f4{0, 0, 0, 0};
      }

    u4 ra[NV], rb[NV];
    big_load<P, A_CONJ>(As, d.lda, d.a_plane, m0, d.M, 0, kcur, ra);
    big_load<P, B_CONJ>(Bs, d.ldb, d.b_plane, n0, d.N, 0, kcur, rb);
    for (int k0 = 0; k0 < kcur; k0 += BK) {
      __syncthreads();
      big_store<P>(sA, ra);
      big_store<P>(sB, rb);
      __syncthreads();
      if (k0 + BK < kcur) {
        big_load<P, A_CONJ>(As, d.lda, d.a_plane, m0, d.M, k0 + BK, kcur, ra);
        big_load<P, B_CONJ>(Bs, d.ldb, d.b_plane, n0, d.N, k0 + BK, kcur, rb);
      }
      {
        // FP32: lane k-set 8*lk + s, s = 0..7, per 32-k quarter
        const float* a = (const float*)sA;
        const float* bb = (const float*)sB;
#pragma unroll
        for (int half = 0; half < 2 * (BK / 32); ++half) {
          float ar[2][4], ai[2][4];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int ra_ = wm * 32 + i * 16 + lr;
            const int ko = (half >> 1) * 32 + 8 * lk + 4 * (half & 1);
            const f4 x0 = *(const f4*)&a[(0 * BT + ra_) * PITCH + ko];
            const f4 x1 = *(const f4*)&a[(1 * BT + ra_) * PITCH + ko];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              ar[i][s] = x0[s];
              ai[i][s] = x1[s];
            }
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int rb_ = wn * 64 + j * 16 + lr;
            const int ko = (half >> 1) * 32 + 8 * lk + 4 * (half & 1);
            const f4 y0 = *(const f4*)&bb[(0 * BT + rb_) * PITCH + ko];
            const f4 y1 = *(const f4*)&bb[(1 * BT + rb_) * PITCH + ko];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
              for (int i = 0; i < 2; ++i) {
                c_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i][s], y0[s], c_re[i][j], 0, 0, 0);
                c_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[i][s], y1[s], c_re[i][j], 0, 0, 0);
                c_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i][s], y1[s], c_im[i][j], 0, 0, 0);
                c_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i][s], y0[s], c_im[i][j], 0, 0, 0);
              }
          }
        }
      }
    }

    // ---- epilogue (FP32 layout: lane l, register v -> row 4*(l/16)+v, column l%16) ----
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + wm * 32 + i * 16 + 4 * lk + v;
          const int n = n0 + wn * 64 + j * 16 + lr;
          if (m >= d.M) continue;
          const float vr = c_re[i][j][v], vi = c_im[i][j][v];
          const long long o = (long long)b * d.sC_bat + (long long)m * d.ldc + n;
          if (d.epi == 3) {
            if (n >= (d.npad ? d.npad : d.ldc)) continue;
            const bool in = n < d.N;
            store_fmt(d.C, o, d.c_plane, P, cmk(in ? vr : 0.0, in ? vi : 0.0));
          } else {
            if (n >= d.N) continue;
            cplx* c = (cplx*)d.C + o;
            cplx x = seg > 0 ? *c : cmk(0.0, 0.0);   // FP64 accumulation across launches
            x.x += (double)vr;
            x.y += (double)vi;
            *c = x;
          }
        }
  }
}

template <int P, int KIND>
hipError_t launch_big(int conj, const NtDesc* descs, int ndesc, long long total, int blocks, int seg,
                      hipStream_t s) {
  dim3 g(blocks), b(NT);
  switch (conj & 3) {
    case 0: hipLaunchKernelGGL((zgemm_big_kernel<P, false, false, KIND>), g, b, 0, s, descs, ndesc, total, seg); break;
    case 1: hipLaunchKernelGGL((zgemm_big_kernel<P, true, false, KIND>), g, b, 0, s, descs, ndesc, total, seg); break;
    case 2: hipLaunchKernelGGL((zgemm_big_kernel<P, false, true, KIND>), g, b, 0, s, descs, ndesc, total, seg); break;
    default: hipLaunchKernelGGL((zgemm_big_kernel<P, true, true, KIND>), g, b, 0, s, descs, ndesc, total, seg); break;
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_big_kind(int kind, int conj, const NtDesc* descs, int ndesc, long long total, int blocks,
                           int seg, hipStream_t s) {
  switch (kind) {
    case 1: return launch_big<P, 1>(conj, descs, ndesc, total, blocks, seg, s);
    case 2: return launch_big<P, 2>(conj, descs, ndesc, total, blocks, seg, s);
    case 3: return launch_big<P, 3>(conj, descs, ndesc, total, blocks, seg, s);
    default: return launch_big<P, 0>(conj, descs, ndesc, total, blocks, seg, s);
  }
}

// Hermitian matrices of which the lower triangle (diagonal included) was
// computed -> full matrix: every upper element is the conjugate of its
// lower mirror (the GEMMs compute lower tiles; in diagonal tiles the blocks
// strictly above the diagonal may be skipped)
__global__ void herm_fill_kernel(cplx* c, int n, long long ld, long long bat, int nbat) {
  const long long per = (long long)n * n;
  const long long total = per * nbat;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(idx / per);
    const long long e = idx - (long long)b * per;
    const int m = (int)(e / n), k = (int)(e - (e / n) * n);
    if (m < k) {
      const cplx v = c[(long long)b * bat + (long long)k * ld + m];
      c[(long long)b * bat + (long long)m * ld + k] = cmk(v.x, -v.y);
    }
  }
}

// E[(pq)][(sr)] (lower triangle computed) -> eri[p][q][r][s], fragment f
// reading e + eoff[f] and writing eri[f]
__global__ void eri_scatter_batch_kernel(const cplx* __restrict__ e, const long long* __restrict__ eoff,
                                         cplx* const* __restrict__ eri, const int* __restrict__ nfa) {
  const int f = blockIdx.y;
  const int nf = nfa[f];
  const cplx* ef = e + eoff[f];
  cplx* out = eri[f];
  const long long n = (long long)nf * nf;
  const long long total = n * n;
  // G[a][b] from the computed lower triangle (G is Hermitian)
  auto g = [&](long long a, long long b) { return a >= b ? ef[a * n + b] : cconj(ef[b * n + a]); };
  // (pq|rs) = G[(pq)][(sr)] + conj(G[(qp)][(rs)]) = v; (qp|sr) = conj(v),
  // (rs|pq) = v, (sr|qp) = conj(v): one thread per orbit {o1, o2, o3, o4}
  // (the smallest of the four output indices) reads G twice and writes all
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    const long long pq = o / n, rs = o - pq * n;
    const int p_ = (int)(pq / nf), q_ = (int)(pq - (long long)p_ * nf);
    const int r_ = (int)(rs / nf), s_ = (int)(rs - (long long)r_ * nf);
    const long long qp = (long long)q_ * nf + p_, sr = (long long)s_ * nf + r_;
    const long long o2 = qp * n + sr, o3 = rs * n + pq, o4 = sr * n + qp;
    if (o2 < o || o3 < o || o4 < o) continue;
    const cplx a = g(pq, sr), b = g(qp, rs);
    const cplx v = cmk(a.x + b.x, a.y - b.y), vc = cmk(v.x, -v.y);
    out[o] = v;
    out[o2] = vc;
    out[o3] = v;
    out[o4] = vc;
  }
}

inline unsigned grid_of(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

long long big_plan(NtDesc* d, int n) {
  long long acc = 0;
  for (int i = 0; i < n; ++i) {
    d[i].tiles_m = ceil_div(d[i].M, BT);
    d[i].tiles_n = ceil_div(d[i].N, BT);
    d[i].tiles_per_batch = d[i].herm ? d[i].tiles_m * (d[i].tiles_m + 1) / 2
                                     : d[i].tiles_m * d[i].tiles_n;
    if (d[i].Klast <= 0 || d[i].Klast > d[i].Kseg) d[i].Klast = d[i].Kseg;
    d[i].tile_begin = acc;
    acc += (long long)d[i].tiles_per_batch * d[i].batch;
  }
  return acc;
}

hipError_t big_launch(int prec, int conj, const NtDesc* descs_dev, int ndesc, long long total,
                      int max_blocks, int seg, hipStream_t s, int kind) {
  if (total <= 0) return hipSuccess;
  // FP32 operands only; bf16 hi+lo operands go through x3_launch
  if (prec != 1) return hipErrorInvalidValue;
  const long long t8 = (total + 7) / 8 * 8;
  max_blocks = max_blocks / 8 * 8;
  const int blocks = (int)(t8 < max_blocks ? t8 : max_blocks);
  return launch_big_kind<1>(kind, conj, descs_dev, ndesc, total, blocks, seg, s);
}

hipError_t herm_fill_launch(cplx* c, int n, long long ld, long long bat, int nbat, hipStream_t s) {
  hipLaunchKernelGGL(herm_fill_kernel, dim3(grid_of((long long)n * n * nbat)), dim3(256), 0, s, c, n, ld,
                     bat, nbat);
  return hipGetLastError();
}

hipError_t eri_scatter_batch_launch(const cplx* e, const long long* eoff, cplx* const* eri, const int* nf,
                                    int n, int maxnf, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long m = (long long)maxnf * maxnf;
  long long bx = (m * m + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(eri_scatter_batch_kernel, dim3((unsigned)bx, n), dim3(256), 0, s, e, eoff, eri, nf);
  return hipGetLastError();
}
