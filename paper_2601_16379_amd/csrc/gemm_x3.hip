// Complex "NT" GEMM on bf16 operands with the 32x32x16 bf16 matrix cores of
// gfx950, in two operand formats: F = 2, bf16 hi+lo (the bf16x3 precision),
// and F = 3, single bf16 (re, im) (the bf16 precision):
//
//   C[m][n] (+)= sum_k opA(A_seg[m][k]) opB(B_seg[n][k])
//
// F = 2: x = hi + lo per real component; every real product keeps hi*hi +
// hi*lo + lo*hi (three bf16 MFMAs, FP32 accumulation), and a complex product
// is four real ones, so one 32x32 complex block costs 12 MFMAs per 16 k.
// F = 3: one bf16 MFMA per real product, 8 MFMAs per 32 k.  In both formats
// one row of one stage is 128 contiguous bytes: 16 k x 4 planes (F = 2) or
// 32 k x 2 planes (F = 3), so the copies and the LDS layout are shared.
//
// Workgroup: 256 threads (4 waves, 2 x 2), 128 x 128 output tile, each wave
// 64 x 64 (2 x 2 blocks of 32 x 32); two workgroups per CU.  K advances in
// stages of 16 (one MFMA step).  In the operand format (bf16 hi/lo
// interleaved by 8-element groups) the 16 k of one row are 128 contiguous
// bytes, so a stage of a 128-row operand tile is 128 whole cache lines; it is
// copied from global memory straight into LDS (global_load_lds_dwordx4, no
// register staging) into one of two LDS stage buffers, one stage ahead of
// the one being multiplied.  Each stage: wait for its copies, one barrier
// (after it every wave has also read the previous stage, whose buffer then
// takes the copies of the next stage, issued first), read the fragments,
// MFMAs.  The stalls of one workgroup's waves are filled by the other
// workgroup's MFMAs.  (Two barriers a stage with the copies two stages
// ahead measured 8 % slower on the 1000-k contraction; so did issuing the
// fragment reads before the copies.)  A launch with fewer tiles than two
// rounds of workgroups leaves workgroups alone on their CUs; its
// contraction runs the two-barrier loop, which hides more latency
// (zgemm_c2b_kernel: 0.143 against 0.126 of peak at 216 k).  Both loops
// issue the same MFMAs in the same order: the results do not depend on the
// choice.  The single-bf16 contraction always runs the two-barrier loop.  In LDS a row keeps its eight 16-byte slots (2 k-groups x 4 planes)
// in an order XOR-permuted by the row, so that the 32x32 fragment reads
// (lane -> row l%32, k-group l/32) hit distinct banks.
//
// Rows beyond M / N are loaded from the last valid row (their outputs are
// dropped); 16-byte vectors that start beyond the segment length are copied
// from a zero block.  Each lane's copy sources are computed once per tile.
// One K segment per launch; epilogues as in the 128-tile FP32 kernel (split
// store, FP64 accumulation across launches).
#include "kernels.hpp"

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

constexpr int XT = 128;               // tile edge
constexpr int XK = 16;                // k per stage of the hi+lo format
// k per stage, u16 per element in the global layout, and log2 of the
// planes per 8-element group, by format
template <int F> struct Fmt;
template <> struct Fmt<2> { static constexpr int K = 16, EU = 4, PL = 2; };
template <> struct Fmt<3> { static constexpr int K = 32, EU = 2, PL = 1; };
constexpr int NBUF = 2;               // LDS stages (two workgroups per CU)
constexpr int XNT = 256;              // threads
constexpr int ROW_B = 128;             // bytes of one row of one stage
constexpr int OPER_B = XT * ROW_B;     // one operand tile of a stage (16 KB)
constexpr int STAGE_B = 2 * OPER_B;    // A and B (32 KB)
constexpr int NCOPY = 4;               // copy instructions per wave per operand and stage

// LDS position of 16-byte slot `slot` (k-group * 4 + plane) of a row
__device__ inline int lds_slot(int row, int slot) { return slot ^ ((row ^ (row >> 3)) & 7); }

__device__ inline bf8 as_bf8(u4 v) { return __builtin_bit_cast(bf8, v); }

// wait until at most n stages of copies (2 * NCOPY instructions each) are in flight
__device__ inline void wait_copies(int n) {
  static_assert(2 * NCOPY == 8, "vmcnt below counts 8 copies a stage");
  if (n >= 2) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
  else if (n == 1) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
  else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// The ring pipeline: one workgroup a CU, RING LDS stage buffers
constexpr int RING = 4;

__device__ inline int isqrt_floor(long long x) {
  long long r = (long long)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return (int)r;
}

// Vectors that start at or past the end of the K segment are copied from
// this zero block instead, so that LDS holds zeros there.
__device__ __attribute__((aligned(16))) unsigned short kZeroVec[8];

// Issue the copies of one operand's stage (128 rows x 128 bytes) into LDS at
// `dst`: 16 wave-instructions of 8 rows, 4 per wave.  src[j]: this lane's
// 16-byte source of the wave's j-th instruction at k = 0 (row base plus the
// slot gslot[j] whose LDS position is this lane's); the address advances by
// 4 u16 an element of k.  In the last stage of a segment, vectors that start
// at or past its end are copied from the zero block.
template <int F>
__device__ inline void stage_copy(const unsigned short* const (&src)[NCOPY], const int (&gslot)[NCOPY], int k0,
                                  int kcur, char* dst, int wave) {
  const bool tail = k0 + Fmt<F>::K > kcur;    // the same for the whole workgroup
#pragma unroll
  for (int j = 0; j < NCOPY; ++j) {
    const int rc = wave + 4 * j;          // rows rc*8 .. rc*8+7
    const unsigned short* g = src[j] + Fmt<F>::EU * k0;
    if (tail && k0 + 8 * (gslot[j] >> Fmt<F>::PL) >= kcur) g = kZeroVec;
    __builtin_amdgcn_global_load_lds((glb_void*)g, (lds_void*)(dst + rc * 8 * ROW_B), 16, 0, 0);
  }
}

// Fragments of one stage for this lane: A rows of the wave's two 32-row
// blocks, B rows of its two 32-column blocks, four planes each (16 bytes =
// 8 k of the lane's k-half).
// Fragments of one stage for this lane: NI 32-row blocks of A (rows rb0 +
// i * 32) and NJ 32-row blocks of B (rows cb0 + j * 32), four planes each
// (16 bytes = 8 k of the lane's k-group l/32).
template <int NI, int NJ>
struct Frag {
  u4 a[NI][4], b[NJ][4];
};

// The four 16-byte slots of a lane's row: F = 2, planes rh rl ih il of k-group
// lk; F = 3, (re, im) of k-group lk for the first MFMA step, then of k-group
// 2 + lk for the second.
template <int F>
__device__ inline int frag_slot(int lk, int x) {
  return F == 2 ? 4 * lk + x : 4 * (x >> 1) + 2 * lk + (x & 1);
}
template <int F, int NI, int NJ>
__device__ inline void read_frags_a(const char* buf, Frag<NI, NJ>& f, int rb0, int lr, int lk) {
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int row = rb0 + i * 32 + lr;
    const char* p = buf + row * ROW_B;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) f.a[i][pl] = *(const u4*)(p + (lds_slot(row, frag_slot<F>(lk, pl)) << 4));
  }
}
template <int F, int NI, int NJ>
__device__ inline void read_frags_b(const char* buf, Frag<NI, NJ>& f, int cb0, int lr, int lk) {
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int row = cb0 + j * 32 + lr;
    const char* p = buf + OPER_B + row * ROW_B;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) f.b[j][pl] = *(const u4*)(p + (lds_slot(row, frag_slot<F>(lk, pl)) << 4));
  }
}

// Pin a stage's fragments: their reads have completed here, and later uses
// do not depend on the loads any more.
template <int NI, int NJ>
__device__ inline void settle(Frag<NI, NJ>& f) {
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int p = 0; p < 4; ++p) asm volatile("" : "+v"(f.a[i][p]));
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int p = 0; p < 4; ++p) asm volatile("" : "+v"(f.b[j][p]));
}

__device__ inline u4 neg_bf(u4 v) {
  return u4{v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u};
}

// The 12 MFMAs of one 32x32 block pair (i, j) and one 16-k step, as six
// (re, im) term pairs: re += a_r b_r - a_i b_i, im += a_r b_i + a_i b_r,
// each real product as hi*hi + hi*lo + lo*hi; conjugation flips the sign of
// the imaginary planes of that operand.
struct BFr {
  bf8 rh, rl, ih, il, nih, nil;
};
template <bool CONJ>
__device__ inline BFr split_a(const u4 (&a)[4]) {
  const u4 ih = CONJ ? neg_bf(a[2]) : a[2];
  const u4 il = CONJ ? neg_bf(a[3]) : a[3];
  return BFr{as_bf8(a[0]), as_bf8(a[1]), as_bf8(ih), as_bf8(il), as_bf8(neg_bf(ih)), as_bf8(neg_bf(il))};
}
#define X3_TERMS(A, BRH, BRL, BIH, BIL, CR, CI, T)                          \
  if ((T) == 0) { CR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.rl, BRH, CR, 0, 0, 0);  \
                  CI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.rl, BIH, CI, 0, 0, 0); }\
  if ((T) == 1) { CR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.rh, BRL, CR, 0, 0, 0);  \
                  CI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.rh, BIL, CI, 0, 0, 0); }\
  if ((T) == 2) { CR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.nil, BIH, CR, 0, 0, 0); \
                  CI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.il, BRH, CI, 0, 0, 0); }\
  if ((T) == 3) { CR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.nih, BIL, CR, 0, 0, 0); \
                  CI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.ih, BRL, CI, 0, 0, 0); }\
  if ((T) == 4) { CR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.rh, BRH, CR, 0, 0, 0);  \
                  CI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.rh, BIH, CI, 0, 0, 0); }\
  if ((T) == 5) { CR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.nih, BIH, CR, 0, 0, 0); \
                  CI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.ih, BRH, CI, 0, 0, 0); }

// MFMAs of one stage for the wave's column block j; with two row blocks
// their four accumulator chains are interleaved (a chain every fourth MFMA).
template <int NI, int NJ, bool A_CONJ, bool B_CONJ>
__device__ inline void mma_half(const Frag<NI, NJ>& f, int j, f16v (&c_re)[NI][NJ], f16v (&c_im)[NI][NJ]) {
  const u4 bi = B_CONJ ? neg_bf(f.b[j][2]) : f.b[j][2];
  const u4 bl = B_CONJ ? neg_bf(f.b[j][3]) : f.b[j][3];
  const bf8 brh = as_bf8(f.b[j][0]), brl = as_bf8(f.b[j][1]), bih = as_bf8(bi), bil = as_bf8(bl);
  if constexpr (NI == 2) {
    const BFr x0 = split_a<A_CONJ>(f.a[0]), x1 = split_a<A_CONJ>(f.a[1]);
    f16v cr0 = c_re[0][j], ci0 = c_im[0][j], cr1 = c_re[1][j], ci1 = c_im[1][j];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      X3_TERMS(x0, brh, brl, bih, bil, cr0, ci0, t)
      X3_TERMS(x1, brh, brl, bih, bil, cr1, ci1, t)
    }
    c_re[0][j] = cr0;
    c_im[0][j] = ci0;
    c_re[1][j] = cr1;
    c_im[1][j] = ci1;
  } else {
    const BFr x0 = split_a<A_CONJ>(f.a[0]);
    f16v cr0 = c_re[0][j], ci0 = c_im[0][j];
#pragma unroll
    for (int t = 0; t < 6; ++t) { X3_TERMS(x0, brh, brl, bih, bil, cr0, ci0, t) }
    c_re[0][j] = cr0;
    c_im[0][j] = ci0;
  }
}
#undef X3_TERMS

// The 8 MFMAs of one stage of the single-bf16 format for the wave's column
// block j: two k steps (fragment slots 0, 1 and 2, 3 hold re, im), each
// re += a_r b_r - a_i b_i, im += a_r b_i + a_i b_r.
// The accumulator chains (re and im of each row block) are issued round
// robin, so that dependent MFMAs are 2 NI apart.
template <int NI, int NJ, bool A_CONJ, bool B_CONJ>
__device__ inline void mma_single(const Frag<NI, NJ>& f, int j, f16v (&c_re)[NI][NJ], f16v (&c_im)[NI][NJ]) {
  f16v cr[NI], ci[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    cr[i] = c_re[i][j];
    ci[i] = c_im[i][j];
  }
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    const u4 bi = B_CONJ ? neg_bf(f.b[j][2 * st + 1]) : f.b[j][2 * st + 1];
    const bf8 br = as_bf8(f.b[j][2 * st]), bim = as_bf8(bi);
    bf8 ar[NI], aim[NI], naim[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const u4 ai = A_CONJ ? neg_bf(f.a[i][2 * st + 1]) : f.a[i][2 * st + 1];
      ar[i] = as_bf8(f.a[i][2 * st]);
      aim[i] = as_bf8(ai);
      naim[i] = as_bf8(neg_bf(ai));
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) cr[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[i], br, cr[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NI; ++i) ci[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[i], bim, ci[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NI; ++i) cr[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(naim[i], bim, cr[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NI; ++i) ci[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aim[i], br, ci[i], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    c_re[i][j] = cr[i];
    c_im[i][j] = ci[i];
  }
}

// Epilogue of one tile (32x32 layout: lane l, register v -> row
// 8(v/4) + 4(l/32) + v%4, column l%32).  epi 3: each wave assembles its
// block 32 rows at a time in LDS (16 KB a wave) in the operand format (a row
// of NJ*32 points is NJ*256 contiguous bytes) and writes it with 16-byte
// stores; otherwise FP64 accumulation across launches (the first K segment,
// `first`, stores).
template <int F, int NI, int NJ>
__device__ inline void tile_epilogue(const NtDesc& d, int b, int m0, int n0, int rb0, int cb0,
                                     const f16v (&c_re)[NI][NJ], const f16v (&c_im)[NI][NJ], char* smem, int wave,
                                     int lane, bool first) {
  const int lr = lane & 31, lk = lane >> 5;
  if (d.epi == 3) {
    __syncthreads();                      // every wave is past its last stage reads
    unsigned short* st = (unsigned short*)(smem + wave * 16384);
    const int npad = d.npad ? d.npad : (int)d.ldc;
    constexpr int EU = Fmt<F>::EU;
    constexpr int RU = NJ * 32 * EU;      // u16 per staged row
    constexpr int PPR = NJ * 4 * EU;      // 16-byte parts per row
    unsigned short* C = (unsigned short*)d.C + EU * ((long long)b * d.sC_bat + n0 + cb0);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int ml = 8 * (v >> 2) + 4 * lk + (v & 3);
          const int nl = j * 32 + lr;
          const bool in = n0 + cb0 + nl < d.N;
          const float re = in ? c_re[i][j][v] : 0.f, im = in ? c_im[i][j][v] : 0.f;
          const unsigned short rh = bf16_bits_of(re), ih = bf16_bits_of(im);
          unsigned short* e = st + ml * RU + (nl >> 3) * (8 * EU) + (nl & 7);
          if constexpr (F == 2) {
            e[0] = rh;
            e[8] = bf16_bits_of(re - bf16_value(rh));
            e[16] = ih;
            e[24] = bf16_bits_of(im - bf16_value(ih));
          } else {
            e[0] = rh;
            e[8] = ih;
          }
        }
      __builtin_amdgcn_wave_barrier();
      // 32 staged rows of PPR parts, 64 lanes a pass
#pragma unroll 4
      for (int h = 0; h < PPR / 2; ++h) {
        const int c = h * 64 + lane, ml = c / PPR, part = c % PPR;
        const int m = m0 + rb0 + i * 32 + ml;
        if (m < d.M && n0 + cb0 + (part >> Fmt<F>::PL) * 8 < npad)
          *(u4*)(C + EU * (long long)m * d.ldc + part * 8) = *(const u4*)(st + ml * RU + part * 8);
      }
      __builtin_amdgcn_wave_barrier();
    }
  } else {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int m = m0 + rb0 + i * 32 + 8 * (v >> 2) + 4 * lk + (v & 3);
          const int n = n0 + cb0 + j * 32 + lr;
          if (m >= d.M || n >= d.N) continue;
          cplx* cp = (cplx*)d.C + (long long)b * d.sC_bat + (long long)m * d.ldc + n;
          cplx x = first ? cmk(0.0, 0.0) : *cp;   // FP64 accumulation across launches
          x.x += (double)c_re[i][j][v];
          x.y += (double)c_im[i][j][v];
          *cp = x;
        }
  }
}

// The MFMAs of one stage of fragments (both column blocks).
template <int F, int NI, int NJ, bool A_CONJ, bool B_CONJ>
__device__ inline void stage_mma(const Frag<NI, NJ>& f, f16v (&c_re)[NI][NJ], f16v (&c_im)[NI][NJ]) {
  if constexpr (F == 2) {
    mma_half<NI, NJ, A_CONJ, B_CONJ>(f, 0, c_re, c_im);
    if (NJ == 2) mma_half<NI, NJ, A_CONJ, B_CONJ>(f, NJ - 1, c_re, c_im);
  } else {
    mma_single<NI, NJ, A_CONJ, B_CONJ>(f, 0, c_re, c_im);
    if (NJ == 2) mma_single<NI, NJ, A_CONJ, B_CONJ>(f, NJ - 1, c_re, c_im);
  }
}

// The same with a triangular B (U^q in the factor form, kind 2): a column
// block whose B rows are all zero over the stage's k range (live0 / live1
// false) is skipped; it would add exact zeros.
template <int F, int NI, int NJ, bool A_CONJ, bool B_CONJ>
__device__ inline void stage_mma_tri(const Frag<NI, NJ>& f, f16v (&c_re)[NI][NJ], f16v (&c_im)[NI][NJ],
                                     bool live0, bool live1) {
  if constexpr (F == 2) {
    if (live0) mma_half<NI, NJ, A_CONJ, B_CONJ>(f, 0, c_re, c_im);
    if (NJ == 2 && live1) mma_half<NI, NJ, A_CONJ, B_CONJ>(f, NJ - 1, c_re, c_im);
  } else {
    if (live0) mma_single<NI, NJ, A_CONJ, B_CONJ>(f, 0, c_re, c_im);
    if (NJ == 2 && live1) mma_single<NI, NJ, A_CONJ, B_CONJ>(f, NJ - 1, c_re, c_im);
  }
}

// With a triangular B (B[n][k] = 0 for k < n; the K range starts at the
// tile's first column), column block j of the wave (columns cb0 + 32 j on)
// has only zeros in B over stage s when (s + 1) SK <= cb0 + 32 j.
__device__ inline void tri_live(bool tri, int s, int sk, int cb0, bool& l0, bool& l1) {
  l0 = !tri || (s + 1) * sk > cb0;
  l1 = !tri || (s + 1) * sk > cb0 + 32;
}

// K loop and epilogue of one tile.  The wave owns the (NI*32) x (NJ*32)
// block at rows rb0, columns cb0 of the tile: 64 x 64 in full tiles (2 x 2
// waves); in tiles with at most 32 valid rows (columns) each wave takes a
// 32 x 32 block of the one 32-row (32-column) strip, so edge tiles cost a
// quarter of the matrix-core work.  Two workgroups share a CU (64 KB of LDS
// each): two LDS stages, each stage's fragments read from LDS at its start
// (the waves of the other workgroup keep the matrix cores busy meanwhile),
// copies one stage ahead, one barrier a stage.
template <int F, int NI, int NJ, bool A_CONJ, bool B_CONJ, bool TRI>
__device__ inline void tile_body(const NtDesc& d, int b, int m0, int n0, int kcur,
                                 const unsigned short* const (&asrc)[NCOPY], const unsigned short* const (&bsrc)[NCOPY],
                                 const int (&gslot)[NCOPY], int rb0, int cb0, char* smem, int wave, int lane,
                                 bool idle, bool first) {
  const int lr = lane & 31, lk = lane >> 5;
  f16v c_re[NI][NJ], c_im[NI][NJ];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        c_re[i][j][v] = 0.f;
        c_im[i][j][v] = 0.f;
      }
  constexpr int SK = Fmt<F>::K;
  const int nst = (kcur + SK - 1) / SK;
  __syncthreads();                        // LDS of the previous tile no longer read
  stage_copy<F>(asrc, gslot, 0, kcur, smem, wave);
  stage_copy<F>(bsrc, gslot, 0, kcur, smem + OPER_B, wave);
  for (int s = 0; s < nst; ++s) {
    char* buf = smem + (s & 1) * STAGE_B;
    // stage s landed (nothing else in flight); after the barrier every wave
    // has read stage s - 1, so its buffer takes stage s + 1
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (s + 1 < nst) {
      char* nb = smem + ((s + 1) & 1) * STAGE_B;
      stage_copy<F>(asrc, gslot, (s + 1) * SK, kcur, nb, wave);
      stage_copy<F>(bsrc, gslot, (s + 1) * SK, kcur, nb + OPER_B, wave);
    }
    Frag<NI, NJ> f;
    read_frags_a<F>(buf, f, rb0, lr, lk);
    read_frags_b<F>(buf, f, cb0, lr, lk);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    settle(f);
    if constexpr (TRI) {
      bool l0, l1;
      tri_live(d.ktri != 0, s, SK, cb0, l0, l1);
      if (!idle) stage_mma_tri<F, NI, NJ, A_CONJ, B_CONJ>(f, c_re, c_im, l0, l1);
    } else {
      if (!idle) stage_mma<F, NI, NJ, A_CONJ, B_CONJ>(f, c_re, c_im);
    }
  }
  if (!idle) tile_epilogue<F, NI, NJ>(d, b, m0, n0, rb0, cb0, c_re, c_im, smem, wave, lane, first);
}

// One step of the ring pipeline: the MFMAs of stage s (fragments in `cur`)
// while the fragments of stage s + 1 are read from LDS into `nxt`.  Before
// them: stage s + 1 has landed (this wave's copies, then the barrier for
// everyone's), and every wave has read stage s, so its buffer takes the
// copies of stage s + RING.  One barrier a stage; the copies run up to
// RING - 1 stages ahead of the MFMAs.
template <int F, int NI, int NJ, bool A_CONJ, bool B_CONJ, bool TRI>
__device__ inline void ring_step(int s, int nst, int kcur, bool tri, Frag<NI, NJ>& cur, Frag<NI, NJ>& nxt,
                                 f16v (&c_re)[NI][NJ], f16v (&c_im)[NI][NJ],
                                 const unsigned short* const (&asrc)[NCOPY],
                                 const unsigned short* const (&bsrc)[NCOPY], const int (&gslot)[NCOPY],
                                 int rb0, int cb0, char* smem, int wave, int lr, int lk, bool idle) {
  constexpr int SK = Fmt<F>::K;
  const bool more = s + 1 < nst;
  if (more) {
    // copies issued so far: stages up to min(nst, s + RING) - 1
    const int last = (nst < s + RING ? nst : s + RING) - 1;
    wait_copies(last - (s + 1));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (s + RING < nst) {
      char* buf = smem + (s % RING) * STAGE_B;
      stage_copy<F>(asrc, gslot, (s + RING) * SK, kcur, buf, wave);
      stage_copy<F>(bsrc, gslot, (s + RING) * SK, kcur, buf + OPER_B, wave);
    }
    const char* nb = smem + ((s + 1) % RING) * STAGE_B;
    read_frags_a<F>(nb, nxt, rb0, lr, lk);
    read_frags_b<F>(nb, nxt, cb0, lr, lk);
  }
  if constexpr (TRI) {
    bool l0, l1;
    tri_live(tri, s, SK, cb0, l0, l1);
    if (!idle) stage_mma_tri<F, NI, NJ, A_CONJ, B_CONJ>(cur, c_re, c_im, l0, l1);
  } else {
    if (!idle) stage_mma<F, NI, NJ, A_CONJ, B_CONJ>(cur, c_re, c_im);
  }
  if (more) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    settle(nxt);
  }
}

// K loop and epilogue of one tile on the ring pipeline (same blocks, MFMA
// order and epilogues as tile_body, so the same results bit for bit).
template <int F, int NI, int NJ, bool A_CONJ, bool B_CONJ, bool TRI>
__device__ inline void tile_body_ring(const NtDesc& d, int b, int m0, int n0, int kcur,
                                      const unsigned short* const (&asrc)[NCOPY],
                                      const unsigned short* const (&bsrc)[NCOPY], const int (&gslot)[NCOPY],
                                      int rb0, int cb0, char* smem, int wave, int lane, bool idle, bool first) {
  const int lr = lane & 31, lk = lane >> 5;
  f16v c_re[NI][NJ], c_im[NI][NJ];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        c_re[i][j][v] = 0.f;
        c_im[i][j][v] = 0.f;
      }
  constexpr int SK = Fmt<F>::K;
  const int nst = (kcur + SK - 1) / SK;
  __syncthreads();                        // LDS of the previous tile no longer read
#pragma unroll
  for (int s = 0; s < RING; ++s)
    if (s < nst) {
      stage_copy<F>(asrc, gslot, s * SK, kcur, smem + s * STAGE_B, wave);
      stage_copy<F>(bsrc, gslot, s * SK, kcur, smem + s * STAGE_B + OPER_B, wave);
    }
  // stage 0 landed: the later stages of the prologue may be in flight
  wait_copies((nst < RING ? nst : RING) - 1);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  Frag<NI, NJ> f0, f1;
  read_frags_a<F>(smem, f0, rb0, lr, lk);
  read_frags_b<F>(smem, f0, cb0, lr, lk);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  settle(f0);
  for (int s = 0; s < nst; s += 2) {
    ring_step<F, NI, NJ, A_CONJ, B_CONJ, TRI>(s, nst, kcur, d.ktri != 0, f0, f1, c_re, c_im, asrc, bsrc, gslot, rb0,
                                              cb0, smem, wave, lr, lk, idle);
    if (s + 1 < nst)
      ring_step<F, NI, NJ, A_CONJ, B_CONJ, TRI>(s + 1, nst, kcur, d.ktri != 0, f1, f0, c_re, c_im, asrc, bsrc, gslot,
                                                rb0, cb0, smem, wave, lr, lk, idle);
  }
  if (!idle) tile_epilogue<F, NI, NJ>(d, b, m0, n0, rb0, cb0, c_re, c_im, smem, wave, lane, first);
}

// The same K loop with two barriers a stage and the copies two stages
// ahead (a buffer is refilled only after every wave has read the stage it
// holds): more tolerant of a workgroup that has its CU to itself, the case
// of launches with fewer tiles than two rounds of workgroups.
// K loop and epilogue of one tile.  The wave owns the (NI*32) x (NJ*32)
// block at rows rb0, columns cb0 of the tile: 64 x 64 in full tiles (2 x 2
// waves); in tiles with at most 32 valid rows (columns) each wave takes a
// 32 x 32 block of the one 32-row (32-column) strip, so edge tiles cost a
// quarter of the matrix-core work.  Two workgroups share a CU (64 KB of LDS
// each): two LDS stages, each stage's fragments read from LDS at its start
// (the waves of the other workgroup keep the matrix cores busy meanwhile),
// copies two stages ahead.
template <int F, int NI, int NJ, bool A_CONJ, bool B_CONJ, bool TRI>
__device__ inline void tile_body_2b(const NtDesc& d, int b, int m0, int n0, int kcur,
                                 const unsigned short* const (&asrc)[NCOPY], const unsigned short* const (&bsrc)[NCOPY],
                                 const int (&gslot)[NCOPY], int rb0, int cb0, char* smem, int wave, int lane,
                                 bool idle, bool first) {
  const int lr = lane & 31, lk = lane >> 5;
  f16v c_re[NI][NJ], c_im[NI][NJ];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        c_re[i][j][v] = 0.f;
        c_im[i][j][v] = 0.f;
      }
  constexpr int SK = Fmt<F>::K;
  const int nst = (kcur + SK - 1) / SK;
  __syncthreads();                        // LDS of the previous tile no longer read
#pragma unroll
  for (int s = 0; s < NBUF; ++s)
    if (s < nst) {
      stage_copy<F>(asrc, gslot, s * SK, kcur, smem + s * STAGE_B, wave);
      stage_copy<F>(bsrc, gslot, s * SK, kcur, smem + s * STAGE_B + OPER_B, wave);
    }
  for (int s = 0; s < nst; ++s) {
    char* buf = smem + (s & 1) * STAGE_B;
    // stage s landed: at most the copies of stage s+1 still in flight
    wait_copies(s + 1 < nst ? 1 : 0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    Frag<NI, NJ> f;
    read_frags_a<F>(buf, f, rb0, lr, lk);
    read_frags_b<F>(buf, f, cb0, lr, lk);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    settle(f);
    // every wave holds its fragments of stage s: its buffer takes stage s+2
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (s + NBUF < nst) {
      stage_copy<F>(asrc, gslot, (s + NBUF) * SK, kcur, buf, wave);
      stage_copy<F>(bsrc, gslot, (s + NBUF) * SK, kcur, buf + OPER_B, wave);
    }
    if constexpr (TRI) {
      bool l0, l1;
      tri_live(d.ktri != 0, s, SK, cb0, l0, l1);
      if (!idle) stage_mma_tri<F, NI, NJ, A_CONJ, B_CONJ>(f, c_re, c_im, l0, l1);
    } else if (!idle) {
      if constexpr (F == 2) {
        mma_half<NI, NJ, A_CONJ, B_CONJ>(f, 0, c_re, c_im);
        if (NJ == 2) mma_half<NI, NJ, A_CONJ, B_CONJ>(f, NJ - 1, c_re, c_im);
      } else {
        mma_single<NI, NJ, A_CONJ, B_CONJ>(f, 0, c_re, c_im);
        if (NJ == 2) mma_single<NI, NJ, A_CONJ, B_CONJ>(f, NJ - 1, c_re, c_im);
      }
    }
  }
  if (!idle) tile_epilogue<F, NI, NJ>(d, b, m0, n0, rb0, cb0, c_re, c_im, smem, wave, lane, first);
}

template <int F, bool A_CONJ, bool B_CONJ, int KIND, bool RINGP, bool TWOB = false>
__device__ inline void x3_tiles(const NtDesc* __restrict__ descs, int ndesc, long long total_tiles, int seg) {
  extern __shared__ __attribute__((aligned(16))) char smem[];   // NBUF (RING) stages x (A, B)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

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
    const int m0 = tm * XT, n0 = tn * XT;
    // interleaved formats: logical element e at u16 EU*e (e a multiple of 8)
    constexpr int EU = Fmt<F>::EU;
    // a triangular B (zero for k < n) contributes from k = n0 on
    const int kstart = d.ktri ? n0 : 0;
    const unsigned short* As =
        (const unsigned short*)d.A + EU * (b * d.sA_bat + (long long)seg * d.sA_seg + kstart);
    const unsigned short* Bs =
        (const unsigned short*)d.B + EU * (b * d.sB_bat + (long long)seg * d.sB_seg + kstart);
    const int kcur = ((seg == d.nseg - 1) ? d.Klast : d.Kseg) - kstart;

    // this lane's sources and slots in its copy instructions; rows past M / N
    // read the last valid row (their outputs are not stored)
    const unsigned short* asrc[NCOPY];
    const unsigned short* bsrc[NCOPY];
    int gslot[NCOPY];
#pragma unroll
    for (int j = 0; j < NCOPY; ++j) {
      const int row = (wave + 4 * j) * 8 + (lane >> 3);
      gslot[j] = lds_slot(row, lane & 7);     // the slot whose LDS position is lane & 7
      const int ra = min(m0 + row, d.M - 1), rb = min(n0 + row, d.N - 1);
      asrc[j] = As + EU * ((long long)ra * d.lda) + 8 * gslot[j];
      bsrc[j] = Bs + EU * ((long long)rb * d.ldb) + 8 * gslot[j];
    }
    // Hermitian outputs (lower tiles; the upper triangle is mirrored later):
    // in a diagonal tile, a wave whose block lies strictly above the
    // diagonal only helps with the copies (FP64 epilogues only; the entries it
    // skips lie above the diagonal, which the consumers never read)
    const bool diag = d.herm && tm == tn && d.epi != 3;
    const bool first = seg == 0;
    if constexpr (RINGP) {
      if (d.M - m0 <= 32)
        tile_body_ring<F, 1, 1, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, 0, wave * 32, smem, wave,
                                                lane, diag && wave > 0, first);
      else if (d.N - n0 <= 32)
        tile_body_ring<F, 1, 1, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, wave * 32, 0, smem, wave,
                                                lane, false, first);
      else
        tile_body_ring<F, 2, 2, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, wm * 64, wn * 64, smem,
                                                wave, lane, diag && wm < wn, first);
    } else if constexpr (TWOB) {
      if (d.M - m0 <= 32)
        tile_body_2b<F, 1, 1, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, 0, wave * 32, smem, wave, lane,
                                              diag && wave > 0, first);
      else if (d.N - n0 <= 32)
        tile_body_2b<F, 1, 1, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, wave * 32, 0, smem, wave, lane,
                                              false, first);
      else
        tile_body_2b<F, 2, 2, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, wm * 64, wn * 64, smem, wave,
                                              lane, diag && wm < wn, first);
    } else {
      if (d.M - m0 <= 32)
        tile_body<F, 1, 1, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, 0, wave * 32, smem, wave, lane,
                                           diag && wave > 0, first);
      else if (d.N - n0 <= 32)
        tile_body<F, 1, 1, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, wave * 32, 0, smem, wave, lane,
                                           false, first);
      else
        tile_body<F, 2, 2, A_CONJ, B_CONJ, KIND == 2>(d, b, m0, n0, kcur, asrc, bsrc, gslot, wm * 64, wn * 64, smem, wave,
                                           lane, diag && wm < wn, first);
    }
  }
}

template <bool A_CONJ, bool B_CONJ, int KIND>
__global__ __launch_bounds__(XNT, 2) void zgemm_x3_kernel(const NtDesc* __restrict__ descs, int ndesc,
                                                          long long total_tiles, int seg) {
  x3_tiles<2, A_CONJ, B_CONJ, KIND, false>(descs, ndesc, total_tiles, seg);
}

template <bool A_CONJ, bool B_CONJ, int KIND>
__global__ __launch_bounds__(XNT, 2) void zgemm_x1_kernel(const NtDesc* __restrict__ descs, int ndesc,
                                                          long long total_tiles, int seg) {
  x3_tiles<3, A_CONJ, B_CONJ, KIND, false>(descs, ndesc, total_tiles, seg);
}

// two barriers a stage: the fragment contraction (kind 3, B conjugated) of
// launches with few tiles, both formats
template <int F>
__global__ __launch_bounds__(XNT, 2) void zgemm_c2b_kernel(const NtDesc* __restrict__ descs, int ndesc,
                                                           long long total_tiles, int seg) {
  x3_tiles<F, false, true, 3, false, true>(descs, ndesc, total_tiles, seg);
}

// ring pipeline (one workgroup a CU): the fragment GEMMs, both formats
template <int F, bool A_CONJ, bool B_CONJ, int KIND>
__global__ __launch_bounds__(XNT, 1) void zgemm_ring_kernel(const NtDesc* __restrict__ descs, int ndesc,
                                                            long long total_tiles, int seg) {
  x3_tiles<F, A_CONJ, B_CONJ, KIND, true>(descs, ndesc, total_tiles, seg);
}

template <int KIND>
hipError_t launch_x3(int conj, const NtDesc* descs, int ndesc, long long total, int blocks, int seg,
                     hipStream_t s) {
  dim3 g(blocks), b(XNT);
  const size_t lds = NBUF * STAGE_B;
  switch (conj & 3) {
    case 0: hipLaunchKernelGGL((zgemm_x3_kernel<false, false, KIND>), g, b, lds, s, descs, ndesc, total, seg); break;
    case 1: hipLaunchKernelGGL((zgemm_x3_kernel<true, false, KIND>), g, b, lds, s, descs, ndesc, total, seg); break;
    case 2: hipLaunchKernelGGL((zgemm_x3_kernel<false, true, KIND>), g, b, lds, s, descs, ndesc, total, seg); break;
    default: hipLaunchKernelGGL((zgemm_x3_kernel<true, true, KIND>), g, b, lds, s, descs, ndesc, total, seg); break;
  }
  return hipGetLastError();
}

// single-bf16 format: the two call sites of the path (U^q = R^q W^q, kind 2,
// no conjugation; the fragment contraction, kind 3, B conjugated)
hipError_t launch_x1(int conj, const NtDesc* descs, int ndesc, long long total, int blocks, int seg, int kind,
                     hipStream_t s) {
  dim3 g(blocks), b(XNT);
  const size_t lds = NBUF * STAGE_B;
  if (kind == 2 && (conj & 3) == 0)
    hipLaunchKernelGGL((zgemm_x1_kernel<false, false, 2>), g, b, lds, s, descs, ndesc, total, seg);
  else if (kind == 3 && (conj & 3) == 2)
    hipLaunchKernelGGL((zgemm_x1_kernel<false, true, 3>), g, b, lds, s, descs, ndesc, total, seg);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ring pipeline: the same two call sites, either format
template <int F>
hipError_t launch_ring(int conj, const NtDesc* descs, int ndesc, long long total, int blocks, int seg, int kind,
                       hipStream_t s) {
  dim3 g(blocks), b(XNT);
  const size_t lds = RING * STAGE_B;
  if (kind == 2 && (conj & 3) == 0)
    hipLaunchKernelGGL((zgemm_ring_kernel<F, false, false, 2>), g, b, lds, s, descs, ndesc, total, seg);
  else if (kind == 3 && (conj & 3) == 2)
    hipLaunchKernelGGL((zgemm_ring_kernel<F, false, true, 3>), g, b, lds, s, descs, ndesc, total, seg);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

bool ring_supported(int conj, int kind) {
  return (kind == 2 && (conj & 3) == 0) || (kind == 3 && (conj & 3) == 2);
}

hipError_t x1_launch(int conj, const NtDesc* descs_dev, int ndesc, long long total, int max_blocks, int seg,
                     hipStream_t s, int kind, bool ring) {
  if (total <= 0) return hipSuccess;
  const long long t8 = (total + 7) / 8 * 8;
  max_blocks = max_blocks / 8 * 8;
  const int blocks = (int)(t8 < max_blocks ? t8 : max_blocks);
  if (ring) return launch_ring<3>(conj, descs_dev, ndesc, total, blocks, seg, kind, s);
  // single bf16: 32 MFMAs a stage (against 48 in bf16x3) leave less time to
  // cover a one-stage prefetch; the contraction always takes the two-barrier
  // loop (0.378 against 0.354 of bf16 peak on the 120-orbital 1000-k shape)
  if (kind == 3 && (conj & 3) == 2) {
    hipLaunchKernelGGL((zgemm_c2b_kernel<3>), dim3(blocks), dim3(XNT), NBUF * STAGE_B, s, descs_dev, ndesc, total,
                       seg);
    return hipGetLastError();
  }
  return launch_x1(conj, descs_dev, ndesc, total, blocks, seg, kind, s);
}

hipError_t x3_launch(int conj, const NtDesc* descs_dev, int ndesc, long long total, int max_blocks, int seg,
                     hipStream_t s, int kind, bool ring) {
  if (total <= 0) return hipSuccess;
  const long long t8 = (total + 7) / 8 * 8;
  max_blocks = max_blocks / 8 * 8;
  const int blocks = (int)(t8 < max_blocks ? t8 : max_blocks);
  if (ring) return launch_ring<2>(conj, descs_dev, ndesc, total, blocks, seg, kind, s);
  if (kind == 3 && (conj & 3) == 2 && total < 2LL * blocks) {
    hipLaunchKernelGGL((zgemm_c2b_kernel<2>), dim3(blocks), dim3(XNT), NBUF * STAGE_B, s, descs_dev, ndesc, total,
                       seg);
    return hipGetLastError();
  }
  switch (kind) {
    case 1: return launch_x3<1>(conj, descs_dev, ndesc, total, blocks, seg, s);
    case 2: return launch_x3<2>(conj, descs_dev, ndesc, total, blocks, seg, s);
    case 3: return launch_x3<3>(conj, descs_dev, ndesc, total, blocks, seg, s);
    default: return launch_x3<0>(conj, descs_dev, ndesc, total, blocks, seg, s);
  }
}
