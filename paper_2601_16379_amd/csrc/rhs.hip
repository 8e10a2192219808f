// T^k_I(r) = sum_mu X^k_{I mu} conj(phi^k_mu(r)) for one tile of grid points
// (Algorithm 1 with Y = phi, the right-hand side of eq. (5)): a contraction
// over only N_orb orbitals whose cost is writing T, so it runs on the FP64
// vector units with every output written once in 4 KB rows.
//
// Workgroup (256 threads): RT = 256 consecutive r x IT interpolation points
// of one k.  The X^k values of the IT points are the same for every lane and
// are read through the scalar cache into SGPRs (the FMAs take them as their
// scalar operand, so no LDS traffic); each thread streams phi^k_mu(r) for its
// r over mu and accumulates its IT outputs in registers.  The mixed-precision
// fit stores T as complex FP32 and computes it on the FP32 matrix cores
// instead (rhs_mfma_kernel below).
#include "kernels.hpp"

namespace {

constexpr int RT = 256;

template <int IT>
__global__ __launch_bounds__(256) void rhs_t_kernel(const cplx* __restrict__ xt, const cplx* __restrict__ phi,
                                                    cplx* __restrict__ out, int norb, int nip, long long ng,
                                                    long long r0, int rcur) {
  const int k = blockIdx.z;
  const int I0 = blockIdx.y * IT;
  const int r = blockIdx.x * RT + threadIdx.x;
  const int ni = (nip - I0) < IT ? (nip - I0) : IT;
  if (r >= rcur) return;
  // X^k_{I mu} rows of this block's points: the same for every lane, read
  // through the scalar cache into SGPRs
  const cplx* X = xt + (long long)k * norb * nip + I0;   // [mu][I]
  const cplx* P = phi + (long long)k * norb * ng + r0 + r;
  double ar[IT], ai[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) ar[i] = ai[i] = 0.0;
  // one phi row per step: loading several orbitals ahead measured slower
  for (int mu = 0; mu < norb; ++mu) {
    const cplx f = P[(long long)mu * ng];
    // rows past N_IP (last block) read the padding after X or the next row;
    // their outputs are not stored
    const cplx* x = X + (long long)mu * nip;
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      // x * conj(f)
      const cplx xv = x[i];
      ar[i] = fma(xv.x, f.x, fma(xv.y, f.y, ar[i]));
      ai[i] = fma(xv.y, f.x, fma(-xv.x, f.y, ai[i]));
    }
  }
  cplx* o = out + ((long long)k * nip + I0) * rcur + r;
#pragma unroll
  for (int i = 0; i < IT; ++i)
    if (i < ni) o[(long long)i * rcur] = cmk(ar[i], ai[i]);
}

// FP32 matrix-core form for the mixed-precision fit (T stored as complex
// FP32).  With conj(phi) the complex product splits into two real products
// over the pair (re, im) of each orbital:
//   Re T = sum_mu Xr phr + Xi phi,   Im T = sum_mu Xi phr - Xr phi,
// so one 32x32x2 FP32 MFMA per orbital and output block takes that pair as
// its K = 2: the A operand [Xr | Xi] (lanes 0-31 | 32-63, one row each) gives
// Re T, [Xi | -Xr] gives Im T, against the shared B operand [phr ; phi]
// (lane n + 32h holds component h of phi^k_mu(r0 + n)).  Workgroup: 128
// points I (four 32-row blocks, X^k staged in LDS as FP32) x 128 grid points
// r (32 per wave); accumulators stay in registers, one 8-byte store per
// output.
constexpr int RM_I = 128, RM_R = 128, RM_CP = 160;   // CP: pitch of the (re | im) halves, 32 banks apart
constexpr int RM_MAXORB = 64;
typedef float f32x16 __attribute__((ext_vector_type(16)));

// One orbital's pair of MFMAs for each of the NIB row blocks.
template <int NIB>
__device__ inline void rhs_mfma_step(const float* own, const float* oth, float sg, float b, f32x16 (&acc_re)[4],
                                     f32x16 (&acc_im)[4]) {
#pragma unroll
  for (int ib = 0; ib < NIB; ++ib) {
    acc_re[ib] = __builtin_amdgcn_mfma_f32_32x32x2f32(own[ib * 32], b, acc_re[ib], 0, 0, 0);
    acc_im[ib] = __builtin_amdgcn_mfma_f32_32x32x2f32(sg * oth[ib * 32], b, acc_im[ib], 0, 0, 0);
  }
}

// The orbital loop: phi loads issued MB at a time (every load unconditional)
// ahead of their MFMAs.
template <int NIB>
__device__ inline void rhs_mfma_loop(const float* own, const float* oth, float sg, const double* P, long long ng2,
                                     int norb, f32x16 (&acc_re)[4], f32x16 (&acc_im)[4]) {
  constexpr int MB = 8;
  int mu0 = 0;
  for (; mu0 + MB <= norb; mu0 += MB) {
    double b[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) b[j] = P[(long long)(mu0 + j) * ng2];
#pragma unroll
    for (int j = 0; j < MB; ++j)
      rhs_mfma_step<NIB>(own + (mu0 + j) * 2 * RM_CP, oth + (mu0 + j) * 2 * RM_CP, sg, (float)b[j], acc_re, acc_im);
  }
  for (; mu0 < norb; ++mu0)
    rhs_mfma_step<NIB>(own + mu0 * 2 * RM_CP, oth + mu0 * 2 * RM_CP, sg, (float)P[(long long)mu0 * ng2], acc_re,
                       acc_im);
}

// Whole workgroup for NIB row blocks present (uniform over the workgroup).
template <int NIB>
__device__ inline void rhs_mfma_tile(const cplx* __restrict__ xt, const cplx* __restrict__ phi,
                                     float2* __restrict__ out32, float* xs, int norb, int nip, long long ng,
                                     long long r0, int rcur, int k, int I0, int rw, int n, int h) {
  const cplx* X = xt + (long long)k * norb * nip;
  // columns past rcur read the last valid column and are not stored
  const int rc = rw + n < rcur ? rw + n : rcur - 1;
  const float* own = xs + h * RM_CP + n;          // Xr (lanes 0-31) / Xi (lanes 32-63)
  const float* oth = xs + (1 - h) * RM_CP + n;    // the other component, times sg: Xi / -Xr
  const float sg = h ? -1.f : 1.f;
  f32x16 acc_re[4], acc_im[4];
#pragma unroll
  for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc_re[ib][v] = acc_im[ib][v] = 0.f;
  const long long ng2 = 2 * ng;
  // orbitals in chunks of at most RM_MAXORB (the X^k rows staged in LDS)
  for (int c0 = 0; c0 < norb; c0 += RM_MAXORB) {
    const int nc = norb - c0 < RM_MAXORB ? norb - c0 : RM_MAXORB;
    if (c0 > 0) __syncthreads();          // the previous chunk is no longer read
    for (int idx = threadIdx.x; idx < nc * RM_I; idx += 256) {
      const int mu = idx / RM_I, m = idx - (idx / RM_I) * RM_I;
      const cplx x = I0 + m < nip ? X[(long long)(c0 + mu) * nip + I0 + m] : cmk(0.0, 0.0);
      xs[mu * 2 * RM_CP + m] = (float)x.x;
      xs[mu * 2 * RM_CP + RM_CP + m] = (float)x.y;
    }
    __syncthreads();
    const double* P = (const double*)(phi + ((long long)k * norb + c0) * ng + r0 + rc) + h;
    rhs_mfma_loop<NIB>(own, oth, sg, P, ng2, nc, acc_re, acc_im);
  }
  if (rw + n >= rcur) return;
  // output block layout: lane l, register v -> row 8(v/4) + 4(l/32) + v%4, column l%32
  float2* o = out32 + (long long)k * nip * rcur + rw + n;
#pragma unroll
  for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int I = I0 + ib * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
      if (I < nip) o[(long long)I * rcur] = make_float2(acc_re[ib][v], acc_im[ib][v]);
    }
}

__global__ __launch_bounds__(256, 2) void rhs_mfma_kernel(const cplx* __restrict__ xt, const cplx* __restrict__ phi,
                                                        float2* __restrict__ out32, int norb, int nip,
                                                        long long ng, long long r0, int rcur) {
  extern __shared__ float xs[];          // [orbital chunk][2][RM_CP]: Xr, Xi of rows I0 .. I0 + 127 (zero past N_IP)
  const int k = blockIdx.z;
  const int I0 = blockIdx.y * RM_I;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 31, h = lane >> 5;
  const int rw = blockIdx.x * RM_R + wave * 32;
  const int nib = (nip - I0 + 31) / 32;   // row blocks present (uniform over the workgroup)
  if (nib >= 4) rhs_mfma_tile<4>(xt, phi, out32, xs, norb, nip, ng, r0, rcur, k, I0, rw, n, h);
  else if (nib == 3) rhs_mfma_tile<3>(xt, phi, out32, xs, norb, nip, ng, r0, rcur, k, I0, rw, n, h);
  else if (nib == 2) rhs_mfma_tile<2>(xt, phi, out32, xs, norb, nip, ng, r0, rcur, k, I0, rw, n, h);
  else rhs_mfma_tile<1>(xt, phi, out32, xs, norb, nip, ng, r0, rcur, k, I0, rw, n, h);
}

}  // namespace

hipError_t rhs_t_launch(const cplx* xt, const cplx* phi, cplx* out, float2* out32, int nk, int norb, int nip,
                        long long ng, long long r0, int rcur, hipStream_t s) {
  if (nk <= 0 || rcur <= 0) return hipSuccess;
  constexpr int IT = 16;
  static_assert(IT <= RHS_X_PAD, "X padding covers one block of points");
  dim3 g((rcur + RT - 1) / RT, (nip + IT - 1) / IT, nk);
  if (out32) {
    dim3 gm((rcur + RM_R - 1) / RM_R, (nip + RM_I - 1) / RM_I, nk);
    const int nc = norb < RM_MAXORB ? norb : RM_MAXORB;
    hipLaunchKernelGGL(rhs_mfma_kernel, gm, dim3(256), (size_t)nc * 2 * RM_CP * sizeof(float), s, xt, phi, out32,
                       norb, nip, ng, r0, rcur);
  } else {
    hipLaunchKernelGGL(rhs_t_kernel<IT>, g, dim3(RT), 0, s, xt, phi, out, norb, nip, ng, r0, rcur);
  }
  return hipGetLastError();
}
