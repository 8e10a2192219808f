// T^k_I(r) = sum_mu X^k_{I mu} conj(phi^k_mu(r)) for one tile of grid points
// (Algorithm 1 with Y = phi, the right-hand side of eq. (5)): a contraction
// over only N_orb orbitals whose cost is writing T, so it runs on the FP64
// vector units with every output written once in 4 KB rows.
//
// Workgroup (256 threads): RT = 256 consecutive r x IT interpolation points
// of one k.  A tile covers the points [i0, i0 + icur) and rcur grid points
// (out[k][I - i0][r]).  The X^k values of the IT points are the same for every lane and
// are read through the scalar cache into SGPRs (the FMAs take them as their
// scalar operand, so no LDS traffic); each thread streams phi^k_mu(r) for its
// r over mu and accumulates its IT outputs in registers.
#include "kernels.hpp"

namespace {

constexpr int RT = 256;

template <int IT>
__global__ __launch_bounds__(256) void rhs_t_kernel(const cplx* __restrict__ xt, const cplx* __restrict__ phi,
                                                    cplx* __restrict__ out, int norb, int nip, long long ng,
                                                    long long r0, int rcur, int i0, int icur) {
  const int k = blockIdx.z;
  const int I0 = blockIdx.y * IT;                        // within the tile's points
  const int r = blockIdx.x * RT + threadIdx.x;
  const int ni = (icur - I0) < IT ? (icur - I0) : IT;
  if (r >= rcur) return;
  // X^k_{I mu} rows of this block's points: the same for every lane, read
  // through the scalar cache into SGPRs
  const cplx* X = xt + (long long)k * norb * nip + i0 + I0;   // [mu][I]
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
  cplx* o = out + ((long long)k * icur + I0) * rcur + r;
#pragma unroll
  for (int i = 0; i < IT; ++i)
    if (i < ni) o[(long long)i * rcur] = cmk(ar[i], ai[i]);
}

}  // namespace

hipError_t rhs_t_launch(const cplx* xt, const cplx* phi, cplx* out, int nk, int norb, int nip, long long ng,
                        long long r0, int rcur, int i0, int icur, hipStream_t s) {
  if (nk <= 0 || rcur <= 0 || icur <= 0) return hipSuccess;
  if (i0 < 0 || i0 + icur > nip) return hipErrorInvalidValue;
  constexpr int IT = 16;
  static_assert(IT <= RHS_X_PAD, "X padding covers one block of points");
  dim3 g((rcur + RT - 1) / RT, (icur + IT - 1) / IT, nk);
  hipLaunchKernelGGL(rhs_t_kernel<IT>, g, dim3(RT), 0, s, xt, phi, out, norb, nip, ng, r0, rcur, i0, icur);
  return hipGetLastError();
}
