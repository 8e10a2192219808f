// Transforms over the k mesh (the convolution theorem of Algorithm 1 and the
// k <-> R transforms of Algorithm 2), staged through LDS.
//
// A workgroup loads a tile of `etile` independent elements for every k of
// the m1 x m2 x m3 mesh (k-major rows of contiguous elements, so every HBM
// row access is coalesced), applies the 3-D DFT over the mesh one axis at a
// time inside LDS (each thread owns one length-m line in registers), applies
// the pointwise step, transforms back and stores: one HBM read and one HBM
// write per element, however many mesh axes there are.
#include "kernels.hpp"
#include "dft_small.hpp"

namespace {

constexpr int MAXM = 16;

// Length-M DFT of lines p[j * estride], j < M, for the lines `line` owned by
// this thread: each line in registers, transformed by dft_line with
// compile-time length, sign and twiddles.
template <int M, int S>
__device__ void axis_dft_s(cplx* buf, int nlines, int eshift, int ax, int m2, int m3) {
  const int etile = 1 << eshift;
#pragma unroll 1
  for (int line = threadIdx.x; line < nlines; line += blockDim.x) {
    const int e = line & (etile - 1);
    const int rest = line >> eshift;
    int base, stride;
    if (ax == 0) { base = rest; stride = m2 * m3; }
    else if (ax == 1) { base = (rest / m3) * m2 * m3 + (rest % m3); stride = m3; }
    else { base = rest * M; stride = 1; }
    const int estride = stride << eshift;
    cplx* p = buf + (base << eshift) + e;
    cplx x[M];
#pragma unroll
    for (int j = 0; j < M; ++j) x[j] = p[j * estride];
    dft_line<M, S>(x);
#pragma unroll
    for (int t = 0; t < M; ++t) p[t * estride] = x[t];
  }
}

template <int M>
__device__ void axis_dft(cplx* buf, int nlines, int eshift, int ax, int m2, int m3, int sign) {
  if (sign > 0) axis_dft_s<M, 1>(buf, nlines, eshift, ax, m2, m3);
  else axis_dft_s<M, -1>(buf, nlines, eshift, ax, m2, m3);
}

// In-place 3-D DFT over the mesh for every element column of buf[k][etile]:
// buf[k][e] <- sum_j exp(sign * 2 pi i sum_d j_d k_d / m_d) buf[j][e].
// etile is a power of two.
// MAXA: largest axis length of the mesh (4, 8 or 16): only the axis
// transforms up to it are instantiated, which keeps the register count of
// the kernels (and so their occupancy) set by the mesh actually used.
template <int MAXA>
__device__ void mesh_dft(cplx* buf, int etile, int m1, int m2, int m3, int sign) {
  const int eshift = __builtin_ctz(etile);
  const int nk = m1 * m2 * m3;
  const int ms[3] = {m1, m2, m3};
  for (int ax = 0; ax < 3; ++ax) {
    const int m = ms[ax];
    if (m == 1) continue;
    const int nlines = (nk / m) << eshift;
    switch (m) {
#define AXIS_CASE(M) \
  case M: if constexpr (M <= MAXA) axis_dft<M>(buf, nlines, eshift, ax, m2, m3, sign); break;
      AXIS_CASE(2) AXIS_CASE(3) AXIS_CASE(4) AXIS_CASE(5) AXIS_CASE(6) AXIS_CASE(7) AXIS_CASE(8)
      AXIS_CASE(9) AXIS_CASE(10) AXIS_CASE(11) AXIS_CASE(12) AXIS_CASE(13) AXIS_CASE(14)
      AXIS_CASE(15) AXIS_CASE(16)
#undef AXIS_CASE
      default: break;
    }
    __syncthreads();
  }
}

template <int MAXA>
__global__ __launch_bounds__(256) void kconv_kernel(KconvArgs a, int etile) {
  // blockDim.x == 256; etile a power of two
  extern __shared__ cplx buf[];
  const int eshift = __builtin_ctz(etile);
  const int nk = a.m1 * a.m2 * a.m3;
  const long long e0 = (long long)blockIdx.x * etile;
  const long long rem = a.n_elem - e0;
  const int ne = rem < etile ? (int)rem : etile;
  // element e0 + e maps to in/out offsets base + e when the tile does not cross
  // a row of the (inner, outer) maps (the host guarantees it when fast != 0)
  const bool fast = (a.in_inner % etile == 0) && (a.out_inner % etile == 0);
  const long long in0 = (e0 / a.in_inner) * a.in_outer + e0 % a.in_inner;
  const long long out0 = (e0 / a.out_inner) * a.out_outer + e0 % a.out_inner;
  constexpr int UNR = 8;
  const int total = nk << eshift;
  for (int b0 = 0; b0 < total; b0 += UNR * 256) {
    cplx v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = b0 + u * 256 + threadIdx.x;
      v[u] = cmk(0.0, 0.0);
      if (idx < total) {
        const int k = idx >> eshift, e = idx & (etile - 1);
        if (e < ne) {
          long long off;
          if (fast) {
            off = in0 + e;
          } else {
            const long long ee = e0 + e;
            off = (ee / a.in_inner) * a.in_outer + ee % a.in_inner;
          }
          v[u] = a.in[(long long)k * a.in_kstride + off];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = b0 + u * 256 + threadIdx.x;
      if (idx < total) buf[idx] = v[u];
    }
  }
  __syncthreads();
  if (a.mode == 0) {
    // T^R = sum_k exp(+i k.R) T^k ;  Z^R = |T^R|^2 ;  out^q = scale * sum_R exp(+i q.R) Z^R
    mesh_dft<MAXA>(buf, etile, a.m1, a.m2, a.m3, +1);
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      cplx v = buf[idx];
      buf[idx] = cmk(v.x * v.x + v.y * v.y, 0.0);
    }
    __syncthreads();
    mesh_dft<MAXA>(buf, etile, a.m1, a.m2, a.m3, +1);
  } else {
    mesh_dft<MAXA>(buf, etile, a.m1, a.m2, a.m3, a.sign);
  }
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int q0 = idx >> eshift, e = idx & (etile - 1);
    const int q = (a.mode == 0 && a.qslot) ? a.qslot[q0] : q0;
    if (q >= 0 && e < ne) {
      long long off;
      if (fast) {
        off = out0 + e;
      } else {
        const long long ee = e0 + e;
        off = (ee / a.out_inner) * a.out_outer + ee % a.out_inner;
      }
      const cplx r = cscale(buf[idx], a.scale);
      if (a.out32) a.out32[(long long)q * a.out_qstride + off] = make_float2((float)r.x, (float)r.y);
      else a.out[(long long)q * a.out_qstride + off] = r;
    }
  }
}

// The convolution of mode 0 on a fixed M1 x M2 x M3 mesh with every line in
// registers.  LDS holds the tile [k][etile] with one pad element after each
// (k1, k2) row (rows of M3 etile + 1 elements, an odd stride, so the
// lanes of a line pass fall on distinct banks).  One thread per line:
//   axis-3 lines straight from HBM, forward DFT, to LDS;
//   axis-2 lines, forward DFT;
//   axis-1 lines, forward DFT, |.|^2, inverse DFT (the same line);
//   axis-2 lines, inverse DFT;
//   axis-3 lines, inverse DFT, straight to HBM (classes that qslot selects).
// Four LDS passes and four barriers in all; each workgroup reads its
// elements once and writes them once.  Tiles are mapped XCD-contiguously
// (workgroup b runs on XCD b mod 8), so neighbouring element tiles, which
// share cache lines, are read through one L2.
template <int M1, int M2, int M3>
__global__ __launch_bounds__(512) void kconv_lines_kernel(KconvArgs a, int etile, int ntiles) {
  extern __shared__ cplx buf[];
  constexpr int NK = M1 * M2 * M3;
  const int per = (ntiles + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int eshift = __builtin_ctz(etile);
  const int rs = M3 * etile + 1;                 // LDS row of one (k1, k2)
  const long long e0 = (long long)tile * etile;
  const long long rem = a.n_elem - e0;
  const int ne = rem < etile ? (int)rem : etile;
  const bool fast = (a.in_inner % etile == 0) && (a.out_inner % etile == 0);
  const long long in0 = (e0 / a.in_inner) * a.in_outer + e0 % a.in_inner;
  const long long out0 = (e0 / a.out_inner) * a.out_outer + e0 % a.out_inner;
  const int tid = threadIdx.x, nt = blockDim.x;

  // axis 3 from HBM: line (k1, k2, e)
  for (int l = tid; l < (NK / M3) << eshift; l += nt) {
    const int e = l & (etile - 1), k12 = l >> eshift;
    cplx x[M3];
    long long off = 0;
    if (e < ne) off = fast ? in0 + e : ((e0 + e) / a.in_inner) * a.in_outer + (e0 + e) % a.in_inner;
#pragma unroll
    for (int j = 0; j < M3; ++j)
      x[j] = e < ne ? a.in[(long long)(k12 * M3 + j) * a.in_kstride + off] : cmk(0.0, 0.0);
    dft_line<M3, 1>(x);
    cplx* p = buf + k12 * rs + e;
#pragma unroll
    for (int j = 0; j < M3; ++j) p[j * etile] = x[j];
  }
  __syncthreads();
  // axis 2: line (k1, k3, e)
  for (int l = tid; l < (NK / M2) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    cplx* p = buf + (r / M3) * M2 * rs + (r % M3) * etile + e;
    cplx x[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) x[j] = p[j * rs];
    dft_line<M2, 1>(x);
#pragma unroll
    for (int j = 0; j < M2; ++j) p[j * rs] = x[j];
  }
  __syncthreads();
  // axis 1: line (k2, k3, e); T^R -> |T^R|^2 -> back along the same line
  for (int l = tid; l < (NK / M1) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    cplx* p = buf + (r / M3) * rs + (r % M3) * etile + e;
    cplx x[M1];
#pragma unroll
    for (int j = 0; j < M1; ++j) x[j] = p[j * M2 * rs];
    dft_line<M1, 1>(x);
#pragma unroll
    for (int j = 0; j < M1; ++j) x[j] = cmk(x[j].x * x[j].x + x[j].y * x[j].y, 0.0);
    dft_line<M1, 1>(x);
#pragma unroll
    for (int j = 0; j < M1; ++j) p[j * M2 * rs] = x[j];
  }
  __syncthreads();
  for (int l = tid; l < (NK / M2) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    cplx* p = buf + (r / M3) * M2 * rs + (r % M3) * etile + e;
    cplx x[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) x[j] = p[j * rs];
    dft_line<M2, 1>(x);
#pragma unroll
    for (int j = 0; j < M2; ++j) p[j * rs] = x[j];
  }
  __syncthreads();
  // axis 3 to HBM: line (q1, q2, e)
  for (int l = tid; l < (NK / M3) << eshift; l += nt) {
    const int e = l & (etile - 1), q12 = l >> eshift;
    if (e >= ne) continue;
    const cplx* p = buf + q12 * rs + e;
    cplx x[M3];
#pragma unroll
    for (int j = 0; j < M3; ++j) x[j] = p[j * etile];
    dft_line<M3, 1>(x);
    const long long off = fast ? out0 + e : ((e0 + e) / a.out_inner) * a.out_outer + (e0 + e) % a.out_inner;
#pragma unroll
    for (int j = 0; j < M3; ++j) {
      const int q0 = q12 * M3 + j;
      const int q = a.qslot ? a.qslot[q0] : q0;
      if (q < 0) continue;
      const cplx r = cscale(x[j], a.scale);
      if (a.out32) a.out32[(long long)q * a.out_qstride + off] = make_float2((float)r.x, (float)r.y);
      else a.out[(long long)q * a.out_qstride + off] = r;
    }
  }
}

template <int M1, int M2, int M3>
hipError_t kconv_lines_launch(const KconvArgs& a, hipStream_t s) {
  constexpr int NK = M1 * M2 * M3;
  constexpr int LMAX = NK / (M1 < M2 ? (M1 < M3 ? M1 : M3) : (M2 < M3 ? M2 : M3));   // most lines of one axis
  // largest power-of-two element tile with at most 512 lines an axis pass
  // and at most 80 KB of LDS (two workgroups a CU)
  int etile = 1;
  while (LMAX * etile * 2 <= 512 && (size_t)M1 * M2 * (M3 * etile * 2 + 1) * sizeof(cplx) <= 80 * 1024) etile *= 2;
  const long long ntiles = (a.n_elem + etile - 1) / etile;
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > (1LL << 28)) return hipErrorInvalidValue;
  const long long blocks = ((ntiles + 7) / 8) * 8;
  const int threads = (LMAX * etile + 63) / 64 * 64;
  const size_t lds = (size_t)M1 * M2 * (M3 * etile + 1) * sizeof(cplx);
  hipLaunchKernelGGL((kconv_lines_kernel<M1, M2, M3>), dim3((unsigned)blocks), dim3(threads), lds, s, a, etile,
                     (int)ntiles);
  return hipGetLastError();
}

// The exchange convolution of eq. (10), in place:
//   rho[k][e] <- scale * sum_R exp(+i k.R) Wt(R) rhot(R),
//   rhot(R) = sum_k exp(-i k.R) rho[k][e],  Wt(R) = sum_q exp(+i q.R) W^q[e],
// which is scale * N_k * sum_q W^q[e] rho[k+q][e].  W^q is read from the
// class storage: W^q[e] = w[wsel[q] >> 1][e], conjugated when wsel[q] & 1.
// Both mesh columns of a tile of `etile` elements sit in LDS ([k][etile]
// each); a workgroup reads and writes only its own elements.
template <int MAXA>
__global__ __launch_bounds__(256) void xconv_kernel(XconvArgs a, int etile) {
  extern __shared__ cplx xbuf[];
  const int eshift = __builtin_ctz(etile);
  const int nk = a.m1 * a.m2 * a.m3;
  const int total = nk << eshift;
  cplx* br = xbuf;
  cplx* bw = xbuf + total;
  const long long e0 = (long long)blockIdx.x * etile;
  const long long rem = a.n_elem - e0;
  const int ne = rem < etile ? (int)rem : etile;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int k = idx >> eshift, e = idx & (etile - 1);
    cplx r = cmk(0.0, 0.0), w = cmk(0.0, 0.0);
    if (e < ne) {
      r = a.rho[(long long)k * a.n_elem + e0 + e];
      const int sel = a.wsel[k];
      w = a.w[(long long)(sel >> 1) * a.n_elem + e0 + e];
      if (sel & 1) w.y = -w.y;
    }
    br[idx] = r;
    bw[idx] = w;
  }
  __syncthreads();
  mesh_dft<MAXA>(br, etile, a.m1, a.m2, a.m3, -1);
  mesh_dft<MAXA>(bw, etile, a.m1, a.m2, a.m3, +1);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) br[idx] = cmul(br[idx], bw[idx]);
  __syncthreads();
  mesh_dft<MAXA>(br, etile, a.m1, a.m2, a.m3, +1);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int k = idx >> eshift, e = idx & (etile - 1);
    if (e < ne) a.rho[(long long)k * a.n_elem + e0 + e] = cscale(br[idx], a.scale);
  }
}

// The exchange convolution on a fixed M1 x M2 x M3 mesh with every line in
// registers (as kconv_lines_kernel): LDS holds the tiles of rho and W, each
// [k][etile] with rows padded to an odd stride.  The axis-3 lines of rho
// and of W come straight from HBM and are transformed (rho with exp(-i k.R),
// W with exp(+i q.R)), the axis-2 lines of both pass through LDS, the
// axis-1 lines of both are transformed, multiplied and transformed back in
// registers, and the product goes back along axes 2 and 3, the last
// straight to HBM: five LDS passes and four barriers a tile.
template <int M1, int M2, int M3>
__global__ __launch_bounds__(512) void xconv_lines_kernel(XconvArgs a, int etile, int ntiles) {
  extern __shared__ cplx xl[];
  constexpr int NK = M1 * M2 * M3;
  const int per = (ntiles + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int eshift = __builtin_ctz(etile);
  const int rs = M3 * etile + 1;
  cplx* br = xl;
  cplx* bw = xl + M1 * M2 * rs;
  const long long e0 = (long long)tile * etile;
  const long long rem = a.n_elem - e0;
  const int ne = rem < etile ? (int)rem : etile;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int l = tid; l < (NK / M3) << eshift; l += nt) {
    const int e = l & (etile - 1), k12 = l >> eshift;
    cplx x[M3], y[M3];
#pragma unroll
    for (int j = 0; j < M3; ++j) {
      x[j] = y[j] = cmk(0.0, 0.0);
      if (e < ne) {
        const int k = k12 * M3 + j;
        x[j] = a.rho[(long long)k * a.n_elem + e0 + e];
        const int sel = a.wsel[k];
        y[j] = a.w[(long long)(sel >> 1) * a.n_elem + e0 + e];
        if (sel & 1) y[j].y = -y[j].y;
      }
    }
    dft_line<M3, -1>(x);
    dft_line<M3, 1>(y);
    const int o = k12 * rs + e;
#pragma unroll
    for (int j = 0; j < M3; ++j) {
      br[o + j * etile] = x[j];
      bw[o + j * etile] = y[j];
    }
  }
  __syncthreads();
  for (int l = tid; l < (NK / M2) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    const int o = (r / M3) * M2 * rs + (r % M3) * etile + e;
    cplx x[M2], y[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) {
      x[j] = br[o + j * rs];
      y[j] = bw[o + j * rs];
    }
    dft_line<M2, -1>(x);
    dft_line<M2, 1>(y);
#pragma unroll
    for (int j = 0; j < M2; ++j) {
      br[o + j * rs] = x[j];
      bw[o + j * rs] = y[j];
    }
  }
  __syncthreads();
  for (int l = tid; l < (NK / M1) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    const int o = (r / M3) * rs + (r % M3) * etile + e;
    cplx x[M1], y[M1];
#pragma unroll
    for (int j = 0; j < M1; ++j) {
      x[j] = br[o + j * M2 * rs];
      y[j] = bw[o + j * M2 * rs];
    }
    dft_line<M1, -1>(x);
    dft_line<M1, 1>(y);
#pragma unroll
    for (int j = 0; j < M1; ++j) x[j] = cmul(x[j], y[j]);
    dft_line<M1, 1>(x);
#pragma unroll
    for (int j = 0; j < M1; ++j) br[o + j * M2 * rs] = x[j];
  }
  __syncthreads();
  for (int l = tid; l < (NK / M2) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    const int o = (r / M3) * M2 * rs + (r % M3) * etile + e;
    cplx x[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) x[j] = br[o + j * rs];
    dft_line<M2, 1>(x);
#pragma unroll
    for (int j = 0; j < M2; ++j) br[o + j * rs] = x[j];
  }
  __syncthreads();
  for (int l = tid; l < (NK / M3) << eshift; l += nt) {
    const int e = l & (etile - 1), k12 = l >> eshift;
    if (e >= ne) continue;
    cplx x[M3];
#pragma unroll
    for (int j = 0; j < M3; ++j) x[j] = br[k12 * rs + e + j * etile];
    dft_line<M3, 1>(x);
#pragma unroll
    for (int j = 0; j < M3; ++j) a.rho[(long long)(k12 * M3 + j) * a.n_elem + e0 + e] = cscale(x[j], a.scale);
  }
}

template <int M1, int M2, int M3>
hipError_t xconv_lines_launch(const XconvArgs& a, hipStream_t s) {
  constexpr int NK = M1 * M2 * M3;
  constexpr int LMAX = NK / (M1 < M2 ? (M1 < M3 ? M1 : M3) : (M2 < M3 ? M2 : M3));
  // largest power-of-two element tile with at most 512 lines an axis pass
  // and both padded tiles in at most 160 KB of LDS
  int etile = 1;
  while (LMAX * etile * 2 <= 512 && 2 * (size_t)M1 * M2 * (M3 * etile * 2 + 1) * sizeof(cplx) <= 160 * 1024)
    etile *= 2;
  const long long ntiles = (a.n_elem + etile - 1) / etile;
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > (1LL << 28)) return hipErrorInvalidValue;
  const long long blocks = ((ntiles + 7) / 8) * 8;
  const int threads = (LMAX * etile + 63) / 64 * 64;
  const size_t lds = 2 * (size_t)M1 * M2 * (M3 * etile + 1) * sizeof(cplx);
  hipLaunchKernelGGL((xconv_lines_kernel<M1, M2, M3>), dim3((unsigned)blocks), dim3(threads), lds, s, a, etile,
                     (int)ntiles);
  return hipGetLastError();
}

// The two polarisabilities of the opposite-spin MP2 energy, in place:
//   A(R) = sum_k exp(+i k.R) gv[k][e],  B(R) = sum_k exp(+i k.R) go[k][e],
//   Z(R) = A(R) conj(B(R)),
//   chi^q  = scale * sum_R exp(+i q.R) Z(R)        -> gv[qslot[q]][e]
//   chit^q = scale * sum_R exp(+i q.R) conj(Z(R))  -> go[qslot[q]][e]
// (with scale N_k^-2: chi^q = N_k^-1 sum_k gv^k conj(go^{k+q}), chit^q the
// same with gv and go exchanged), for the q with qslot[q] >= 0.  Both mesh
// columns of a tile of `etile` elements sit in LDS; a workgroup reads and
// writes only its own elements.
template <int MAXA>
__global__ __launch_bounds__(256) void pconv_kernel(PconvArgs a, int etile) {
  extern __shared__ cplx pbuf[];
  const int eshift = __builtin_ctz(etile);
  const int nk = a.m1 * a.m2 * a.m3;
  const int total = nk << eshift;
  cplx* ba = pbuf;
  cplx* bb = pbuf + total;
  const long long e0 = (long long)blockIdx.x * etile;
  const long long rem = a.n_elem - e0;
  const int ne = rem < etile ? (int)rem : etile;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int k = idx >> eshift, e = idx & (etile - 1);
    cplx v = cmk(0.0, 0.0), o = cmk(0.0, 0.0);
    if (e < ne) {
      v = a.gv[(long long)k * a.n_elem + e0 + e];
      o = a.go[(long long)k * a.n_elem + e0 + e];
    }
    ba[idx] = v;
    bb[idx] = o;
  }
  __syncthreads();
  mesh_dft<MAXA>(ba, etile, a.m1, a.m2, a.m3, +1);
  mesh_dft<MAXA>(bb, etile, a.m1, a.m2, a.m3, +1);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const cplx z = cmulc(ba[idx], bb[idx]);
    ba[idx] = z;
    bb[idx] = cmk(z.x, -z.y);
  }
  __syncthreads();
  mesh_dft<MAXA>(ba, etile, a.m1, a.m2, a.m3, +1);
  mesh_dft<MAXA>(bb, etile, a.m1, a.m2, a.m3, +1);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int q = idx >> eshift, e = idx & (etile - 1);
    const int slot = a.qslot[q];
    if (slot >= 0 && e < ne) {
      a.gv[(long long)slot * a.n_elem + e0 + e] = cscale(ba[idx], a.scale);
      a.go[(long long)slot * a.n_elem + e0 + e] = cscale(bb[idx], a.scale);
    }
  }
}

// One workgroup: a tile of `tp` pairs of one fragment times `ti` consecutive
// interpolation points; LDS holds [R][tp*ti] so that the output rows (pair,
// I-range) are written as contiguous runs of I.
// The polarisabilities on a fixed M1 x M2 x M3 mesh with every line in
// registers (as kconv_lines_kernel): the axis-3 lines of gv and go come from
// HBM and are transformed, the axis-2 lines of both pass through LDS, the
// axis-1 lines of both are transformed, Z = A conj(B) formed and transformed
// back, and Z goes back along axes 2 and 3 inside LDS.  chit^q, the
// transform of conj(Z), is conj(chi^{-q}), so one inverse transform serves
// both: the store pass reads q and -q from LDS.
template <int M1, int M2, int M3>
__global__ __launch_bounds__(512) void pconv_lines_kernel(PconvArgs a, int etile, int ntiles) {
  extern __shared__ cplx pl2[];
  constexpr int NK = M1 * M2 * M3;
  const int per = (ntiles + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int eshift = __builtin_ctz(etile);
  const int rs = M3 * etile + 1;
  cplx* ba = pl2;
  cplx* bb = pl2 + M1 * M2 * rs;
  const long long e0 = (long long)tile * etile;
  const long long rem = a.n_elem - e0;
  const int ne = rem < etile ? (int)rem : etile;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int l = tid; l < (NK / M3) << eshift; l += nt) {
    const int e = l & (etile - 1), k12 = l >> eshift;
    cplx x[M3], y[M3];
#pragma unroll
    for (int j = 0; j < M3; ++j) {
      x[j] = y[j] = cmk(0.0, 0.0);
      if (e < ne) {
        const long long off = (long long)(k12 * M3 + j) * a.n_elem + e0 + e;
        x[j] = a.gv[off];
        y[j] = a.go[off];
      }
    }
    dft_line<M3, 1>(x);
    dft_line<M3, 1>(y);
    const int o = k12 * rs + e;
#pragma unroll
    for (int j = 0; j < M3; ++j) {
      ba[o + j * etile] = x[j];
      bb[o + j * etile] = y[j];
    }
  }
  __syncthreads();
  for (int l = tid; l < (NK / M2) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    const int o = (r / M3) * M2 * rs + (r % M3) * etile + e;
    cplx x[M2], y[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) {
      x[j] = ba[o + j * rs];
      y[j] = bb[o + j * rs];
    }
    dft_line<M2, 1>(x);
    dft_line<M2, 1>(y);
#pragma unroll
    for (int j = 0; j < M2; ++j) {
      ba[o + j * rs] = x[j];
      bb[o + j * rs] = y[j];
    }
  }
  __syncthreads();
  for (int l = tid; l < (NK / M1) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    const int o = (r / M3) * rs + (r % M3) * etile + e;
    cplx x[M1], y[M1];
#pragma unroll
    for (int j = 0; j < M1; ++j) {
      x[j] = ba[o + j * M2 * rs];
      y[j] = bb[o + j * M2 * rs];
    }
    dft_line<M1, 1>(x);
    dft_line<M1, 1>(y);
#pragma unroll
    for (int j = 0; j < M1; ++j) x[j] = cmulc(x[j], y[j]);
    dft_line<M1, 1>(x);
#pragma unroll
    for (int j = 0; j < M1; ++j) ba[o + j * M2 * rs] = x[j];
  }
  __syncthreads();
  for (int l = tid; l < (NK / M2) << eshift; l += nt) {
    const int e = l & (etile - 1), r = l >> eshift;
    const int o = (r / M3) * M2 * rs + (r % M3) * etile + e;
    cplx x[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) x[j] = ba[o + j * rs];
    dft_line<M2, 1>(x);
#pragma unroll
    for (int j = 0; j < M2; ++j) ba[o + j * rs] = x[j];
  }
  __syncthreads();
  for (int l = tid; l < (NK / M3) << eshift; l += nt) {
    const int e = l & (etile - 1), k12 = l >> eshift;
    cplx x[M3];
    const int o = k12 * rs + e;
#pragma unroll
    for (int j = 0; j < M3; ++j) x[j] = ba[o + j * etile];
    dft_line<M3, 1>(x);
#pragma unroll
    for (int j = 0; j < M3; ++j) ba[o + j * etile] = x[j];
  }
  __syncthreads();
  // chi^q -> gv[qslot[q]], chit^q = conj(chi^{-q}) -> go[qslot[q]]
  for (int l = tid; l < NK << eshift; l += nt) {
    const int e = l & (etile - 1), q = l >> eshift;
    const int slot = a.qslot[q];
    if (slot < 0 || e >= ne) continue;
    const int q1 = q / (M2 * M3), q2 = (q / M3) % M2, q3 = q % M3;
    const int n1 = (M1 - q1) % M1, n2 = (M2 - q2) % M2, n3 = (M3 - q3) % M3;
    const cplx v = ba[(q1 * M2 + q2) * rs + q3 * etile + e];
    const cplx w = ba[(n1 * M2 + n2) * rs + n3 * etile + e];
    const long long off = (long long)slot * a.n_elem + e0 + e;
    a.gv[off] = cscale(v, a.scale);
    a.go[off] = cmk(a.scale * w.x, -a.scale * w.y);
  }
}

template <int M1, int M2, int M3>
hipError_t pconv_lines_launch(const PconvArgs& a, hipStream_t s) {
  constexpr int NK = M1 * M2 * M3;
  constexpr int LMAX = NK / (M1 < M2 ? (M1 < M3 ? M1 : M3) : (M2 < M3 ? M2 : M3));
  int etile = 1;
  while (LMAX * etile * 2 <= 512 && 2 * (size_t)M1 * M2 * (M3 * etile * 2 + 1) * sizeof(cplx) <= 160 * 1024)
    etile *= 2;
  const long long ntiles = (a.n_elem + etile - 1) / etile;
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > (1LL << 28)) return hipErrorInvalidValue;
  const long long blocks = ((ntiles + 7) / 8) * 8;
  const int threads = (LMAX * etile + 63) / 64 * 64;
  const size_t lds = 2 * (size_t)M1 * M2 * (M3 * etile + 1) * sizeof(cplx);
  hipLaunchKernelGGL((pconv_lines_kernel<M1, M2, M3>), dim3((unsigned)blocks), dim3(threads), lds, s, a, etile,
                     (int)ntiles);
  return hipGetLastError();
}

template <int MAXA>
__global__ __launch_bounds__(256) void pair_kernel(PairArgs a) {
  extern __shared__ cplx buf[];
  const int nk = a.m1 * a.m2 * a.m3;
  // consecutive workgroups walk the pair blocks of one interpolation-point
  // tile, so psi rows of that tile stay in L2 while they are reused
  const int blk = blockIdx.x % a.nblocks;
  const int it = blockIdx.x / a.nblocks;
  const PairBlock pb = a.blocks[blk];
  const int nf = a.frag_nf[pb.frag];
  const int col = a.frag_col[pb.frag];
  const long long poff = a.frag_pair[pb.frag];
  const int w = a.tp * a.ti;           // power of two
  const int wshift = __builtin_ctz(w), tshift = __builtin_ctz(a.ti);
  const int I0 = it * a.ti;
  __shared__ int sp[8], sq[8];          // (p, q) of the block's pairs (tp <= 8)
  if (threadIdx.x < a.tp) {
    const int P = pb.pair0 + threadIdx.x;
    sp[threadIdx.x] = P / nf;
    sq[threadIdx.x] = P - (P / nf) * nf;
  }
  __syncthreads();
  constexpr int UNR = 4;
  const int total = nk * w;
  for (int b0 = 0; b0 < total; b0 += UNR * 256) {
    cplx xp[UNR], xq[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = b0 + u * 256 + threadIdx.x;
      xp[u] = cmk(0.0, 0.0);
      xq[u] = cmk(0.0, 0.0);
      if (idx < total) {
        const int R = idx >> wshift, e = idx & (w - 1);
        const int j = e >> tshift, i = e & (a.ti - 1);
        const int I = I0 + i;
        if (j < pb.npair && I < a.n_ip) {
          const cplx* base = a.psi + ((long long)R * a.ncol + col) * a.n_ip + I;
          xp[u] = base[(long long)sp[j] * a.n_ip];
          xq[u] = base[(long long)sq[j] * a.n_ip];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = b0 + u * 256 + threadIdx.x;
      if (idx < total) buf[idx] = cmulc(xq[u], xp[u]);   // conj(psi_p) psi_q
    }
  }
  __syncthreads();
  mesh_dft<MAXA>(buf, w, a.m1, a.m2, a.m3, -1);
  for (int idx = threadIdx.x; idx < nk * w; idx += blockDim.x) {
    const int Q = idx >> wshift, e = idx & (w - 1);
    const int j = e >> tshift, i = e & (a.ti - 1);
    const int I = I0 + i;
    const int slot = a.qslot[Q];
    if (slot >= 0 && j < pb.npair && I < a.ld) {
      const long long off = (long long)slot * a.q_stride + (poff + pb.pair0 + j) * a.p_stride + I;
      store_fmt(a.out, off, a.plane, a.fmt, cscale(buf[idx], a.scale));
    }
  }
}

// ---- pair transform for the mixed formats on meshes with an axis longer
// than 4 (the register path holds at most 4 x 4 x 4 values a lane) ----
// Same tiling as pair_kernel (a tile of tp pairs x ti interpolation points
// for every R, LDS [R][tp*ti]) with complex FP32 values: psi is read from its
// complex FP32 copy, the products and the mesh DFT are FP32 (the outputs are
// rounded to FP32 or bf16 hi + lo anyway), which doubles the tile that fits
// in 64 KB.  Each axis DFT holds one line of M values in registers with
// compile-time twiddles.
template <int M>
__device__ void axis_dft32(float2* buf, int nlines, int eshift, int ax, int m2, int m3) {
  const int etile = 1 << eshift;
#pragma unroll 1
  for (int line = threadIdx.x; line < nlines; line += blockDim.x) {
    const int e = line & (etile - 1);
    const int rest = line >> eshift;
    int base, stride;
    if (ax == 0) { base = rest; stride = m2 * m3; }
    else if (ax == 1) { base = (rest / m3) * m2 * m3 + (rest % m3); stride = m3; }
    else { base = rest * M; stride = 1; }
    const int estride = stride << eshift;
    float2* p = buf + (base << eshift) + e;
    float2 x[M], y[M];
#pragma unroll
    for (int j = 0; j < M; ++j) x[j] = p[j * estride];
    dft_any_f<M>(x, y);
#pragma unroll
    for (int t = 0; t < M; ++t) p[t * estride] = y[t];
  }
}

template <int MAXA>
__device__ void mesh_dft32(float2* buf, int etile, int m1, int m2, int m3) {
  const int eshift = __builtin_ctz(etile);
  const int nk = m1 * m2 * m3;
  const int ms[3] = {m1, m2, m3};
  for (int ax = 0; ax < 3; ++ax) {
    const int m = ms[ax];
    if (m == 1) continue;
    const int nlines = (nk / m) << eshift;
    switch (m) {
#define AXIS32_CASE(M) \
  case M: if constexpr (M <= MAXA) axis_dft32<M>(buf, nlines, eshift, ax, m2, m3); break;
      AXIS32_CASE(2) AXIS32_CASE(3) AXIS32_CASE(4) AXIS32_CASE(5) AXIS32_CASE(6) AXIS32_CASE(7) AXIS32_CASE(8)
      AXIS32_CASE(9) AXIS32_CASE(10) AXIS32_CASE(11) AXIS32_CASE(12) AXIS32_CASE(13) AXIS32_CASE(14)
      AXIS32_CASE(15) AXIS32_CASE(16)
#undef AXIS32_CASE
      default: break;
    }
    __syncthreads();
  }
}

template <int MAXA>
__global__ __launch_bounds__(256) void pair32_kernel(PairArgs a) {
  extern __shared__ float2 buf32[];
  const int nk = a.m1 * a.m2 * a.m3;
  // consecutive workgroups walk the pair blocks of one interpolation-point
  // tile, so psi rows of that tile stay in L2 while they are reused
  const int blk = blockIdx.x % a.nblocks;
  const int it = blockIdx.x / a.nblocks;
  const PairBlock pb = a.blocks[blk];
  const int nf = a.frag_nf[pb.frag];
  const int col = a.frag_col[pb.frag];
  const long long poff = a.frag_pair[pb.frag];
  const int w = a.tp * a.ti;           // power of two
  const int wshift = __builtin_ctz(w), tshift = __builtin_ctz(a.ti);
  const int I0 = it * a.ti;
  __shared__ int sp[8], sq[8];          // (p, q) of the block's pairs (tp <= 8)
  if (threadIdx.x < a.tp) {
    const int P = pb.pair0 + threadIdx.x;
    sp[threadIdx.x] = P / nf;
    sq[threadIdx.x] = P - (P / nf) * nf;
  }
  __syncthreads();
  constexpr int UNR = 8;
  const int total = nk * w;
  for (int b0 = 0; b0 < total; b0 += UNR * 256) {
    float2 xp[UNR], xq[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = b0 + u * 256 + threadIdx.x;
      xp[u] = make_float2(0.f, 0.f);
      xq[u] = make_float2(0.f, 0.f);
      if (idx < total) {
        const int R = idx >> wshift, e = idx & (w - 1);
        const int j = e >> tshift, i = e & (a.ti - 1);
        const int I = I0 + i;
        if (j < pb.npair && I < a.n_ip) {
          const float2* base = a.psi32 + ((long long)R * a.ncol + col) * a.n_ip + I;
          xp[u] = base[(long long)sp[j] * a.n_ip];
          xq[u] = base[(long long)sq[j] * a.n_ip];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = b0 + u * 256 + threadIdx.x;
      // conj(psi_p) psi_q
      if (idx < total)
        buf32[idx] = make_float2(fmaf(xp[u].x, xq[u].x, xp[u].y * xq[u].y), fmaf(xp[u].x, xq[u].y, -(xp[u].y * xq[u].x)));
    }
  }
  __syncthreads();
  mesh_dft32<MAXA>(buf32, w, a.m1, a.m2, a.m3);
  const float sc = (float)a.scale;
  for (int idx = threadIdx.x; idx < nk * w; idx += blockDim.x) {
    const int Q = idx >> wshift, e = idx & (w - 1);
    const int j = e >> tshift, i = e & (a.ti - 1);
    const int I = I0 + i;
    const int slot = a.qslot[Q];
    if (slot >= 0 && j < pb.npair && I < a.ld) {
      const long long off = (long long)slot * a.q_stride + (poff + pb.pair0 + j) * a.p_stride + I;
      const float2 v = buf32[idx];
      store_fmt(a.out, off, a.plane, a.fmt, cmk((double)(v.x * sc), (double)(v.y * sc)));
    }
  }
}

// ---- pair transform of the mixed formats on the 6^3, 8^3 and 10^3 meshes,
// one line a thread ----
// The tile of pair_kernel (tp pairs x ti interpolation points for every R)
// in complex FP32: the axis-3 lines of conj(psi_p) psi_q are formed from HBM
// in registers and transformed, the axis-2 lines pass once through LDS
// (rows padded by one value to an odd stride), and the axis-1 lines are
// transformed and written straight to the operand format: two LDS passes
// and two barriers a tile.  Tiles are mapped XCD-contiguously (workgroup b
// on XCD b mod 8 takes a contiguous range), so that consecutive pair blocks
// of one point tile, which share orbitals, are read through one L2.  With
// ipair the point tiles come in pairs (the two halves of a 2 ti range,
// neighbours in that order): half tiles, whose LDS lets two workgroups
// share a CU, still read and write whole cache lines between two
// workgroups that run together.
template <int M1, int M2, int M3>
__global__ __launch_bounds__(1024) void pair_lines_kernel(PairArgs a, int ntot) {
  extern __shared__ float2 pl[];
  constexpr int NK = M1 * M2 * M3;
  const int per = (ntot + 7) >> 3;
  const int v = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (v >= ntot) return;
  int blk, it;
  if (a.ipair) {
    const int rest = v >> 1;
    blk = rest % a.nblocks;
    it = (rest / a.nblocks) * 2 + (v & 1);
  } else {
    blk = v % a.nblocks;
    it = v / a.nblocks;
  }
  const PairBlock pb = a.blocks[blk];
  const int nf = a.frag_nf[pb.frag];
  const int col = a.frag_col[pb.frag];
  const long long poff = a.frag_pair[pb.frag];
  const int w = a.tp * a.ti;           // power of two
  const int wshift = __builtin_ctz(w), tshift = __builtin_ctz(a.ti);
  const int I0 = it * a.ti;
  const int rs = M3 * w + 1;           // LDS row of one (R1, R2)
  const long long rstride = (long long)a.ncol * a.n_ip;   // psi32 between consecutive R
  const int tid = threadIdx.x, nt = blockDim.x;
  // axis 3 from HBM: line (R1, R2, e)
  for (int l = tid; l < (NK / M3) << wshift; l += nt) {
    const int e = l & (w - 1), r12 = l >> wshift;
    const int j = e >> tshift, I = I0 + (e & (a.ti - 1));
    float2 x[M3];
    if (j < pb.npair && I < a.n_ip) {
      const int P = pb.pair0 + j, pp = P / nf, qq = P - pp * nf;
      const float2* bp = a.psi32 + ((long long)r12 * M3 * a.ncol + col + pp) * a.n_ip + I;
      const float2* bq = a.psi32 + ((long long)r12 * M3 * a.ncol + col + qq) * a.n_ip + I;
#pragma unroll
      for (int t = 0; t < M3; ++t) {
        const float2 xp = bp[t * rstride], xq = bq[t * rstride];
        // conj(psi_p) psi_q
        x[t] = make_float2(fmaf(xp.x, xq.x, xp.y * xq.y), fmaf(xp.x, xq.y, -(xp.y * xq.x)));
      }
    } else {
#pragma unroll
      for (int t = 0; t < M3; ++t) x[t] = make_float2(0.f, 0.f);
    }
    float2 y[M3];
    dft_any_f<M3>(x, y);
    float2* p = pl + r12 * rs + e;
#pragma unroll
    for (int t = 0; t < M3; ++t) p[t * w] = y[t];
  }
  __syncthreads();
  // axis 2: line (R1, R3, e)
  for (int l = tid; l < (NK / M2) << wshift; l += nt) {
    const int e = l & (w - 1), r = l >> wshift;
    float2* p = pl + (r / M3) * M2 * rs + (r % M3) * w + e;
    float2 x[M2], y[M2];
#pragma unroll
    for (int t = 0; t < M2; ++t) x[t] = p[t * rs];
    dft_any_f<M2>(x, y);
#pragma unroll
    for (int t = 0; t < M2; ++t) p[t * rs] = y[t];
  }
  __syncthreads();
  // axis 1 to the output: line (Q2, Q3, e)
  const float sc = (float)a.scale;
  for (int l = tid; l < (NK / M1) << wshift; l += nt) {
    const int e = l & (w - 1), r = l >> wshift;
    const int j = e >> tshift, I = I0 + (e & (a.ti - 1));
    if (j >= pb.npair || I >= a.ld) continue;
    const float2* p = pl + (r / M3) * rs + (r % M3) * w + e;
    float2 x[M1], y[M1];
#pragma unroll
    for (int t = 0; t < M1; ++t) x[t] = p[t * M2 * rs];
    dft_any_f<M1>(x, y);
    const long long row = (poff + pb.pair0 + j) * a.p_stride + I;
#pragma unroll
    for (int t = 0; t < M1; ++t) {
      const int slot = a.qslot[t * M2 * M3 + r];
      if (slot < 0) continue;
      store_fmt(a.out, (long long)slot * a.q_stride + row, a.plane, a.fmt,
                cmk((double)(y[t].x * sc), (double)(y[t].y * sc)));
    }
  }
}

template <int M1, int M2, int M3>
hipError_t pair_lines_launch(const PairArgs& a, hipStream_t s) {
  constexpr int NK = M1 * M2 * M3;
  const int w = a.tp * a.ti;
  // with ipair, point tiles in pairs (an odd count gains one empty tile)
  const long long ntot = (long long)a.nblocks * (a.ipair ? (a.n_itiles + 1) / 2 * 2 : a.n_itiles);
  if (ntot <= 0) return hipSuccess;
  if (ntot > (1LL << 30) || w > pair_lines_wmax(M1, M2, M3)) return hipErrorInvalidValue;
  const int lmax = NK / (M1 < M2 ? (M1 < M3 ? M1 : M3) : (M2 < M3 ? M2 : M3)) * w;
  const int threads = lmax <= 1024 ? (lmax + 63) / 64 * 64 : ((lmax + 1) / 2 + 63) / 64 * 64;   // <= 1024
  const size_t lds = (size_t)M1 * M2 * (M3 * w + 1) * sizeof(float2);
  const long long blocks = (ntot + 7) / 8 * 8;
  hipLaunchKernelGGL((pair_lines_kernel<M1, M2, M3>), dim3((unsigned)blocks), dim3(threads), lds, s, a, (int)ntot);
  return hipGetLastError();
}

// ---- register path of the k convolution (mode 0), mesh M1 x M2 x M3 with
// M1 in {1, 2, 4} and M2, M3 <= 4 ----
// M1 lanes per element (lane l: element l / M1, k1 = l % M1): the M2 x M3
// values of a k1 plane sit in the lane's registers (FP64), the k1 axis is a
// radix-2 transform across the lanes of a quad (DPP, no LDS).  Both
// transforms have the sign +1: T^R = sum_k exp(+ik.R) T^k, then
// out^q = scale * sum_R exp(+iq.R) |T^R|^2.
// y_k = sum_j x_j exp(+2 pi i jk / R) for R <= 4: butterflies (no
// multiplications except the two of radix 3)
template <int R>
__device__ inline void dft_pos(cplx (&x)[R]) {
  static_assert(R >= 1 && R <= 4, "register k transforms take mesh axes of length <= 4");
  if constexpr (R == 2) {
    const cplx a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 3) {
    // y0 = x0 + s, y1,2 = (x0 - s/2) +- i (sqrt(3)/2) d, s = x1 + x2, d = x1 - x2
    constexpr double h = 0.8660254037844386;
    const cplx s_ = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    const cplx t = cmk(fma(-0.5, s_.x, x[0].x), fma(-0.5, s_.y, x[0].y));
    x[0] = cadd(x[0], s_);
    x[1] = cmk(fma(-h, d.y, t.x), fma(h, d.x, t.y));
    x[2] = cmk(fma(h, d.y, t.x), fma(-h, d.x, t.y));
  } else if constexpr (R == 4) {
    // a = x0 + x2, b = x0 - x2, c = x1 + x3, d = x1 - x3:
    // y0 = a + c, y2 = a - c, y1 = b + i d, y3 = b - i d
    const cplx a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    const cplx c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cmk(b.x - d.y, b.y + d.x);
    x[3] = cmk(b.x + d.y, b.y - d.x);
  }
}

template <int M2, int M3>
__device__ inline void dft23_pos(cplx (&x)[M2 * M3]) {
#pragma unroll
  for (int a = 0; a < M2; ++a) {
    cplx t[M3];
#pragma unroll
    for (int j = 0; j < M3; ++j) t[j] = x[a * M3 + j];
    dft_pos<M3>(t);
#pragma unroll
    for (int j = 0; j < M3; ++j) x[a * M3 + j] = t[j];
  }
#pragma unroll
  for (int b = 0; b < M3; ++b) {
    cplx t[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) t[j] = x[j * M3 + b];
    dft_pos<M2>(t);
#pragma unroll
    for (int j = 0; j < M2; ++j) x[j * M3 + b] = t[j];
  }
}

// value of the lane (l ^ 1) or (l ^ 2) of the quad
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int2 u = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_mov_dpp(u.x, CTRL, 0xF, 0xF, true);
  r.y = __builtin_amdgcn_mov_dpp(u.y, CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, r);
}
constexpr int DPP_XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]
template <int CTRL>
__device__ inline cplx dpp_c(cplx v) { return cmk(dpp_d<CTRL>(v.x), dpp_d<CTRL>(v.y)); }

// radix-2 step across lanes l, l ^ X: even lanes v + p, odd lanes p - v
// (or, with twist, the odd lanes of the second half p - i v and v + i p)
template <int CTRL>
__device__ inline cplx bfly(cplx v, bool hi) {
  const cplx p = dpp_c<CTRL>(v);
  // selects, not branches: hi ? p - v : p + v
  const double sg = hi ? -1.0 : 1.0;
  return cmk(fma(sg, v.x, p.x), fma(sg, v.y, p.y));
}

template <int M1, int M2, int M3>
__global__ __launch_bounds__(256) void kconv_reg_kernel(KconvArgs a) {
  constexpr int NV = M2 * M3, EPW = 64 / M1;
  const int lane = threadIdx.x & 63;
  const int k1 = lane % M1;
  const long long e = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * EPW + lane / M1;
  const bool in = e < a.n_elem;
  const long long ie = in ? (e / a.in_inner) * a.in_outer + e % a.in_inner : 0;
  cplx x[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    // every lane loads (ie = 0 is in bounds for lanes past the end, whose
    // quads only exchange among themselves and store nothing): a load under
    // a branch is waited for inside it, one round trip per value
    x[v] = a.in[(long long)(k1 * NV + v) * a.in_kstride + ie];
  }
  dft23_pos<M2, M3>(x);
  // k1 axis across the quad; M1 = 4 leaves the lanes in bit-reversed order
  if constexpr (M1 == 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = bfly<DPP_XOR1>(x[v], k1 & 1);
  } else if constexpr (M1 == 4) {
    // lanes 0..3 -> y0 = s0 + s1, y2 = s0 - s1, y1 = d0 + i d1, y3 = d0 - i d1;
    // lane k1 forms z = s + rho p with rho = 1, -1, i, i (y = gamma z with
    // gamma = 1, -1, 1, -i): only |y|^2 = |z|^2 is used, so gamma is dropped
    // and the step is two FMAs a component, no selects
    const double rr = k1 == 0 ? 1.0 : (k1 == 1 ? -1.0 : 0.0), ri = k1 >= 2 ? 1.0 : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const cplx s_ = bfly<DPP_XOR2>(x[v], k1 >= 2);     // x_j +- x_{j^2}
      const cplx p = dpp_c<DPP_XOR1>(s_);
      const double zr = fma(rr, p.x, fma(-ri, p.y, s_.x));
      const double zi = fma(rr, p.y, fma(ri, p.x, s_.y));
      x[v] = cmk(zr * zr + zi * zi, 0.0);
    }
  }
  // |T^R|^2
  if constexpr (M1 != 4) {
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = cmk(x[v].x * x[v].x + x[v].y * x[v].y, 0.0);
  }
  // R1 axis: input lanes hold R1 = bitrev(k1) for M1 = 4; output in natural order
  if constexpr (M1 == 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = bfly<DPP_XOR1>(x[v], k1 & 1);
  } else if constexpr (M1 == 4) {
    // real inputs: s = p1 +- x across lanes (l, l ^ 1), then with p the value
    // of lane l ^ 2: y0 = s + p, y1 = p - s (real), y2 = s + i p, y3 = p - i s,
    // as lane-constant coefficients of s and p
    const int role = ((k1 & 1) << 1) | (k1 >> 1);
    const double sg = (k1 & 1) ? -1.0 : 1.0;
    const double ar = role == 0 || role == 2 ? 1.0 : (role == 1 ? -1.0 : 0.0);
    const double br = role <= 1 || role == 3 ? 1.0 : 0.0;
    const double ai = role == 3 ? -1.0 : 0.0, bi = role == 2 ? 1.0 : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double s_ = fma(sg, x[v].x, dpp_d<DPP_XOR1>(x[v].x));   // a, b (lanes 0, 1), c, d (lanes 2, 3)
      const double p = dpp_d<DPP_XOR2>(s_);
      // y0 = a + c, y1 = b + i d, y2 = a - c, y3 = b - i d
      x[v] = cmk(fma(ar, s_, br * p), fma(ai, s_, bi * p));
    }
  }
  dft23_pos<M2, M3>(x);
  if (!in) return;
  const long long oe = (e / a.out_inner) * a.out_outer + e % a.out_inner;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int slot = a.qslot ? a.qslot[k1 * NV + v] : k1 * NV + v;
    if (slot < 0) continue;
    const long long off = (long long)slot * a.out_qstride + oe;
    a.out[off] = cscale(x[v], a.scale);
  }
}

template <int M1, int M2, int M3>
hipError_t launch_kconv_reg(const KconvArgs& a, hipStream_t s) {
  constexpr int EPB = 4 * (64 / M1);
  const long long blocks = (a.n_elem + EPB - 1) / EPB;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((kconv_reg_kernel<M1, M2, M3>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <int M1, int M2>
hipError_t kconv_reg_m3(const KconvArgs& a, hipStream_t s) {
  switch (a.m3) {
    case 1: return launch_kconv_reg<M1, M2, 1>(a, s);
    case 2: return launch_kconv_reg<M1, M2, 2>(a, s);
    case 3: return launch_kconv_reg<M1, M2, 3>(a, s);
    default: return launch_kconv_reg<M1, M2, 4>(a, s);
  }
}
template <int M1>
hipError_t kconv_reg_m2(const KconvArgs& a, hipStream_t s) {
  switch (a.m2) {
    case 1: return kconv_reg_m3<M1, 1>(a, s);
    case 2: return kconv_reg_m3<M1, 2>(a, s);
    case 3: return kconv_reg_m3<M1, 3>(a, s);
    default: return kconv_reg_m3<M1, 4>(a, s);
  }
}

// ---- register path of the pair transform (mixed precisions) ----
// 3-D forward DFT over an M1 x M2 x M3 mesh held in registers,
// x[(j1 * M2 + j2) * M3 + j3], one axis at a time.
template <int M1, int M2, int M3>
__device__ inline void mesh_dft_reg(float2 (&x)[M1 * M2 * M3]) {
  if constexpr (M3 > 1) {
#pragma unroll
    for (int a = 0; a < M1 * M2; ++a) {
      float2 t[M3], y[M3];
#pragma unroll
      for (int j = 0; j < M3; ++j) t[j] = x[a * M3 + j];
      small_dft_f<M3>(t, y);
#pragma unroll
      for (int j = 0; j < M3; ++j) x[a * M3 + j] = y[j];
    }
  }
  if constexpr (M2 > 1) {
#pragma unroll
    for (int j1 = 0; j1 < M1; ++j1)
#pragma unroll
      for (int j3 = 0; j3 < M3; ++j3) {
        float2 t[M2], y[M2];
#pragma unroll
        for (int j = 0; j < M2; ++j) t[j] = x[(j1 * M2 + j) * M3 + j3];
        small_dft_f<M2>(t, y);
#pragma unroll
        for (int j = 0; j < M2; ++j) x[(j1 * M2 + j) * M3 + j3] = y[j];
      }
  }
  if constexpr (M1 > 1) {
#pragma unroll
    for (int b = 0; b < M2 * M3; ++b) {
      float2 t[M1], y[M1];
#pragma unroll
      for (int j = 0; j < M1; ++j) t[j] = x[j * M2 * M3 + b];
      small_dft_f<M1>(t, y);
#pragma unroll
      for (int j = 0; j < M1; ++j) x[j * M2 * M3 + b] = y[j];
    }
  }
}

// One wave per (pair (p, q) of a fragment, 64 consecutive interpolation
// points): lane I loads psi_p(r_I + R) and psi_q(r_I + R) for every R from the
// complex FP32 copy of psi (each load instruction reads 64 consecutive I),
// forms conj(psi_p) psi_q in FP32, transforms R -> q in registers and writes
// the N_k outputs of its I (each store instruction covers 64 consecutive I
// of one row).  Workgroups are mapped XCD-contiguously so the psi rows of
// one fragment and I chunk stay in one L2 while all its pairs use them.
constexpr int PAIR_RB = 8;   // lattice vectors whose loads are issued together
template <int M1, int M2, int M3>
__global__ __launch_bounds__(256, 2) void pair_reg_kernel(PairArgs a, int nblocks) {
  constexpr int NK = M1 * M2 * M3;
  // output staging: per wave 8 rows (q) of 64 points in the operand format
  __shared__ __attribute__((aligned(16))) unsigned short stage[4][8][256];
  const int g8 = gridDim.x >> 3;
  const int blk = (int)(blockIdx.x & 7) * g8 + (int)(blockIdx.x >> 3);
  if (blk >= nblocks) return;
  const long long item = (long long)blk * 4 + (threadIdx.x >> 6);
  if (item >= a.nitems) return;                      // whole wave
  const int lane = threadIdx.x & 63;
  int lo = 0, hi = a.nfrag - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.item_off[mid] <= item) lo = mid; else hi = mid - 1;
  }
  const int f = lo;
  const int nf = a.frag_nf[f];
  const int np = a.frag_np ? a.frag_np[f] : nf * nf;     // pairs of this fragment in the launch
  const int pbeg = a.frag_p0 ? a.frag_p0[f] : 0;
  const long long local = item - a.item_off[f];
  const int chunk = (int)(local / np);
  const int pp = pbeg + (int)(local - (long long)chunk * np);
  const int p = pp / nf, q = pp - (pp / nf) * nf;
  const int I = chunk * 64 + lane;
  const bool in = I < a.n_ip;
  const int col = a.frag_col[f];
  const long long rstride = (long long)a.ncol * a.n_ip;
  float2 x[NK];
  // loads in batches of RB lattice vectors, all issued before the first use
  // (left to itself the compiler waits for every pair of loads in turn)
  // complex FP32 psi (the register path serves the mixed precisions only)
  const float2* fp = a.psi32 + (long long)(col + p) * a.n_ip + (in ? I : 0);
  const float2* fq = a.psi32 + (long long)(col + q) * a.n_ip + (in ? I : 0);
  constexpr int RB = NK < PAIR_RB ? NK : PAIR_RB;
#pragma unroll
  for (int R0 = 0; R0 < NK; R0 += RB) {
    float2 u[RB], v[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      if (R0 + j < NK) {
        u[j] = fp[(R0 + j) * rstride];
        v[j] = fq[(R0 + j) * rstride];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      if (R0 + j < NK) {
        // conj(u) v
        const float re = fmaf(u[j].x, v[j].x, u[j].y * v[j].y), im = fmaf(u[j].x, v[j].y, -(u[j].y * v[j].x));
        x[R0 + j] = in ? make_float2(re, im) : make_float2(0.f, 0.f);
      }
    }
  }
  mesh_dft_reg<M1, M2, M3>(x);
  const float sc = (float)a.scale;
  const long long base = (a.frag_pair[f] + pp) * a.p_stride + chunk * 64;   // row start of this chunk
  const int nI = (a.ld - chunk * 64) < 64 ? (int)(a.ld - chunk * 64) : 64;  // a multiple of 16
  if (a.fmt == 1) {
    if (I >= a.ld) return;
    float* o = (float*)a.out;
#pragma unroll
    for (int Q = 0; Q < NK; ++Q) {
      const int slot = a.qslot[Q];
      if (slot < 0) continue;
      const long long off = base + lane + slot * a.q_stride;
      o[off] = x[Q].x * sc;
      o[a.plane + off] = x[Q].y * sc;
    }
    return;
  }
  if (a.fmt == 3) {
    // single bf16: each row (q) of the chunk is 64 points x 4 bytes = 256
    // contiguous bytes; rows assembled in LDS, 8 at a time, written with
    // 16-byte stores (four rows per wave instruction)
    unsigned short (*st3)[256] = stage[threadIdx.x >> 6];
    const int e3 = (lane >> 3) * 16 + (lane & 7);
#pragma unroll
    for (int Q0 = 0; Q0 < NK; Q0 += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (Q0 + u >= NK) break;
        st3[u][e3] = bf16_bits_of(x[Q0 + u].x * sc);
        st3[u][e3 + 8] = bf16_bits_of(x[Q0 + u].y * sc);
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int u = 4 * h + (lane >> 4), part = lane & 15;   // row u, 16-byte part
        const int sq = Q0 + u < NK ? a.qslot[Q0 + u] : -1;
        if (sq >= 0 && (part >> 1) * 8 < nI) {
          const uint4 v = *(const uint4*)&st3[u][part * 8];
          *(uint4*)((unsigned short*)a.out + 2 * (base + (long long)sq * a.q_stride) + part * 8) = v;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    return;
  }
  // bf16 hi/lo: each row (q) of the chunk is 64 points x 8 bytes = 512
  // contiguous bytes; rows are assembled in LDS, 8 at a time, and written
  // with 16-byte stores (two rows per wave instruction)
  unsigned short (*st)[256] = stage[threadIdx.x >> 6];
  const int e = (lane >> 3) * 32 + (lane & 7);
#pragma unroll
  for (int Q0 = 0; Q0 < NK; Q0 += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (Q0 + u >= NK) break;
      const float re = x[Q0 + u].x * sc, im = x[Q0 + u].y * sc;
      const unsigned short rh = bf16_bits_of(re), ih = bf16_bits_of(im);
      st[u][e] = rh;
      st[u][e + 8] = bf16_bits_of(re - bf16_value(rh));
      st[u][e + 16] = ih;
      st[u][e + 24] = bf16_bits_of(im - bf16_value(ih));
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int u = 2 * h + (lane >> 5), part = lane & 31;   // row u, 16-byte part
      // output block of row u (uniform loads, one per half wave)
      const int s0 = Q0 + 2 * h < NK ? a.qslot[Q0 + 2 * h] : -1;
      const int s1 = Q0 + 2 * h + 1 < NK ? a.qslot[Q0 + 2 * h + 1] : -1;
      const int slot = (lane >> 5) ? s1 : s0;
      if (slot >= 0 && part * 2 < nI) {
        const uint4 v = *(const uint4*)&st[u][part * 8];
        *(uint4*)((unsigned short*)a.out + 4 * (base + (long long)slot * a.q_stride) + part * 8) = v;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int M1, int M2, int M3>
hipError_t launch_pair_reg(const PairArgs& a, hipStream_t s) {
  const long long nb = (a.nitems + 3) / 4;
  if (nb <= 0) return hipSuccess;
  if (nb > (1LL << 30)) return hipErrorInvalidValue;
  const long long g = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((pair_reg_kernel<M1, M2, M3>), dim3((unsigned)g), dim3(256), 0, s, a, (int)nb);
  return hipGetLastError();
}

template <int M1, int M2>
hipError_t pair_reg_m3(const PairArgs& a, hipStream_t s) {
  switch (a.m3) {
    case 1: return launch_pair_reg<M1, M2, 1>(a, s);
    case 2: return launch_pair_reg<M1, M2, 2>(a, s);
    case 3: return launch_pair_reg<M1, M2, 3>(a, s);
    default: return launch_pair_reg<M1, M2, 4>(a, s);
  }
}
template <int M1>
hipError_t pair_reg_m2(const PairArgs& a, hipStream_t s) {
  switch (a.m2) {
    case 1: return pair_reg_m3<M1, 1>(a, s);
    case 2: return pair_reg_m3<M1, 2>(a, s);
    case 3: return pair_reg_m3<M1, 3>(a, s);
    default: return pair_reg_m3<M1, 4>(a, s);
  }
}

}  // namespace

hipError_t kconv_launch(const KconvArgs& a, hipStream_t s) {
  if (a.mode == 0 && !a.out32 && (a.m1 == 1 || a.m1 == 2 || a.m1 == 4) && a.m2 <= 4 && a.m3 <= 4) {
    if (a.m1 == 1) return kconv_reg_m2<1>(a, s);
    if (a.m1 == 2) return kconv_reg_m2<2>(a, s);
    return kconv_reg_m2<4>(a, s);
  }
  if (a.mode == 0 && a.m1 == a.m2 && a.m2 == a.m3) {
    if (a.m1 == 6) return kconv_lines_launch<6, 6, 6>(a, s);
    if (a.m1 == 8) return kconv_lines_launch<8, 8, 8>(a, s);
    if (a.m1 == 10) return kconv_lines_launch<10, 10, 10>(a, s);
  }
  const int nk = a.m1 * a.m2 * a.m3;
  if (a.m1 > MAXM || a.m2 > MAXM || a.m3 > MAXM) return hipErrorInvalidValue;
  int etile = 1;                        // largest power of two with nk*etile <= 4096 (64 KB)
  while (etile < 256 && (long long)nk * etile * 2 <= 4096) etile *= 2;
  const long long blocks = (a.n_elem + etile - 1) / etile;
  if (blocks <= 0) return hipSuccess;
  const size_t lds = (size_t)nk * etile * sizeof(cplx);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const int mx = std::max(a.m1, std::max(a.m2, a.m3));
  if (mx <= 4) hipLaunchKernelGGL(kconv_kernel<4>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  else if (mx <= 8) hipLaunchKernelGGL(kconv_kernel<8>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  // axes up to 12 (the 10^3 mesh) without the registers of the longer lines
  else if (mx <= 12) hipLaunchKernelGGL(kconv_kernel<12>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  else hipLaunchKernelGGL(kconv_kernel<16>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  return hipGetLastError();
}

hipError_t xconv_launch(const XconvArgs& a, hipStream_t s) {
  if (!a.rho || !a.w || !a.wsel) return hipErrorInvalidValue;
  if (a.m1 > MAXM || a.m2 > MAXM || a.m3 > MAXM || a.m1 < 1 || a.m2 < 1 || a.m3 < 1) return hipErrorInvalidValue;
  if (a.m1 == a.m2 && a.m2 == a.m3) {
    if (a.m1 == 6) return xconv_lines_launch<6, 6, 6>(a, s);
    if (a.m1 == 8) return xconv_lines_launch<8, 8, 8>(a, s);
    if (a.m1 == 10) return xconv_lines_launch<10, 10, 10>(a, s);
  }
  const int nk = a.m1 * a.m2 * a.m3;
  int etile = 1;                        // two [nk][etile] columns in at most 64 KB
  while (etile < 256 && (long long)nk * etile * 2 <= 2048) etile *= 2;
  const long long blocks = (a.n_elem + etile - 1) / etile;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)nk * etile * sizeof(cplx);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const int mx = std::max(a.m1, std::max(a.m2, a.m3));
  if (mx <= 4) hipLaunchKernelGGL(xconv_kernel<4>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  else if (mx <= 8) hipLaunchKernelGGL(xconv_kernel<8>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  else hipLaunchKernelGGL(xconv_kernel<16>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  return hipGetLastError();
}

hipError_t pconv_launch(const PconvArgs& a, hipStream_t s) {
  if (!a.gv || !a.go || !a.qslot) return hipErrorInvalidValue;
  if (a.m1 > MAXM || a.m2 > MAXM || a.m3 > MAXM || a.m1 < 1 || a.m2 < 1 || a.m3 < 1) return hipErrorInvalidValue;
  if (a.m1 == a.m2 && a.m2 == a.m3) {
    if (a.m1 == 6) return pconv_lines_launch<6, 6, 6>(a, s);
    if (a.m1 == 8) return pconv_lines_launch<8, 8, 8>(a, s);
    if (a.m1 == 10) return pconv_lines_launch<10, 10, 10>(a, s);
  }
  const int nk = a.m1 * a.m2 * a.m3;
  int etile = 1;                        // two [nk][etile] columns in at most 64 KB
  while (etile < 256 && (long long)nk * etile * 2 <= 2048) etile *= 2;
  const long long blocks = (a.n_elem + etile - 1) / etile;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)nk * etile * sizeof(cplx);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const int mx = std::max(a.m1, std::max(a.m2, a.m3));
  if (mx <= 4) hipLaunchKernelGGL(pconv_kernel<4>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  else if (mx <= 8) hipLaunchKernelGGL(pconv_kernel<8>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  else hipLaunchKernelGGL(pconv_kernel<16>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  return hipGetLastError();
}

bool pair_reg_supported(int fmt, int m1, int m2, int m3) {
  return fmt != 0 && m1 <= 4 && m2 <= 4 && m3 <= 4;
}

bool pair32_supported(int fmt, int m1, int m2, int m3) {
  return fmt != 0 && !pair_reg_supported(fmt, m1, m2, m3);
}

bool pair_lines_supported(int fmt, int m1, int m2, int m3) {
  return fmt != 0 && m1 == m2 && m2 == m3 && (m1 == 6 || m1 == 8 || m1 == 10);
}

hipError_t pair_launch(const PairArgs& a, hipStream_t s) {
  if (!a.qslot) return hipErrorInvalidValue;
  if (pair_reg_supported(a.fmt, a.m1, a.m2, a.m3)) {
    if (!a.psi32 || !a.item_off) return hipErrorInvalidValue;
    switch (a.m1) {
      case 1: return pair_reg_m2<1>(a, s);
      case 2: return pair_reg_m2<2>(a, s);
      case 3: return pair_reg_m2<3>(a, s);
      default: return pair_reg_m2<4>(a, s);
    }
  }
  const int nk = a.m1 * a.m2 * a.m3;
  if (a.m1 > MAXM || a.m2 > MAXM || a.m3 > MAXM) return hipErrorInvalidValue;
  const long long blocks = (long long)a.nblocks * a.n_itiles;
  if (blocks <= 0) return hipSuccess;
  const int mx = std::max(a.m1, std::max(a.m2, a.m3));
  if (pair_lines_supported(a.fmt, a.m1, a.m2, a.m3)) {
    if (!a.psi32) return hipErrorInvalidValue;
    if (a.m1 == 6) return pair_lines_launch<6, 6, 6>(a, s);
    if (a.m1 == 8) return pair_lines_launch<8, 8, 8>(a, s);
    return pair_lines_launch<10, 10, 10>(a, s);
  }
  if (pair32_supported(a.fmt, a.m1, a.m2, a.m3)) {
    if (!a.psi32) return hipErrorInvalidValue;
    const size_t lds32 = (size_t)nk * a.tp * a.ti * sizeof(float2);
    if (lds32 > 64 * 1024) return hipErrorInvalidValue;
    if (mx <= 8) hipLaunchKernelGGL(pair32_kernel<8>, dim3((unsigned)blocks), dim3(256), lds32, s, a);
    else hipLaunchKernelGGL(pair32_kernel<16>, dim3((unsigned)blocks), dim3(256), lds32, s, a);
    return hipGetLastError();
  }
  const size_t lds = (size_t)nk * a.tp * a.ti * sizeof(cplx);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (mx <= 4) hipLaunchKernelGGL(pair_kernel<4>, dim3((unsigned)blocks), dim3(256), lds, s, a);
  else if (mx <= 8) hipLaunchKernelGGL(pair_kernel<8>, dim3((unsigned)blocks), dim3(256), lds, s, a);
  else hipLaunchKernelGGL(pair_kernel<16>, dim3((unsigned)blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}
