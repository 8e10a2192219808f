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

namespace {

constexpr int MAXM = 16;

// In-place 3-D DFT over the mesh for every element column of buf[k][etile]:
// buf[k][e] <- sum_j exp(sign * 2 pi i sum_d j_d k_d / m_d) buf[j][e].
// tw[ax][t] = exp(2 pi i t / m_ax), filled by init_twiddles.
__device__ void init_twiddles(cplx (*tw)[MAXM], int m1, int m2, int m3) {
  const int ms[3] = {m1, m2, m3};
  if (threadIdx.x < 3 * MAXM) {
    const int ax = threadIdx.x / MAXM, t = threadIdx.x % MAXM;
    if (t < ms[ax]) tw[ax][t] = cexpipi(2.0 * (double)t / (double)ms[ax]);
  }
}

// Length-M DFT of lines p[j * estride], j < M, for the lines `line` owned by
// this thread; M is a compile-time constant so the loops unroll and the
// twiddle indices (j t mod M) are constants; twiddles live in registers for
// M <= 8 and are read from the LDS table (one broadcast read) above.
template <int M>
__device__ void axis_dft(cplx* buf, const cplx* twa, int nlines, int eshift, int ax, int m2, int m3,
                         int sign) {
  constexpr int MW = M <= 8 ? M : 1;
  cplx w[MW];
#pragma unroll
  for (int t = 0; t < MW; ++t) {
    w[t] = twa[t];
    if (sign < 0) w[t].y = -w[t].y;
  }
  const double sy = sign < 0 ? -1.0 : 1.0;
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
#pragma unroll
    for (int t = 0; t < M; ++t) {
      cplx acc = x[0];
#pragma unroll
      for (int j = 1; j < M; ++j) {
        if constexpr (M <= 8) {
          cfma(acc, x[j], w[(j * t) % M]);
        } else {
          const cplx wt = twa[(j * t) % M];
          cfma(acc, x[j], cmk(wt.x, sy * wt.y));
        }
      }
      p[t * estride] = acc;
    }
  }
}

// In-place 3-D DFT over the mesh for every element column of buf[k][etile]:
// buf[k][e] <- sum_j exp(sign * 2 pi i sum_d j_d k_d / m_d) buf[j][e].
// etile is a power of two; tw[ax][t] = exp(2 pi i t / m_ax).
// MAXA: largest axis length of the mesh (4, 8 or 16): only the axis
// transforms up to it are instantiated, which keeps the register count of
// the kernels (and so their occupancy) set by the mesh actually used.
template <int MAXA>
__device__ void mesh_dft(cplx* buf, const cplx (*tw)[MAXM], int etile, int m1, int m2, int m3,
                         int sign) {
  const int eshift = __builtin_ctz(etile);
  const int nk = m1 * m2 * m3;
  const int ms[3] = {m1, m2, m3};
  for (int ax = 0; ax < 3; ++ax) {
    const int m = ms[ax];
    if (m == 1) continue;
    const int nlines = (nk / m) << eshift;
    switch (m) {
#define AXIS_CASE(M) \
  case M: if constexpr (M <= MAXA) axis_dft<M>(buf, tw[ax], nlines, eshift, ax, m2, m3, sign); break;
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
  __shared__ cplx tw[3][MAXM];
  init_twiddles(tw, a.m1, a.m2, a.m3);
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
    mesh_dft<MAXA>(buf, tw, etile, a.m1, a.m2, a.m3, +1);
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      cplx v = buf[idx];
      buf[idx] = cmk(v.x * v.x + v.y * v.y, 0.0);
    }
    __syncthreads();
    mesh_dft<MAXA>(buf, tw, etile, a.m1, a.m2, a.m3, +1);
  } else {
    mesh_dft<MAXA>(buf, tw, etile, a.m1, a.m2, a.m3, a.sign);
  }
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int q = idx >> eshift, e = idx & (etile - 1);
    if (e < ne) {
      long long off;
      if (fast) {
        off = out0 + e;
      } else {
        const long long ee = e0 + e;
        off = (ee / a.out_inner) * a.out_outer + ee % a.out_inner;
      }
      a.out[(long long)q * a.out_qstride + off] = cscale(buf[idx], a.scale);
    }
  }
}

// One workgroup: a tile of `tp` pairs of one fragment times `ti` consecutive
// interpolation points; LDS holds [R][tp*ti] so that the output rows (pair,
// I-range) are written as contiguous runs of I.
template <int MAXA>
__global__ __launch_bounds__(256) void pair_kernel(PairArgs a) {
  extern __shared__ cplx buf[];
  __shared__ cplx tw[3][MAXM];
  init_twiddles(tw, a.m1, a.m2, a.m3);
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
  mesh_dft<MAXA>(buf, tw, w, a.m1, a.m2, a.m3, -1);
  for (int idx = threadIdx.x; idx < nk * w; idx += blockDim.x) {
    const int Q = idx >> wshift, e = idx & (w - 1);
    const int j = e >> tshift, i = e & (a.ti - 1);
    const int I = I0 + i;
    if (j < pb.npair && I < a.ld) {
      const long long off = (long long)Q * a.q_stride + (poff + pb.pair0 + j) * a.p_stride + I;
      store_fmt(a.out, off, a.plane, a.fmt, cscale(buf[idx], a.scale));
    }
  }
}

}  // namespace

hipError_t kconv_launch(const KconvArgs& a, hipStream_t s) {
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
  else hipLaunchKernelGGL(kconv_kernel<16>, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  return hipGetLastError();
}

hipError_t pair_launch(const PairArgs& a, hipStream_t s) {
  const int nk = a.m1 * a.m2 * a.m3;
  if (a.m1 > MAXM || a.m2 > MAXM || a.m3 > MAXM) return hipErrorInvalidValue;
  const size_t lds = (size_t)nk * a.tp * a.ti * sizeof(cplx);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const long long blocks = (long long)a.nblocks * a.n_itiles;
  if (blocks <= 0) return hipSuccess;
  const int mx = std::max(a.m1, std::max(a.m2, a.m3));
  if (mx <= 4) hipLaunchKernelGGL(pair_kernel<4>, dim3((unsigned)blocks), dim3(256), lds, s, a);
  else if (mx <= 8) hipLaunchKernelGGL(pair_kernel<8>, dim3((unsigned)blocks), dim3(256), lds, s, a);
  else hipLaunchKernelGGL(pair_kernel<16>, dim3((unsigned)blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}
