// Unit-cell 3-D FFT with the Bloch phase and the Coulomb kernel fused in
// (eqs. (6)-(7) "computed by FFT").
//
// For every (q, I) the function f(r) exp(-i q.r) on the n1 x n2 x n3 grid is
// transformed, and each coefficient at G is scaled by
// sqrt(Omega 4 pi/|G+q|^2)/N_g (0 at G+q = 0), so that the Coulomb matrix of
// eq. (7) is a plain Hermitian product of the result.  Two HBM passes:
//   pass A: one or more contiguous (i2, i3) slabs per workgroup, phase applied
//           on load, FFT along i3 then i2 inside LDS;
//   pass B: 64 consecutive (i2, i3) columns per workgroup, FFT along i1
//           inside LDS, Coulomb factor applied on store.
// Every HBM access is a contiguous row.  Each 1-D transform of length
// n = na * nb is a two-factor Cooley-Tukey (na-point DFTs, twiddle, nb-point
// DFTs) read from and written to LDS, with the twiddles in an LDS table.
#include "kernels.hpp"
#include "dft_small.hpp"

namespace {

__device__ inline void factor2(int n, int& na, int& nb) {
  na = 1;
  for (int f = 2; f * f <= n; ++f)
    if (n % f == 0) na = f;
  nb = n / na;
}

// Forward DFT (exp(-2 pi i jk/n)) of nlines lines held in buf; element j of
// line l at buf[base(l) + j*estride], base(l) = (l / L1)*S1 + (l % L1)*S2.
// tmp has the same layout; tw[t] = exp(-2 pi i t/n).  Result back in buf.
__device__ void fft_lines(cplx* buf, cplx* tmp, const cplx* tw, int n, int nlines, int L1,
                          int S1, int S2, int estride) {
  int na, nb;
  factor2(n, na, nb);
  const int total = nlines * n;
  for (int o = threadIdx.x; o < total; o += blockDim.x) {
    const int l = o / n, r = o - (o / n) * n;
    const int base = (l / L1) * S1 + (l % L1) * S2;
    const int j2 = r / na, k1 = r - (r / na) * na;
    cplx acc = cmk(0.0, 0.0);
    for (int j1 = 0; j1 < na; ++j1)
      cfma(acc, buf[base + (nb * j1 + j2) * estride], tw[(j1 * k1 * nb) % n]);
    tmp[base + r * estride] = cmul(acc, tw[(j2 * k1) % n]);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < total; o += blockDim.x) {
    const int l = o / n, r = o - (o / n) * n;
    const int base = (l / L1) * S1 + (l % L1) * S2;
    const int k1 = r % na, k2 = r / na;
    cplx acc = cmk(0.0, 0.0);
    for (int j2 = 0; j2 < nb; ++j2)
      cfma(acc, tmp[base + (j2 * na + k1) * estride], tw[(j2 * k2 * na) % n]);
    buf[base + r * estride] = acc;
  }
  __syncthreads();
}

__device__ inline double wrap_frac(int j, int m) {
  // representative of j modulo m in [-m/2, m/2), divided by m
  int w = ((j + m / 2) % m) - m / 2;
  return (double)w / (double)m;
}

__device__ inline int q_of(const GridFftArgs& a, int qi) { return a.qlist ? a.qlist[qi] : a.q0 + qi; }

__device__ inline void q_frac(const GridFftArgs& a, int q, double qf[3]) {
  const int j1 = q / (a.m2 * a.m3), j2 = (q / a.m3) % a.m2, j3 = q % a.m3;
  qf[0] = wrap_frac(j1, a.m1);
  qf[1] = wrap_frac(j2, a.m2);
  qf[2] = wrap_frac(j3, a.m3);
}

__device__ inline int wrap_int(int g, int n) { return ((g + n / 2) % n) - n / 2; }

// Wrapped mesh integers of q (the Bloch phase uses jw/m).
__device__ inline void q_wrapped(const GridFftArgs& a, int q, int jw[3]) {
  const int j[3] = {q / (a.m2 * a.m3), (q / a.m3) % a.m2, q % a.m3};
  const int m[3] = {a.m1, a.m2, a.m3};
  for (int d = 0; d < 3; ++d) jw[d] = ((j[d] + m[d] / 2) % m[d]) - m[d] / 2;
}

// Axis d of K = G + q for DFT index i (frequency i after the Bloch phase
// exp(-i q.r), q = jw/m): the representative of the class i + jw/m (mod n)
// nearest zero, in units of b_d.  It is unique except at +-n/2 (the Nyquist
// plane of an even grid, or a zone-boundary q on an odd one): there `tie`
// is set and the returned -n/2 stands with +n/2.  Integer arithmetic in
// units of 1/m, so ties are found exactly.
__device__ inline double k_axis(int i, int jw, int n, int m, bool& tie) {
  const int P = n * m;
  int r = (i * m + jw) % P;
  if (r < 0) r += P;
  if (2 * r >= P) r -= P;
  tie = (2 * r == -P);
  return (double)r / (double)m;
}

// 4 pi/|K|^2 factor of eq. (7) up to the constant: the mean of 1/|K|^2 over
// the representatives of K (each tied axis doubles them, with the opposite
// sign), 0 at K = 0.  b: reciprocal rows b1 b2 b3.
__device__ inline double inv_k2_mean(const double x[3], const bool t[3], const double* b) {
  double acc = 0.0;
  int cnt = 0;
  for (int s = 0; s < 8; ++s) {
    if (((s & 1) && !t[0]) || ((s & 2) && !t[1]) || ((s & 4) && !t[2])) continue;
    const double y0 = (s & 1) ? -x[0] : x[0], y1 = (s & 2) ? -x[1] : x[1], y2 = (s & 4) ? -x[2] : x[2];
    const double kx = y0 * b[0] + y1 * b[3] + y2 * b[6];
    const double ky = y0 * b[1] + y1 * b[4] + y2 * b[7];
    const double kz = y0 * b[2] + y1 * b[5] + y2 * b[8];
    const double k2 = kx * kx + ky * ky + kz * kz;
    if (k2 > 1e-20) acc += 1.0 / k2;
    ++cnt;
  }
  return acc / cnt;
}

__global__ __launch_bounds__(256) void slab_kernel(GridFftArgs a, int S) {
  extern __shared__ cplx sm[];
  const int n23 = a.n2 * a.n3;
  cplx* buf = sm;
  cplx* tmp = sm + S * n23;
  cplx* tw2 = tmp + S * n23;
  cplx* tw3 = tw2 + a.n2;
  for (int t = threadIdx.x; t < a.n2; t += blockDim.x) tw2[t] = cexpipi(-2.0 * t / a.n2);
  for (int t = threadIdx.x; t < a.n3; t += blockDim.x) tw3[t] = cexpipi(-2.0 * t / a.n3);
  const long long nslab = (long long)a.nq * a.n_ip * a.n1;
  const long long s0 = (long long)blockIdx.x * S;
  const int ns = (int)((nslab - s0) < S ? (nslab - s0) : S);
  for (int idx = threadIdx.x; idx < ns * n23; idx += blockDim.x) {
    const int s = idx / n23, p = idx - (idx / n23) * n23;
    const long long slab = s0 + s;
    const int i1 = (int)(slab % a.n1);
    const long long qI = slab / a.n1;
    const int I = (int)(qI % a.n_ip);
    const int qi = (int)(qI / a.n_ip);
    double qf[3];
    q_frac(a, q_of(a, qi), qf);
    const int i2 = p / a.n3, i3 = p - (p / a.n3) * a.n3;
    const double ph = qf[0] * i1 / a.n1 + qf[1] * i2 / a.n2 + qf[2] * i3 / a.n3;
    const cplx v = a.data[(long long)qi * a.q_stride + ((long long)I * a.n1 + i1) * n23 + p];
    buf[idx] = cmul(v, cexpipi(-2.0 * ph));
  }
  __syncthreads();
  fft_lines(buf, tmp, tw3, a.n3, ns * a.n2, 1, a.n3, 0, 1);          // along i3
  fft_lines(buf, tmp, tw2, a.n2, ns * a.n3, a.n3, n23, 1, a.n3);     // along i2
  for (int idx = threadIdx.x; idx < ns * n23; idx += blockDim.x) {
    const int s = idx / n23, p = idx - (idx / n23) * n23;
    const long long slab = s0 + s;
    const int i1 = (int)(slab % a.n1);
    const long long qI = slab / a.n1;
    const int I = (int)(qI % a.n_ip);
    const int qi = (int)(qI / a.n_ip);
    a.data[(long long)qi * a.q_stride + ((long long)I * a.n1 + i1) * n23 + p] = buf[idx];
  }
}

constexpr int COLS = 64;

__global__ __launch_bounds__(256) void col_kernel(GridFftArgs a) {
  extern __shared__ cplx sm[];
  const int n23 = a.n2 * a.n3;
  const int ncb = (n23 + COLS - 1) / COLS;
  cplx* buf = sm;
  cplx* tmp = sm + a.n1 * COLS;
  cplx* tw1 = tmp + a.n1 * COLS;
  for (int t = threadIdx.x; t < a.n1; t += blockDim.x) tw1[t] = cexpipi(-2.0 * t / a.n1);
  const int cb = blockIdx.x % ncb;
  const long long qI = blockIdx.x / ncb;
  const int I = (int)(qI % a.n_ip);
  const int qi = (int)(qI / a.n_ip);
  const int c0 = cb * COLS;
  const int nc = (n23 - c0) < COLS ? (n23 - c0) : COLS;
  cplx* base = a.data + (long long)qi * a.q_stride + (long long)I * a.n1 * n23;
  for (int idx = threadIdx.x; idx < a.n1 * COLS; idx += blockDim.x) {
    const int i1 = idx / COLS, c = idx - (idx / COLS) * COLS;
    buf[idx] = (c < nc) ? base[(long long)i1 * n23 + c0 + c] : cmk(0.0, 0.0);
  }
  __syncthreads();
  fft_lines(buf, tmp, tw1, a.n1, COLS, 1, 1, 0, COLS);                 // along i1
  int jw[3];
  q_wrapped(a, q_of(a, qi), jw);
  const double coef = sqrt(4.0 * M_PI * a.volume) / ((double)a.n1 * n23);
  for (int idx = threadIdx.x; idx < a.n1 * COLS; idx += blockDim.x) {
    const int i1 = idx / COLS, c = idx - (idx / COLS) * COLS;
    if (c >= nc) continue;
    const int col = c0 + c;
    double x[3];
    bool t[3];
    x[0] = k_axis(i1, jw[0], a.n1, a.m1, t[0]);
    x[1] = k_axis(col / a.n3, jw[1], a.n2, a.m2, t[1]);
    x[2] = k_axis(col % a.n3, jw[2], a.n3, a.m3, t[2]);
    const double f = coef * sqrt(inv_k2_mean(x, t, a.recip));
    base[(long long)i1 * n23 + col] = cscale(buf[idx], f);
  }
}

// ---- compile-time-size variants (cubic grids): every index division is by a
// constant, and the radix loops unroll ----
template <int N> constexpr int fac_a() {
  int na = 1;
  for (int f = 2; f * f <= N; ++f)
    if (N % f == 0) na = f;
  return na;
}

// Same transform as fft_lines with the line geometry fixed at compile time:
// element j of line l at buf[(l / L1) * S1 + (l % L1) * S2 + j * ES].
template <int N, int L1, int S1, int S2, int ES>
__device__ void fft_lines_c(cplx* buf, cplx* tmp, const cplx* tw, int nlines) {
  constexpr int NA = fac_a<N>(), NB = N / NA;
  const int total = nlines * N;
  for (int o = threadIdx.x; o < total; o += blockDim.x) {
    const int l = o / N, r = o % N;
    const int base = (l / L1) * S1 + (l % L1) * S2;
    const int j2 = r / NA, k1 = r % NA;
    cplx acc = cmk(0.0, 0.0);
#pragma unroll
    for (int j1 = 0; j1 < NA; ++j1) cfma(acc, buf[base + (NB * j1 + j2) * ES], tw[(j1 * k1 * NB) % N]);
    tmp[base + r * ES] = cmul(acc, tw[(j2 * k1) % N]);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < total; o += blockDim.x) {
    const int l = o / N, r = o % N;
    const int base = (l / L1) * S1 + (l % L1) * S2;
    const int k1 = r % NA, k2 = r / NA;
    cplx acc = cmk(0.0, 0.0);
#pragma unroll
    for (int j2 = 0; j2 < NB; ++j2) cfma(acc, tmp[base + (j2 * NA + k1) * ES], tw[(j2 * k2 * NA) % N]);
    buf[base + r * ES] = acc;
  }
  __syncthreads();
}

// ---- two-stage radix transforms with the small DFTs in registers ----
// factor N = NA * NB with both <= 8 (NA <= NB), or 0 if impossible
template <int N> constexpr int radix_a() {
  int best = 0;
  for (int a = 2; a <= 8; ++a)
    if (N % a == 0 && N / a <= 8 && a <= N / a) best = a;
  return best;
}

// Same transform as fft_lines_c: stage 1, one thread per (line, j2), does an
// NA-point DFT over j1 in registers and the twiddle w^{j2 k1}; stage 2, one
// thread per (line, k1), an NB-point DFT over j2.  Two LDS reads and two LDS
// writes per point and axis.
template <int N, int L1, int S1, int S2, int ES>
__device__ void fft_lines_r(cplx* buf, cplx* tmp, const cplx* tw, int nlines) {
  constexpr int NA = radix_a<N>(), NB = N / NA;
  const int n1 = nlines * NB;
  for (int it = threadIdx.x; it < n1; it += blockDim.x) {
    const int l = it / NB, j2 = it % NB;
    const int base = (l / L1) * S1 + (l % L1) * S2;
    cplx x[NA], y[NA];
#pragma unroll
    for (int j1 = 0; j1 < NA; ++j1) x[j1] = buf[base + (NB * j1 + j2) * ES];
    small_dft<NA>(x, y);
    tmp[base + (j2 * NA) * ES] = y[0];
#pragma unroll
    for (int k1 = 1; k1 < NA; ++k1) tmp[base + (j2 * NA + k1) * ES] = cmul(y[k1], tw[(j2 * k1) % N]);
  }
  __syncthreads();
  const int n2 = nlines * NA;
  for (int it = threadIdx.x; it < n2; it += blockDim.x) {
    const int l = it / NA, k1 = it % NA;
    const int base = (l / L1) * S1 + (l % L1) * S2;
    cplx x[NB], y[NB];
#pragma unroll
    for (int j2 = 0; j2 < NB; ++j2) x[j2] = tmp[base + (j2 * NA + k1) * ES];
    small_dft<NB>(x, y);
#pragma unroll
    for (int k2 = 0; k2 < NB; ++k2) buf[base + (k1 + NA * k2) * ES] = y[k2];
  }
  __syncthreads();
}

// radix path when N factors into two factors <= 8, generic otherwise
template <int N, int L1, int S1, int S2, int ES>
__device__ inline void fft_axis(cplx* buf, cplx* tmp, const cplx* tw, int nlines) {
  if constexpr (radix_a<N>() != 0) fft_lines_r<N, L1, S1, S2, ES>(buf, tmp, tw, nlines);
  else fft_lines_c<N, L1, S1, S2, ES>(buf, tmp, tw, nlines);
}

// The Bloch phase exp(-2 pi i (qf0 i1 + qf1 i2 + qf2 i3) / N) of a slab is
// the product of an (i1, i2) factor and an i3 factor, 2 N values a slab
// computed once into LDS (a sine and cosine per value, not per point).
template <int N>
__global__ __launch_bounds__(256) void slab_kernel_c(GridFftArgs a, int S) {
  constexpr int N2 = N * N;
  extern __shared__ cplx sm[];
  cplx* buf = sm;
  cplx* tmp = sm + S * N2;
  cplx* tw = tmp + S * N2;
  cplx* ph = tw + N;                    // [S][2N]: (i1, i2) factors, then i3 factors
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw[t] = cexpipi(-2.0 * t / N);
  const long long nslab = (long long)a.nq * a.n_ip * N;
  const long long s0 = (long long)blockIdx.x * S;
  const int ns = (int)((nslab - s0) < S ? (nslab - s0) : S);
  for (int t = threadIdx.x; t < ns * 2 * N; t += blockDim.x) {
    const int s = t / (2 * N), r = t % (2 * N);
    const long long slab = s0 + s;
    const int i1 = (int)(slab % N);
    const int qi = (int)(slab / N / a.n_ip);
    double qf[3];
    q_frac(a, q_of(a, qi), qf);
    ph[t] = r < N ? cexpipi(-2.0 * (qf[0] * i1 + qf[1] * r) / N) : cexpipi(-2.0 * (qf[2] * (r - N)) / N);
  }
  __syncthreads();
  for (int s = 0; s < ns; ++s) {
    const long long slab = s0 + s;
    const int i1 = (int)(slab % N);
    const long long qI = slab / N;
    const int I = (int)(qI % a.n_ip);
    const int qi = (int)(qI / a.n_ip);
    const cplx* src = a.data + (long long)qi * a.q_stride + ((long long)I * N + i1) * N2;
    const cplx* phs = ph + s * 2 * N;
    for (int p = threadIdx.x; p < N2; p += blockDim.x) {
      const int i2 = p / N, i3 = p % N;
      buf[s * N2 + p] = cmul(src[p], cmul(phs[i2], phs[N + i3]));
    }
  }
  __syncthreads();
  fft_axis<N, 1, N, 0, 1>(buf, tmp, tw, ns * N);    // along i3
  fft_axis<N, N, N2, 1, N>(buf, tmp, tw, ns * N);   // along i2
  for (int s = 0; s < ns; ++s) {
    const long long slab = s0 + s;
    const int i1 = (int)(slab % N);
    const long long qI = slab / N;
    const int I = (int)(qI % a.n_ip);
    const int qi = (int)(qI / a.n_ip);
    cplx* dst = a.data + (long long)qi * a.q_stride + ((long long)I * N + i1) * N2;
    for (int p = threadIdx.x; p < N2; p += blockDim.x) dst[p] = buf[s * N2 + p];
  }
}

// One workgroup takes a block of COLS_C columns of one q for up to `ipb`
// interpolation points in turn: the Coulomb factor of its elements depends on
// (q, i1, column) only, so it is formed once and kept in registers.  32
// columns (512-byte rows) keep the LDS at 42 KB for N = 40, three workgroups
// a CU.
constexpr int COLS_C = 32;
template <int N>
__global__ __launch_bounds__(256) void col_kernel_c(GridFftArgs a, int ipb) {
  constexpr int N2 = N * N;
  constexpr int NCB = (N2 + COLS_C - 1) / COLS_C;
  constexpr int PER = (N * COLS_C + 255) / 256;   // elements of a thread
  extern __shared__ cplx sm[];
  cplx* buf = sm;
  cplx* tmp = sm + N * COLS_C;
  cplx* tw = tmp + N * COLS_C;
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw[t] = cexpipi(-2.0 * t / N);
  const int cb = blockIdx.x % NCB;
  const long long rest = blockIdx.x / NCB;
  const int nib = (a.n_ip + ipb - 1) / ipb;
  const int ib = (int)(rest % nib);
  const int qi = (int)(rest / nib);
  const int I0 = ib * ipb, I1 = min(I0 + ipb, a.n_ip);
  const int c0 = cb * COLS_C;
  const int nc = (N2 - c0) < COLS_C ? (N2 - c0) : COLS_C;
  int jw[3];
  q_wrapped(a, q_of(a, qi), jw);
  const double coef = sqrt(4.0 * M_PI * a.volume) / ((double)N * N2);
  double fac[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int idx = threadIdx.x + 256 * u;
    fac[u] = 0.0;
    const int i1 = idx / COLS_C, c = idx % COLS_C;
    if (idx < N * COLS_C && c < nc) {
      const int col = c0 + c;
      double x[3];
      bool t[3];
      x[0] = k_axis(i1, jw[0], N, a.m1, t[0]);
      x[1] = k_axis(col / N, jw[1], N, a.m2, t[1]);
      x[2] = k_axis(col % N, jw[2], N, a.m3, t[2]);
      fac[u] = coef * sqrt(inv_k2_mean(x, t, a.recip));
    }
  }
  for (int I = I0; I < I1; ++I) {
    cplx* base = a.data + (long long)qi * a.q_stride + (long long)I * N * N2;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = threadIdx.x + 256 * u;
      if (idx < N * COLS_C) {
        const int i1 = idx / COLS_C, c = idx % COLS_C;
        buf[idx] = (c < nc) ? base[(long long)i1 * N2 + c0 + c] : cmk(0.0, 0.0);
      }
    }
    __syncthreads();
    fft_axis<N, 1, 1, 0, COLS_C>(buf, tmp, tw, COLS_C);   // along i1
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = threadIdx.x + 256 * u;
      const int i1 = idx / COLS_C, c = idx % COLS_C;
      if (idx < N * COLS_C && c < nc) base[(long long)i1 * N2 + c0 + c] = cscale(buf[idx], fac[u]);
    }
    __syncthreads();                      // buf is read before the next point's loads
  }
}

template <int N>
hipError_t launch_cubic(const GridFftArgs& a, hipStream_t s) {
  constexpr int N2 = N * N;
  int S = 2048 / N2;
  if (S < 1) S = 1;
  size_t ldsA = (2 * (size_t)S * N2 + N + 2 * (size_t)S * N) * sizeof(cplx);
  while (ldsA > 150 * 1024 && S > 1) {
    --S;
    ldsA = (2 * (size_t)S * N2 + N + 2 * (size_t)S * N) * sizeof(cplx);
  }
  if (ldsA > 160 * 1024) return hipErrorInvalidValue;
  const long long nslab = (long long)a.nq * a.n_ip * N;
  if (nslab <= 0) return hipSuccess;
  hipLaunchKernelGGL(slab_kernel_c<N>, dim3((unsigned)((nslab + S - 1) / S)), dim3(256), ldsA, s, a, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t ldsB = (2 * (size_t)N * COLS_C + N) * sizeof(cplx);
  if (ldsB > 160 * 1024) return hipErrorInvalidValue;
  const long long ncb = (N2 + COLS_C - 1) / COLS_C;
  const int ipb = 8;                    // interpolation points a workgroup (Coulomb factor reused)
  const long long nib = (a.n_ip + ipb - 1) / ipb;
  const long long nblk = ncb * a.nq * nib;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(col_kernel_c<N>, dim3((unsigned)nblk), dim3(256), ldsB, s, a, ipb);
  return hipGetLastError();
}

}  // namespace

hipError_t gridfft_launch(const GridFftArgs& a, hipStream_t s) {
  if (a.n1 == a.n2 && a.n2 == a.n3) {
    switch (a.n1) {
      case 6: return launch_cubic<6>(a, s);
      case 8: return launch_cubic<8>(a, s);
      case 10: return launch_cubic<10>(a, s);
      case 12: return launch_cubic<12>(a, s);
      case 16: return launch_cubic<16>(a, s);
      case 18: return launch_cubic<18>(a, s);
      case 20: return launch_cubic<20>(a, s);
      case 24: return launch_cubic<24>(a, s);
      case 30: return launch_cubic<30>(a, s);
      case 32: return launch_cubic<32>(a, s);
      case 36: return launch_cubic<36>(a, s);
      case 40: return launch_cubic<40>(a, s);
      case 48: return launch_cubic<48>(a, s);
      case 60: return launch_cubic<60>(a, s);
      case 64: return launch_cubic<64>(a, s);
      default: break;
    }
  }
  const int n23 = a.n2 * a.n3;
  int S = 2048 / n23;
  if (S < 1) S = 1;
  size_t ldsA = (2 * (size_t)S * n23 + a.n2 + a.n3) * sizeof(cplx);
  while (ldsA > 150 * 1024 && S > 1) {
    --S;
    ldsA = (2 * (size_t)S * n23 + a.n2 + a.n3) * sizeof(cplx);
  }
  if (ldsA > 160 * 1024) return hipErrorInvalidValue;
  const long long nslab = (long long)a.nq * a.n_ip * a.n1;
  if (nslab <= 0) return hipSuccess;
  hipLaunchKernelGGL(slab_kernel, dim3((unsigned)((nslab + S - 1) / S)), dim3(256), ldsA, s, a, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t ldsB = (2 * (size_t)a.n1 * COLS + a.n1) * sizeof(cplx);
  if (ldsB > 160 * 1024) return hipErrorInvalidValue;
  const long long ncb = (n23 + COLS - 1) / COLS;
  hipLaunchKernelGGL(col_kernel, dim3((unsigned)(ncb * a.nq * a.n_ip)), dim3(256), ldsB, s, a);
  return hipGetLastError();
}
