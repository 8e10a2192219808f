// Host-visible declarations of the gfx950 kernels' launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.hpp"

// ---------------------------------------------------------------------------
// Complex GEMM on MFMA (grouped, batched, K-segmented).
//   C[m][n] (+)= sum_{s<nseg} sum_{k<Kseg} opA(m, s, k) * opB(s, k, n)
// opA element (m, k) of segment s: A + s*sA_seg + (A_KM ? k*lda + m : m*lda + k),
// conjugated if a_conj; opB element (k, n): B + s*sB_seg + (B_KN ? k*ldb + n :
// n*ldb + k), conjugated if b_conj.  Batch b offsets A, B, C by sX_bat.
// Precisions: 0 = FP64 MFMA, 1 = FP32 MFMA, 2 = bf16 x3 split MFMA; in 1 and
// 2 each K segment is accumulated in FP32 and added into FP64 registers.
// herm: M == N and only tiles with tm >= tn are computed, mirrored as
// conj(value) at (n, m).  epi: 0 store, 1 accumulate, 2 ERI scatter
// (row P = p*nf+q, column P' = s*nf+r -> eri[((p*nf+q)*nf+r)*nf+s]).
// ---------------------------------------------------------------------------
struct GemmDesc {
  const cplx* A;
  const cplx* B;
  cplx* C;
  long long lda, ldb, ldc;
  long long sA_seg, sB_seg;
  long long sA_bat, sB_bat, sC_bat;
  int M, N, Kseg, nseg, batch;
  int Klast;              // length of the last K segment (<= Kseg)
  int tiles_m, tiles_n, tiles_per_batch;
  int herm, epi, nf;
  long long tile_begin;   // first global tile of this descriptor
};

enum { GEMM_A_KM = 1, GEMM_B_KN = 2, GEMM_A_CONJ = 4, GEMM_B_CONJ = 8 };

// Fills tile counts and tile_begin of every descriptor; returns total tiles.
long long gemm_plan(GemmDesc* d, int n);
// descs_dev: device copy of the planned descriptors.
hipError_t gemm_launch(int prec, int layout_flags, const GemmDesc* descs_dev, int ndesc,
                       long long total_tiles, int max_blocks, hipStream_t s);

// ---------------------------------------------------------------------------
// k-mesh transforms (Algorithm 1 and 2 in the k/R domain), LDS-staged.
// ---------------------------------------------------------------------------
struct KconvArgs {
  const cplx* in;       // in[k*in_kstride + in_map(e)]
  cplx* out;            // out[q*out_qstride + out_map(e)]
  long long in_kstride, out_qstride;
  long long n_elem;
  long long in_inner, in_outer;    // in_map(e)  = (e / in_inner)*in_outer + e % in_inner
  long long out_inner, out_outer;  // out_map(e) = (e / out_inner)*out_outer + e % out_inner
  int m1, m2, m3;
  int mode;        // 0: out = scale * DFT_{+}( |DFT_{+}(in)|^2 ) ; 1: out = scale * DFT_{sign}(in)
  int sign;        // +1 / -1 for mode 1
  double scale;
};
hipError_t kconv_launch(const KconvArgs& a, hipStream_t s);

// Fragment pair transform: M[Q][I][pair_off_f + p*nf + q] =
//   scale * sum_R exp(-2 pi i jQ.jR/m) conj(psi[R][I][col_f + p]) psi[R][I][col_f + q]
struct PairBlock { int frag; int pair0; int npair; };
struct PairArgs {
  const cplx* psi;         // [N_R][n_ip][ncol]
  cplx* out;               // [N_q][n_ip][ptot]
  const PairBlock* blocks; // device
  const int* frag_nf; const int* frag_col; const long long* frag_pair;  // device
  int nblocks, n_ip, ncol, pb_max;
  long long ptot;
  int m1, m2, m3;
  double scale;
};
hipError_t pair_launch(const PairArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Unit-cell grid FFT of f_{q,I}(r) exp(-i q.r) with the Coulomb factor
// sqrt(Omega 4 pi/|G+q|^2)/N_g applied (0 at G+q = 0), in place on
// data[q][I][N_g], q = q0 .. q0+nq-1 (q0 selects the mesh point).
// ---------------------------------------------------------------------------
struct GridFftArgs {
  cplx* data;
  int n1, n2, n3;
  int m1, m2, m3;
  int q0, nq, n_ip;
  long long q_stride;     // elements between consecutive q in data
  double recip[9];        // rows b1 b2 b3
  double volume;
};
hipError_t gridfft_launch(const GridFftArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// FP64 pivoted Cholesky of Pi^q (one workgroup per q) and the two-sided
// solve W = Pi^+ V Pi^+ through the factor.
// ---------------------------------------------------------------------------
hipError_t chol_launch(const cplx* pi, cplx* work, cplx* lt, int* perm, int* rank,
                       int n, int nq, double rtol, int pivot, hipStream_t s);
// stage 1: Z = Pi~^-1 (P^T V P)   stage 2: W = P (Pi~^-1 Z^H) P^T
hipError_t wsolve_launch(const cplx* v, cplx* z, cplx* w, const cplx* lt, const int* perm,
                         const int* rank, int n, int nq, hipStream_t s);

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
// Xt[k][mu][I] = phi[k][mu][ip[I]]
hipError_t gather_launch(const cplx* phi, const int* ip, cplx* xt, int nk, int norb,
                         long long ng, int nip, hipStream_t s);
// out[k][mu][col0 + p] = in[k][mu][p] for a fragment's coefficients (device copy
// into the batch matrix)
hipError_t copy_cols_launch(const cplx* in, cplx* out, int nk, int norb, int nf,
                            int ncol, int col0, hipStream_t s);
// count non-finite entries (real or imaginary) of n complex values into *flag
hipError_t nonfinite_launch(const cplx* x, long long n, int* flag, hipStream_t s);
