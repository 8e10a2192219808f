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
// "NT" complex GEMM (both operands k-contiguous rows) for the large
// contractions:  C[m][n] (+)= sum_s sum_k opA(A_s[m][k]) opB(B_s[n][k]).
// Operand formats by precision: 0 complex128 rows (ld in complex elements);
// 1 two float planes re|im; 2 four bf16 planes re_hi|re_lo|im_hi|im_lo (ld and
// plane strides in scalar elements; rows zero-padded to a multiple of 8).
// epi: 0 store c128, 1 accumulate c128, 2 ERI scatter c128, 3 store in the
// split format of the precision (plane stride c_plane), zero-filling columns
// N..ldc-1, 4 subtract from c128.  herm: 1 lower tiles mirrored as conj to the
// upper triangle; 2 lower tiles only, no mirror.
// ---------------------------------------------------------------------------
struct NtDesc {
  const void* A;
  const void* B;
  void* C;
  long long lda, ldb, ldc;
  long long a_plane, b_plane, c_plane;
  long long sA_seg, sB_seg;
  long long sA_bat, sB_bat, sC_bat;
  int M, N, Kseg, nseg, Klast, batch;
  int tiles_m, tiles_n, tiles_per_batch;
  int herm, epi, nf;
  int npad;               // epi 3: columns written (zeros from N on); 0 = ldc
  int ktri;               // B[n][k] = 0 for k < n: the mixed kernels start each column
                          // tile's K range at its first column (FP64 reads the zeros)
  long long tile_begin;
};
long long nt_plan(NtDesc* d, int n);
// conj: bit 0 conjugates A, bit 1 conjugates B
// kind names the call site in profiles: 0 generic, 1 V^q, 2 U^q, 3 fragment contraction
hipError_t nt_launch(int prec, int conj, const NtDesc* descs_dev, int ndesc, long long total,
                     int max_blocks, hipStream_t s, int kind = 0);

// Large-tile (128x128, 512 threads) NT GEMM for the mixed precisions (1, 2):
// one K segment `seg` per launch; epi 1 accumulates the FP32 partials in an
// FP64 c128 output (segment 0 stores, later segments add), epi 3 stores the
// split format; herm 2 computes lower tiles only (entries above the diagonal
// inside diagonal tiles are left unwritten).
long long big_plan(NtDesc* d, int n);
hipError_t big_launch(int prec, int conj, const NtDesc* descs_dev, int ndesc, long long total,
                      int max_blocks, int seg, hipStream_t s, int kind = 0);
// Fill the upper triangles of nbat Hermitian n x n matrices (pitch ld,
// batch stride bat) from their computed lower triangles.
hipError_t herm_fill_launch(cplx* c, int n, long long ld, long long bat, int nbat, hipStream_t s);
// G[(pq)][(sr)] (Hermitian, lower triangle computed; the contraction over the
// classes {q, -q}) -> eri[p][q][r][s] = G[(pq)][(sr)] + conj(G[(qp)][(rs)])
// for n fragments in one launch: fragment f reads e + eoff[f] and writes
// eri[f]; nf, eoff, eri are device arrays
hipError_t eri_scatter_batch_launch(const cplx* e, const long long* eoff, cplx* const* eri, const int* nf,
                                    int n, int maxnf, hipStream_t s);
// bf16x3 NT GEMM on the 32x32x16 matrix cores (128 x 128 tiles, 256
// threads, direct-to-LDS operand copies): same descriptors and epilogues as
// big_launch for precision 2; plan with big_plan.
// ring: the ring pipeline (four LDS stages, one workgroup a CU, the next
// stage's fragments read during the MFMAs; same results bit for bit), for
// the call sites ring_supported accepts.
hipError_t x3_launch(int conj, const NtDesc* descs_dev, int ndesc, long long total, int max_blocks, int seg,
                     hipStream_t s, int kind, bool ring = false);
// The same kernel on the single-bf16 operand format (fmt 3): kind 2 without
// conjugation (U^q) and kind 3 with B conjugated (the contraction) only.
hipError_t x1_launch(int conj, const NtDesc* descs_dev, int ndesc, long long total, int max_blocks, int seg,
                     hipStream_t s, int kind, bool ring = false);
bool ring_supported(int conj, int kind);
// mixed-precision fragment contraction: classes {q, -q} summed in FP32 per
// launch (one contiguous K range of the classes of a group, the classes
// split into balanced groups), FP64 across launches.  The initial tiling of
// a context: the most classes a launch, at most ERI_QGROUP, whose K range
// of one operand row in the 8-byte mixed formats stays within ERI_ROW_BYTES
// (12 up to N_IP = 768, 11 at 800, 8 at 1040: the rows of the tiles an XCD runs
// together then stay within the last-level cache; at the 1000-k workload 8
// classes measured 1.7 % faster than 12, and 24 or 42 slower), and 2
// workgroups per CU for the fragment GEMMs (one resident wave of
// workgroups).  At 12 classes and 2 per CU it is also what the launch-tiling
// autotuner picks on a 4x4x4 mesh with 64 fragments of 12-40 orbitals.
constexpr int ERI_QGROUP = 12;
constexpr long long ERI_ROW_BYTES = 73728;
inline int initial_qgroup(long long ld) {
  const long long g = ERI_ROW_BYTES / (ld * 8);
  return (int)(g < 1 ? 1 : (g > ERI_QGROUP ? ERI_QGROUP : g));
}
constexpr int FRAG_WG_PER_CU = 2;

// W (c128 [h][n][n], one q per class {q, -q}) -> transposed copies
// Wt[h][J][I] = w_h W[h][I][J], w_h = 1/2 where q = -q (hself: device), with
// row pitch ld in c128, two-float-plane, four-bf16-plane and two-bf16-plane
// formats (any output pointer may be null); pad columns are zero.
// The mixed operand copies of the Cholesky factor of W (W^h = L L^H): the
// operand B of Y = R L, Bt[h][j][a] = sqrt(w_h) L^h[a][j] (a >= j, zero
// elsewhere and for a >= n), from lt[h][j][a] = L^h[a][j].
hipError_t lt_convert_launch(const cplx* lt, float* wt32, unsigned short* wt16, unsigned short* wt16s, int n, int ld,
                             int nh, const int* hself, hipStream_t s);
hipError_t wt_convert_launch(const cplx* w, cplx* wt64, float* wt32, unsigned short* wt16, unsigned short* wt16s,
                             int n, int ld, int nh, const int* hself, hipStream_t s);

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
  float2* out32;        // when set, the result goes here as complex FP32 (same offsets), not to out
  const int* qslot;     // mode 0, device, optional: output q goes to block qslot[q] (skipped if < 0)
};
hipError_t kconv_launch(const KconvArgs& a, hipStream_t s);

// Exchange convolution of eq. (10), in place over rho [N_k][n_elem]:
//   rho[k][e] <- scale * N_k * sum_q W^q[e] rho[k+q][e]   (k + q on the mesh),
// W^q[e] = w[wsel[q] >> 1][e], conjugated when wsel[q] & 1 (device table).
struct XconvArgs {
  cplx* rho;
  const cplx* w;
  const int* wsel;
  long long n_elem;
  int m1, m2, m3;
  double scale;
};
hipError_t xconv_launch(const XconvArgs& a, hipStream_t s);

// Polarisabilities of the opposite-spin MP2 energy, in place over gv, go
// [N_k][n_elem]: for every q with qslot[q] >= 0 (device table),
//   gv[qslot[q]][e] <- scale * N_k * sum_k gv[k][e] conj(go[k+q][e])
//   go[qslot[q]][e] <- scale * N_k * sum_k go[k][e] conj(gv[k+q][e])
struct PconvArgs {
  cplx* gv;
  cplx* go;
  long long n_elem;
  int m1, m2, m3;
  double scale;
  const int* qslot;
};
hipError_t pconv_launch(const PconvArgs& a, hipStream_t s);

// Fragment pair transform (eq. (20)):
//   R[Q][pair_off_f + p*nf + q][I] =
//     scale * sum_R exp(-2 pi i jQ.jR/m) conj(psi[R][col_f + p][I]) psi[R][col_f + q][I]
// written in format fmt (0 c128, 1 float planes, 2 bf16 hi/lo planes) with
// rows of pitch ld (>= n_ip, zero padded) and plane stride plane.
struct PairBlock { int frag; int pair0; int npair; };
struct PairArgs {
  const cplx* psi;         // [N_R][ncol][n_ip]
  const float2* psi32;     // register path (required there): psi as complex FP32, same layout
  void* out;               // element (q, pair, I) at qslot[q]*q_stride + pair*p_stride + I (per plane)
  const PairBlock* blocks; // device
  const int* frag_nf; const int* frag_col; const long long* frag_pair;  // device
  int nblocks, n_ip, ncol, tp, ti, n_itiles;
  long long ld, plane, q_stride, p_stride;
  int fmt;
  const int* qslot;        // device: output block of each q (rows q with qslot < 0 are not written)
  // register path (mixed precisions, mesh axes <= 4): one wave per (pair,
  // 64 interpolation points); items ordered (fragment, I chunk, pair),
  // item_off[f] = first item of fragment f (nfrag + 1 entries, device).
  // A fragment's pairs may be a range: pairs frag_p0[f] .. frag_p0[f] +
  // frag_np[f] - 1 (device arrays; null = all nf^2 pairs from 0); the output
  // row of pair P is frag_pair[f] + P in both paths.
  const long long* item_off;
  const int* frag_p0;
  const int* frag_np;
  int nfrag;
  long long nitems;
  int m1, m2, m3;
  double scale;
  // line path: 1 = consecutive workgroups take the two halves (ti points
  // each) of one 2 ti point range, so that two neighbouring workgroups
  // complete each 2 ti x 8-byte line of psi and of the output between them
  int ipair;
};
hipError_t pair_launch(const PairArgs& a, hipStream_t s);

// out[k][I - i0][r] = sum_mu xt[k][mu][I] conj(phi[k][mu][r0 + r]), r < rcur,
// i0 <= I < i0 + icur (the right-hand side's T^k_I(r) on one tile of points
// and grid points); FP64 vector units.  xt must stay readable for RHS_X_PAD
// elements past its end (blocks of points read whole rows; the extra outputs
// are not stored).
constexpr int RHS_X_PAD = 16;
hipError_t rhs_t_launch(const cplx* xt, const cplx* phi, cplx* out, int nk, int norb, int nip, long long ng,
                        long long r0, int rcur, int i0, int icur, hipStream_t s);
// true when pair_launch takes the register path (needs item_off / nitems)
bool pair_reg_supported(int fmt, int m1, int m2, int m3);
// true when pair_launch takes the FP32 LDS path (mixed formats, a mesh axis
// longer than 4): psi32 required, tp * ti * N_k <= 8192
bool pair32_supported(int fmt, int m1, int m2, int m3);
// the line pair transform (mixed formats, 6^3, 8^3 and 10^3 meshes) and the
// largest tile (tp * ti, a power of two) it takes: at most 2048 lines an
// axis pass (two a thread) and 160 KB of LDS
bool pair_lines_supported(int fmt, int m1, int m2, int m3);
constexpr int pair_lines_wmax(int m1, int m2, int m3) {
  int w = 1;
  const int nk = m1 * m2 * m3, mn = m1 < m2 ? (m1 < m3 ? m1 : m3) : (m2 < m3 ? m2 : m3);
  while (w < 16 && nk / mn * w * 2 <= 2048 && m1 * m2 * (m3 * w * 2 + 1) * 8 <= 160 * 1024) w *= 2;
  return w;
}
// LDS bytes of one line pair-transform tile of w values a mesh point
constexpr long long pair_lines_lds(int m1, int m2, int m3, int w) { return (long long)m1 * m2 * (m3 * w + 1) * 8; }

// ---------------------------------------------------------------------------
// Unit-cell grid FFT of f_{q,I}(r) exp(-i q.r) with the Coulomb factor
// sqrt(Omega 4 pi/|G+q|^2)/N_g applied (0 at G+q = 0), in place on
// data[q][I][N_g], q = q0 .. q0+nq-1 (q0 selects the mesh point).
// ---------------------------------------------------------------------------
struct GridFftArgs {
  cplx* data;
  const int* qlist;       // device, optional: item qi is momentum qlist[qi] (else q0 + qi)
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
// qlist: device list of the nq matrices to factor (null = 0..nq-1)
hipError_t chol_launch(const cplx* pi, cplx* work, cplx* lt, int* perm, int* rank,
                       int n, int nq, double rtol, int pivot, hipStream_t s,
                       const int* qlist = nullptr);
// Blocked (unpivoted) Cholesky pieces, batched over nq matrices A[q] (n x n,
// lower triangle used): setup copies Pi into A, records the largest diagonal,
// sets perm = identity, rank = n and clears the breakdown flags; diag factors
// the NB x NB diagonal block at jb in LDS (flagging q when a pivot is not
// above rtol * max diagonal); panel computes L21 = A21 L11^{-H}.  Both also
// store the columns of L transposed into lt.  The trailing update is an NT
// GEMM.
constexpr int CHOL_NB = 64;
hipError_t bchol_setup_launch(const cplx* pi, cplx* a, int* perm, int* rank, double* dmax, int* flag,
                              int n, int nq, hipStream_t s);
hipError_t bchol_diag_launch(cplx* a, cplx* lt, const double* dmax, int* flag, int n, int nq, int jb,
                             double rtol, hipStream_t s);
hipError_t bchol_panel_launch(cplx* a, cplx* lt, const int* flag, int n, int nq, int jb, hipStream_t s);
// Blocked L^{-1} pieces: setup writes the row-major factor lrow (zero outside
// the rank block) and clears yt; diag inverts the 64 x 64 diagonal block at
// jb into yt (transposed) and yd[q] (row-major 64 x 64).  The off-diagonal
// block rows are two NT GEMMs per block row.
hipError_t tri_setup_launch(const cplx* lt, const int* rank, cplx* lrow, cplx* yt, int n, int nq,
                            hipStream_t s);
hipError_t tri_inv_diag_launch(const cplx* lrow, const int* rank, cplx* yt, cplx* yd, int n, int nq, int jb,
                               hipStream_t s);
// dir 0: out[q][i][j] = in[q][perm[i]][perm[j]] (i, j < rank);
// dir 1: out[q][perm[i]][perm[j]] = in[q][i][j], zero outside the rank block.
hipError_t permute_launch(const cplx* in, cplx* out, const int* perm, const int* rank, int n, int nq,
                          int dir, hipStream_t s);

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
// Xt[k][mu][I] = phi[k][mu][ip[I]]
hipError_t gather_launch(const cplx* phi, const int* ip, cplx* xt, int nk, int norb,
                         long long ng, int nip, hipStream_t s);
// out[k][mu][col0 + p] = in[k][mu][p] for a fragment's coefficients (device copy
// into the batch matrix)
// fragment f: in[f] [nk][norb][nf[f]] -> out[k][mu][col[f] + p], one launch
hipError_t copy_cols_batch_launch(const cplx* const* in, cplx* out, int nk, int norb, const int* nf,
                                  const int* col, int n, int maxnf, int ncol, hipStream_t s);
hipError_t copy_cols_launch(const cplx* in, cplx* out, int nk, int norb, int nf,
                            int ncol, int col0, hipStream_t s);
// x[i] = 0 for i < n (complex128)
hipError_t zero_launch(cplx* x, long long n, hipStream_t s);
// count non-finite entries (real or imaginary) of n complex values into *flag
hipError_t nonfinite_launch(const cplx* x, long long n, int* flag, hipStream_t s);

// ---------------------------------------------------------------------------
// interpolation-point selection (pivoted Cholesky of the pair products)
// ---------------------------------------------------------------------------
// Launch shape of one step: xblocks workgroups of 256 grid points, each of
// the nslice row slices rows_per rows long.
struct SelPlan {
  int xblocks = 0;
  int nslice = 0;
  long long rows_per = 0;
};
SelPlan sel_plan(long long nrows, long long ng);
// phi [nrows][ng]; part [nslice][ng]; d [ng]; bv, bi [xblocks]; piv, dmax
// [n_ip].  Start: d = rho^2, piv[0] / dmax[0] = first pivot and its residual.
hipError_t sel_start_launch(const SelPlan& pl, const cplx* phi, long long nrows, long long ng, cplx* part, double* d,
                            double* bv, long long* bi, int* piv, double* dmax, hipStream_t s);
// Step `step`: column lf[step][ng] and residual update; with pick_next the
// pivot of step + 1 into piv / dmax.
hipError_t sel_step_launch(const SelPlan& pl, const cplx* phi, long long nrows, long long ng, cplx* part, double* lf,
                           double* d, double* bv, long long* bi, int* piv, double* dmax, int step, bool pick_next,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// k-point Hartree-Fock Coulomb matrix helpers
// ---------------------------------------------------------------------------
// n[J] = sum_k rho[k][J][J]   (rho [nk][nip][nip])
hipError_t hf_diag_sum_launch(const cplx* rho, int nk, int nip, cplx* n, hipStream_t s);
// v[I] = scale * sum_J W[I][J] n[J], W conjugated when conj
hipError_t hf_matvec_launch(const cplx* w, int conj, const cplx* n, int nip, double scale, cplx* v, hipStream_t s);
// out[r][I] = v[I] xt[r][I] for rows r < rows
hipError_t hf_scale_launch(const cplx* xt, const cplx* v, long long rows, int nip, cplx* out, hipStream_t s);

// ---------------------------------------------------------------------------
// opposite-spin MP2 helpers
// ---------------------------------------------------------------------------
// y [nk][nip][nmo] -> yo [nk][nip][nocc] (x exp(tau (e - mu)/2)) and
// yv [nk][nip][nmo - nocc] (x exp(-tau (e - mu)/2)); e [nk][nmo]
hipError_t mp2_scale_launch(const cplx* y, const double* e, int nk, int nip, int nmo, int nocc, double tau, double mu,
                            cplx* yo, cplx* yv, hipStream_t s);
// part[h][b] = partial sums over nblk chunks of sum_i t1[h][i] conj(t2[h][i])
hipError_t mp2_dot_launch(const cplx* t1, const cplx* t2, long long n_elem, int nclass, int nblk, cplx* part,
                          hipStream_t s);

// ---------------------------------------------------------------------------
// direct RPA helpers
// ---------------------------------------------------------------------------
// out[m][e] -= ph[m] chi[e] + conj(ph[m]) chit[e] for m < nw (ph device)
hipError_t drpa_accum_launch(const cplx* chi, const cplx* chit, long long n_elem, const cplx* ph, int nw, cplx* out,
                             hipStream_t s);
// a[h] <- 1 - a[h] for nmat n x n matrices
hipError_t drpa_one_minus_launch(cplx* a, int n, int nmat, hipStream_t s);
// tr[h] = trace of a[h]
hipError_t drpa_trace_launch(const cplx* a, int n, int nmat, cplx* tr, hipStream_t s);
// part[h][t] (drpa_trace2_tiles(n) per matrix): partial sums of tr(a[h] a[h])
int drpa_trace2_tiles(int n);
hipError_t drpa_trace2_launch(const cplx* a, int n, int nmat, cplx* part, hipStream_t s);
// ld[h] = 2 sum_j ln a[h][j][j] (Cholesky factor in the lower triangle), NaN where flag[h]
hipError_t drpa_logdet_launch(const cplx* a, const int* flag, int n, int nmat, double* ld, hipStream_t s);
