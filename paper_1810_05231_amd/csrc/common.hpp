// Shared constants and device-side layouts of libproxsdp.
//
// Memory layout (device, carved from the caller's workspace):
//  * W, the matrix the primal step projects (Algorithm 1: X - alpha (C - M*(y))
//    in the dual sign of Section 1.3), is npad x npad row-major, npad = n
//    rounded up to TILE.  Rows/columns >= n are zero.
//  * Subspace blocks (basis B, product Z = W B, Chebyshev iterates) are
//    npad x k row-major with row stride k; rows >= n are zero.
//  * Factors V of X = V diag(lambda) V^T are npad x KMAX (row stride KMAX).
//  * Small matrices (k x k) are row-major with row stride KMAX.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace proxsdp {

typedef double d4 __attribute__((ext_vector_type(4)));   // FP64 MFMA accumulator

constexpr int TILE = 64;      // dense write tile and padding unit
constexpr int KMAX = 64;      // largest subspace width / largest n of the full-eig path
constexpr int SLICE = 64;     // rows per workgroup in the row-wise kernels
constexpr int MAX_R1 = 4;     // largest number of rank-one constraint terms
constexpr int RING = 1024;    // per-iteration record ring

// Offsets (in doubles) inside the `small` device block.
struct SL {
  static constexpr int kk = KMAX * KMAX;
  static constexpr int S = 0;                  // Ritz coefficients, V = B S
  static constexpr int MZ = S + kk;            // next basis Bn = Z MZ + B MB
  static constexpr int MB = MZ + kk;
  static constexpr int THETA = MB + kk;        // Ritz values, decreasing
  static constexpr int RES = THETA + KMAX;     // relative Ritz residuals
  static constexpr int LAM = RES + KMAX;       // 2 x KMAX: lambda_+ by iteration parity
  static constexpr int GG = LAM + 2 * KMAX;    // reduced Grams B^T B, B^T Z, Z^T Z
  static constexpr int TG = GG + kk;
  static constexpr int PG = TG + kk;
  static constexpr int SC = PG + kk;           // named scalars
  static constexpr int FR = SC + 64;           // reduced factor partials (FAC_RES + KMAX values)
  static constexpr int VB = FR + 2 * kk + MAX_R1 * KMAX + KMAX;  // V^T B (KMAX x KMAX) then u_q^T B
  static constexpr int TOTAL = VB + kk + MAX_R1 * KMAX;
};

enum Scalar {
  S_ALPHA = 0,    // step size
  S_GERSH,        // lower bound of lambda_min(W) from the sparse + rank-one part
  S_MAXRES,       // largest relative Ritz residual of the kept pairs (last RR)
  S_LAMR,         // r-th Ritz value
  S_LAMR1,        // (r+1)-th Ritz value (NaN if none)
  S_NORMW,        // max |theta|
  S_EPSP,         // residuals of the last finalised iteration
  S_EPSD,
  S_OBJ,
  S_DOBJ,
  S_DX2,
  S_X2,           // 2 slots by parity: ||X||_F^2
  S_X2B,
  S_NONFINITE,    // 0 ok; 1 Rayleigh-Ritz, 2 full eig, 3 dual step, 4 residuals
  S_CHOLFIX,      // number of regularised Cholesky pivots in the last RR
  S_FILTC,
  S_FILTE,
  S_SWEEPS,       // Jacobi sweeps of the last small eigensolve
  S_RRPATH,       // last Rayleigh-Ritz: Newton steps taken (>= 0) or -1 (Cholesky path)
  S_RRCHOL,       // number of Rayleigh-Ritz calls that took the Cholesky path
  S_RRCOUNT,      // number of Rayleigh-Ritz calls
  S_ITER,         // iterations finalised (ring slot of the next record)
  S_RRWHY1,       // Rayleigh-Ritz calls that left the Newton path because G stayed
  S_RRWHY2,       //   non-orthonormal / kept couplings stayed large / the tail
  S_RRWHY3,       //   bound exceeded the r-th value (counts since create/reset)
  S_RRT0,         // Rayleigh-Ritz seconds (wave 0's clock, summed since create/reset):
  S_RRT1,         //   Newton steps / Cholesky path / diagonalisation and sort /
  S_RRT2,         //   coefficients, residual estimates and next-basis matrices
  S_RRT3,
  S_NPOS,         // leading positive Ritz values among the kept ones (last Rayleigh-Ritz)
  S_FILTX1,       // (theta_1 - c) / e: the largest Ritz value in the filter's scaled variable
  S_RRSTEPS,      // Newton refinement steps of all Rayleigh-Ritz calls since create/reset
  S_RRCAP,        // Rayleigh-Ritz calls whose Newton steps reached the step limit
  S_RRJSW,        // Jacobi sweeps after an accepted Newton path (summed)
  S_COUNT
};

// One record per iteration (written by the finalising workgroup).
struct IterRecord {
  double eps_p, eps_d, obj, dual_obj;
  double lambda_r, lambda_r1, maxres, normw;   // maxres relative to normw = max |theta|
  double npos;                                 // positive kept Ritz values
  double filt_x1;                              // (theta_1 - c) / e of the Chebyshev filter
};

// Device views of the preprocessed problem.
struct DevProblem {
  int n, npad, rows, m, p;
  int n_pat;
  const int* pat_a;       // entry (a, b), a <= b
  const int* pat_b;
  const double* pat_c;    // C on the entry
  const int* pat_rptr;    // entry -> rows CSR
  const int* pat_row;
  const double* pat_val;  // scaled coefficient (matrix value, not doubled)
  const int* row_ptr;     // row -> entries CSR
  const int* row_a;
  const int* row_b;
  const double* row_w;    // scaled coefficient, x2 off the diagonal
  const int* sym_ptr;     // symmetric rows of the pattern (n + 1)
  const int* sym_e;
  // per slot of sym_e: the entry's other index (the row itself on the diagonal),
  // C value, row range [t0, t1) and first row / value (-1 / 0 if none)
  const int* slot_other;
  const int* slot_t0;
  const int* slot_t1;
  const int* slot_row0;
  const double* slot_c;
  const double* slot_val0;
  int tiles_side;         // npad / TILE
  const int* tile_ptr;    // full (mirrored) pattern bucketed by tile
  const int* tile_item;   // (local row << 8) | local col
  const int* tile_e;
  int n_r1;
  int r1_row[MAX_R1];
  double r1_sigma[MAX_R1];  // scaled sigma
  double r1_norm2[MAX_R1];  // ||u||^2
  double r1_gram[MAX_R1 * MAX_R1];  // (u_s^T u_t)^2
  const double* r1_u;     // n_r1 x npad
  const int* row_r1;      // rows: rank-one term index or -1
  const double* rhs;      // [b; h] scaled
  double norm_c;          // ||C||_F, an upper bound of lambda_max(C)
};

// Partial-buffer strides (doubles per slice / per block).
constexpr int FAC_RES = 2 * KMAX * KMAX + MAX_R1 * KMAX;   // Ritz residual norms^2 (k values)
constexpr int FAC_STRIDE = FAC_RES + KMAX;
constexpr int VB_STRIDE = KMAX * KMAX + MAX_R1 * KMAX;  // per-slice partials of V^T B, u^T B
constexpr int ROW_PART = 5;                 // eps_d^2, <dMX, dy>, dual obj, nonfinite, <y, M(X+)>
constexpr int ROW_LANES = 8;                // threads per constraint row in the dual step
constexpr int ROWS_PER_BLOCK = 256 / ROW_LANES;
constexpr int PAT_PART = 4 + MAX_R1;        // min gersh of D, ||M*dy||^2 (sparse), min gersh of M*(y), unused, cross_q

// Number of SLICE-row workgroups covering npad rows.
inline int n_slices(int npad) { return (npad + SLICE - 1) / SLICE; }

}  // namespace proxsdp
