// Low-precision pieces of the inner operator (lowprec.hip): FP32 / BF16 GEMMs
// on the matrix cores with FP32 accumulation, precision conversions, and the
// two packed constraint passes over an FP32 copy of the packed rows.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace wc {

// Storage precision of a low-precision operand.
enum class Lp { F32 = 1, BF16 = 2 };

// Bytes per element of a low-precision operand.
inline int lp_bytes(Lp p) { return p == Lp::F32 ? 4 : 2; }

// How the GEMM result is written: as FP32, as BF16 (round to nearest even), as
// FP64, or added in FP64 to an existing FP64 matrix (C += A B).
enum class LpOut { F32, BF16, F64, ADD_F64 };

// C = A B for column-major A (M x K), B (K x N) stored in precision `in`
// (FP32 or BF16 bit patterns), accumulated in FP32 on the matrix cores.
void lp_gemm_nn(hipStream_t st, Lp in, LpOut out, int M, int N, int K, const void* A, long lda, const void* B,
                long ldb, void* C, long ldc);

// C = A B with A symmetric (M x M), B (M x N), in FP32 or BF16 on the matrix
// cores: A is read by rows, so both operands load k-contiguous.  Returns false
// (nothing launched) unless lda and ldb are multiples of the elements in 16
// bytes, A, B are 16-byte aligned and the product has at least 64 tiles of
// 128 x 128; the caller then uses lp_gemm_nn.
bool lp_gemm_sym(hipStream_t st, Lp in, LpOut out, int M, int N, const void* A, long lda, const void* B, long ldb,
                 void* C, long ldc);

// Entry sampling: Y = A^T(u) scattered into a zeroed low-precision n x n
// matrix (each entry rounded as to_lowp rounds it); `count` elements of a
// low-precision buffer (16-byte aligned) set to zero; out_i = alpha (M_jk +
// M_kj) / 2 + beta out_i read from an FP32 matrix at the m sampled pairs.
void entry_scatter_lp(hipStream_t st, Lp p, int m, const int* jk, const double* u, void* Y, long ldy);
void zero_lowp(hipStream_t st, Lp p, long count, void* X);
void entry_gather_f32(hipStream_t st, int m, const int* jk, const float* M, long ldm, double* out, double alpha,
                      double beta);

// B = A rounded to precision p (column-major, rows x cols).
void to_lowp(hipStream_t st, Lp p, int rows, int cols, const double* A, long lda, void* B, long ldb);
// y = x rounded to FP32 (count elements).
void to_f32(hipStream_t st, long count, const double* x, float* y);

// Packed constraint passes over FP32 rows P (m x ldp row-major, ldp a multiple
// of 4, zero padded), accumulated in FP64:
//   packed_rows_f32: y = alpha P x + beta y with x FP32, readable and zero
//     padded up to round_up(k, 4);
//   packed_cols_partial_f32: packed_cols_parts_f32(m) slab partial sums of
//     P^T x into `part` with row pitch round_up(k, 4).
int packed_cols_parts_f32(int m);
void packed_rows_f32(hipStream_t st, int m, int k, const float* P, long ldp, const float* x, double* y,
                     double alpha, double beta);
void packed_cols_partial_f32(hipStream_t st, int m, int k, const float* P, long ldp, const double* x, double* part);

// Packed weights of a symmetric M in FP32 (mw[p] = M_jj, or M_jk + M_kj off
// the diagonal), zero padded to ldp.
void pack_weighted_f32(hipStream_t st, long N2, long ldp, const double* M, long ldm, const int* pj, const int* pk,
                       float* mw);

// Y = sum over slabs of the partial column sums, unpacked to a full symmetric
// FP64 matrix (skipped when Y is null), plus the same matrix rounded to
// precision p in Ylp.
void at_reduce_unpack_lp(hipStream_t st, Lp p, long N2, int nparts, const double* part, long pstride, const int* pj,
                         const int* pk, double* Y, long ldy, void* Ylp);

}  // namespace wc
