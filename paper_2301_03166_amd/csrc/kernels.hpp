// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/abft.h"

namespace abft {

// C = beta*C + alpha*op(A)*op(B) on FP64 MFMA.  ta/tb: 0 = N, 1 = T.  fa/fb:
// 0 plain, 1 unit-lower mask on the stored operand, 2 absolute values,
// 3 unit-lower mask then absolute values.
// lower: write only C(i,j) with i + doff >= j.  With a scratch buffer `ws`
// (ws_elems doubles) a launch with few output tiles and a long K is split
// along K and reduced in a fixed order.  atype/btype: 0 double,
// 1 float (rounded to bf16 / fp16 when rnd = 1 / 2).
int gemm64(hipStream_t s, int ta, int tb, int fa, int fb, int lower, int m, int n, int k, double alpha, const void* A,
           int64_t lda, const void* B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t doff, int atype = 0,
           int btype = 0, int rnd = 0, double* ws = nullptr, size_t ws_elems = 0, int role = 0,
           int* split_out = nullptr);
// C = beta C + sum of the S split-K partials in P (m x n each, leading dimension m)
int splitk_reduce(hipStream_t s, const double* P, int S, int m, int n, double beta, double* C, int64_t ldc);

// binary32 data GEMM for the mixed-precision trailing update:
// C -= op(A) op(B) with C, A, B float; op in FP32 MFMA (prec ABFT_F32) or
// bf16 / fp16 MFMA with FP32 accumulation (ABFT_BF16 / ABFT_F16).
// FP64 MFMA GEMM for the large plain products (aligned operands); returns 1
// if launched, 0 if the option combination is not covered, <0 on error
int dgemm_fast(hipStream_t s, int ta, int tb, int fa, int fb, int lower, int m, int n, int k, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
               int64_t doff, int S, int kc, double* ws, int role);
int gemm32(hipStream_t s, int prec, int ta, int tb, int lower, int m, int n, int k, float alpha, const float* A,
           int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int64_t doff);

template <typename T>
int verify_tiles(hipStream_t s, const T* A, int64_t lda, int64_t nr, int64_t nc, int nb, int I0, int J0, int sym,
                 int mode, double* colchk, int64_t ldc, double* rowchk, int64_t ldr, const double* gc,
                 const double* gr, double tsu, int* tflags, abft_report* rep, int iter, int level = 2,
                 int64_t frow = -1, int64_t fcol = -1);
template <typename T>
int correct_tiles(hipStream_t s, T* A, int64_t lda, int64_t nr, int64_t nc, int nb, int I0, int J0, int sym,
                  double* colchk, int64_t ldc, double* rowchk, int64_t ldr, const double* gc, const double* gr,
                  double tsu, const int* tflags, abft_report* rep, int iter, int level = 2);
template <typename T>
int xsums(hipStream_t s, const T* A, int64_t lda, int64_t n, int nb, int I0, int64_t xc0, int kw, int dI, int mode,
          double* S, double* Sa, int ldS, int rnd);
template <typename T>
int ysums(hipStream_t s, const T* Y, int64_t ldy, int64_t n, int nb, int J0, int kw, double* Tm, double* Ta, int ldT,
          int rnd);
template <typename MT>
int panel_check(hipStream_t s, const double* S, const double* Sa, int ldS, int I0, int I1, int kw, const MT* Mp,
                int64_t msp, int64_t msj, int tri, int pjoff, double mscale, const double* Mabs, const double* E,
                const double* bt, int Ik, const double* colchk, int64_t ldc, int64_t cj0, int ncols, double tsu_p,
                abft_report* rep, int iter, int nb, int* pflags = nullptr);
int qr_check_prep(hipStream_t s, const double* A, int64_t lda, int64_t c0, int w, int64_t m, const double* T, int ldt,
                  double* scratch, double* Z, double* Zabs, double* E, double* bt);
int inject(hipStream_t s, void* p, int is_float, int bit, abft_report* rep = nullptr);
int report_init(hipStream_t s, abft_report* r, int32_t* info);
int report_fini(hipStream_t s, abft_report* r);

template <typename T>
int potrf_leaf(hipStream_t s, T* A, int64_t lda, int64_t c0, int w, int32_t* info);
template <typename T>
int trsm_rlt_leaf(hipStream_t s, T* A, int64_t lda, int64_t r0, int64_t r1, int64_t c0, int w);
template <typename T>
int trsm_llu_leaf(hipStream_t s, T* A, int64_t lda, int64_t c0, int w, int64_t j0, int64_t j1);
template <typename T>
int trsm_llu_blk(hipStream_t s, T* A, int64_t lda, int64_t c0, int w, int64_t j0, int64_t j1);
// cooperative-leaf exchange area, in 8-byte words (the LU leaf's records are
// cleared at the start of each factorization: their sequence numbers restart)
constexpr size_t SLOT_WORDS = (size_t)3 << 20;
template <typename T>
int getrf_leaf(hipStream_t s, T* A, int64_t lda, int64_t m, int64_t c0, int w, int32_t* ipiv, int32_t* info,
               double* slots, unsigned* ctr, unsigned* ctr_base, abft_report* rep, int maxg);
int geqrf_leaf(hipStream_t s, double* A, int64_t lda, int64_t m, int64_t c0, int w, double* tau, double* Tm, int ldt,
               int toff, double* slots, unsigned* ctr, unsigned* ctr_base, abft_report* rep, int maxg);
int perm_build(hipStream_t s, const int32_t* ipiv, int64_t c0, int w, int64_t n, int* moves);
template <typename T>
int laswp(hipStream_t s, T* A, int64_t lda, int64_t j0, int64_t j1, const int* moves, T* stage, double* colchk,
          int64_t ldc, int nb);

int fill_zero(hipStream_t s, void* p, size_t bytes);

// mixed-precision solve helpers
int convert_f64_f32(hipStream_t s, const double* A, int64_t lda, float* B, int64_t ldb, int64_t m, int64_t n);
int perm_vector(hipStream_t s, const int32_t* ipiv, int n, int* perm);
int gather_scale(hipStream_t s, const double* x, const int* perm, double scale, float* y, int n);
int gather64(hipStream_t s, const double* x, const int* perm, double* y, int n);
// solution words xw: 2n 64-bit words, zero before the first call of a
// sequence; seq > 0 distinct per call
template <typename T>
int trsv(hipStream_t s, const T* F, int64_t ld, int n, int kind, T* x, unsigned* counter, uint64_t* xw,
         uint32_t seq, abft_report* rep);
int residual(hipStream_t s, const double* A, int64_t lda, int n, const double* x, const double* b, double* r,
             double* part, int nsplit, double* norms);
int update_x(hipStream_t s, double* x, const float* d32, double scale, int n, double* norms);
int anorm(hipStream_t s, const double* A, int64_t lda, int n, double* part, int nsplit, double* norms);
int copy_f64(hipStream_t s, const double* a, double* b, int n);

// batched factorizations (one persistent kernel)
size_t batched_ws_bytes(int batch);
int batched_factor(hipStream_t s, int chol, int prec, int batch, const int32_t* dn, void* const* dA,
                   const int32_t* dlda, int32_t* const* dipiv, void* dwork, int protect, double ts,
                   const abft_fault* hfaults, int nfaults, int32_t* dinfo, abft_report* dreps, int wgs);
int f32_to_f64(hipStream_t s, const float* a, double* b, int n);

}  // namespace abft
