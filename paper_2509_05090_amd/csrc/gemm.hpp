// Batched, strided matrix products on CDNA4 matrix cores (MFMA).
//
// Every tensor contraction of the CTMRG step is one of these products after
// a choice of index grouping; see engine.cpp for the mapping of each step.
#pragma once
#include "common.hpp"

namespace ctm {

// Operand of a product: element (r, c) of the logical matrix lives at
// p[r * ld + c] (trans = false) or p[c * ld + r] (trans = true); batch
// (b0, b1) adds b0 * s0 + b1 * s1 elements to p.
struct Operand {
  const void* p;
  int64_t ld;
  bool trans;
  int64_t s0 = 0, s1 = 0;
};

// Output: element (r, c) at p[r * ld + c] + batch offsets, of type t.
struct Output {
  void* p;
  int64_t ld;
  DType t;
  int64_t s0 = 0, s1 = 0;
};

// Device scratch for split-K partial sums (and the norm partials of the
// reduction kernels).
struct Scratch {
  void* p = nullptr;
  size_t bytes = 0;
};

// C = alpha * op(A) op(B) + beta * C for nb0 x nb1 batches.  A and B hold
// elements of type e (F64, F32 or BF16); products accumulate in FP64 for
// e = F64 and in FP32 otherwise.  Split-K (ksplit > 1, only for nb0*nb1 = 1)
// writes partial sums to scratch and reduces them in a fixed order, so
// results are deterministic.  ksplit = 0 picks a split that fills the GPU.
// If sumsq is non-null (unbatched products only) the reduction also writes
// per-block partial sums of squares of the final C there (see
// sumsq_blocks()).
// Optional HIP events recorded right before and after the product kernel
// (not the split-K reduction).
struct KernelEvents {
  hipEvent_t begin = nullptr, end = nullptr;
};

void gemm(hipStream_t s, DType e, int M, int N, int K, const Operand& A, const Operand& B,
          const Output& C, int nb0, int nb1, double alpha, double beta, const Scratch& ws,
          int ksplit = 0, double* sumsq = nullptr, const KernelEvents* ev = nullptr);

// Number of partial sums written to `sumsq` by gemm() for an M x N output.
int sumsq_blocks(int M, int N);

// Bytes of scratch gemm() may need for an unbatched M x N product in
// element type e.
size_t gemm_scratch_bytes(DType e, int M, int N);

}  // namespace ctm
