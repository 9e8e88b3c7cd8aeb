// CTMRG engine and C interface (see include/ctm.h).
//
// One step of the C3v-symmetric CTMRG on the honeycomb lattice (Sec. II.B,
// Fig. 3), as a schedule of MFMA matrix products.  Indices: chi_c = current
// corner dimension, D2 = D^2, n = chi_c * D2.
//
//   1. TCp[beta][gamma][j]  = sum_delta C[gamma][delta] T[beta][j][delta]
//        chi_c products of (chi_c x D2), k = chi_c: corner onto the column edge
//   2. V[(alpha,m)][(gamma,j)] = sum_i T[alpha][i][gamma] a[m][i][j]
//        chi_c*D2 products of (chi_c x D2), k = D2: outer site of the pair on
//        the row edge (the double layer is symmetric in its legs)
//   3. W[(alpha,m)][beta]   = V . TCp^T               (n x chi_c, k = n)
//   4. Ct[(alpha,k)][(beta,l)] = sum_m W[(alpha,m)][beta] a[m][k][l]
//        chi_c*D2 products (chi_c x D2), k = D2: inner site; Ct is the n x n
//        enlarged corner, symmetric
//   5. projector Q (n x chi): identity while n <= chi; else the thin QR of
//        the reduced corner M = Ct . P_prev (n x chi, k = n), FP64 blocked
//        Householder, Q1; its basis is tied to P_prev: Q = Q1 gs(Q1^T P_prev)
//        with gs the Gram-Schmidt basis (QR with positive diagonal of the
//        chi x chi overlap); P_prev <- Q
//   6. Gm = Ct . Q                                    (n x chi, k = n)
//   7. C' = Q^T . Gm, then (C' + C'^T)/2 / ||.||_F     (chi x chi, k = n)
//   8. V2 = V . Q                                     (n x chi, k = n)
//   9. V3[alpha][(k,l)][nu] = sum_m a[k][l][m] V2[(alpha,m)][nu], stored
//        transposed as [(l,nu)][(alpha,k)] (chi_c D2 batches of chi x D2,
//        k = D2)
//  10. T' = Q^T . V3 (V3 read as n x (D2 chi), from its transposed store),
//        then / ||.||_F
//
// Steps 1-4 and 6-10 run in the context's arithmetic (FP64, or FP32/BF16
// matrix cores with FP32 accumulation); the QR, sign gauge and norms are
// FP64, as are the master copies of C, T and P_prev.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctm.h"
#include "chol.hpp"
#include "gemm.hpp"
#include "kernels.hpp"
#include "qr.hpp"
#include "spectrum.hpp"
#include "context.hpp"

using namespace ctm;

namespace {

thread_local std::string g_error;

}  // namespace

namespace ctm {
void set_global_error(const std::string& s) { g_error = s; }
}  // namespace ctm

namespace {

template <typename F>
int guarded(ctm_ctx* c, F&& f) {
  if (!c) {
    g_error = "null context";
    return CTM_EINVAL;
  }
  if (c->poisoned) {
    c->err = "context unusable after a device error: " + c->err;
    return CTM_EDEVICE;
  }
  try {
    return f();
  } catch (const DeviceError& e) {
    c->poisoned = true;
    c->err = e.what();
    return CTM_EDEVICE;
  } catch (const OutOfMemory& e) {
    c->err = e.what();
    return CTM_ENOMEM;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return CTM_ENOMEM;
  } catch (const std::exception& e) {
    c->err = e.what();
    return CTM_EINVAL;
  }
}

DType to_dtype(int prec) {
  if (prec == CTM_PREC_LADDER) return DType::BF16;  // the ladder starts on BF16
  return prec == CTM_PREC_FP32 ? DType::F32 : (prec == CTM_PREC_BF16 ? DType::BF16 : DType::F64);
}

// View of FP64 data in arithmetic e: the FP64 buffer itself for e = F64,
// else a converted copy in `scratch`.
bool read_flag(ctm_ctx* c) {
  int f = 0;
  CTM_HIP(hipMemcpyAsync(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  CTM_HIP(hipStreamSynchronize(c->stream));
  return f != 0;
}

void stage_begin(ctm_ctx* c, int stage) {
  if (!c->prof_active) return;
  c->stage_open[stage] = c->next_event();
  CTM_HIP(hipEventRecord(c->stage_open[stage], c->stream));
}

void stage_end(ctm_ctx* c, int stage) {
  if (!c->prof_active) return;
  hipEvent_t e = c->next_event();
  CTM_HIP(hipEventRecord(e, c->stream));
  c->intervals.push_back({stage, c->stage_open[stage], e});
}

// Events around one of the big (n x chi x n) matrix-core kernels, or null.
const KernelEvents* big_gemm_events(ctm_ctx* c, KernelEvents& ev, double M, double N, double K) {
  if (!c->prof_active) return nullptr;
  ev.begin = c->next_event();
  ev.end = c->next_event();
  c->intervals.push_back({CTM_STAGE_BIG_GEMM, ev.begin, ev.end});
  c->big_flops += 2.0 * M * N * K;
  return &ev;
}

std::vector<double> current_spectrum(ctm_ctx* c) {
  std::vector<double> h((size_t)c->chi_c * c->chi_c);
  CTM_HIP(hipMemcpyAsync(h.data(), c->C, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  CTM_HIP(hipStreamSynchronize(c->stream));
  return normalized_spectrum(h, c->chi_c);
}

// P_prev <- Gram-Schmidt basis of the first n rows of G (unique: diag(R) > 0),
// written to `dst` (n x chi).
void start_projector(ctm_ctx* c, int n, double* dst) {
  hipStream_t s = c->stream;
  const int chi = c->chi;
  CTM_HIP(hipMemcpyAsync(c->M, c->G, (size_t)n * chi * sizeof(double), hipMemcpyDeviceToDevice, s));
  householder_qr(s, c->M, chi, n, chi, c->qr);
  householder_form_q(s, c->qr, n, chi, dst, chi);
  launch_diag_signs(s, c->M, chi, chi, c->sgn);
  launch_apply_signs(s, dst, n, chi, c->sgn, nullptr);
}

// Enlarged corner of the current state into c->Ct (steps 1-4), arithmetic e.
// Leaves TCp, V, W valid.
void enlarged_corner(ctm_ctx* c, DType e) {
  hipStream_t s = c->stream;
  const int x = c->chi_c, D2 = c->D2;
  const int64_t n = (int64_t)x * D2;
  const void *CE, *TE, *aE;
  if (e == DType::F64) {
    CE = c->C;
    TE = c->T;
    aE = c->a;
  } else {
    launch_cast(s, c->C, c->CE, e, (int64_t)x * x);
    launch_cast(s, c->T, c->TE, e, (int64_t)x * D2 * x);
    CE = c->CE;
    TE = c->TE;
    aE = c->aE;
    if (c->aE_type != (int)e) {  // a changes only with the site tensor
      launch_cast(s, c->a, c->aE, e, (int64_t)D2 * D2 * D2);
      c->aE_type = (int)e;
    }
  }
  // 1. TCp[beta][gamma][j]
  gemm(s, e, x, D2, x, Operand{CE, x, false}, Operand{TE, x, true, (int64_t)D2 * x},
       Output{c->TCp, D2, e, (int64_t)x * D2}, x, 1, 1.0, 0.0, c->ws);
  // 2. V[(alpha,m)][(gamma,j)]
  gemm(s, e, x, D2, D2, Operand{TE, x, true, (int64_t)D2 * x, 0},
       Operand{aE, D2, false, 0, (int64_t)D2 * D2}, Output{c->V, D2, e, D2 * n, n}, x, D2, 1.0,
       0.0, c->ws);
  // 3. W = V TCp^T
  gemm(s, e, (int)n, x, (int)n, Operand{c->V, n, false}, Operand{c->TCp, n, true},
       Output{c->W, x, e}, 1, 1, 1.0, 0.0, c->ws);
  // 4. Ct[(alpha,k)][(beta,l)]
  gemm(s, e, x, D2, D2, Operand{c->W, x, true, (int64_t)D2 * x, 0},
       Operand{aE, (int64_t)D2 * D2, false, 0, D2}, Output{c->Ct, D2, e, D2 * n, n}, x, D2, 1.0,
       0.0, c->ws);
}

// Gram-Schmidt basis of the columns of the k x k matrix X (leading
// dimension ld; QR with a positive diagonal of R), into Qx (ld k).  X is
// overwritten.  Uses the second QR workspace.
void gram_schmidt_small(ctm_ctx* c, double* X, int ld, int k, double* Qx,
                        hipStream_t s = nullptr) {
  if (!s) s = c->stream;
  householder_qr(s, X, ld, k, k, c->qr2);
  householder_form_q(s, c->qr2, k, k, Qx, k);
  launch_diag_signs(s, X, ld, k, c->sgn);
  launch_apply_signs(s, Qx, k, k, c->sgn, nullptr);
}

// Projector of the QR rule for the current Ct (FP64, n x chi, ld chi): thin
// QR of M = Ct P_prev, basis tied to P_prev (or to the start projector when
// P_prev does not match n).  Written into c->P (the new P_prev) if update,
// else into c->Q; returns where.
//
// M and P_prev sit side by side in c->MP (n x 2 chi) and P_prev is carried
// through the factorization's trailing updates, which leaves X = Q1^T P_prev
// in the top chi rows of the carried block.  X no longer waits for Q1:
// the explicit Q1 is formed on the second stream while X is factored on
// this one, and the two meet before Q = Q1 gs(X).
const double* qr_projector(ctm_ctx* c, DType e, bool update) {
  hipStream_t s = c->stream;
  const int chi = c->chi;
  const int n = c->chi_c * c->D2;
  double* Pref = c->P;
  if (c->p_rows != n) {
    if (update) {
      start_projector(c, n, c->P);
      c->p_rows = n;
    } else {
      Pref = (double*)c->PE;  // 8-byte scratch of n x chi (the energy runs in FP64)
      start_projector(c, n, Pref);
    }
  }
  // P_prev^T in the product's arithmetic (into W, which is free between the
  // enlarged corner and the next step): both operands of the product below
  // are then contiguous along its summed index.
  launch_cast_transpose(s, Pref, c->W, e, n, chi);
  // 5. [M | P_prev], M = Ct P_prev (FP64 result); thin QR of M with P_prev
  //    carried
  const int ldmp = 2 * chi;
  double* X = c->MP + chi;
  KernelEvents ev;
  gemm(s, e, n, chi, n, Operand{c->Ct, n, false}, Operand{c->W, n, true},
       Output{c->MP, ldmp, DType::F64}, 1, 1, 1.0, 0.0, c->ws, 0, nullptr,
       big_gemm_events(c, ev, n, chi, n));
  launch_copy_block(s, Pref, chi, X, ldmp, n, chi);
  householder_qr(s, c->MP, ldmp, n, chi, c->qr, ldmp);
  // Q1 into M on the second stream
  CTM_HIP(hipEventRecord(c->ev_fork, s));
  CTM_HIP(hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
  householder_form_q(c->stream2, c->qr, n, chi, c->M, chi);
  CTM_HIP(hipEventRecord(c->ev_join, c->stream2));
  // basis: Q = Q1 gs(X), X = Q1^T P_prev
  gram_schmidt_small(c, X, ldmp, chi, c->Xq);
  CTM_HIP(hipStreamWaitEvent(s, c->ev_join, 0));
  // P_prev has been read by now (into MP and W), so with update the new
  // projector goes straight into its place
  double* Qout = update ? c->P : c->Q;
  gemm(s, DType::F64, n, chi, chi, Operand{c->M, chi, false}, Operand{c->Xq, chi, false},
       Output{Qout, chi, DType::F64}, 1, 1, 1.0, 0.0, c->ws, 1);
  return Qout;
}

// One Cholesky QR pass: Out = In R^{-1} with R^T R = In^T In (n x chi, ld
// chi, FP64); the factorization shifts a numerically singular Gram matrix.
void chol_pass(ctm_ctx* c, const double* In, double* Out, int n, int chi) {
  hipStream_t s = c->stream;
  gemm(s, DType::F64, chi, chi, n, Operand{In, chi, true}, Operand{In, chi, false},
       Output{c->cg, chi, DType::F64}, 1, 1, 1.0, 0.0, c->ws);
  launch_cholesky(s, c->cg, chi, chi, n, nullptr, 0, c->cri, chi, c->chol_status, c->flag);
  gemm(s, DType::F64, n, chi, chi, Operand{In, chi, false}, Operand{c->cri, chi, false},
       Output{Out, chi, DType::F64}, 1, 1, 1.0, 0.0, c->ws, 1);
}

// The QR projector with Q1 from Cholesky QR instead of Householder: three
// passes (the first shifted if M^T M is numerically singular) give an
// orthonormal basis of span(M) to working precision for cond(M) below about
// 1/u.  The isometry Q = Q1 gs(Q1^T P_prev) depends on Q1 only through
// span(Q1) = span(M), so it is the same as with the Householder Q1 up to
// rounding.  gs(X) stays a Householder QR: for the chi x chi matrix X that
// is cheaper than three more Cholesky passes.
const double* chol_projector(ctm_ctx* c, DType e, bool update) {
  hipStream_t s = c->stream;
  const int chi = c->chi;
  const int n = c->chi_c * c->D2;
  double* Pref = c->P;
  if (c->p_rows != n) {
    if (update) {
      start_projector(c, n, c->P);
      c->p_rows = n;
    } else {
      Pref = (double*)c->PE;
      start_projector(c, n, Pref);
    }
  }
  launch_cast_transpose(s, Pref, c->W, e, n, chi);
  // 5. M = Ct P_prev (FP64 result), then Q1 by three Cholesky QR passes
  double* M0 = c->MP;
  double* M1 = c->MP + (int64_t)n * chi;
  KernelEvents ev;
  gemm(s, e, n, chi, n, Operand{c->Ct, n, false}, Operand{c->W, n, true},
       Output{M0, chi, DType::F64}, 1, 1, 1.0, 0.0, c->ws, 0, nullptr,
       big_gemm_events(c, ev, n, chi, n));
  chol_pass(c, M0, M1, n, chi);
  chol_pass(c, M1, M0, n, chi);
  chol_pass(c, M0, c->M, n, chi);
  // basis: Q = Q1 gs(X), X = Q1^T P_prev
  gemm(s, DType::F64, chi, chi, n, Operand{c->M, chi, true}, Operand{Pref, chi, false},
       Output{c->cx, chi, DType::F64}, 1, 1, 1.0, 0.0, c->ws);
  if (update && c->overlap && e != DType::BF16) {
    // G1 = Ct Q1 and W1 = V Q1 on the products' CUs while gs(X) runs on the
    // reserved ones; the renormalization finishes Gm = G1 Qx and V2 = W1 Qx
    CTM_HIP(hipEventRecord(c->ev_fork, s));
    CTM_HIP(hipStreamWaitEvent(c->stream_big, c->ev_fork, 0));
    CTM_HIP(hipStreamWaitEvent(c->stream_small, c->ev_fork, 0));
    hipStream_t sb = c->stream_big;
    launch_cast_transpose(sb, c->M, c->W, e, n, chi);
    KernelEvents ev1, ev2;
    gemm(sb, e, n, chi, n, Operand{c->Ct, n, false}, Operand{c->W, n, true},
         Output{c->G1, chi, e}, 1, 1, 1.0, 0.0, c->ws_big, 0, nullptr,
         big_gemm_events(c, ev1, n, chi, n));
    gemm(sb, e, n, chi, n, Operand{c->V, n, false}, Operand{c->W, n, true},
         Output{c->W1, chi, e}, 1, 1, 1.0, 0.0, c->ws_big, 0, nullptr,
         big_gemm_events(c, ev2, n, chi, n));
    CTM_HIP(hipEventRecord(c->ev_big, sb));
    gram_schmidt_small(c, c->cx, chi, chi, c->Xq, c->stream_small);
    CTM_HIP(hipEventRecord(c->ev_small, c->stream_small));
    CTM_HIP(hipStreamWaitEvent(s, c->ev_small, 0));
    c->pre_q1 = true;
  } else {
    gram_schmidt_small(c, c->cx, chi, chi, c->Xq);
  }
  double* Qout = update ? c->P : c->Q;
  gemm(s, DType::F64, n, chi, chi, Operand{c->M, chi, false}, Operand{c->Xq, chi, false},
       Output{Qout, chi, DType::F64}, 1, 1, 1.0, 0.0, c->ws, 1);
  return Qout;
}

// Projector of the eigendecomposition rule (Fig. 3c) into c->Q: the chi
// eigenvectors of Ct of largest |eigenvalue|, column signs following P_prev
// when it matches n (else largest entry positive).  If update, P_prev <- Q.
void evd_projector(ctm_ctx* c, DType e, bool update) {
  const int chi = c->chi;
  const int n = c->chi_c * c->D2;
  const double* Pref = c->p_rows == n ? c->P : nullptr;
  std::vector<double> lam;
  eigh_top(c->stream, c->Ct, e, n, chi, c->evd, c->ws, c->Q, chi, Pref, lam);
  if (update) {
    CTM_HIP(hipMemcpyAsync(c->P, c->Q, (size_t)n * chi * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
    c->p_rows = n;
  }
}

// Projector for the current Ct; returns where it is (c->Q, or c->P for the
// QR rule with update).
const double* projector(ctm_ctx* c, DType e, bool update) {
  if (c->cfg.proj == CTM_PROJ_EVD) {
    evd_projector(c, e, update);
    return c->Q;
  }
  if (c->cfg.proj == CTM_PROJ_QR_CHOL) return chol_projector(c, e, update);
  return qr_projector(c, e, update);
}

void step_once(ctm_ctx* c) {
  hipStream_t s = c->stream;
  const DType e = c->prec;
  const int x = c->chi_c, D2 = c->D2, chi = c->chi;
  const int64_t n = (int64_t)x * D2;
  c->prof_active = c->prof_on;
  stage_begin(c, CTM_STAGE_CORNER);
  enlarged_corner(c, e);
  stage_end(c, CTM_STAGE_CORNER);
  stage_begin(c, CTM_STAGE_PROJECTOR);
  int xn;
  const double* Qp = c->Q;
  if (n <= chi) {
    xn = (int)n;
    launch_eye(s, c->Q, DType::F64, (int)n, (int)n, n);
  } else {
    xn = chi;
    Qp = projector(c, e, true);
  }
  stage_end(c, CTM_STAGE_PROJECTOR);
  stage_begin(c, CTM_STAGE_RENORM_C);
  // Q^T in the products' arithmetic (xn x n), contiguous along n for all four
  // products that use it
  void* QT = c->QE;
  launch_cast_transpose(s, Qp, QT, e, (int)n, xn);
  KernelEvents ev1, ev2;
  const bool pre = c->pre_q1;  // Gm = (Ct Q1) Qx and V2 = (V Q1) Qx
  c->pre_q1 = false;
  const void* QxE = c->Xq;
  if (pre) {
    CTM_HIP(hipStreamWaitEvent(s, c->ev_big, 0));
    if (e != DType::F64) {
      launch_cast(s, c->Xq, c->cg, e, (int64_t)xn * xn);
      QxE = c->cg;
    }
  }
  // 6. Gm = Ct Q
  if (pre)
    gemm(s, e, (int)n, xn, xn, Operand{c->G1, xn, false}, Operand{QxE, xn, false},
         Output{c->Gm, xn, e}, 1, 1, 1.0, 0.0, c->ws, 1);
  else
    gemm(s, e, (int)n, xn, (int)n, Operand{c->Ct, n, false}, Operand{QT, n, true},
         Output{c->Gm, xn, e}, 1, 1, 1.0, 0.0, c->ws, 0, nullptr,
         big_gemm_events(c, ev1, n, xn, n));
  // 7. C' = Q^T Gm, symmetrized and normalized
  gemm(s, e, xn, xn, (int)n, Operand{QT, n, false}, Operand{c->Gm, xn, false},
       Output{c->Cp, xn, DType::F64}, 1, 1, 1.0, 0.0, c->ws);
  launch_corner_finalize(s, c->Cp, c->Cn, xn, c->sumsq, c->flag);
  stage_end(c, CTM_STAGE_RENORM_C);
  stage_begin(c, CTM_STAGE_RENORM_T);
  // 8. V2 = V Q
  if (pre)
    gemm(s, e, (int)n, xn, xn, Operand{c->W1, xn, false}, Operand{QxE, xn, false},
         Output{c->V2, xn, e}, 1, 1, 1.0, 0.0, c->ws, 1);
  else
    gemm(s, e, (int)n, xn, (int)n, Operand{c->V, n, false}, Operand{QT, n, true},
         Output{c->V2, xn, e}, 1, 1, 1.0, 0.0, c->ws, 0, nullptr,
         big_gemm_events(c, ev2, n, xn, n));
  // 9. V3 stored transposed, V3t[(l,nu)][(alpha,k)] = sum_m a[k][l][m] V2[(alpha,m)][nu],
  //    into the Ct buffer (Ct is no longer needed): batches (alpha, l) of
  //    xn x D2 x D2 products, A[alpha](nu, m) = V2[alpha][m][nu],
  //    B[l](m, k) = a[k][l][m]
  const void* aE = e == DType::F64 ? (const void*)c->a : c->aE;
  void* V3t = c->Ct;
  gemm(s, e, xn, D2, D2, Operand{c->V2, xn, true, (int64_t)D2 * xn, 0},
       Operand{aE, (int64_t)D2 * D2, true, 0, D2}, Output{V3t, n, e, D2, (int64_t)xn * n}, x, D2,
       1.0, 0.0, c->ws);
  // 10. T'[mu][(l,nu)] = sum_(alpha,k) Q[(alpha,k)][mu] V3t[(l,nu)][(alpha,k)], normalized
  const int64_t tn = (int64_t)xn * D2 * xn;
  gemm(s, e, xn, D2 * xn, (int)n, Operand{QT, n, false}, Operand{V3t, n, true},
       Output{c->Tp, (int64_t)D2 * xn, DType::F64}, 1, 1, 1.0, 0.0, c->ws, 0, c->sumsq);
  launch_scale_by_norm(s, c->Tp, c->Tn, tn, c->sumsq, sumsq_blocks(xn, D2 * xn), c->flag);
  stage_end(c, CTM_STAGE_RENORM_T);
  c->prof_active = false;
  std::swap(c->C, c->Cn);
  std::swap(c->T, c->Tn);
  c->chi_c = xn;
  c->steps += 1;
}

int do_steps(ctm_ctx* c, int n_steps, double* delta) {
  if (n_steps < 0) throw std::invalid_argument("n_steps < 0");
  int pend_x = 0;  // corner dimension of a pending copy taken before the last step
  for (int i = 0; i < n_steps; ++i) {
    if (delta && i == n_steps - 1 && c->spec_step != c->steps) {
      // the corner before the last step goes to pinned host memory without a
      // stream synchronization; its spectrum is computed while the GPU runs
      // the last step
      pend_x = c->chi_c;
      CTM_HIP(hipMemcpyAsync(c->hostC, c->C, (size_t)pend_x * pend_x * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
      CTM_HIP(hipEventRecord(c->ev_spec, c->stream));
    }
    step_once(c);
  }
  if (pend_x > 0) {
    CTM_HIP(hipEventSynchronize(c->ev_spec));
    c->spec = normalized_spectrum(
        std::vector<double>(c->hostC, c->hostC + (size_t)pend_x * pend_x), pend_x);
    c->spec_step = c->steps - 1;
  }
  if (delta) {
    if (n_steps == 0 || c->spec_step != c->steps - 1) {
      *delta = std::numeric_limits<double>::infinity();
      if (n_steps > 0) {
        c->spec = current_spectrum(c);
        c->spec_step = c->steps;
      }
    } else {
      std::vector<double> sn = current_spectrum(c);
      *delta = spectrum_change(sn, c->spec);
      c->spec = std::move(sn);
      c->spec_step = c->steps;
    }
    if (read_flag(c)) {
      c->err = "non-finite or zero norm in C or T";
      return CTM_ENONFINITE;
    }
  }
  return CTM_OK;
}

}  // namespace

void ctm::ensure_energy_buffers(ctm_ctx* c) {
  if (c->XO) return;
  const int64_t x2 = (int64_t)c->chi * c->chi;
  const int64_t dd = (int64_t)c->d * c->d;
  c->XO = c->allocd(x2 * c->D2 * dd);
  c->EO = c->allocd(x2 * c->D2 * dd);
  c->aO = c->allocd((int64_t)c->D2 * c->D2 * c->D2 * dd);
  c->aOr = c->allocd((int64_t)c->D2 * c->D2 * c->D2 * dd);
  c->Cr2 = c->allocd(x2);
  c->Cr4 = c->allocd(x2);
  c->Cr5 = c->allocd(x2);
  c->rho_raw = c->allocd(dd * dd);
  c->h_dev = c->allocd(dd * dd);
  c->e_out = c->allocd(1 + dd * dd);
  launch_double_layer_open(c->stream, c->A, c->d, c->D, 0, c->aO);
  launch_double_layer_open(c->stream, c->A, c->d, c->D, 1, c->aOr);
}

namespace {

// Bond density matrix of the apex pair on the six-corner ring (FP64).
int do_energy(ctm_ctx* c, const double* h_host, double* e_host, double* rho_host) {
  hipStream_t s = c->stream;
  ensure_energy_buffers(c);
  const DType f = DType::F64;
  const int x = c->chi_c, D2 = c->D2, chi = c->chi, d = c->d;
  const int dd = d * d;
  const int64_t n = (int64_t)x * D2;
  CTM_HIP(hipMemcpyAsync(c->h_dev, h_host, (size_t)dd * dd * sizeof(double), hipMemcpyHostToDevice, s));
  enlarged_corner(c, f);
  int xm;
  if (n <= chi) {
    xm = (int)n;
    launch_eye(s, c->Q, f, (int)n, (int)n, n);
  } else {
    xm = chi;
    projector(c, f, false);
  }
  double* Ct = (double*)c->Ct;
  double* Gm = (double*)c->Gm;
  // Cr = Q^T Ct Q, scaled; its fifth power
  gemm(s, f, (int)n, xm, (int)n, Operand{Ct, n, false}, Operand{c->Q, xm, false}, Output{Gm, xm, f},
       1, 1, 1.0, 0.0, c->ws);
  gemm(s, f, xm, xm, (int)n, Operand{c->Q, xm, true}, Operand{Gm, xm, false}, Output{c->Cp, xm, f},
       1, 1, 1.0, 0.0, c->ws);
  launch_scale_by_maxabs(s, c->Cp, xm);
  gemm(s, f, xm, xm, xm, Operand{c->Cp, xm, false}, Operand{c->Cp, xm, false},
       Output{c->Cr2, xm, f}, 1, 1, 1.0, 0.0, c->ws);
  gemm(s, f, xm, xm, xm, Operand{c->Cr2, xm, false}, Operand{c->Cr2, xm, false},
       Output{c->Cr4, xm, f}, 1, 1, 1.0, 0.0, c->ws);
  gemm(s, f, xm, xm, xm, Operand{c->Cr4, xm, false}, Operand{c->Cp, xm, false},
       Output{c->Cr5, xm, f}, 1, 1, 1.0, 0.0, c->ws);
  // QC5 = Q Cr^5 (into W)
  double* QC5 = (double*)c->W;
  gemm(s, f, (int)n, xm, xm, Operand{c->Q, xm, false}, Operand{c->Cr5, xm, false},
       Output{QC5, xm, f}, 1, 1, 1.0, 0.0, c->ws);
  // EnvP[alpha][beta][K][L] = Env[(beta,L),(alpha,K)] = sum_nu Q[(alpha,K)][nu] QC5[(beta,L)][nu]
  double* EnvP = (double*)c->V;
  gemm(s, f, D2, D2, xm, Operand{c->Q, xm, false, (int64_t)D2 * xm, 0},
       Operand{QC5, xm, true, 0, (int64_t)D2 * xm},
       Output{EnvP, D2, f, (int64_t)x * D2 * D2, (int64_t)D2 * D2}, x, x, 1.0, 0.0, c->ws);
  // TCTp[alpha][beta][I][J] = sum_gamma T[alpha][I][gamma] TCp[beta][gamma][J]  (into Ct)
  double* TCTp = Ct;
  gemm(s, f, D2, D2, x, Operand{c->T, x, false, (int64_t)D2 * x, 0},
       Operand{c->TCp, D2, false, 0, (int64_t)x * D2},
       Output{TCTp, D2, f, (int64_t)x * D2 * D2, (int64_t)D2 * D2}, x, x, 1.0, 0.0, c->ws);
  // outer site open: XO[(alpha,beta)][(M,s,s')]; inner site open with the ring: EO
  const int64_t x2 = (int64_t)x * x;
  gemm(s, f, (int)x2, D2 * dd, D2 * D2, Operand{TCTp, (int64_t)D2 * D2, false},
       Operand{c->aO, (int64_t)D2 * dd, false}, Output{c->XO, (int64_t)D2 * dd, f}, 1, 1, 1.0, 0.0,
       c->ws);
  gemm(s, f, (int)x2, D2 * dd, D2 * D2, Operand{EnvP, (int64_t)D2 * D2, false},
       Operand{c->aOr, (int64_t)D2 * dd, false}, Output{c->EO, (int64_t)D2 * dd, f}, 1, 1, 1.0,
       0.0, c->ws);
  // R[(s,s')][(t,t')] = sum_{(alpha,beta,M)} XO[..][(s,s')] EO[..][(t,t')]
  gemm(s, f, dd, dd, (int)(x2 * D2), Operand{c->XO, dd, true}, Operand{c->EO, dd, false},
       Output{c->rho_raw, dd, f}, 1, 1, 1.0, 0.0, c->ws);
  launch_energy_finalize(s, c->rho_raw, c->h_dev, d, c->e_out, c->flag);
  std::vector<double> out(1 + (size_t)dd * dd);
  CTM_HIP(hipMemcpyAsync(out.data(), c->e_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CTM_HIP(hipStreamSynchronize(s));
  if (read_flag(c)) {
    c->err = "non-finite or zero norm in C, T or the density matrix";
    return CTM_ENONFINITE;
  }
  if (e_host) *e_host = out[0];
  if (rho_host) std::memcpy(rho_host, out.data() + 1, (size_t)dd * dd * sizeof(double));
  return CTM_OK;
}

bool valid_cfg(const ctm_config* cfg, std::string& why) {
  if (!cfg) return why = "null config", false;
  if (cfg->d < 1 || cfg->D < 1 || cfg->chi < 1) return why = "d, D and chi must be >= 1", false;
  if ((int64_t)cfg->d * cfg->D * cfg->D * cfg->D > 16384) return why = "d*D^3 > 16384", false;
  if ((int64_t)cfg->chi * cfg->D * cfg->D > QR_MAX_ROWS) return why = "chi*D^2 > 32768", false;
  if (cfg->proj != CTM_PROJ_QR && cfg->proj != CTM_PROJ_EVD && cfg->proj != CTM_PROJ_QR_CHOL)
    return why = "bad projector", false;
  if (cfg->proj == CTM_PROJ_QR_CHOL && cfg->chi > CHOL_KMAX)
    return why = "the Cholesky QR projector needs chi <= " + std::to_string(CHOL_KMAX), false;
  if (cfg->proj == CTM_PROJ_EVD && (int64_t)cfg->chi * cfg->D * cfg->D > 8192)
    return why = "the eigendecomposition projector needs chi*D^2 <= 8192", false;
  if (cfg->prec < CTM_PREC_FP64 || cfg->prec > CTM_PREC_LADDER) return why = "bad precision", false;
  return true;
}

// The pair of CU-masked streams of the current device (16 CUs for the basis
// factorization, the others for the products), created on first use and
// kept for the life of the process: every context on the device shares
// them, since the runtime gives each masked stream hardware queue resources
// of its own and creating a pair per context slowed later contexts down.
// Work from different contexts on the pair is ordered by each context's own
// events, so sharing costs at most false dependencies.  False if the device
// has fewer than 64 CUs or the runtime refuses the masks.
bool masked_streams(hipStream_t* small_s, hipStream_t* big_s) {
  static std::mutex mu;
  static std::map<int, std::pair<hipStream_t, hipStream_t>> pool;
  int dev = 0, ncu = 0;
  CTM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = pool.find(dev);
  if (it == pool.end()) {
    std::pair<hipStream_t, hipStream_t> q{nullptr, nullptr};
    CTM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu >= 64) {
      std::vector<uint32_t> small((ncu + 31) / 32, 0u), big((ncu + 31) / 32, 0u);
      for (int i = 0; i < ncu; ++i) (i < 16 ? small : big)[i / 32] |= 1u << (i % 32);
      if (hipExtStreamCreateWithCUMask(&q.first, (uint32_t)small.size(), small.data()) != hipSuccess ||
          hipExtStreamCreateWithCUMask(&q.second, (uint32_t)big.size(), big.data()) != hipSuccess) {
        (void)hipGetLastError();
        if (q.first) (void)hipStreamDestroy(q.first);
        q = {nullptr, nullptr};
      }
    }
    it = pool.emplace(dev, q).first;
  }
  *small_s = it->second.first;
  *big_s = it->second.second;
  return *small_s != nullptr && *big_s != nullptr;
}

void allocate(ctm_ctx* c) {
  const int64_t D2 = c->D2, chi = c->chi, nmax = c->nmax;
  const int64_t dA = (int64_t)c->d * c->D * c->D * c->D;
  c->A = c->allocd(dA);
  c->Anext = c->allocd(dA);
  c->a = c->allocd(D2 * D2 * D2);
  c->G = c->allocd(nmax * chi);
  c->C = c->allocd(chi * chi);
  c->Cn = c->allocd(chi * chi);
  c->T = c->allocd(chi * D2 * chi);
  c->Tn = c->allocd(chi * D2 * chi);
  c->P = c->allocd(nmax * chi);
  c->M = c->allocd(nmax * chi);
  c->MP = c->allocd(nmax * 2 * chi);
  c->Q = c->allocd(nmax * chi);
  c->Cp = c->allocd(chi * chi);
  c->Xs = c->allocd(chi * chi);
  c->Xq = c->allocd(chi * chi);
  if (c->cfg.proj == CTM_PROJ_QR_CHOL) {
    c->cg = c->allocd(chi * chi);
    c->cri = c->allocd(chi * chi);
    c->cx = c->allocd(chi * chi);
    c->G1 = c->allocd(nmax * chi);
    c->W1 = c->allocd(nmax * chi);
    c->ws_big = Scratch{c->alloc(gemm_scratch_bytes(DType::F64, (int)nmax, (int)chi)),
                        gemm_scratch_bytes(DType::F64, (int)nmax, (int)chi)};
    // CU masks: the first 16 CUs for the basis factorization, the rest for
    // the products.  Streams made with a CU mask are blocking streams, which
    // the legacy default stream would synchronize with at every launch, so
    // with the null stream (or no masked streams) there is no overlap.
    if (c->stream != nullptr &&
        masked_streams(&c->stream_small, &c->stream_big)) {
      CTM_HIP(hipEventCreateWithFlags(&c->ev_big, hipEventDisableTiming | hipEventDisableSystemFence));
      CTM_HIP(hipEventCreateWithFlags(&c->ev_small, hipEventDisableTiming | hipEventDisableSystemFence));
      c->overlap = true;
    }
    c->chol_status = (int*)c->alloc(sizeof(int) * 4);
  }
  c->Tp = c->allocd(chi * D2 * chi);
  c->sgn = c->allocd(chi);
  c->sumsq = c->allocd(1024);
  c->dev_small = c->allocd(8);
  c->flag = (int*)c->alloc(sizeof(int) * 4);
  c->aE = c->allocd(D2 * D2 * D2);
  c->CE = c->allocd(chi * chi);
  c->TE = c->allocd(chi * D2 * chi);
  c->PE = c->allocd(nmax * chi);
  c->QE = c->allocd(nmax * chi);
  c->TCp = c->allocd(chi * nmax);
  c->V = c->allocd(nmax * nmax);
  c->W = c->allocd(nmax * chi);
  c->Ct = c->allocd(nmax * nmax);
  c->Gm = c->allocd(nmax * chi);
  c->V2 = c->allocd(nmax * chi);
  c->qr = qr_work_carve(c->stream, c->alloc(qr_work_bytes((int)nmax, (int)chi)), (int)nmax,
                        (int)chi);
  c->qr2 = qr_work_carve(c->stream, c->alloc(qr_work_bytes((int)chi, (int)chi)), (int)chi,
                         (int)chi);
  // the Householder projector's second stream (the Cholesky projector has
  // its own pair below); every stream a context creates takes a hardware
  // queue of the process's few
  if (c->cfg.proj != CTM_PROJ_QR_CHOL)
    CTM_HIP(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
  // fork/join of the projector's two streams: an ordering within the device,
  // so no system-scope fence (host and other devices never read through them)
  CTM_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming | hipEventDisableSystemFence));
  CTM_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming | hipEventDisableSystemFence));
  CTM_HIP(hipEventCreateWithFlags(&c->ev_spec, hipEventDisableTiming));
  CTM_HIP(hipHostMalloc((void**)&c->hostC, (size_t)chi * chi * sizeof(double), hipHostMallocDefault));
  if (c->cfg.proj == CTM_PROJ_EVD)
    c->evd = evd_work_carve(c->alloc(evd_work_bytes((int)nmax, (int)chi)), (int)nmax, (int)chi);
  size_t wsb = std::max(gemm_scratch_bytes(DType::F64, (int)nmax, (int)chi),
                        gemm_scratch_bytes(DType::F64, (int)chi, (int)chi));
  c->ws.bytes = wsb;
  c->ws.p = c->alloc(wsb);
}

}  // namespace

extern "C" {

int ctm_symmetrize(const double* raw_dev, double* A_dev, int d, int D, void* stream) {
  if (!raw_dev || !A_dev || d < 1 || D < 1 || (int64_t)d * D * D * D > 16384) {
    g_error = "ctm_symmetrize: bad arguments";
    return CTM_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    double* tmp = nullptr;
    CTM_HIP(hipMalloc(&tmp, sizeof(double)));
    launch_symmetrize(s, raw_dev, A_dev, d, D, tmp);
    double n2 = 0.0;
    CTM_HIP(hipMemcpyAsync(&n2, tmp, sizeof(double), hipMemcpyDeviceToHost, s));
    CTM_HIP(hipStreamSynchronize(s));
    CTM_HIP(hipFree(tmp));
    if (!(n2 > 0.0) || !std::isfinite(n2)) {
      g_error = "ctm_symmetrize: the symmetric projection is zero or not finite";
      return CTM_ENONFINITE;
    }
    return CTM_OK;
  } catch (const std::exception& e) {
    g_error = e.what();
    return CTM_EDEVICE;
  }
}

int ctm_init(ctm_ctx** out, const ctm_config* cfg, const double* A_dev, const double* G_dev,
             void* stream) {
  if (!out || !A_dev || !G_dev) {
    g_error = "ctm_init: null pointer";
    return CTM_EINVAL;
  }
  *out = nullptr;
  std::string why;
  if (!valid_cfg(cfg, why)) {
    g_error = "ctm_init: " + why;
    return CTM_EINVAL;
  }
  std::unique_ptr<ctm_ctx> c(new (std::nothrow) ctm_ctx());
  if (!c) {
    g_error = "ctm_init: host allocation failed";
    return CTM_ENOMEM;
  }
  c->cfg = *cfg;
  c->stream = (hipStream_t)stream;
  c->d = cfg->d;
  c->D = cfg->D;
  c->D2 = cfg->D * cfg->D;
  c->chi = cfg->chi;
  c->nmax = (int64_t)cfg->chi * c->D2;
  c->prec = to_dtype(cfg->prec);
  int rc = guarded(c.get(), [&]() -> int {
    allocate(c.get());
    hipStream_t s = c->stream;
    const int64_t dA = (int64_t)c->d * c->D * c->D * c->D;
    CTM_HIP(hipMemcpyAsync(c->A, A_dev, dA * sizeof(double), hipMemcpyDeviceToDevice, s));
    CTM_HIP(hipMemcpyAsync(c->G, G_dev, (size_t)c->nmax * c->chi * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    launch_symmetry_defect(s, c->A, c->d, c->D, c->dev_small);
    double sd[2];
    CTM_HIP(hipMemcpyAsync(sd, c->dev_small, sizeof(sd), hipMemcpyDeviceToHost, s));
    CTM_HIP(hipStreamSynchronize(s));
    if (!(sd[1] > 0.0) || !std::isfinite(sd[0]) || !std::isfinite(sd[1])) {
      c->err = "site tensor is zero or not finite";
      return CTM_ENONFINITE;
    }
    if (std::sqrt(sd[0]) > 1e-12 * std::sqrt(sd[1])) {
      c->err = "site tensor is not C3v-symmetric: ||A - sym(A)|| / ||A|| = " +
               std::to_string(std::sqrt(sd[0] / sd[1]));
      return CTM_ENOTSYM;
    }
    launch_double_layer(s, c->A, c->d, c->D, c->a);
    c->aE_type = -1;
    launch_init_env(s, c->D, c->C, c->T);
    CTM_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), s));
    CTM_HIP(hipStreamSynchronize(s));
    c->chi_c = 1;
    c->steps = 0;
    c->p_rows = 0;
    return CTM_OK;
  });
  if (rc != CTM_OK) {
    g_error = "ctm_init: " + c->err;
    return rc;
  }
  *out = c.release();
  return CTM_OK;
}

int ctm_step(ctm_ctx* c, int n_steps, double* delta_host) {
  return guarded(c, [&]() { return do_steps(c, n_steps, delta_host); });
}

int ctm_converge(ctm_ctx* c, double tol, int max_steps, int n_check, int* steps_host,
                 double* delta_host) {
  return guarded(c, [&]() -> int {
    if (max_steps < 0 || n_check < 1) throw std::invalid_argument("max_steps < 0 or n_check < 1");
    int taken = 0;
    double delta = std::numeric_limits<double>::infinity();
    int rc = CTM_OK;
    // Precision ladder: BF16, then FP32, then FP64; a rung is left when the
    // spectrum change falls below its threshold or stops improving (the
    // best change not halved in 8 checks).  Convergence counts on FP64 only.
    const bool ladder = c->cfg.prec == CTM_PREC_LADDER;
    double best = std::numeric_limits<double>::infinity();
    int stale = 0;
    while (taken < max_steps) {
      const int k = std::min(n_check, max_steps - taken);
      rc = do_steps(c, k, &delta);
      taken += k;
      if (rc != CTM_OK) break;
      if (ladder && c->prec != DType::F64) {
        if (delta < 0.5 * best) {
          best = delta;
          stale = 0;
        } else {
          ++stale;
        }
        const double rung_tol = c->prec == DType::BF16 ? 1e-4 : 1e-9;
        if (delta < rung_tol || stale >= 8) {
          c->prec = c->prec == DType::BF16 ? DType::F32 : DType::F64;
          best = std::numeric_limits<double>::infinity();
          stale = 0;
        }
        continue;
      }
      if (delta < tol) break;
    }
    if (steps_host) *steps_host = taken;
    if (delta_host) *delta_host = delta;
    if (rc != CTM_OK) return rc;
    if (!(delta < tol)) {
      c->err = "tolerance not reached in max_steps";
      return CTM_ENOTCONV;
    }
    return CTM_OK;
  });
}

int ctm_energy(ctm_ctx* c, const double* h_host, double* e_host, double* rho_host) {
  return guarded(c, [&]() -> int {
    if (!h_host) throw std::invalid_argument("null operator");
    return do_energy(c, h_host, e_host, rho_host);
  });
}

int ctm_grad(ctm_ctx* c, const double* h_host, int mode, double tol, int max_iter,
             double* gradA_dev, double* e_host, int* iters_host) {
  return guarded(c, [&]() -> int {
    return do_grad(c, h_host, mode, tol, max_iter, gradA_dev, e_host, iters_host);
  });
}

int ctm_spectrum(ctm_ctx* c, double* s_host, int* n_host) {
  return guarded(c, [&]() -> int {
    if (!s_host) throw std::invalid_argument("null output");
    std::vector<double> sp = current_spectrum(c);
    std::memcpy(s_host, sp.data(), sp.size() * sizeof(double));
    if (n_host) *n_host = c->chi_c;
    return CTM_OK;
  });
}

int ctm_query(const ctm_ctx* c, int* chi_c, int* steps, int* p_rows) {
  if (!c) {
    g_error = "null context";
    return CTM_EINVAL;
  }
  if (chi_c) *chi_c = c->chi_c;
  if (steps) *steps = c->steps;
  if (p_rows) *p_rows = c->p_rows;
  return CTM_OK;
}

int ctm_get_env(ctm_ctx* c, double* C_dev, double* T_dev, double* P_dev) {
  return guarded(c, [&]() -> int {
    hipStream_t s = c->stream;
    const size_t x = c->chi_c;
    if (C_dev) CTM_HIP(hipMemcpyAsync(C_dev, c->C, x * x * 8, hipMemcpyDeviceToDevice, s));
    if (T_dev) CTM_HIP(hipMemcpyAsync(T_dev, c->T, x * c->D2 * x * 8, hipMemcpyDeviceToDevice, s));
    if (P_dev && c->p_rows > 0)
      CTM_HIP(hipMemcpyAsync(P_dev, c->P, (size_t)c->p_rows * c->chi * 8, hipMemcpyDeviceToDevice, s));
    return CTM_OK;
  });
}

int ctm_set_env(ctm_ctx* c, int chi_c, const double* C_dev, const double* T_dev, int p_rows,
                const double* P_dev) {
  return guarded(c, [&]() -> int {
    if (chi_c < 1 || chi_c > c->chi || !C_dev || !T_dev || p_rows < 0 || p_rows > c->nmax ||
        (p_rows > 0 && !P_dev))
      throw std::invalid_argument("ctm_set_env: bad arguments");
    hipStream_t s = c->stream;
    const size_t x = chi_c;
    CTM_HIP(hipMemcpyAsync(c->C, C_dev, x * x * 8, hipMemcpyDeviceToDevice, s));
    CTM_HIP(hipMemcpyAsync(c->T, T_dev, x * c->D2 * x * 8, hipMemcpyDeviceToDevice, s));
    if (p_rows > 0)
      CTM_HIP(hipMemcpyAsync(c->P, P_dev, (size_t)p_rows * c->chi * 8, hipMemcpyDeviceToDevice, s));
    c->chi_c = chi_c;
    c->p_rows = p_rows;
    c->spec_step = -1;
    return CTM_OK;
  });
}

int ctm_update_tensor(ctm_ctx* c, const double* A_dev) {
  if (!c || !A_dev) {
    g_error = "ctm_update_tensor: null pointer";
    return CTM_EINVAL;
  }
  return guarded(c, [&]() -> int {
    hipStream_t s = c->stream;
    const int64_t dA = (int64_t)c->d * c->D * c->D * c->D;
    // checked in a scratch copy first, so a rejected tensor leaves the state as it was
    double* chk = c->Anext;
    CTM_HIP(hipMemcpyAsync(chk, A_dev, dA * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_symmetry_defect(s, chk, c->d, c->D, c->dev_small);
    double sd[2];
    CTM_HIP(hipMemcpyAsync(sd, c->dev_small, sizeof(sd), hipMemcpyDeviceToHost, s));
    CTM_HIP(hipStreamSynchronize(s));
    if (!(sd[1] > 0.0) || !std::isfinite(sd[0]) || !std::isfinite(sd[1])) {
      c->err = "site tensor is zero or not finite";
      return CTM_ENONFINITE;
    }
    if (std::sqrt(sd[0]) > 1e-12 * std::sqrt(sd[1])) {
      c->err = "site tensor is not C3v-symmetric: ||A - sym(A)|| / ||A|| = " +
               std::to_string(std::sqrt(sd[0] / sd[1]));
      return CTM_ENOTSYM;
    }
    CTM_HIP(hipMemcpyAsync(c->A, A_dev, dA * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_double_layer(s, c->A, c->d, c->D, c->a);
    c->aE_type = -1;
    if (c->aO) {
      launch_double_layer_open(s, c->A, c->d, c->D, 0, c->aO);
      launch_double_layer_open(s, c->A, c->d, c->D, 1, c->aOr);
    }
    c->spec_step = -1;
    return CTM_OK;
  });
}

int ctm_set_precision(ctm_ctx* c, int prec) {
  return guarded(c, [&]() -> int {
    if (prec < CTM_PREC_FP64 || prec > CTM_PREC_LADDER) throw std::invalid_argument("bad precision");
    c->prec = to_dtype(prec);
    c->cfg.prec = prec;
    return CTM_OK;
  });
}

int ctm_profile(ctm_ctx* c, int enable) {
  return guarded(c, [&]() -> int {
    CTM_HIP(hipStreamSynchronize(c->stream));
    c->prof_on = enable != 0;
    c->intervals.clear();
    c->events_used = 0;
    c->big_flops = 0.0;
    return CTM_OK;
  });
}

int ctm_profile_read(ctm_ctx* c, double* ms_host, int64_t* launches_host, double* flops_host) {
  return guarded(c, [&]() -> int {
    CTM_HIP(hipStreamSynchronize(c->stream));
    double ms[CTM_NSTAGES] = {};
    int64_t cnt[CTM_NSTAGES] = {};
    for (const auto& iv : c->intervals) {
      float t = 0.0f;
      CTM_HIP(hipEventElapsedTime(&t, iv.begin, iv.end));
      ms[iv.stage] += t;
      cnt[iv.stage] += 1;
    }
    if (ms_host) std::memcpy(ms_host, ms, sizeof(ms));
    if (launches_host) std::memcpy(launches_host, cnt, sizeof(cnt));
    if (flops_host) *flops_host = c->big_flops;
    return CTM_OK;
  });
}

void ctm_free(ctm_ctx* c) { delete c; }

const char* ctm_last_error(const ctm_ctx* c) {
  if (!c) return g_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
