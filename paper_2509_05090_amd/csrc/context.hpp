// The CTMRG context shared by the forward engine and the adjoint.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ctm.h"
#include "gemm.hpp"
#include "qr.hpp"
#include "evd.hpp"

namespace ctm {

struct OutOfMemory : std::runtime_error {
  explicit OutOfMemory(const std::string& s) : std::runtime_error(s) {}
};

struct GradBuffers;
void free_grad(GradBuffers* g);

}  // namespace ctm

using ctm::DType;
using ctm::QrWork;
using ctm::Scratch;

struct ctm_ctx {
  ctm_config cfg{};
  hipStream_t stream = nullptr;
  // second stream of the projector (the explicit Q1 is formed there while
  // the basis matrix is factored on `stream`), joined by ev_fork / ev_join
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Cholesky QR projector, update steps (FP64, FP32): while the basis matrix
  // X is factored on stream_small (a few CUs), the products Ct Q1 and V Q1
  // run on stream_big (the other CUs); disjoint CU masks keep the
  // latency-bound factorization off the products' CUs.  overlap is false if
  // the masked streams are unavailable.  The two streams belong to the
  // process (one pair per device, shared by all contexts); a context's work
  // on them is joined into `stream` by ev_small and ev_big.
  hipStream_t stream_big = nullptr, stream_small = nullptr;
  hipEvent_t ev_big = nullptr, ev_small = nullptr;
  bool overlap = false;
  bool pre_q1 = false;  // G1 = Ct Q1 and W1 = V Q1 pending for the renormalization
  double *G1 = nullptr, *W1 = nullptr;
  Scratch ws_big;  // split-K scratch of the products on stream_big
  // convergence test: pinned host copy of the corner taken before a batch's
  // last step, and the event marking the copy
  double* hostC = nullptr;
  hipEvent_t ev_spec = nullptr;
  std::string err;
  bool poisoned = false;
  int d = 0, D = 0, D2 = 0, chi = 0;
  int64_t nmax = 0;
  int chi_c = 1, steps = 0, p_rows = 0;
  DType prec = DType::F64;

  std::vector<void*> allocations;

  // FP64 state and inputs
  double *A = nullptr, *a = nullptr, *aO = nullptr, *aOr = nullptr, *G = nullptr;
  double* Anext = nullptr;  // site tensor under check by ctm_update_tensor
  double *C = nullptr, *T = nullptr, *Cn = nullptr, *Tn = nullptr, *P = nullptr;
  // FP64 work
  double *M = nullptr, *MP = nullptr, *Q = nullptr, *Cp = nullptr, *Tp = nullptr, *Xs = nullptr, *Xq = nullptr;
  double *sgn = nullptr, *sumsq = nullptr, *dev_small = nullptr;
  int* flag = nullptr;
  // Cholesky QR projector: Gram matrix, inverse of its factor, X = Q1^T P_prev
  double *cg = nullptr, *cri = nullptr, *cx = nullptr;
  int* chol_status = nullptr;
  // Intermediates; allocated with 8-byte elements so that they hold any precision.
  void *aE = nullptr, *CE = nullptr, *TE = nullptr, *PE = nullptr, *QE = nullptr;
  int aE_type = -1;  // DType held in aE (a cast of a), -1 if none
  void *TCp = nullptr, *V = nullptr, *W = nullptr, *Ct = nullptr, *Gm = nullptr, *V2 = nullptr;
  // energy
  double *XO = nullptr, *EO = nullptr, *Cr2 = nullptr, *Cr4 = nullptr, *Cr5 = nullptr;
  double *rho_raw = nullptr, *h_dev = nullptr, *e_out = nullptr;
  QrWork qr;
  QrWork qr2;  // chi x chi factorizations (the basis of the QR projector)
  ctm::EvdWork evd;  // eigendecomposition projector (CTM_PROJ_EVD only)
  Scratch ws;
  ctm::GradBuffers* grad = nullptr;  // adjoint workspace, allocated by the first ctm_grad

  // spectrum cache (host)
  std::vector<double> spec;
  int spec_step = -1;

  // stage timing (HIP events on the stream)
  struct TimedInterval {
    int stage;
    hipEvent_t begin, end;
  };
  bool prof_on = false, prof_active = false;
  std::vector<hipEvent_t> event_pool;
  size_t events_used = 0;
  std::vector<TimedInterval> intervals;
  double big_flops = 0.0;
  hipEvent_t stage_open[CTM_NSTAGES] = {};

  hipEvent_t next_event() {
    if (events_used == event_pool.size()) {
      hipEvent_t e;
      CTM_HIP(hipEventCreate(&e));
      event_pool.push_back(e);
    }
    return event_pool[events_used++];
  }

  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw ctm::OutOfMemory("hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e));
    }
    allocations.push_back(p);
    return p;
  }
  double* allocd(int64_t n) { return (double*)alloc((size_t)n * sizeof(double)); }

  ~ctm_ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (stream2) {
      (void)hipStreamSynchronize(stream2);
      (void)hipStreamDestroy(stream2);
    }
    // the last work this context put on the shared masked streams
    for (hipEvent_t e : {ev_big, ev_small})
      if (e) {
        (void)hipEventSynchronize(e);
        (void)hipEventDestroy(e);
      }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_spec) (void)hipEventDestroy(ev_spec);
    if (hostC) (void)hipHostFree(hostC);
    ctm::free_grad(grad);
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    for (void* p : allocations) (void)hipFree(p);
  }
};


namespace ctm {

// Energy gradient of the current environment (see ctm_grad in ctm.h).
int do_grad(ctm_ctx* c, const double* h_host, int mode, double tol, int max_iter, double* gradA_dev,
            double* e_host, int* iters_host);

// Open double layers for the energy (engine.cpp); idempotent.
void ensure_energy_buffers(ctm_ctx* c);

}  // namespace ctm
