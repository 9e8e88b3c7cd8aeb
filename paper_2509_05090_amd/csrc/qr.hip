// Blocked Householder QR (FP64) for tall-skinny matrices.
//
// Panels of QR_NB columns are factored by one workgroup: for every column
// the squared norm, the inner products with the panel's later columns and
// with the panel's earlier Householder vectors are reduced in one pass
// (wavefront shuffles, then LDS across the 16 wavefronts), the reflector is
// formed as in LAPACK's dlarfg (beta = -sign(x0) ||x||), and the pass that
// applies it also accumulates the sums for the next column.  The same pass
// builds the triangular factor T of the compact WY form H_1...H_w = I - Y T Y^T
// column by column.  The trailing columns are then updated with two MFMA
// products, A <- A - Y (T^T (Y^T A)), and the explicit Q is accumulated
// backwards, Q <- Q - Y (T (Y^T Q)), starting from the first k columns of
// the identity.
#include "qr.hpp"

namespace ctm {

constexpr int PT = 512;  // threads of the panel workgroup

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// State of one panel factorization shared by the per-column steps.
template <int NB>
struct PanelCtx {
  double* __restrict__ M;
  int ld, n, j0, w;
  double* __restrict__ Y;
  int ldy;
  double* __restrict__ tau;
  double (*red)[NB];
  double* fin;
  double (*Tsh)[NB];
  int tid, lane, wid;
  // part[0] = sum x_r^2, part[k - c] = sum x_r a_k[r] (k > c),
  // part[NB - c + i] = sum Y[r][i] x_r (i < c), all over rows r > pivot.
  double part[NB];
};

// Column c of the panel; c is a template parameter so that every register
// array is indexed with constants.
template <int NB, int c>
__device__ inline void panel_column(PanelCtx<NB>& x) {
  const int pr = x.j0 + c;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const double s = wave_sum(x.part[q]);
    if (x.lane == 0) x.red[x.wid][q] = s;
  }
  __syncthreads();
  if (x.tid < NB) {
    double s = 0.0;
    for (int i = 0; i < PT / 64; ++i) s += x.red[i][x.tid];
    x.fin[x.tid] = s;
  }
  __syncthreads();

  const double* prow = x.M + (size_t)pr * x.ld + x.j0;
  double pv[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) pv[k] = k < x.w ? prow[k] : 0.0;
  const double x0 = pv[c], sigma = x.fin[0];
  double beta, tc, scale;
  if (sigma == 0.0) {
    tc = 0.0;
    beta = x0;
    scale = 0.0;
  } else {
    const double nrm = sqrt(x0 * x0 + sigma);
    beta = x0 >= 0.0 ? -nrm : nrm;
    tc = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
  }
  double vta[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) vta[k] = k > c ? pv[k] + scale * x.fin[k - c] : 0.0;

  if (x.tid == 0) {
    double yv[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) yv[i] = i < c ? pv[i] + scale * x.fin[NB - c + i] : 0.0;
#pragma unroll
    for (int i = 0; i < c; ++i) {
      double t = 0.0;
#pragma unroll
      for (int i2 = i; i2 < c; ++i2) t += x.Tsh[i][i2] * yv[i2];
      x.Tsh[i][c] = -tc * t;
    }
    x.Tsh[c][c] = tc;
#pragma unroll
    for (int i = c + 1; i < NB; ++i) x.Tsh[i][c] = 0.0;
    x.tau[pr] = tc;
  }

#pragma unroll
  for (int q = 0; q < NB; ++q) x.part[q] = 0.0;
  for (int r = pr + 1 + x.tid; r < x.n; r += PT) {
    double* row = x.M + (size_t)r * x.ld + x.j0;
    double v[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) v[k] = k < x.w ? row[k] : 0.0;
    const double vr = v[c] * scale;
    v[c] = vr;
#pragma unroll
    for (int k = c + 1; k < NB; ++k) v[k] -= tc * vr * vta[k];
#pragma unroll
    for (int k = c; k < NB; ++k)
      if (k < x.w) row[k] = v[k];
    x.Y[(size_t)r * x.ldy + x.j0 + c] = vr;
    if (c + 1 < NB && r > pr + 1) {
      const double xn = v[(c + 1) % NB];
      x.part[0] += xn * xn;
#pragma unroll
      for (int k = c + 2; k < NB; ++k) x.part[k - (c + 1)] += xn * v[k];
#pragma unroll
      for (int i = 0; i <= c; ++i) x.part[(NB - (c + 1) + i) % NB] += v[i] * xn;
    }
  }
  if (x.tid == 0) {
    double* prw = x.M + (size_t)pr * x.ld + x.j0;
    prw[c] = beta;
#pragma unroll
    for (int k = c + 1; k < NB; ++k)
      if (k < x.w) prw[k] = pv[k] - tc * vta[k];
    x.Y[(size_t)pr * x.ldy + x.j0 + c] = 1.0;
    for (int r = x.j0; r < pr; ++r) x.Y[(size_t)r * x.ldy + x.j0 + c] = 0.0;
  }
  __syncthreads();
}

template <int NB, int c>
struct PanelColumns {
  __device__ static inline void run(PanelCtx<NB>& x) {
    if (c < x.w) {
      panel_column<NB, c>(x);
      PanelColumns<NB, c + 1>::run(x);
    }
  }
};
template <int NB>
struct PanelColumns<NB, NB> {
  __device__ static inline void run(PanelCtx<NB>&) {}
};

template <int NB>
__global__ __launch_bounds__(PT) void qr_panel_kernel(double* __restrict__ M, int ld, int n, int j0,
                                                      int w, double* __restrict__ Y, int ldy,
                                                      double* __restrict__ tau,
                                                      double* __restrict__ Tf) {
  __shared__ double red[PT / 64][NB];
  __shared__ double fin[NB];
  __shared__ double Tsh[NB][NB];
  PanelCtx<NB> x{M, ld, n, j0, w, Y, ldy, tau, red, fin, Tsh};
  x.tid = threadIdx.x;
  x.lane = x.tid & 63;
  x.wid = x.tid >> 6;
#pragma unroll
  for (int q = 0; q < NB; ++q) x.part[q] = 0.0;
  for (int r = j0 + 1 + x.tid; r < n; r += PT) {
    const double* row = M + (size_t)r * ld + j0;
    double v[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) v[k] = k < w ? row[k] : 0.0;
    x.part[0] += v[0] * v[0];
#pragma unroll
    for (int k = 1; k < NB; ++k) x.part[k] += v[0] * v[k];
  }
  PanelColumns<NB, 0>::run(x);
  for (int i = x.tid; i < NB * NB; i += PT) {
    const int a = i / NB, b = i % NB;
    Tf[i] = (a < w && b < w) ? Tsh[a][b] : 0.0;
  }
}

// Wout = op(T) Win for the w x w upper-triangular T (op = T^T if trans).
__global__ void tri_apply_kernel(const double* __restrict__ T, int nbT, bool trans,
                                 const double* __restrict__ Win, double* __restrict__ Wout, int w,
                                 int N) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double x[QR_NB];
#pragma unroll
  for (int i = 0; i < QR_NB; ++i) x[i] = i < w ? Win[(size_t)i * N + j] : 0.0;
#pragma unroll
  for (int c = 0; c < QR_NB; ++c) {
    double s = 0.0;
    if (trans) {
#pragma unroll
      for (int i = 0; i <= c; ++i) s += T[i * nbT + c] * x[i];
    } else {
#pragma unroll
      for (int i = c; i < QR_NB; ++i)
        if (i < w) s += T[c * nbT + i] * x[i];
    }
    if (c < w) Wout[(size_t)c * N + j] = s;
  }
}

__global__ void fill_eye_kernel(double* Q, int n, int k, int ldq) {
  const int64_t total = (int64_t)n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / k, c = i % k;
    Q[r * ldq + c] = r == c ? 1.0 : 0.0;
  }
}

static void tri_apply(hipStream_t s, const double* T, bool trans, const double* Win, double* Wout,
                      int w, int N) {
  tri_apply_kernel<<<(unsigned)cdiv(N, 256), 256, 0, s>>>(T, QR_NB, trans, Win, Wout, w, N);
  CTM_LAUNCHED();
}

void householder_qr(hipStream_t s, double* M, int ld, int n, int k, QrWork& w) {
  if (n < k) throw std::invalid_argument("householder_qr: needs n >= k");
  for (int p = 0, j0 = 0; j0 < k; ++p, j0 += QR_NB) {
    const int wp = std::min(QR_NB, k - j0);
    double* Tp = w.Tf + (size_t)p * QR_NB * QR_NB;
    qr_panel_kernel<QR_NB><<<1, PT, 0, s>>>(M, ld, n, j0, wp, w.Y, k, w.tau, Tp);
    CTM_LAUNCHED();
    const int rest = k - j0 - wp;
    if (rest <= 0) continue;
    const double* Yp = w.Y + (size_t)j0 * k + j0;
    double* Arest = M + (size_t)j0 * ld + j0 + wp;
    gemm(s, DType::F64, wp, rest, n - j0, Operand{Yp, k, true}, Operand{Arest, ld, false},
         Output{w.W, rest, DType::F64}, 1, 1, 1.0, 0.0, w.ws);
    tri_apply(s, Tp, true, w.W, w.W2, wp, rest);
    gemm(s, DType::F64, n - j0, rest, wp, Operand{Yp, k, false}, Operand{w.W2, rest, false},
         Output{Arest, ld, DType::F64}, 1, 1, -1.0, 1.0, w.ws, 1);
  }
}

void householder_form_q(hipStream_t s, const QrWork& w, int n, int k, double* Q, int ldq) {
  fill_eye_kernel<<<(unsigned)std::min<int64_t>(4096, cdiv((int64_t)n * k, 256)), 256, 0, s>>>(
      Q, n, k, ldq);
  CTM_LAUNCHED();
  const int np = (int)cdiv(k, QR_NB);
  for (int p = np - 1; p >= 0; --p) {
    const int j0 = p * QR_NB, wp = std::min(QR_NB, k - j0), cols = k - j0;
    const double* Tp = w.Tf + (size_t)p * QR_NB * QR_NB;
    const double* Yp = w.Y + (size_t)j0 * k + j0;
    double* Qs = Q + (size_t)j0 * ldq + j0;
    gemm(s, DType::F64, wp, cols, n - j0, Operand{Yp, k, true}, Operand{Qs, ldq, false},
         Output{w.W, cols, DType::F64}, 1, 1, 1.0, 0.0, w.ws);
    tri_apply(s, Tp, false, w.W, w.W2, wp, cols);
    gemm(s, DType::F64, n - j0, cols, wp, Operand{Yp, k, false}, Operand{w.W2, cols, false},
         Output{Qs, ldq, DType::F64}, 1, 1, -1.0, 1.0, w.ws, 1);
  }
}

}  // namespace ctm
