// Blocked Householder QR (FP64) for tall-skinny matrices, with each panel
// factored as a tall-skinny QR (TSQR) over row blocks.
//
// Panel kernel: one workgroup of 512 threads per leaf (row block of up to
// 512 or 1024 rows) holds its block of the panel in registers, one or two
// rows per thread, and factors it column by column.  Per column a single
// reduction gives, for the rows below the pivot, the column's squared norm,
// its inner products with the later panel columns and with the earlier
// Householder vectors (the latter build the compact WY factor T).  The
// reduction is a reduce-scatter across the 64 lanes of a wavefront (the
// 32 partial sums are halved at each exchange, 32 exchanges instead of
// 32 x 6), then one LDS pass across the 8 wavefronts.  The reflector
// follows LAPACK's dlarfg (beta = -sign(x0) ||x||).  Leaves write their
// triangular factors to a stack; the last leaf to finish (atomic counter,
// no waiting) factors the stack in the same way.
//
// Apply kernel: B <- (I - Y op(T) Y^T) B on a range of columns, per leaf
// (row block) or on the stacked rows, 32 columns per workgroup: W = Y^T B,
// W <- op(T) W, B <- B - Y W, with LDS-staged 64-row tiles.
#include "qr.hpp"

namespace ctm {

namespace {

constexpr int NB = QR_NB;
constexpr int QT = 512;  // threads of the panel workgroups
constexpr int NW = QT / 64;

struct QrShared {
  double red[2][NW][NB];
  double fin[2][NB];
  double prow[2][NB];
  double T[NB][NB + 1];
  int last;
};

// Lane l ends the reduce-scatter holding the wavefront sum of this index.
__device__ inline int rs_index(int lane) {
  return ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 +
         ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
}

template <int N>
__device__ __forceinline__ void rs_halve(const double (&in)[2 * N], double (&out)[N], bool up, int off) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double keep = up ? in[j + N] : in[j], send = up ? in[j] : in[j + N];
    out[j] = keep + __shfl_xor(send, off);
  }
}

// Column c of a local Householder QR of the rows held by this workgroup
// (row t = tid + r * QT in a[r][*]); w = columns in use.
template <int RPT, int c>
__device__ __forceinline__ void qr_column(double (&a)[RPT][NB], int w, QrShared& sh, int tid) {
  const int lane = tid & 63, wid = tid >> 6;
  constexpr int buf = c & 1;
  double x[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) x[r] = tid + r * QT > c ? a[r][c] : 0.0;
  double h16[16];
  {
    const bool up = lane & 32;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double lo = 0.0, hi = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        lo += x[r] * a[r][j];
        hi += x[r] * a[r][j + 16];
      }
      const double keep = up ? hi : lo, send = up ? lo : hi;
      h16[j] = keep + __shfl_xor(send, 32);
    }
  }
  double h8[8], h4[4], h2[2], h1[1];
  rs_halve<8>(h16, h8, lane & 16, 16);
  rs_halve<4>(h8, h4, lane & 8, 8);
  rs_halve<2>(h4, h2, lane & 4, 4);
  rs_halve<1>(h2, h1, lane & 2, 2);
  const double hsum = h1[0] + __shfl_xor(h1[0], 1);
  if ((lane & 1) == 0) sh.red[buf][wid][rs_index(lane)] = hsum;
  if (tid == c) {
#pragma unroll
    for (int q = 0; q < NB; ++q) sh.prow[buf][q] = a[0][q];
  }
  __syncthreads();
  if (tid < NB) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) s += sh.red[buf][v][tid];
    sh.fin[buf][tid] = s;
  }
  __syncthreads();
  const double x0 = sh.prow[buf][c], sigma = sh.fin[buf][c];
  double beta, tau, scale;
  if (sigma == 0.0) {
    tau = 0.0;
    beta = x0;
    scale = 0.0;
  } else {
    const double nrm = sqrt(x0 * x0 + sigma);
    beta = x0 >= 0.0 ? -nrm : nrm;
    tau = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
  }
  // column c of T: T[i][c] = -tau sum_{i2 = i..c-1} T[i][i2] (y_i2 . v_c),
  // y_i2 . v_c = Y[c][i2] + scale * (sum over rows below c of Y[.][i2] x)
  if (tid < c) {
    double t = 0.0;
    for (int i2 = tid; i2 < c; ++i2)
      t += sh.T[tid][i2] * (sh.prow[buf][i2] + scale * sh.fin[buf][i2]);
    sh.T[tid][c] = -tau * t;
  }
  if (tid == c) sh.T[c][c] = tau;
  double v[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const bool below = tid + r * QT > c;
    v[r] = below ? a[r][c] * scale : 0.0;
    if (below) a[r][c] = v[r];
  }
#pragma unroll
  for (int k = c + 1; k < NB; ++k) {
    if (k < w) {
      const double wk = sh.prow[buf][k] + scale * sh.fin[buf][k];
#pragma unroll
      for (int r = 0; r < RPT; ++r) a[r][k] -= tau * v[r] * wk;
      if (tid == c) a[0][k] = sh.prow[buf][k] - tau * wk;
    }
  }
  if (tid == c) a[0][c] = beta;
}

template <int RPT, int c>
struct QrCols {
  __device__ static __forceinline__ void run(double (&a)[RPT][NB], int w, QrShared& sh, int tid) {
    if (c < w) {
      qr_column<RPT, c>(a, w, sh, tid);
      QrCols<RPT, c + 1>::run(a, w, sh, tid);
    }
  }
};
template <int RPT>
struct QrCols<RPT, NB> {
  __device__ static inline void run(double (&)[RPT][NB], int, QrShared&, int) {}
};

// Writes this workgroup's Householder vectors (unit diagonal, zeros above)
// and its T factor.
template <int RPT>
__device__ __forceinline__ void store_reflectors(const double (&a)[RPT][NB], int m, int w, double* Y,
                                        int64_t ldy, double* Tout, const QrShared& sh, int tid) {
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int t = tid + r * QT;
    if (t < m) {
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < w) Y[(int64_t)t * ldy + q] = t > q ? a[r][q] : (t == q ? 1.0 : 0.0);
    }
  }
  for (int i = tid; i < NB * NB; i += QT) {
    const int r = i / NB, cc = i % NB;
    Tout[i] = (r < w && cc < w && cc >= r) ? sh.T[r][cc] : 0.0;
  }
}

template <int RL, int RT>
__global__ __launch_bounds__(QT) void qr_panel_kernel(double* __restrict__ A, int ld, int n, int j0,
                                                      int w, int rpl, int L, double* __restrict__ Y,
                                                      int ldy, double* __restrict__ Tl,
                                                      double* __restrict__ S, double* __restrict__ Yt,
                                                      double* __restrict__ Tt,
                                                      unsigned* __restrict__ counter) {
  __shared__ QrShared sh;
  const int tid = threadIdx.x, leaf = blockIdx.x;
  const int r0 = j0 + leaf * rpl;
  const int m = min(rpl, n - r0);
  {
    double a[RL][NB];
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int t = tid + r * QT;
      const double* row = A + (int64_t)(r0 + t) * ld + j0;
#pragma unroll
      for (int q = 0; q < NB; ++q) a[r][q] = (t < m && q < w) ? row[q] : 0.0;
    }
    QrCols<RL, 0>::run(a, w, sh, tid);
    __syncthreads();
    store_reflectors<RL>(a, m, w, Y + (int64_t)r0 * ldy + j0, ldy, Tl + (int64_t)leaf * NB * NB, sh,
                         tid);
    if (L == 1) {
      if (tid < w) {
        double* row = A + (int64_t)(r0 + tid) * ld + j0;
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < w) row[q] = q >= tid ? a[0][q] : 0.0;
      }
      return;
    }
    if (tid < w) {
      double* srow = S + (int64_t)(leaf * w + tid) * NB;
#pragma unroll
      for (int q = 0; q < NB; ++q) srow[q] = (q >= tid && q < w) ? a[0][q] : 0.0;
    }
  }
  // Publish the stacked factor; the last leaf to arrive factors the stack.
  __threadfence();
  __syncthreads();
  if (tid == 0) sh.last = atomicAdd(counter, 1u) == (unsigned)(L - 1);
  __syncthreads();
  if (!sh.last) return;
  __threadfence();
  const int Sm = L * w;
  double b[RT][NB];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int t = tid + r * QT;
#pragma unroll
    for (int q = 0; q < NB; ++q) b[r][q] = (t < Sm && q < w) ? S[(int64_t)t * NB + q] : 0.0;
  }
  QrCols<RT, 0>::run(b, w, sh, tid);
  __syncthreads();
  store_reflectors<RT>(b, Sm, w, Yt, NB, Tt, sh, tid);
  if (tid < w) {
    double* row = A + (int64_t)(j0 + tid) * ld + j0;
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (q < w) row[q] = q >= tid ? b[0][q] : 0.0;
  }
  if (tid == 0) atomicExch(counter, 0u);
}

constexpr int AT = 256;   // threads of the apply workgroups
constexpr int ACW = 32;   // columns per workgroup
constexpr int ART = 64;   // rows per LDS tile

// B <- (I - Y op(T) Y^T) B on columns [c0, c1), op(T) = T^T if TRANS.  Leaf
// mode (STACKED = false): workgroup x handles leaf x, rows [j0 + x rpl, ...)
// of B, reflectors Y[row][j0 + q] (leading dimension ldy), T = Tsrc + x NB^2.
// Stacked mode: the L*w stacked rows (leaf i, offset t) -> row j0 + i rpl + t,
// reflectors Ysrc[(i w + t) NB + q], T = Tsrc.
template <bool STACKED, bool TRANS>
__global__ __launch_bounds__(AT) void qr_apply_kernel(double* __restrict__ B, int ldb, int c0, int c1,
                                                      const double* __restrict__ Ysrc, int ldy,
                                                      const double* __restrict__ Tsrc, int n, int j0,
                                                      int w, int rpl, int L) {
  __shared__ double Ys[ART][NB + 1];
  __shared__ double Bs[ART][ACW + 1];
  __shared__ double W[NB][ACW + 1];
  __shared__ double Tsh[NB][NB + 1];
  const int tid = threadIdx.x;
  int rows, rbase = 0;
  const double* Yb;
  const double* T;
  int64_t ys;
  if (STACKED) {
    rows = L * w;
    Yb = Ysrc;
    ys = NB;
    T = Tsrc;
  } else {
    rbase = j0 + blockIdx.x * rpl;
    rows = min(rpl, n - rbase);
    Yb = Ysrc + (int64_t)rbase * ldy + j0;
    ys = ldy;
    T = Tsrc + (int64_t)blockIdx.x * NB * NB;
  }
  const int cb = c0 + blockIdx.y * ACW;
  const int nc = min(ACW, c1 - cb);
  auto grow = [&](int r) -> int64_t {
    return STACKED ? (int64_t)(j0 + (r / w) * rpl + r % w) : (int64_t)(rbase + r);
  };
  auto load_tiles = [&](int r0) {
    for (int i = tid; i < ART * NB; i += AT) {
      const int rr = i / NB, q = i % NB, r = r0 + rr;
      Ys[rr][q] = (r < rows && q < w) ? Yb[(int64_t)r * ys + q] : 0.0;
    }
    for (int i = tid; i < ART * ACW; i += AT) {
      const int rr = i / ACW, j = i % ACW, r = r0 + rr;
      Bs[rr][j] = (r < rows && j < nc) ? B[grow(r) * ldb + cb + j] : 0.0;
    }
  };
  for (int i = tid; i < NB * NB; i += AT) Tsh[i / NB][i % NB] = T[i];
  // W = Y^T B: thread (tq, tj) owns rows 2tq, 2tq+1 and columns 2tj, 2tj+1 of W
  const int tq = tid / 16, tj = tid % 16;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int r0 = 0; r0 < rows; r0 += ART) {
    load_tiles(r0);
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < ART; ++rr) {
      const double y0 = Ys[rr][2 * tq], y1 = Ys[rr][2 * tq + 1];
      const double b0 = Bs[rr][2 * tj], b1 = Bs[rr][2 * tj + 1];
      acc[0][0] += y0 * b0;
      acc[0][1] += y0 * b1;
      acc[1][0] += y1 * b0;
      acc[1][1] += y1 * b1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) W[2 * tq + a][2 * tj + b] = acc[a][b];
  __syncthreads();
  // W <- op(T) W (T upper triangular)
  double w2[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int q = 2 * tq + a;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = 2 * tj + b;
      double s = 0.0;
      if (TRANS) {
        for (int i = 0; i <= q; ++i) s += Tsh[i][q] * W[i][j];
      } else {
        for (int i = q; i < NB; ++i) s += Tsh[q][i] * W[i][j];
      }
      w2[a][b] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) W[2 * tq + a][2 * tj + b] = w2[a][b];
  __syncthreads();
  // B <- B - Y W: thread owns row tid/4 of the tile and 8 columns
  const int rr = tid / 4, jb = (tid % 4) * 8;
  for (int r0 = 0; r0 < rows; r0 += ART) {
    load_tiles(r0);
    __syncthreads();
    double o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = Bs[rr][jb + j];
#pragma unroll 4
    for (int q = 0; q < NB; ++q) {
      const double y = Ys[rr][q];
#pragma unroll
      for (int j = 0; j < 8; ++j) o[j] -= y * W[q][jb + j];
    }
    const int r = r0 + rr;
    if (r < rows) {
      double* dst = B + grow(r) * ldb + cb + jb;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (jb + j < nc) dst[j] = o[j];
    }
    __syncthreads();
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

__global__ void zero_u32_kernel(unsigned* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

int panels_of(int k) { return (int)cdiv(k, NB); }

void launch_panel(hipStream_t s, const QrPanel& p, double* A, int ld, int n, QrWork& w,
                  int panel) {
  double* Tl = w.Tl + (int64_t)panel * QR_MAX_LEAVES * NB * NB;
  double* Yt = w.Yt + (int64_t)panel * QR_MAX_STACK * NB;
  double* Tt = w.Tt + (int64_t)panel * NB * NB;
  unsigned* cnt = w.counter + panel;
  const dim3 grid(p.L);
#define CTM_QR_PANEL(RL, RT)                                                                  \
  qr_panel_kernel<RL, RT><<<grid, QT, 0, s>>>(A, ld, n, p.j0, p.w, p.rpl, p.L, w.Y, w.k, Tl, \
                                               w.S, Yt, Tt, cnt)
  if (p.rpt_leaf == 1 && p.rpt_tree == 1) CTM_QR_PANEL(1, 1);
  else if (p.rpt_leaf == 1) CTM_QR_PANEL(1, 2);
  else if (p.rpt_tree == 1) CTM_QR_PANEL(2, 1);
  else CTM_QR_PANEL(2, 2);
#undef CTM_QR_PANEL
  CTM_LAUNCHED();
}

void launch_apply(hipStream_t s, bool stacked, bool trans, const QrPanel& p, double* B, int ldb,
                  int c0, int c1, int n, const QrWork& w, int panel) {
  if (c1 <= c0) return;
  const dim3 grid(stacked ? 1 : p.L, (unsigned)cdiv(c1 - c0, ACW));
  const double* Y = stacked ? w.Yt + (int64_t)panel * QR_MAX_STACK * NB : w.Y;
  const double* T = stacked ? w.Tt + (int64_t)panel * NB * NB
                            : w.Tl + (int64_t)panel * QR_MAX_LEAVES * NB * NB;
#define CTM_QR_APPLY(ST, TR)                                                                    \
  qr_apply_kernel<ST, TR><<<grid, AT, 0, s>>>(B, ldb, c0, c1, Y, w.k, T, n, p.j0, p.w, p.rpl, \
                                              p.L)
  if (stacked && trans) CTM_QR_APPLY(true, true);
  else if (stacked) CTM_QR_APPLY(true, false);
  else if (trans) CTM_QR_APPLY(false, true);
  else CTM_QR_APPLY(false, false);
#undef CTM_QR_APPLY
  CTM_LAUNCHED();
}

}  // namespace

size_t qr_work_bytes(int n, int k) {
  const int64_t P = panels_of(k);
  const int64_t doubles = (int64_t)n * k + P * QR_MAX_LEAVES * NB * NB + P * QR_MAX_STACK * NB +
                          P * NB * NB + (int64_t)QR_MAX_STACK * NB;
  return (size_t)doubles * sizeof(double) + (size_t)P * sizeof(unsigned) + 256;
}

QrWork qr_work_carve(hipStream_t s, void* p, int n, int k) {
  const int64_t P = panels_of(k);
  QrWork w;
  w.n = n;
  w.k = k;
  double* d = (double*)p;
  w.Y = d;
  d += (int64_t)n * k;
  w.Tl = d;
  d += P * QR_MAX_LEAVES * NB * NB;
  w.Yt = d;
  d += P * QR_MAX_STACK * NB;
  w.Tt = d;
  d += P * NB * NB;
  w.S = d;
  d += (int64_t)QR_MAX_STACK * NB;
  w.counter = (unsigned*)d;
  zero_u32_kernel<<<1, 256, 0, s>>>(w.counter, (int)P);
  CTM_LAUNCHED();
  return w;
}

QrPanel qr_panel_plan(int n, int k, int j0) {
  QrPanel p;
  p.j0 = j0;
  p.w = std::min(NB, k - j0);
  const int m = n - j0;
  p.rpt_leaf = m > 8192 ? 2 : 1;
  const int b = QT * p.rpt_leaf;
  p.L = (int)cdiv(m, b);
  p.rpl = (int)cdiv(m, p.L);
  p.rpt_tree = p.L * p.w > QT ? 2 : 1;
  return p;
}

void householder_qr(hipStream_t s, double* M, int ld, int n, int k, QrWork& w) {
  if (n < k || k < 1) throw std::invalid_argument("householder_qr: needs n >= k >= 1");
  if (n > QR_MAX_ROWS) throw std::invalid_argument("householder_qr: n > 32768");
  if (n > w.n || k != w.k) throw std::invalid_argument("householder_qr: workspace shape mismatch");
  for (int panel = 0, j0 = 0; j0 < k; ++panel, j0 += NB) {
    const QrPanel p = qr_panel_plan(n, k, j0);
    launch_panel(s, p, M, ld, n, w, panel);
    const int c0 = j0 + p.w;
    if (c0 >= k) continue;
    launch_apply(s, false, true, p, M, ld, c0, k, n, w, panel);
    if (p.L > 1) launch_apply(s, true, true, p, M, ld, c0, k, n, w, panel);
  }
}

void householder_form_q(hipStream_t s, const QrWork& w, int n, int k, double* Q, int ldq) {
  fill_eye_kernel<<<(unsigned)std::min<int64_t>(4096, cdiv((int64_t)n * k, 256)), 256, 0, s>>>(
      Q, n, k, ldq);
  CTM_LAUNCHED();
  for (int panel = panels_of(k) - 1; panel >= 0; --panel) {
    const QrPanel p = qr_panel_plan(n, k, panel * NB);
    if (p.L > 1) launch_apply(s, true, false, p, Q, ldq, p.j0, k, n, w, panel);
    launch_apply(s, false, false, p, Q, ldq, p.j0, k, n, w, panel);
  }
}

}  // namespace ctm
