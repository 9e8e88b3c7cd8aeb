// Blocked Householder QR (FP64) for tall-skinny matrices, with each panel
// factored as a tall-skinny QR (TSQR) over row blocks.
//
// Panel kernel: one workgroup of 256 threads (one wavefront per SIMD) per
// leaf holds its row block of the panel in registers, RPT rows per thread,
// and runs the Householder column loop.  The register window rotates: the
// columns are processed four at a time at fixed register positions 0..3, and
// after each group the finished columns (reflectors below the diagonal, R on
// and above it) are written out and the window shifts by four.  Per column a
// single reduction gives, for the rows below the pivot, the column's squared
// norm and its inner products with the later columns; it is a
// reduce-scatter across the 64 lanes of a wavefront (permlane swaps across
// the 32- and 16-lane halves, DPP within rows of 16), then one LDS pass
// across the four wavefronts.  The reflector follows LAPACK's dlarfg
// (beta = -sign(x0) ||x||); an already-zero column gets the reflector
// I - 2 e e^T, which keeps every reflector's tau in [1, 2].  The compact WY
// factor comes from the Gram matrix of the reflectors (Joffrain, Low,
// Quintana-Orti, van de Geijn, van Zee, ACM TOMS 32 (2006)):
// T^{-1} = diag(1/tau) + strictly-upper(Y^T Y), the Gram matrix on the
// matrix cores, the triangular inverse by one wavefront.  Leaves write their
// triangular factors to a stack; the last leaf to finish (atomic counter,
// no waiting) factors the stack in the same way.
//
// Apply kernel: B <- (I - Y op(T) Y^T) B on a range of columns, per leaf
// (row block) or on the stacked rows, 16 columns and 16 wavefronts per
// workgroup: W = Y^T B, W <- op(T) W, B <- B - Y W on the FP64 matrix cores.
#include "qr.hpp"

namespace ctm {

namespace {

constexpr int QT = 256;  // threads of the panel workgroups
constexpr int QW = QT / 64;

typedef double d4v __attribute__((ext_vector_type(4)));

template <int NBT>
struct QrShared {
  double red[2][QW][NBT];   // per-wavefront partial sums per window position
  double piv[2][NBT];       // pivot row
  double tau[NBT];
  double G[NBT][NBT + 1];   // Gram matrix of the reflectors
  double Gp[QW][NBT][NBT + 1];
  int last;
};

__device__ __forceinline__ unsigned lo32(double v) {
  return (unsigned)__builtin_bit_cast(unsigned long long, v);
}
__device__ __forceinline__ unsigned hi32(double v) {
  return (unsigned)(__builtin_bit_cast(unsigned long long, v) >> 32);
}
__device__ __forceinline__ double mk64(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Exchange across the two halves of the wavefront (lanes l and l^32) or of
// each 32-lane half (l and l^16): with x the value of the lower index half
// and y that of the upper, the permlane swaps leave in every lane its own
// kept value plus its partner's copy of it, so the sum is the pair sum of
// the half the lane keeps (lower half if the lane's bit is 0).
__device__ __forceinline__ double pair_sum32(double x, double y) {
  const auto l = __builtin_amdgcn_permlane32_swap(lo32(x), lo32(y), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi32(x), hi32(y), false, false);
  return mk64(l[0], h[0]) + mk64(l[1], h[1]);
}
__device__ __forceinline__ double pair_sum16(double x, double y) {
  const auto l = __builtin_amdgcn_permlane16_swap(lo32(x), lo32(y), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi32(x), hi32(y), false, false);
  return mk64(l[0], h[0]) + mk64(l[1], h[1]);
}

// Value of the partner lane within a row of 16 lanes through DPP: row_ror:8
// (partner l^8), row_half_mirror (partner 7-l within 8: differs in bit 2),
// quad_perm [2,3,0,1] (l^2) and [1,0,3,2] (l^1).
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const int l = __builtin_amdgcn_update_dpp(0, (int)lo32(v), CTRL, 0xF, 0xF, false);
  const int h = __builtin_amdgcn_update_dpp(0, (int)hi32(v), CTRL, 0xF, 0xF, false);
  return mk64((unsigned)l, (unsigned)h);
}

// Value of lane k (uniform) of v, in every lane.
__device__ __forceinline__ double bcast64(double v, int k) {
  return mk64((unsigned)__builtin_amdgcn_readlane((int)lo32(v), k),
              (unsigned)__builtin_amdgcn_readlane((int)hi32(v), k));
}

template <int N, int CTRL>
__device__ __forceinline__ void rs_halve(const double (&in)[2 * N], double (&out)[N], bool up) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double keep = up ? in[j + N] : in[j], send = up ? in[j] : in[j + N];
    out[j] = keep + dpp64<CTRL>(send);
  }
}

// Reduce-scatter of NBT per-lane values f[0..NBT) over the wavefront.  On
// return every lane holds the wavefront sum of index rs_index<NBT>(lane).
template <int NBT>
__device__ __forceinline__ int rs_index(int lane) {
  if constexpr (NBT == 32)
    return ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 +
           ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
  else
    return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
           ((lane >> 2) & 1);
}
// Lanes holding a distinct index (the others hold copies).
template <int NBT>
__device__ __forceinline__ bool rs_writer(int lane) {
  return NBT == 32 ? (lane & 1) == 0 : (lane & 3) == 0;
}

// Column at window position P (absolute column c) of the local Householder
// QR; rows t = tid + r * QT held in a[r][*].
template <int NBT, int RPT, int P>
__device__ __forceinline__ void qr_column(double (&a)[RPT][NBT], int c, QrShared<NBT>& sh,
                                          int tid) {
  const int lane = tid & 63, wid = tid >> 6;
  const int buf = c & 1;
  double x[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) x[r] = tid + r * QT > c ? a[r][P] : 0.0;
  double hsum;
  if constexpr (NBT == 32) {
    double h16[16], h8[8], h4[4], h2[2], h1[1];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double lo = 0.0, hi = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        if (j >= P) lo += x[r] * a[r][j];
        hi += x[r] * a[r][j + 16];
      }
      h16[j] = pair_sum32(lo, hi);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) h8[j] = pair_sum16(h16[j], h16[j + 8]);
    rs_halve<4, 0x128>(h8, h4, lane & 8);
    rs_halve<2, 0x141>(h4, h2, lane & 4);
    rs_halve<1, 0x4E>(h2, h1, lane & 2);
    hsum = h1[0] + dpp64<0xB1>(h1[0]);
  } else {
    double h8[8], h4[4], h2[2], h1[1];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      double lo = 0.0, hi = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        if (j >= P) lo += x[r] * a[r][j];
        hi += x[r] * a[r][j + 8];
      }
      h8[j] = pair_sum32(lo, hi);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) h4[j] = pair_sum16(h8[j], h8[j + 4]);
    rs_halve<2, 0x128>(h4, h2, lane & 8);
    rs_halve<1, 0x141>(h2, h1, lane & 4);
    hsum = h1[0] + dpp64<0x4E>(h1[0]);
    hsum = hsum + dpp64<0xB1>(hsum);
  }
  if (rs_writer<NBT>(lane)) sh.red[buf][wid][rs_index<NBT>(lane)] = hsum;
  const bool pivot = tid == c;
  if (pivot) {
#pragma unroll
    for (int q = 0; q < NBT; ++q) sh.piv[buf][q] = a[0][q];
  }
  __syncthreads();
  // Every wavefront forms the full sums itself: lane k < NBT holds the sum and
  // the pivot row value of window position k; the rest is read by broadcast.
  const int kl = lane & (NBT - 1);
  double f = 0.0;
#pragma unroll
  for (int v = 0; v < QW; ++v) f += sh.red[buf][v][kl];
  const double pk = sh.piv[buf][kl];
  const double x0 = bcast64(pk, P), sigma = bcast64(f, P);
  double beta, tau, scale;
  if (sigma == 0.0) {
    tau = 2.0;
    beta = -x0;
    scale = 0.0;
  } else {
    const double nrm = sqrt(x0 * x0 + sigma);
    beta = x0 >= 0.0 ? -nrm : nrm;
    tau = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
  }
  if (tid == 0) sh.tau[c & (NBT - 1)] = tau;
  const double wlane = pk + scale * f;  // v^T a_k for k = lane
  // reflector entries of this thread's rows: x scale below the pivot, 1 on
  // it, 0 above
  double tv[RPT], v[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    v[r] = x[r] * scale;
    if (r == 0 && pivot) v[r] = 1.0;
    tv[r] = tau * v[r];
  }
  // later columns: a_k -= tau v (v^T a_k)
#pragma unroll
  for (int k = P + 1; k < NBT; ++k) {
    const double wk = bcast64(wlane, k);
#pragma unroll
    for (int r = 0; r < RPT; ++r) a[r][k] -= tv[r] * wk;
  }
  // column c: the reflector below the pivot, beta on it
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    if (tid + r * QT > c) a[r][P] = v[r];
  if (pivot) a[0][P] = beta;
}

// Local Householder QR of m rows x w columns held in registers.  Writes the
// reflectors to Y (m x w, unit diagonal, zeros above; leading dimension
// ldy), R to Rd (w x w upper triangle, zeros below; leading dimension ldr)
// and the compact WY factor to Tout (NBT x NBT, zero outside w x w).
template <int NBT, int RPT>
__device__ __forceinline__ void local_qr(double (&a)[RPT][NBT], int m, int w, QrShared<NBT>& sh,
                                         int tid, double* __restrict__ Y, int64_t ldy,
                                         double* __restrict__ Rd, int64_t ldr,
                                         double* __restrict__ Tout) {
#pragma unroll 1
  for (int c0 = 0; c0 < w; c0 += 4) {
    qr_column<NBT, RPT, 0>(a, c0, sh, tid);
    if (c0 + 1 < w) qr_column<NBT, RPT, 1>(a, c0 + 1, sh, tid);
    if (c0 + 2 < w) qr_column<NBT, RPT, 2>(a, c0 + 2, sh, tid);
    if (c0 + 3 < w) qr_column<NBT, RPT, 3>(a, c0 + 3, sh, tid);
    // write out the four finished columns, then shift the window
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int t = tid + r * QT;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int c = c0 + p;
        if (c < w && t < m) {
          Y[(int64_t)t * ldy + c] = t > c ? a[r][p] : (t == c ? 1.0 : 0.0);
          if (t < w) Rd[(int64_t)t * ldr + c] = t <= c ? a[r][p] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q + 4 < NBT; ++q) a[r][q] = a[r][q + 4];
#pragma unroll
      for (int q = NBT - 4; q < NBT; ++q) a[r][q] = 0.0;
    }
  }
  __syncthreads();  // Y written by this workgroup is read back below
  // Gram matrix G = Y^T Y on the matrix cores: 16x16 tiles (ti, tj), ti <= tj;
  // wavefront wid takes the 4-row steps k0 = 4 (wid + QW s).
  const int lane = tid & 63, wid = tid >> 6, i16 = lane & 15, grp = lane >> 4;
  constexpr int NT = NBT / 16;
  d4v acc[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
  // The loads of a batch of steps are all issued before its products (Y was
  // just written, so each load is a full trip to the L2).
  constexpr int KB = 8;
  for (int kb = 4 * wid; kb < m; kb += 4 * QW * KB) {
    double y[KB][NT];
#pragma unroll
    for (int s = 0; s < KB; ++s) {
      const int t = kb + 4 * QW * s + grp;
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const int q = 16 * i + i16;
        y[s][i] = (t < m && q < w) ? Y[(int64_t)t * ldy + q] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < KB; ++s) {
      if (kb + 4 * QW * s < m) {
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
          for (int j = i; j < NT; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[s][i], y[s][j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // result layout: register e of lane (grp, i16) holds row 4 e + grp, column i16
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = i; j < NT; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) sh.Gp[wid][16 * i + 4 * e + grp][16 * j + i16] = acc[i][j][e];
  __syncthreads();
  for (int idx = tid; idx < NBT * NBT; idx += QT) {
    const int i = idx / NBT, j = idx % NBT;
    double g = 0.0;
#pragma unroll
    for (int v = 0; v < QW; ++v) g += sh.Gp[v][i][j];
    sh.G[i][j] = g;  // valid for i, j in the computed (upper) tiles
  }
  __syncthreads();
  // T = (diag(1/tau) + strictly-upper(G))^{-1}, by back substitution with
  // one column of T per lane of wavefront 0.
  if (tid < 64) {
    const int j = tid;
    double tc[NBT];
#pragma unroll
    for (int i = NBT - 1; i >= 0; --i) {
      double s0 = i == j ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
      for (int k = i + 1; k < NBT; ++k) {
        if ((k - i) & 1) s0 -= sh.G[i][k] * tc[k];
        else s1 -= sh.G[i][k] * tc[k];
      }
      tc[i] = (i < w && j < w && i <= j) ? sh.tau[i] * (s0 + s1) : 0.0;
    }
    if (j < NBT) {
#pragma unroll
      for (int i = 0; i < NBT; ++i) Tout[i * NBT + j] = tc[i];
    }
  }
}

template <int NBT, int RL, int RT>
__global__ __launch_bounds__(QT) void qr_panel_kernel(double* __restrict__ A, int ld, int n, int j0,
                                                      int w, int rpl, int L, double* __restrict__ Y,
                                                      int ldy, double* __restrict__ Tl,
                                                      double* __restrict__ S, double* __restrict__ Yt,
                                                      double* __restrict__ Tt,
                                                      unsigned* __restrict__ counter) {
  __shared__ QrShared<NBT> sh;
  const int tid = threadIdx.x, leaf = blockIdx.x;
  const int r0 = j0 + leaf * rpl;
  const int m = min(rpl, n - r0);
  {
    double a[RL][NBT];
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int t = tid + r * QT;
      const double* row = A + (int64_t)(r0 + t) * ld + j0;
#pragma unroll
      for (int q = 0; q < NBT; ++q) a[r][q] = (t < m && q < w) ? row[q] : 0.0;
    }
    double* Rd = L == 1 ? A + (int64_t)r0 * ld + j0 : S + (int64_t)leaf * w * NBT;
    const int64_t ldr = L == 1 ? ld : NBT;
    local_qr<NBT, RL>(a, m, w, sh, tid, Y + (int64_t)r0 * ldy + j0, ldy, Rd, ldr,
                      Tl + (int64_t)leaf * NBT * NBT);
  }
  if (L == 1) return;
  // Publish the stacked factor; the last leaf to arrive factors the stack.
  __threadfence();
  __syncthreads();
  if (tid == 0) sh.last = atomicAdd(counter, 1u) == (unsigned)(L - 1);
  __syncthreads();
  if (!sh.last) return;
  __threadfence();
  const int Sm = L * w;
  double b[RT][NBT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int t = tid + r * QT;
#pragma unroll
    for (int q = 0; q < NBT; ++q) b[r][q] = (t < Sm && q < w) ? S[(int64_t)t * NBT + q] : 0.0;
  }
  local_qr<NBT, RT>(b, Sm, w, sh, tid, Yt, NBT, A + (int64_t)j0 * ld + j0, ld, Tt);
  if (tid == 0) atomicExch(counter, 0u);
}

constexpr int AT = 1024;  // threads of the apply workgroups (16 wavefronts)
constexpr int AW = AT / 64;
constexpr int ACW = 16;   // columns per workgroup

// B <- (I - Y op(T) Y^T) B on columns [c0, c1), op(T) = T^T if TRANS, on the
// FP64 matrix cores (16x16x4).  Leaf mode (STACKED = false): workgroup x
// handles leaf x, rows [j0 + x rpl, ...) of B, reflectors Y[row][j0 + q]
// (leading dimension ldy), T = Tsrc + x NBT^2.  Stacked mode: the L*w stacked
// rows (leaf i, offset t) -> row j0 + i rpl + t, reflectors
// Ysrc[(i w + t) NBT + q], T = Tsrc.  Each workgroup owns 16 columns:
//   W = Y^T B (NBT x 16): the wavefronts split the rows, partial tiles are
//       summed in LDS in a fixed order;
//   W <- op(T) W;
//   B <- B - Y W: 16-row tiles distributed over the wavefronts.
template <int NBT, bool STACKED, bool TRANS>
__global__ __launch_bounds__(AT) void qr_apply_kernel(double* __restrict__ B, int ldb, int c0, int c1,
                                                      const double* __restrict__ Ysrc, int ldy,
                                                      const double* __restrict__ Tsrc, int n, int j0,
                                                      int w, int rpl, int L) {
  constexpr int NT = NBT / 16;
  __shared__ double Wp[AW][NBT][ACW + 1];
  __shared__ double W[NBT][ACW + 1];
  __shared__ double Tsh[NBT][NBT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i16 = lane & 15, grp = lane >> 4;
  int rows, rbase = 0;
  const double* Yb;
  const double* T;
  int64_t ys;
  if (STACKED) {
    rows = L * w;
    Yb = Ysrc;
    ys = NBT;
    T = Tsrc;
  } else {
    rbase = j0 + blockIdx.x * rpl;
    rows = min(rpl, n - rbase);
    Yb = Ysrc + (int64_t)rbase * ldy + j0;
    ys = ldy;
    T = Tsrc + (int64_t)blockIdx.x * NBT * NBT;
  }
  const int cb = c0 + blockIdx.y * ACW;
  const int col = cb + i16;
  const bool colok = col < c1;
  auto grow = [&](int r) -> int64_t {
    return STACKED ? (int64_t)(j0 + (r / w) * rpl + r % w) : (int64_t)(rbase + r);
  };
  auto yat = [&](int r, int q) -> double {
    return (r < rows && q < w) ? Yb[(int64_t)r * ys + q] : 0.0;
  };
  auto bat = [&](int r) -> double { return (r < rows && colok) ? B[grow(r) * ldb + col] : 0.0; };
  for (int i = tid; i < NBT * NBT; i += AT) Tsh[i / NBT][i % NBT] = T[i];

  // W = Y^T B: wavefront wv takes the 4-row steps k0 = 4 (wv + AW s); the
  // loads of a batch of steps are issued before its products.
  d4v acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
  constexpr int KB = 8;  // steps per batch
  for (int k0 = 4 * wv; k0 < rows; k0 += 4 * AW * KB) {
    double yb[KB][NT], bb[KB];
#pragma unroll
    for (int it = 0; it < KB; ++it) {
      const int r = k0 + 4 * AW * it + grp;
      bb[it] = bat(r);
#pragma unroll
      for (int t = 0; t < NT; ++t) yb[it][t] = yat(r, 16 * t + i16);
    }
#pragma unroll
    for (int it = 0; it < KB; ++it)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[it][t], bb[it], acc[t], 0, 0, 0);
  }
  // result layout: register e of lane (grp, i16) holds row 4 e + grp, column i16
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) Wp[wv][16 * t + 4 * e + grp][i16] = acc[t][e];
  __syncthreads();
  if (tid < NBT * ACW) {
    const int q = tid / ACW, j = tid % ACW;
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < AW; ++v) s += Wp[v][q][j];
    W[q][j] = s;
  }
  __syncthreads();
  // W <- op(T) W (T upper triangular, zeros below the diagonal)
  double w2 = 0.0;
  if (tid < NBT * ACW) {
    const int q = tid / ACW, j = tid % ACW;
#pragma unroll
    for (int p = 0; p < NBT; ++p) w2 += (TRANS ? Tsh[p][q] : Tsh[q][p]) * W[p][j];
  }
  __syncthreads();
  if (tid < NBT * ACW) W[tid / ACW][tid % ACW] = w2;
  __syncthreads();
  // B <- B - Y W on 16-row tiles: A operand Y[r0 + i16][k], B operand W[k][i16]
  double wop[NBT / 4];
#pragma unroll
  for (int s = 0; s < NBT / 4; ++s) wop[s] = W[4 * s + grp][i16];
  for (int r0 = 16 * wv; r0 < rows; r0 += 16 * AW) {
    double ya[NBT / 4], bo[4];
#pragma unroll
    for (int s = 0; s < NBT / 4; ++s) ya[s] = yat(r0 + i16, 4 * s + grp);
#pragma unroll
    for (int e = 0; e < 4; ++e) bo[e] = bat(r0 + 4 * e + grp);
    d4v acc3 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NBT / 4; ++s)
      acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[s], wop[s], acc3, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = r0 + 4 * e + grp;
      if (r < rows && colok) B[grow(r) * ldb + col] = bo[e] - acc3[e];
    }
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

int nb_of(int n) { return n > 8192 ? 16 : 32; }
int panels_of(int n, int k) { return (int)cdiv(k, nb_of(n)); }
int max_panels(int k) { return (int)cdiv(k, 16); }

// Offsets of panel `panel` in the per-panel workspace arrays.
double* tl_of(const QrWork& w, int nb, int panel) {
  return w.Tl + (int64_t)panel * QR_MAX_LEAVES * nb * nb;
}
double* yt_of(const QrWork& w, int nb, int panel) {
  return w.Yt + (int64_t)panel * QR_MAX_LEAVES * nb * nb;
}
double* tt_of(const QrWork& w, int nb, int panel) { return w.Tt + (int64_t)panel * nb * nb; }

void launch_panel(hipStream_t s, const QrPanel& p, double* A, int ld, int n, QrWork& w,
                  int panel) {
  double* Tl = tl_of(w, p.nb, panel);
  double* Yt = yt_of(w, p.nb, panel);
  double* Tt = tt_of(w, p.nb, panel);
  unsigned* cnt = w.counter + panel;
  const dim3 grid(p.L);
#define CTM_QR_PANEL(NBT, RL, RT)                                                            \
  qr_panel_kernel<NBT, RL, RT><<<grid, QT, 0, s>>>(A, ld, n, p.j0, p.w, p.rpl, p.L, w.Y, w.k, \
                                                    Tl, w.S, Yt, Tt, cnt)
  if (p.nb == 32) {
    if (p.rpt_leaf == 1) CTM_QR_PANEL(32, 1, 1);
    else if (p.rpt_tree == 1) CTM_QR_PANEL(32, 2, 1);
    else CTM_QR_PANEL(32, 2, 2);
  } else {
    if (p.rpt_tree == 1) CTM_QR_PANEL(16, 4, 1);
    else CTM_QR_PANEL(16, 4, 2);
  }
#undef CTM_QR_PANEL
  CTM_LAUNCHED();
}

template <int NBT>
void launch_apply_nb(hipStream_t s, bool stacked, bool trans, const QrPanel& p, double* B, int ldb,
                     int c0, int c1, int n, const QrWork& w, int panel) {
  const dim3 grid(stacked ? 1 : p.L, (unsigned)cdiv(c1 - c0, ACW));
  const double* Y = stacked ? yt_of(w, NBT, panel) : w.Y;
  const double* T = stacked ? tt_of(w, NBT, panel) : tl_of(w, NBT, panel);
#define CTM_QR_APPLY(ST, TR)                                                                  \
  qr_apply_kernel<NBT, ST, TR><<<grid, AT, 0, s>>>(B, ldb, c0, c1, Y, w.k, T, n, p.j0, p.w, \
                                                   p.rpl, p.L)
  if (stacked && trans) CTM_QR_APPLY(true, true);
  else if (stacked) CTM_QR_APPLY(true, false);
  else if (trans) CTM_QR_APPLY(false, true);
  else CTM_QR_APPLY(false, false);
#undef CTM_QR_APPLY
  CTM_LAUNCHED();
}

void launch_apply(hipStream_t s, bool stacked, bool trans, const QrPanel& p, double* B, int ldb,
                  int c0, int c1, int n, const QrWork& w, int panel) {
  if (c1 <= c0) return;
  if (p.nb == 32) launch_apply_nb<32>(s, stacked, trans, p, B, ldb, c0, c1, n, w, panel);
  else launch_apply_nb<16>(s, stacked, trans, p, B, ldb, c0, c1, n, w, panel);
}

}  // namespace

// Per-panel arrays are sized for the larger of the two panel widths:
// ceil(k/16) panels of width 16 need at most as much as ceil(k/32) of 32.
size_t qr_work_bytes(int n, int k) {
  const int64_t P = max_panels(k);
  const int64_t per_panel = (int64_t)QR_MAX_LEAVES * QR_NB_MAX * QR_NB_MAX;
  const int64_t doubles = (int64_t)n * k + 2 * P * per_panel + P * QR_NB_MAX * QR_NB_MAX +
                          (int64_t)QR_MAX_STACK * QR_NB_MAX;
  return (size_t)doubles * sizeof(double) + (size_t)P * sizeof(unsigned) + 256;
}

QrWork qr_work_carve(hipStream_t s, void* p, int n, int k) {
  const int64_t P = max_panels(k);
  const int64_t per_panel = (int64_t)QR_MAX_LEAVES * QR_NB_MAX * QR_NB_MAX;
  QrWork w;
  w.n = n;
  w.k = k;
  double* d = (double*)p;
  w.Y = d;
  d += (int64_t)n * k;
  w.Tl = d;
  d += P * per_panel;
  w.Yt = d;
  d += P * per_panel;
  w.Tt = d;
  d += P * QR_NB_MAX * QR_NB_MAX;
  w.S = d;
  d += (int64_t)QR_MAX_STACK * QR_NB_MAX;
  w.counter = (unsigned*)d;
  zero_u32_kernel<<<1, 256, 0, s>>>(w.counter, (int)P);
  CTM_LAUNCHED();
  return w;
}

QrPanel qr_panel_plan(int n, int k, int j0) {
  QrPanel p;
  p.nb = nb_of(n);
  p.j0 = j0;
  p.w = std::min(p.nb, k - j0);
  const int m = n - j0;
  p.rpt_leaf = p.nb == 32 ? (m <= QT ? 1 : 2) : 4;
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
  const int nb = nb_of(n);
  for (int panel = 0, j0 = 0; j0 < k; ++panel, j0 += nb) {
    const QrPanel p = qr_panel_plan(n, k, j0);
    if (p.L > QR_MAX_LEAVES || p.L * p.w > QT * 2 || p.rpl < p.w)
      throw std::logic_error("householder_qr: bad panel plan");
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
  for (int panel = panels_of(n, k) - 1; panel >= 0; --panel) {
    const QrPanel p = qr_panel_plan(n, k, panel * nb_of(n));
    if (p.L > 1) launch_apply(s, true, false, p, Q, ldq, p.j0, k, n, w, panel);
    launch_apply(s, false, false, p, Q, ldq, p.j0, k, n, w, panel);
  }
}

}  // namespace ctm
