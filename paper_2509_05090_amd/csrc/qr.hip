// Blocked Householder QR (FP64) for tall-skinny matrices, with each panel
// factored as a tall-skinny QR (TSQR) over row blocks.
//
// Panel kernel: one workgroup of four wavefronts (one per SIMD) per leaf
// holds its row block of the panel in registers and runs the Householder
// column loop.  In each wavefront, lane 16 g + i holds column i (and i + 16)
// of the rows in row group g.  Per column, the pivot column below the
// diagonal goes to every lane of its row group through wavefront-private
// LDS; each lane forms its partial inner products with its columns (which
// give the column's squared norm and its products with the other columns),
// sums them over the four row groups with permlane swaps and over the
// wavefronts through one LDS pass, and applies the reflector to its rows.
// The reflector follows LAPACK's dlarfg (beta = -sign(x0) ||x||); an
// already-zero column gets the reflector I - 2 e e^T, which keeps every
// reflector's tau in [1, 2].  The compact WY factor comes from the Gram
// matrix of the reflectors (Joffrain, Low, Quintana-Orti, van de Geijn, van
// Zee, ACM TOMS 32 (2006)): T^{-1} = diag(1/tau) + strictly-upper(Y^T Y),
// the Gram matrix assembled from the same inner products, the triangular
// inverse by one wavefront.  Leaves write their triangular factors to a
// stack; the last leaf to finish (atomic counter, no waiting) factors the
// stack in the same way.
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

constexpr int QTR_MAX = 64;  // most register rows per lane group

template <int NBT>
struct __attribute__((aligned(16))) QrShared {
  alignas(16) double xs[QW][4][QTR_MAX];  // per wavefront and row group: the pivot column
  double red[2][QW][NBT];     // per-wavefront partial dots (by column parity)
  double piv[2][NBT];         // pivot row (by column parity)
  double R[NBT][NBT + 1];     // rows of R as they are finished
  double G[NBT][NBT + 1];     // Gram matrix of the reflectors (strictly upper part)
  double tau[NBT];
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

// Sum of v over lanes l and l^32 (permlane32 swap), resp. l and l^16
// (permlane16 swap), in every lane.
__device__ __forceinline__ double sum_x32(double v) {
  const auto l = __builtin_amdgcn_permlane32_swap(lo32(v), lo32(v), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi32(v), hi32(v), false, false);
  return mk64(l[0], h[0]) + mk64(l[1], h[1]);
}
__device__ __forceinline__ double sum_x16(double v) {
  const auto l = __builtin_amdgcn_permlane16_swap(lo32(v), lo32(v), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi32(v), hi32(v), false, false);
  return mk64(l[0], h[0]) + mk64(l[1], h[1]);
}

// Register layout of a row block of at most 16 TR rows held by the 256
// threads: lane l = 16 g + i of wavefront v holds, in a[t][h], row
// 16 t + 4 v + g (t < TR) of column i + 16 h (h < NBT / 16).  A column is
// then spread over the 4 row groups g and the 4 wavefronts, a row over the
// 16 lanes i of a row group.  Rows 0 .. NBT-1 (the diagonal block) are in
// registers t < NBT / 16 of every wavefront, so the per-column work on the
// diagonal block (masking the pivot column, picking the pivot row) is
// spread over the wavefronts instead of lengthening one of them.
template <int NBT>
constexpr int slots_of() { return NBT / 16; }

// Householder step for column k (slot H = k / 16) of the row block.
//   - lanes holding column k publish it below the diagonal (x, zero at and
//     above row k) through wavefront-private LDS; every lane reads the
//     values of its own row group;
//   - partial dots x . a_c over the lane's rows, summed over the 4 row groups
//     of the wavefront (permlane swaps), then over the wavefronts through
//     LDS: one barrier per column;
//   - the reflector follows LAPACK's dlarfg (beta = -sign(x0) ||(x0, x)||,
//     v = (1, x / (x0 - beta)), tau = (beta - x0) / beta); a column that is
//     already zero below the diagonal gets I - 2 e e^T (tau = 2);
//   - row k of R is final and goes to LDS; rows below are updated,
//     a_c -= tau v (v . a_c) for the later columns c; the earlier columns and
//     column k itself keep their values (column k keeps x, the reflector up
//     to its scale);
//   - v_c . v_k = scale_c w_c for the earlier columns c, where w_c = v . a_c,
//     so the Gram matrix of the reflectors is filled in on the way.
template <int NBT, int TR, int H>
__device__ __forceinline__ void qr_column(double (&a)[TR][NBT / 16], double (&sc)[NBT / 16],
                                          int k, QrShared<NBT>& sh) {
  constexpr int SL = NBT / 16;
  constexpr int TD = NBT / 16;  // registers holding rows of the diagonal block
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
  const int g = lane >> 4, i = lane & 15;
  const int par = k & 1;
  // 1. the pivot column below the diagonal, to the lanes of each row group
  //    (rows at or above the pivot are in registers t < TD)
  if (i == (k & 15)) {
#pragma unroll
    for (int t = 0; t < TR; t += 2) {
      double x0 = a[t][H], x1 = a[t + 1][H];
      if (t < TD && 16 * t + 4 * v + g <= k) x0 = 0.0;
      if (t + 1 < TD && 16 * (t + 1) + 4 * v + g <= k) x1 = 0.0;
      *(double2*)&sh.xs[v][g][t] = double2{x0, x1};
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double x[TR];
#pragma unroll
  for (int t = 0; t < TR; t += 2) {
    const double2 p = *(const double2*)&sh.xs[v][g][t];
    x[t] = p.x;
    x[t + 1] = p.y;
  }
  // 2. partial dots with the lane's columns, summed over the wavefront
  double d[SL];
#pragma unroll
  for (int h = 0; h < SL; ++h) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int t = 0; t < TR; t += 2) {
      s0 += x[t] * a[t][h];
      s1 += x[t + 1] * a[t + 1][h];
    }
    d[h] = sum_x16(sum_x32(s0 + s1));
  }
  if (g == 0) {
#pragma unroll
    for (int h = 0; h < SL; ++h) sh.red[par][v][i + 16 * h] = d[h];
  }
  // the pivot row (row k: wavefront (k >> 2) & 3, row group k & 3,
  // register k >> 4)
  if (v == ((k >> 2) & 3) && g == (k & 3)) {
    const int tk = k >> 4;
#pragma unroll
    for (int h = 0; h < SL; ++h) {
      double pv = a[0][h];
#pragma unroll
      for (int t = 1; t < TD; ++t)
        if (t == tk) pv = a[t][h];
      sh.piv[par][i + 16 * h] = pv;
    }
  }
  __syncthreads();
  // 3. full dots of the lane's columns and the reflector
  double f[SL], p[SL];
#pragma unroll
  for (int h = 0; h < SL; ++h) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < QW; ++u) s += sh.red[par][u][i + 16 * h];
    f[h] = s;
    p[h] = sh.piv[par][i + 16 * h];
  }
  double sigma = 0.0;
#pragma unroll
  for (int u = 0; u < QW; ++u) sigma += sh.red[par][u][k];
  const double x0 = sh.piv[par][k];
  // beta, tau, the reflector's scale 1 / (x0 - beta) and tau scale = -1 / beta.
  // With y = 1 / ||(x0, x)||: tau = 1 + |x0| y, tau scale = sign(x0) y and
  // scale = sign(x0) / (|x0| + ||(x0, x)||); y and the reciprocal come from
  // the hardware estimates refined by two Newton steps each.  Outside a safe
  // exponent range (a uniform branch) the library square root and divisions.
  double beta, tau, scale, ts;
  const double s2 = fma(x0, x0, sigma);
  if (sigma == 0.0) {
    tau = 2.0;
    beta = -x0;
    scale = 0.0;
    ts = 0.0;
  } else if (s2 >= 0x1p-960 && s2 <= 0x1p960) {
    double y = __builtin_amdgcn_rsq(s2);
    double e = fma(-s2 * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-s2 * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    const double nrm = s2 * y, ax = fabs(x0);
    const double d = ax + nrm;
    double r = __builtin_amdgcn_rcp(d);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    const bool pos = x0 >= 0.0;
    beta = pos ? -nrm : nrm;
    tau = fma(ax, y, 1.0);
    scale = pos ? r : -r;
    ts = pos ? y : -y;
  } else {
    const double nrm = sqrt(s2);
    beta = x0 >= 0.0 ? -nrm : nrm;
    tau = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
    ts = tau * scale;
  }
  if (i == (k & 15)) sc[H] = scale;
  double wv[SL], uv[SL];
#pragma unroll
  for (int h = 0; h < SL; ++h) {
    wv[h] = p[h] + scale * f[h];  // v . a_c
    uv[h] = (i + 16 * h > k) ? ts * wv[h] : 0.0;
  }
  // row k of R, column k of the Gram matrix and tau: every wavefront holds
  // these values; the writer rotates over the wavefronts, two away from the
  // one that picked the pivot row
  if (v == (((k >> 2) + 2) & 3) && g == 0) {
#pragma unroll
    for (int h = 0; h < SL; ++h) {
      const int c = i + 16 * h;
      sh.R[k][c] = c > k ? p[h] - tau * wv[h] : (c == k ? beta : 0.0);
      if (c < k) sh.G[c][k] = sc[h] * wv[h];
    }
    if (i == 0) sh.tau[k] = tau;
  }
  // 4. rows below the pivot (x is zero at and above it); slots before H
  //    hold finished columns only
#pragma unroll
  for (int t = 0; t < TR; ++t)
#pragma unroll
    for (int h = H; h < SL; ++h) a[t][h] -= x[t] * uv[h];
}

// Householder QR of a block of m rows x w columns held in registers (layout
// above).  Writes the reflectors to Y (m x w, unit diagonal, zeros above;
// leading dimension ldy), R to Rd (w x w upper triangle, zeros below;
// leading dimension ldr) and the compact WY factor to Tout (NBT x NBT, zero
// outside w x w): T^{-1} = diag(1/tau) + strictly-upper(Y^T Y) (Joffrain,
// Low, Quintana-Orti, van de Geijn, Van Zee, ACM TOMS 32 (2006)).
template <int NBT, int TR>
__device__ __forceinline__ void local_qr(double (&a)[TR][NBT / 16], int m, int w,
                                         QrShared<NBT>& sh, double* __restrict__ Y, int64_t ldy,
                                         double* __restrict__ Rd, int64_t ldr,
                                         double* __restrict__ Tout) {
  constexpr int SL = NBT / 16;
  const int tid = threadIdx.x, lane = tid & 63, v = tid >> 6;
  const int g = lane >> 4, i = lane & 15;
  double sc[SL];
#pragma unroll
  for (int h = 0; h < SL; ++h) sc[h] = 0.0;
  // G is written only for column pairs inside w; the rest must read as zero
  for (int idx = tid; idx < NBT * (NBT + 1); idx += QT) (&sh.G[0][0])[idx] = 0.0;
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < min(w, 16); ++k) qr_column<NBT, TR, 0>(a, sc, k, sh);
  if constexpr (SL == 2) {
#pragma unroll 1
    for (int k = 16; k < w; ++k) qr_column<NBT, TR, 1>(a, sc, k, sh);
  }
  // reflectors: Y[r][c] = scale_c x_c[r] below the diagonal, 1 on it
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int r = 16 * t + 4 * v + g;
#pragma unroll
    for (int h = 0; h < SL; ++h) {
      const int c = i + 16 * h;
      if (r < m && c < w) Y[(int64_t)r * ldy + c] = r > c ? sc[h] * a[t][h] : (r == c ? 1.0 : 0.0);
    }
  }
  __syncthreads();  // R, G and tau complete
  for (int idx = tid; idx < w * w; idx += QT) {
    const int r = idx / w, c = idx % w;
    Rd[(int64_t)r * ldr + c] = sh.R[r][c];
  }
  // T = U^{-1}, U = diag(1/tau) + strictly-upper(G), zero outside w x w.
  if constexpr (NBT == 32) {
    // By 16 x 16 blocks: T11 = U11^{-1} and T22 = U22^{-1} by back
    // substitution (one column per lane, wavefronts 0 and 1 at once), then
    // T12 = -T11 (U12 T22), one element per thread.  The pivot-column
    // staging area (free after the column loop) holds T11, T22 and U12 T22.
    constexpr int HB = 16;
    double* st = &sh.xs[0][0][0];
    if (tid < 128) {
      const int v = tid >> 6, j = tid & 63, o = HB * v;
      if (j < HB) {
        double tc[HB];
#pragma unroll
        for (int ii = HB - 1; ii >= 0; --ii) {
          double s0 = ii == j ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
          for (int kk = ii + 1; kk < HB; ++kk) {
            if ((kk - ii) & 1) s0 -= sh.G[o + ii][o + kk] * tc[kk];
            else s1 -= sh.G[o + ii][o + kk] * tc[kk];
          }
          tc[ii] = (o + ii < w && o + j < w && ii <= j) ? sh.tau[o + ii] * (s0 + s1) : 0.0;
        }
#pragma unroll
        for (int ii = 0; ii < HB; ++ii) {
          st[v * HB * HB + ii * HB + j] = tc[ii];
          Tout[(o + ii) * NBT + o + j] = tc[ii];
          if (v == 1) Tout[(HB + ii) * NBT + j] = 0.0;  // lower-left block
        }
      }
    }
    __syncthreads();
    const int r = tid >> 4, cc = tid & 15;  // 256 threads: one element of a 16 x 16 block
    {
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < HB; ++k) x += sh.G[r][HB + k] * st[HB * HB + k * HB + cc];
      st[2 * HB * HB + r * HB + cc] = x;  // U12 T22
    }
    __syncthreads();
    {
      double t12 = 0.0;
#pragma unroll
      for (int k = 0; k < HB; ++k) t12 -= st[r * HB + k] * st[2 * HB * HB + k * HB + cc];
      Tout[r * NBT + HB + cc] = t12;
    }
  } else if (tid < 64) {
    // one column of T per lane of wavefront 0, by back substitution
    const int j = tid;
    double tc[NBT];
#pragma unroll
    for (int ii = NBT - 1; ii >= 0; --ii) {
      double s0 = ii == j ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
      for (int kk = ii + 1; kk < NBT; ++kk) {
        if ((kk - ii) & 1) s0 -= sh.G[ii][kk] * tc[kk];
        else s1 -= sh.G[ii][kk] * tc[kk];
      }
      tc[ii] = (ii < w && j < w && ii <= j) ? sh.tau[ii] * (s0 + s1) : 0.0;
    }
    if (j < NBT) {
#pragma unroll
      for (int ii = 0; ii < NBT; ++ii) Tout[ii * NBT + j] = tc[ii];
    }
  }
  __syncthreads();  // LDS reused by the next block
}

template <int NBT, int TR>
__device__ __forceinline__ void load_block(double (&a)[TR][NBT / 16], const double* __restrict__ src,
                                           int64_t ld, int m, int w) {
  constexpr int SL = NBT / 16;
  const int lane = threadIdx.x & 63, v = threadIdx.x >> 6;
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int r = 16 * t + 4 * v + g;
#pragma unroll
    for (int h = 0; h < SL; ++h) {
      const int c = i + 16 * h;
      a[t][h] = (r < m && c < w) ? src[(int64_t)r * ld + c] : 0.0;
    }
  }
}

// Panel factorization: workgroup `leaf` factors rows [j0 + leaf rpl, ...) of
// columns [j0, j0 + w) (TRL register rows per lane group); the last leaf to
// finish factors the L stacked w x w triangles (TRT register rows).
template <int NBT, int TRL, int TRT>
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
    double a[TRL][NBT / 16];
    load_block<NBT, TRL>(a, A + (int64_t)r0 * ld + j0, ld, m, w);
    double* Rd = L == 1 ? A + (int64_t)r0 * ld + j0 : S + (int64_t)leaf * w * NBT;
    const int64_t ldr = L == 1 ? ld : NBT;
    local_qr<NBT, TRL>(a, m, w, sh, Y + (int64_t)r0 * ldy + j0, ldy, Rd, ldr,
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
  double b[TRT][NBT / 16];
  load_block<NBT, TRT>(b, S, NBT, Sm, w);
  local_qr<NBT, TRT>(b, Sm, w, sh, Yt, NBT, A + (int64_t)j0 * ld + j0, ld, Tt);
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
// Ysrc[(i w + t) NBT + q], T = Tsrc.  Each workgroup owns 16 columns and at
// most 64 RB rows; lane (g, i) of wavefront v holds B at rows
// 4 v + 64 s + g (s < RB), column i, loaded once:
//   W = Y^T B (NBT x 16): MFMAs over the lane's rows, partial tiles summed
//       in LDS in a fixed order;
//   W <- op(T) W;
//   B <- B - Y W: 16-row tiles made of the lane's own rows s = 4 l .. 4 l + 3
//       (output register e of lane (g, i) is row 4 v + 64 (4 l + e) + g), so
//       B is updated from the registers it was loaded into; the Y operands
//       of this phase are loaded before the reduction of W.
template <int NBT>
constexpr int apply_row_steps() { return NBT == 32 ? 8 : 16; }

template <int NBT, bool STACKED, bool TRANS>
__global__ __launch_bounds__(AT) void qr_apply_kernel(double* __restrict__ B, int ldb, int c0, int c1,
                                                      const double* __restrict__ Ysrc, int ldy,
                                                      const double* __restrict__ Tsrc, int n, int j0,
                                                      int w, int rpl, int L) {
  constexpr int NT = NBT / 16;
  constexpr int RB = apply_row_steps<NBT>();
  constexpr int TL = RB / 4;  // 16-row tiles per lane set
  __shared__ double Wp[AW][NBT][ACW + 1];
  __shared__ double W[NBT][ACW + 1];
  __shared__ double W2[NBT][ACW + 1];
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
  auto lrow = [&](int st) -> int { return 4 * wv + 64 * st + grp; };

  double bb[RB], yb[RB][NT];
#pragma unroll
  for (int st = 0; st < RB; ++st) {
    bb[st] = bat(lrow(st));
#pragma unroll
    for (int t = 0; t < NT; ++t) yb[st][t] = yat(lrow(st), 16 * t + i16);
  }
  for (int i = tid; i < NBT * NBT; i += AT) Tsh[i / NBT][i % NBT] = T[i];

  // W = Y^T B over the lane's rows; result register e of lane (grp, i16)
  // holds W[16 t + 4 e + grp][i16]
  d4v acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < RB; ++st)
#pragma unroll
    for (int t = 0; t < NT; ++t)
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[st][t], bb[st], acc[t], 0, 0, 0);
  // Y operands of the update: tile l, row index i16 -> lane row set
  // 4 wv + 64 (4 l + (i16 >> 2)) + (i16 & 3), reflector 4 s + grp
  double ya[TL][NBT / 4];
#pragma unroll
  for (int l = 0; l < TL; ++l) {
    const int rr = 4 * wv + 64 * (4 * l + (i16 >> 2)) + (i16 & 3);
#pragma unroll
    for (int s = 0; s < NBT / 4; ++s) ya[l][s] = yat(rr, 4 * s + grp);
  }
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
  // W2 = op(T) W (T upper triangular, zeros below the diagonal)
  if (tid < NBT * ACW) {
    const int q = tid / ACW, j = tid % ACW;
    double w2 = 0.0;
#pragma unroll
    for (int p = 0; p < NBT; ++p) w2 += (TRANS ? Tsh[p][q] : Tsh[q][p]) * W[p][j];
    W2[q][j] = w2;
  }
  __syncthreads();
  // B <- B - Y W2 on the lane's rows
  double wop[NBT / 4];
#pragma unroll
  for (int s = 0; s < NBT / 4; ++s) wop[s] = W2[4 * s + grp][i16];
#pragma unroll
  for (int l = 0; l < TL; ++l) {
    d4v acc3 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NBT / 4; ++s)
      acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[l][s], wop[s], acc3, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = lrow(4 * l + e);
      if (r < rows && colok) B[grow(r) * ldb + col] = bb[4 * l + e] - acc3[e];
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
#define CTM_QR_PANEL(NBT, TRL, TRT)                                                             \
  qr_panel_kernel<NBT, TRL, TRT><<<grid, QT, 0, s>>>(A, ld, n, p.j0, p.w, p.rpl, p.L, w.Y, w.k, \
                                                      Tl, w.S, Yt, Tt, cnt)
  if (p.nb == 32) {
    if (p.tr_leaf == 8) CTM_QR_PANEL(32, 8, 8);
    else if (p.tr_leaf == 16) CTM_QR_PANEL(32, 16, 8);
    else if (p.tr_leaf == 24) CTM_QR_PANEL(32, 24, 8);
    else if (p.tr_tree == 8) CTM_QR_PANEL(32, 32, 8);
    else if (p.tr_tree == 16) CTM_QR_PANEL(32, 32, 16);
    else if (p.tr_tree == 24) CTM_QR_PANEL(32, 32, 24);
    else CTM_QR_PANEL(32, 32, 32);
  } else {
    if (p.tr_leaf == 16) CTM_QR_PANEL(16, 16, 16);
    else if (p.tr_leaf == 32) CTM_QR_PANEL(16, 32, 16);
    else if (p.tr_tree == 16) CTM_QR_PANEL(16, 64, 16);
    else CTM_QR_PANEL(16, 64, 32);
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
  const int maxrows = 64 * (p.nb == 32 ? apply_row_steps<32>() : apply_row_steps<16>());
  if ((stacked ? p.L * p.w : p.rpl) > maxrows)
    throw std::logic_error("qr apply: more rows per workgroup than the kernel holds");
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
  // register rows per lane group (a workgroup holds 16 tr rows): the
  // smallest instance that holds the rows
  auto fit = [&](int rows) {
    if (p.nb == 32) return rows <= 128 ? 8 : rows <= 256 ? 16 : rows <= 384 ? 24 : 32;
    return rows <= 256 ? 16 : rows <= 512 ? 32 : 64;
  };
  const int big = p.nb == 32 ? 32 : 64;
  p.tr_leaf = fit(m);
  p.L = p.tr_leaf < big ? 1 : (int)cdiv(m, 16 * big);
  p.rpl = (int)cdiv(m, p.L);
  p.tr_leaf = fit(p.rpl);
  if (p.L > 1 && p.tr_leaf != big) p.tr_leaf = big;  // leaf instances exist for big only
  p.tr_tree = p.L == 1 ? (p.nb == 32 ? 8 : 16) : fit(p.L * p.w);
  return p;
}

void householder_qr(hipStream_t s, double* M, int ld, int n, int k, QrWork& w, int kx) {
  if (kx < 0) kx = k;
  if (n < k || k < 1) throw std::invalid_argument("householder_qr: needs n >= k >= 1");
  if (kx < k || ld < kx) throw std::invalid_argument("householder_qr: needs ld >= kx >= k");
  if (n > QR_MAX_ROWS) throw std::invalid_argument("householder_qr: n > 32768");
  if (n > w.n || k != w.k) throw std::invalid_argument("householder_qr: workspace shape mismatch");
  const int nb = nb_of(n);
  for (int panel = 0, j0 = 0; j0 < k; ++panel, j0 += nb) {
    const QrPanel p = qr_panel_plan(n, k, j0);
    if (p.L > QR_MAX_LEAVES || p.L * p.w > 16 * p.tr_tree || p.rpl > 16 * p.tr_leaf ||
        p.rpl < p.w || (p.nb == 32 && p.tr_tree > 32))
      throw std::logic_error("householder_qr: bad panel plan");
    launch_panel(s, p, M, ld, n, w, panel);
    const int c0 = j0 + p.w;
    if (c0 >= kx) continue;
    launch_apply(s, false, true, p, M, ld, c0, kx, n, w, panel);
    if (p.L > 1) launch_apply(s, true, true, p, M, ld, c0, kx, n, w, panel);
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
