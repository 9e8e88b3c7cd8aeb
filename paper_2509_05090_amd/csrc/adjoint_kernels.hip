// Element-wise, permutation and reduction kernels of the CTMRG adjoint.
#include "adjoint_kernels.hpp"

namespace ctm {

namespace {

constexpr int BT = 1024;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Sum over the block (blockDim.x a multiple of 64, fixed order); every
// thread gets it.
__device__ double block_sum(double v, double* sh) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

__device__ double block_max(double v, double* sh) {
  v = wmax(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = fmax(t, sh[i]);
  __syncthreads();
  return t;
}

inline unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 16384) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, cdiv(n, threads)));
}

// One workgroup per (a, b) row of the input: reads in[a][b][*][*] (C*Dd
// contiguous) and writes Dd-long runs out[a][c][b][*].
__global__ void swap_mid_kernel(const double* __restrict__ in, double* __restrict__ out, int A,
                                int B, int C, int Dd, int acc) {
  const int64_t ab = blockIdx.x;
  const int a = (int)(ab / B), b = (int)(ab % B);
  const double* src = in + ab * C * Dd;
  const int64_t run = (int64_t)C * Dd;
  for (int64_t i = threadIdx.x; i < run; i += blockDim.x) {
    const int c = (int)(i / Dd), d = (int)(i % Dd);
    double* dst = out + (((int64_t)a * C + c) * B + b) * Dd + d;
    *dst = acc ? *dst + src[i] : src[i];
  }
}

__global__ void copyltu_kernel(const double* in, double* out, int k) {
  const int64_t total = (int64_t)k * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / k), c = (int)(i % k);
    out[i] = r >= c ? in[i] : in[(int64_t)c * k + r];
  }
}

// Column j of R^{-1} diag(sgn), one wave per column, k <= 64 S: x = R^{-1} e_j
// lives in registers (lane L holds rows L, L + 64, ...) and is found by
// column back substitution, x_i <- x_i / R_ii then x_l -= R_li x_i for
// l < i, over i = j, ..., 0.  The columns of R are read CH at a time, all
// loads of a chunk in flight together; x_i reaches the wave by readlane.
// Only the upper triangle of R is read (the strict lower part may hold
// anything, e.g. Householder vectors).
template <int S>
__global__ __launch_bounds__(256) void tri_inv_upper_wave_kernel(const double* __restrict__ R,
                                                                 int ldr, int k,
                                                                 const double* __restrict__ sgn,
                                                                 double* __restrict__ out) {
  constexpr int CH = 16;
  const int lane = threadIdx.x & 63;
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (j >= k) return;  // whole wave
  double x[S];
#pragma unroll
  for (int s = 0; s < S; ++s) x[s] = s * 64 + lane == j ? 1.0 : 0.0;
  for (int i0 = j / CH * CH; i0 >= 0; i0 -= CH) {
    double r[CH][S], dinv[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int i = i0 + c;
      const bool live = i <= j;
      dinv[c] = live ? 1.0 / R[(int64_t)i * ldr + i] : 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int row = s * 64 + lane;
        r[c][s] = live && row < i ? R[(int64_t)row * ldr + i] : 0.0;
      }
    }
#pragma unroll
    for (int c = CH - 1; c >= 0; --c) {
      const int i = i0 + c;
      if (i > j) continue;  // uniform
      double xv = x[0];
#pragma unroll
      for (int s = 1; s < S; ++s)
        if ((i >> 6) == s) xv = x[s];
      const unsigned long long bits = __builtin_bit_cast(unsigned long long, xv);
      const unsigned lo = __builtin_amdgcn_readlane((unsigned)bits, i & 63);
      const unsigned hi = __builtin_amdgcn_readlane((unsigned)(bits >> 32), i & 63);
      const double xi =
          __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo) * dinv[c];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int row = s * 64 + lane;
        x[s] = row == i ? xi : fma(-r[c][s], xi, x[s]);  // r = 0 for rows >= i
      }
    }
  }
  const double sj = sgn ? sgn[j] : 1.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int row = s * 64 + lane;
    if (row < k) out[(int64_t)row * k + j] = row <= j ? x[s] * sj : 0.0;
  }
}

// Column j of R^{-1}: back substitution, one thread per column (any k).
__global__ void tri_inv_upper_kernel(const double* __restrict__ R, int ldr, int k,
                                     const double* __restrict__ sgn, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double sj = sgn ? sgn[j] : 1.0;
  for (int i = k - 1; i > j; --i) out[(int64_t)i * k + j] = 0.0;
  for (int i = j; i >= 0; --i) {
    double s = i == j ? 1.0 : 0.0;
    for (int l = i + 1; l <= j; ++l) s -= R[(int64_t)i * ldr + l] * out[(int64_t)l * k + j];
    out[(int64_t)i * k + j] = s / R[(int64_t)i * ldr + i];
  }
  for (int i = 0; i <= j; ++i) out[(int64_t)i * k + j] *= sj;
}

__global__ __launch_bounds__(256) void dot_parts_kernel(const double* __restrict__ a,
                                                        const double* __restrict__ b, int64_t n,
                                                        double* __restrict__ parts) {
  __shared__ double sh[4];
  double t = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    t += a[i] * b[i];
  t = block_sum(t, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void dot_final_kernel(const double* __restrict__ parts, int np,
                                                        double* __restrict__ out) {
  __shared__ double sh[4];
  double t = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) t += parts[i];
  t = block_sum(t, sh);
  if (threadIdx.x == 0) out[0] = t;
}

__global__ void unit_norm_bwd_kernel(const double* __restrict__ g, const double* __restrict__ y,
                                     const double* __restrict__ dot,
                                     const double* __restrict__ nrm, double* __restrict__ out,
                                     int64_t n) {
  const double d = dot[0], inv = 1.0 / nrm[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (g[i] - y[i] * d) * inv;
}

__global__ __launch_bounds__(BT) void corner_fwd_kernel(const double* Cq, double* Cn, double* nrm,
                                                        int k) {
  __shared__ double sh[BT / 64];
  const int total = k * k;
  double ss = 0.0;
  for (int i = threadIdx.x; i < total; i += BT) {
    const int r = i / k, c = i % k;
    const double v = 0.5 * (Cq[i] + Cq[c * k + r]);
    ss += v * v;
  }
  const double nr = sqrt(block_sum(ss, sh));
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = threadIdx.x; i < total; i += BT) {
    const int r = i / k, c = i % k;
    Cn[i] = 0.5 * (Cq[i] + Cq[c * k + r]) * inv;
  }
  if (threadIdx.x == 0) nrm[0] = nr;
}

__global__ __launch_bounds__(BT) void corner_bwd_kernel(const double* g, const double* Cn,
                                                        const double* nrm, double* out, int k) {
  __shared__ double sh[BT / 64];
  const int total = k * k;
  double t = 0.0;
  for (int i = threadIdx.x; i < total; i += BT) t += g[i] * Cn[i];
  const double d = block_sum(t, sh);
  const double inv = 1.0 / nrm[0];
  for (int i = threadIdx.x; i < total; i += BT) {
    const int r = i / k, c = i % k;
    const int j = c * k + r;
    out[i] = 0.5 * ((g[i] - Cn[i] * d) + (g[j] - Cn[j] * d)) * inv;
  }
}

__global__ __launch_bounds__(BT) void maxabs_scale_kernel(const double* M, double* out, double* sc,
                                                          int k) {
  __shared__ double sh[BT / 64];
  const int total = k * k;
  double m = 0.0;
  for (int i = threadIdx.x; i < total; i += BT) m = fmax(m, fabs(M[i]));
  m = block_max(m, sh);
  const double s = m > 0.0 ? m : 1.0;
  for (int i = threadIdx.x; i < total; i += BT) out[i] = M[i] / s;
  if (threadIdx.x == 0) sc[0] = s;
}

__global__ void sym_scaled_kernel(const double* M, const double* sc, double alpha, double* out,
                                  int k) {
  const double f = alpha / (sc ? sc[0] : 1.0);
  const int64_t total = (int64_t)k * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / k), c = (int)(i % k);
    out[i] = f * (M[i] + M[(int64_t)c * k + r]);
  }
}

__global__ void div_scalar_kernel(const double* M, const double* sc, double* out, int64_t n) {
  const double inv = 1.0 / sc[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = M[i] * inv;
}

__global__ void energy_bwd_kernel(const double* R, const double* h, int d, double* out, double* Rb) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int d2 = d * d;
  auto ridx = [&](int x, int y) {  // x = (s,t), y = (s',t') -> R[(s,s')][(t,t')]
    const int s = x / d, t = x % d, sp = y / d, tp = y % d;
    return (s * d + sp) * d2 + (t * d + tp);
  };
  double tr = 0.0;
  for (int x = 0; x < d2; ++x) tr += R[ridx(x, x)];
  double e = 0.0;
  for (int x = 0; x < d2; ++x)
    for (int y = 0; y < d2; ++y) e += R[ridx(x, y)] / tr * h[y * d2 + x];
  for (int x = 0; x < d2; ++x)
    for (int y = 0; y < d2; ++y) Rb[ridx(x, y)] = (h[y * d2 + x] - (x == y ? e : 0.0)) / tr;
  out[0] = e;
}

__global__ void sum_batches_kernel(const double* __restrict__ in, int nb, int64_t len,
                                   double* __restrict__ out, double beta) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += in[(int64_t)b * len + i];
    out[i] = beta * out[i] + t;
  }
}

// gA[s][(u,v,w)] += sum_{u'v'w'} (ab[(u,u'),(v,v'),(w,w')] + ab[(u',u),(v',v),(w',w)]) A[s][(u',v',w')]
__global__ void double_layer_bwd_kernel(const double* __restrict__ ab, const double* __restrict__ A,
                                        int d, int D, double* __restrict__ gA) {
  const int D2 = D * D, D3 = D2 * D;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * D3) return;
  const int s = idx / D3, p = idx % D3;
  const int u = p / D2, v = (p / D) % D, w = p % D;
  double t = 0.0;
  for (int q = 0; q < D3; ++q) {
    const int u2 = q / D2, v2 = (q / D) % D, w2 = q % D;
    const int I1 = u * D + u2, J1 = v * D + v2, K1 = w * D + w2;
    const int I2 = u2 * D + u, J2 = v2 * D + v, K2 = w2 * D + w;
    t += (ab[((int64_t)I1 * D2 + J1) * D2 + K1] + ab[((int64_t)I2 * D2 + J2) * D2 + K2]) *
         A[s * D3 + q];
  }
  gA[idx] += t;
}

// Open double layer aO[(X,Y,Z)][s][s'] = A[s][ket] A[s'][bra] with
// (I,J,K) = (X,Y,Z) (rot 0) or (Z,X,Y) (rot 1), ket = (I/D, J/D, K/D),
// bra = (I%D, J%D, K%D).  Output gA[t][(p0,p1,p2)]: ket terms with s = t and
// bra terms with s' = t.
__global__ void double_layer_open_bwd_kernel(const double* __restrict__ aOb,
                                             const double* __restrict__ A, int d, int D, int rot,
                                             double* __restrict__ gA) {
  const int D2 = D * D, D3 = D2 * D;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * D3) return;
  const int t = idx / D3, p = idx % D3;
  const int p0 = p / D2, p1 = (p / D) % D, p2 = p % D;
  auto oidx = [&](int I, int J, int K) -> int64_t {
    const int X = rot ? J : I, Y = rot ? K : J, Z = rot ? I : K;
    return (((int64_t)X * D2 + Y) * D2 + Z) * d * d;
  };
  double acc = 0.0;
  for (int q = 0; q < D3; ++q) {
    const int q0 = q / D2, q1 = (q / D) % D, q2 = q % D;
    // ket side: (I,J,K) = (p0 D + q0, ...), partner index q on the bra side
    const int64_t ok = oidx(p0 * D + q0, p1 * D + q1, p2 * D + q2);
    // bra side: (I,J,K) = (q0 D + p0, ...)
    const int64_t ob = oidx(q0 * D + p0, q1 * D + p1, q2 * D + p2);
    for (int s2 = 0; s2 < d; ++s2) {
      acc += aOb[ok + t * d + s2] * A[s2 * D3 + q];
      acc += aOb[ob + s2 * d + t] * A[s2 * D3 + q];
    }
  }
  gA[idx] += acc;
}

__global__ void symmetrize_plain_kernel(const double* g, double* out, int d, int D) {
  const int D2 = D * D, D3 = D2 * D;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * D3) return;
  const int s = idx / D3, r = idx % D3;
  const int u = r / D2, v = (r / D) % D, w = r % D;
  const double* gs = g + (int64_t)s * D3;
  auto at = [&](int x, int y, int z) { return gs[(x * D + y) * D + z]; };
  out[idx] = (at(u, v, w) + at(u, w, v) + at(v, u, w) + at(v, w, u) + at(w, u, v) + at(w, v, u)) /
             6.0;
}

__global__ void copy_kernel(const double* __restrict__ in, double* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

__global__ void zero_kernel(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void axpy_kernel(const double* __restrict__ x, double* __restrict__ y, int64_t n,
                            double alpha) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += alpha * x[i];
}

__global__ void normalize_kernel(const double* __restrict__ in, const double* __restrict__ sumsq,
                                 double* __restrict__ nrm, double* __restrict__ out, int64_t n) {
  const double nr = sqrt(sumsq[0]);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) nrm[0] = nr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i] * inv;
}

}  // namespace

void launch_axpy(hipStream_t s, const double* x, double* y, int64_t n, double alpha) {
  if (n <= 0) return;
  axpy_kernel<<<grid_for(n), 256, 0, s>>>(x, y, n, alpha);
  CTM_LAUNCHED();
}

void launch_normalize(hipStream_t s, const double* in, const double* sumsq, double* nrm, double* out,
                      int64_t n) {
  normalize_kernel<<<grid_for(n), 256, 0, s>>>(in, sumsq, nrm, out, n);
  CTM_LAUNCHED();
}

void launch_swap_mid(hipStream_t s, const double* in, double* out, int A, int B, int C, int Dd,
                     bool accumulate) {
  const int64_t rows = (int64_t)A * B;
  if (rows <= 0 || C <= 0 || Dd <= 0) return;
  swap_mid_kernel<<<(unsigned)rows, 256, 0, s>>>(in, out, A, B, C, Dd, accumulate ? 1 : 0);
  CTM_LAUNCHED();
}

void launch_copyltu(hipStream_t s, const double* in, double* out, int k) {
  copyltu_kernel<<<grid_for((int64_t)k * k), 256, 0, s>>>(in, out, k);
  CTM_LAUNCHED();
}

void launch_tri_inv_upper(hipStream_t s, const double* R, int ldr, int k, const double* sgn,
                          double* out) {
  if (k <= 0) return;
  const unsigned wg = (unsigned)cdiv(k, 4);
  switch (cdiv(k, 64)) {
    case 1: tri_inv_upper_wave_kernel<1><<<wg, 256, 0, s>>>(R, ldr, k, sgn, out); break;
    case 2: tri_inv_upper_wave_kernel<2><<<wg, 256, 0, s>>>(R, ldr, k, sgn, out); break;
    case 3: tri_inv_upper_wave_kernel<3><<<wg, 256, 0, s>>>(R, ldr, k, sgn, out); break;
    case 4: tri_inv_upper_wave_kernel<4><<<wg, 256, 0, s>>>(R, ldr, k, sgn, out); break;
    default: tri_inv_upper_kernel<<<(unsigned)cdiv(k, 64), 64, 0, s>>>(R, ldr, k, sgn, out);
  }
  CTM_LAUNCHED();
}

void launch_dot(hipStream_t s, const double* a, const double* b, int64_t n, double* parts,
                double* out) {
  const int np = (int)std::min<int64_t>(DOT_PARTS, std::max<int64_t>(1, cdiv(n, 1024)));
  dot_parts_kernel<<<np, 256, 0, s>>>(a, b, n, parts);
  CTM_LAUNCHED();
  dot_final_kernel<<<1, 256, 0, s>>>(parts, np, out);
  CTM_LAUNCHED();
}

void launch_unit_norm_bwd(hipStream_t s, const double* g, const double* y, const double* dot,
                          const double* nrm, double* out, int64_t n) {
  unit_norm_bwd_kernel<<<grid_for(n), 256, 0, s>>>(g, y, dot, nrm, out, n);
  CTM_LAUNCHED();
}

void launch_corner_fwd(hipStream_t s, const double* Cq, double* Cn, double* nrm, int k) {
  corner_fwd_kernel<<<1, BT, 0, s>>>(Cq, Cn, nrm, k);
  CTM_LAUNCHED();
}

void launch_corner_bwd(hipStream_t s, const double* g, const double* Cn, const double* nrm,
                       double* out, int k) {
  corner_bwd_kernel<<<1, BT, 0, s>>>(g, Cn, nrm, out, k);
  CTM_LAUNCHED();
}

void launch_maxabs_scale(hipStream_t s, const double* M, double* out, double* sc, int k) {
  maxabs_scale_kernel<<<1, BT, 0, s>>>(M, out, sc, k);
  CTM_LAUNCHED();
}

void launch_sym_scaled(hipStream_t s, const double* M, const double* sc, double alpha, double* out,
                       int k) {
  sym_scaled_kernel<<<grid_for((int64_t)k * k), 256, 0, s>>>(M, sc, alpha, out, k);
  CTM_LAUNCHED();
}

void launch_div_scalar(hipStream_t s, const double* M, const double* sc, double* out, int64_t n) {
  div_scalar_kernel<<<grid_for(n), 256, 0, s>>>(M, sc, out, n);
  CTM_LAUNCHED();
}

void launch_energy_bwd(hipStream_t s, const double* R, const double* h, int d, double* out,
                       double* Rb) {
  energy_bwd_kernel<<<1, 64, 0, s>>>(R, h, d, out, Rb);
  CTM_LAUNCHED();
}

void launch_sum_batches(hipStream_t s, const double* in, int nb, int64_t len, double* out,
                        double beta) {
  sum_batches_kernel<<<grid_for(len), 256, 0, s>>>(in, nb, len, out, beta);
  CTM_LAUNCHED();
}

void launch_double_layer_bwd(hipStream_t s, const double* ab, const double* A, int d, int D,
                             double* gA) {
  const int n = d * D * D * D;
  double_layer_bwd_kernel<<<(unsigned)cdiv(n, 64), 64, 0, s>>>(ab, A, d, D, gA);
  CTM_LAUNCHED();
}

void launch_double_layer_open_bwd(hipStream_t s, const double* aOb, const double* A, int d, int D,
                                  int rot, double* gA) {
  const int n = d * D * D * D;
  double_layer_open_bwd_kernel<<<(unsigned)cdiv(n, 64), 64, 0, s>>>(aOb, A, d, D, rot, gA);
  CTM_LAUNCHED();
}

void launch_symmetrize_plain(hipStream_t s, const double* g, double* out, int d, int D) {
  const int n = d * D * D * D;
  symmetrize_plain_kernel<<<(unsigned)cdiv(n, 64), 64, 0, s>>>(g, out, d, D);
  CTM_LAUNCHED();
}

void launch_copy(hipStream_t s, const double* in, double* out, int64_t n) {
  if (n <= 0) return;
  copy_kernel<<<grid_for(n), 256, 0, s>>>(in, out, n);
  CTM_LAUNCHED();
}

void launch_zero(hipStream_t s, double* p, int64_t n) {
  if (n <= 0) return;
  zero_kernel<<<grid_for(n), 256, 0, s>>>(p, n);
  CTM_LAUNCHED();
}

}  // namespace ctm
