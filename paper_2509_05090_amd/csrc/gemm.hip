// MFMA matrix-product kernels for gfx950.
//
// One templated kernel serves FP64 (v_mfma_f64_16x16x4), FP32
// (v_mfma_f32_16x16x4) and BF16 (v_mfma_f32_16x16x32_bf16, FP32 accumulate).
// A workgroup of four 64-wide wavefronts computes a BM x BN tile; operands
// are staged through LDS in k-chunks of 128 bytes per row (double-buffered),
// with 16 bytes of padding so that the 16-lane row reads of the MFMA operand
// fetch hit distinct banks.  Within a chunk the four 16-lane groups of a
// wavefront each own a contiguous quarter of the k range, so every lane
// fetches its operand bytes with 16-byte LDS reads.  When an operand's rows
// and batch offsets are 16-byte aligned it is fetched from memory with
// 16-byte loads along its contiguous dimension (VEC); an operand contiguous
// along k then lands in LDS with 16-byte stores, one contiguous along m or n
// is scattered into the k-contiguous LDS rows.
#include "gemm.hpp"

#include <algorithm>

namespace ctm {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename E> struct Mfma;

template <> struct Mfma<double> {
  using acc_t = double;
  using accv = d4v;
  static constexpr int KPL = 1;  // operand elements per lane per instruction
  // Result layout: lane (grp, r16), register r holds row 4*r + grp (rows
  // interleaved across the four 16-lane groups), column r16.
  static constexpr bool ROWS_INTERLEAVED = true;
  __device__ static inline accv mma(const double* a, const double* b, accv c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
  }
};

template <> struct Mfma<float> {
  using acc_t = float;
  using accv = f4v;
  static constexpr int KPL = 1;
  // Result layout: lane (grp, r16), register r holds row 4*grp + r, column r16.
  static constexpr bool ROWS_INTERLEAVED = false;
  __device__ static inline accv mma(const float* a, const float* b, accv c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
};

template <> struct Mfma<bf16> {
  using acc_t = float;
  using accv = f4v;
  static constexpr int KPL = 8;
  static constexpr bool ROWS_INTERLEAVED = false;
  __device__ static inline accv mma(const bf16* a, const bf16* b, accv c) {
    bf16x8 av, bv;
    __builtin_memcpy(&av, a, 16);
    __builtin_memcpy(&bv, b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};

struct GemmArgs {
  int M, N, K;
  const void* A;
  int64_t lda, sA0, sA1;
  const void* B;
  int64_t ldb, sB0, sB1;
  void* C;
  int64_t ldc, sC0, sC1;
  int nb1;
  int tiles_m, tiles_n;
  int kchunk;
  double alpha, beta;
};

template <typename E> __device__ inline E zero_of() { return E(0); }
template <> __device__ inline bf16 zero_of<bf16>() { return (bf16)0.0f; }

// Workgroup -> (tile, batch).  Workgroups are dispatched round-robin over the
// 8 XCDs; this order gives each XCD a contiguous range of tiles, so the
// column tiles that re-read one row panel of A share an L2.
__device__ inline int xcd_linear(int x, int nblk) {
  const int per = nblk / 8, rem = nblk % 8, xcd = x % 8, slot = x / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// Vectorized tile loader of one operand for a k-chunk: a ROWS x BK tile
// (ROWS of the logical m or n index) whose memory layout is contiguous along
// k (KC) or along the row index.  Vectors of V elements; every tile is
// ROWS * BK / V vectors, spread over the 256 threads.
template <typename E, int ROWS, int BK, bool KC>
struct VecTile {
  static constexpr int V = 16 / (int)sizeof(E);
  static constexpr int NV = ROWS * BK / V;
  static constexpr int PER = (NV + 255) / 256;
  typedef E vec_t __attribute__((ext_vector_type(V)));
  vec_t r[PER];
  // p: operand base (batch applied); ld: leading dimension; r0: first row
  // index of the tile; rlim: row count; k0, kend: k range of the chunk.
  __device__ inline void load(const E* __restrict__ p, int64_t ld, int r0, int rlim, int k0,
                              int kend) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * 256;
      // KC: vector along k within row rr; else vector along rows at k row kk
      const int rr = KC ? q / (BK / V) : (q % (ROWS / V)) * V;
      const int kk = KC ? (q % (BK / V)) * V : q / (ROWS / V);
      const int gr = r0 + rr, gk = k0 + kk;
      vec_t v;
#pragma unroll
      for (int j = 0; j < V; ++j) v[j] = zero_of<E>();
      if (q < NV) {
        if (KC) {
          if (gr < rlim) {
            const E* src = p + (int64_t)gr * ld + gk;
            if (gk + V <= kend) {
              v = *(const vec_t*)src;
            } else {
#pragma unroll
              for (int j = 0; j < V; ++j)
                if (gk + j < kend) v[j] = src[j];
            }
          }
        } else if (gk < kend) {
          const E* src = p + (int64_t)gk * ld + gr;
          if (gr + V <= rlim) {
            v = *(const vec_t*)src;
          } else {
#pragma unroll
            for (int j = 0; j < V; ++j)
              if (gr + j < rlim) v[j] = src[j];
          }
        }
      }
      r[i] = v;
    }
  }
  // LDS rows of LDK elements, k contiguous.
  __device__ inline void store(E* __restrict__ lds, int LDK) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * 256;
      if (q >= NV) continue;
      if (KC) {
        *(vec_t*)&lds[(q / (BK / V)) * LDK + (q % (BK / V)) * V] = r[i];
      } else {
        const int rr = (q % (ROWS / V)) * V, kk = q / (ROWS / V);
#pragma unroll
        for (int j = 0; j < V; ++j) lds[(rr + j) * LDK + kk] = r[i][j];
      }
    }
  }
};

template <typename E, bool AT, bool BT, int BM, int BN, int WM, int WN, bool SPLIT, bool VEC>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  using MF = Mfma<E>;
  using acc_t = typename MF::acc_t;
  using accv = typename MF::accv;
  constexpr int NT = 256;
  constexpr int BK = 128 / (int)sizeof(E);
  constexpr int LDK = BK + 16 / (int)sizeof(E);
  constexpr int FM = BM / (16 * WM), FN = BN / (16 * WN);
  constexpr int KG = BK / 4;
  constexpr int STEPS = KG / MF::KPL;
  constexpr int EA = BM * BK / NT, EB = BN * BK / NT;
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0 && WM * WN == 4, "tile");
  static_assert(EA * NT == BM * BK && EB * NT == BN * BK, "load split");

  __shared__ __attribute__((aligned(16))) E As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) E Bs[2][BN * LDK];

  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  const int tiles = g.tiles_m * g.tiles_n;
  const int tile = lin % tiles, batch = lin / tiles;
  const int b0 = batch / g.nb1, b1 = batch % g.nb1;
  const int tm = tile / g.tiles_n, tn = tile % g.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const E* __restrict__ A = (const E*)g.A + b0 * g.sA0 + b1 * g.sA1;
  const E* __restrict__ B = (const E*)g.B + b0 * g.sB0 + b1 * g.sB1;
  const int kbeg = blockIdx.y * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int nk = kend > kbeg ? (int)cdiv(kend - kbeg, BK) : 0;

  E ra[EA], rb[EB];
  VecTile<E, BM, BK, !AT> va;
  VecTile<E, BN, BK, BT> vb;
  auto load = [&](int k0) {
    if constexpr (VEC) {
      va.load(A, g.lda, m0, g.M, k0, kend);
      vb.load(B, g.ldb, n0, g.N, k0, kend);
    } else {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = threadIdx.x + i * NT;
        const int mm = AT ? e % BM : e / BK, kk = AT ? e / BM : e % BK;
        const int gm = m0 + mm, gk = k0 + kk;
        E v = zero_of<E>();
        if (gm < g.M && gk < kend)
          v = AT ? A[(int64_t)gk * g.lda + gm] : A[(int64_t)gm * g.lda + gk];
        ra[i] = v;
      }
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = threadIdx.x + i * NT;
        const int nn = BT ? e / BK : e % BN, kk = BT ? e % BK : e / BN;
        const int gn = n0 + nn, gk = k0 + kk;
        E v = zero_of<E>();
        if (gn < g.N && gk < kend)
          v = BT ? B[(int64_t)gn * g.ldb + gk] : B[(int64_t)gk * g.ldb + gn];
        rb[i] = v;
      }
    }
  };
  auto store = [&](int buf) {
    if constexpr (VEC) {
      va.store(As[buf], LDK);
      vb.store(Bs[buf], LDK);
    } else {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = threadIdx.x + i * NT;
        const int mm = AT ? e % BM : e / BK, kk = AT ? e / BM : e % BK;
        As[buf][mm * LDK + kk] = ra[i];
      }
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = threadIdx.x + i * NT;
        const int nn = BT ? e / BK : e % BN, kk = BT ? e % BK : e / BN;
        Bs[buf][nn * LDK + kk] = rb[i];
      }
    }
  };

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid % WM, wn = wid / WM;
  const int r16 = lane & 15, grp = lane >> 4;
  accv acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = accv{0, 0, 0, 0};

  if (nk > 0) {
    load(kbeg);
    store(0);
    __syncthreads();
  }
  for (int c = 0; c < nk; ++c) {
    const int cur = c & 1;
    if (c + 1 < nk) load(kbeg + (c + 1) * BK);
    E af[FM][KG], bfr[FN][KG];
#pragma unroll
    for (int i = 0; i < FM; ++i)
      __builtin_memcpy(&af[i][0], &As[cur][(wm * FM * 16 + i * 16 + r16) * LDK + grp * KG], 32);
#pragma unroll
    for (int j = 0; j < FN; ++j)
      __builtin_memcpy(&bfr[j][0], &Bs[cur][(wn * FN * 16 + j * 16 + r16) * LDK + grp * KG], 32);
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = MF::mma(&af[i][s * MF::KPL], &bfr[j][s * MF::KPL], acc[i][j]);
    if (c + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = MF::ROWS_INTERLEAVED ? r * 4 + grp : grp * 4 + r;
        const int row = m0 + wm * FM * 16 + i * 16 + rr;
        const int col = n0 + wn * FN * 16 + j * 16 + r16;
        if (row < g.M && col < g.N) {
          if constexpr (SPLIT) {
            acc_t* W = (acc_t*)g.C + (int64_t)blockIdx.y * g.M * g.N;
            W[(int64_t)row * g.N + col] = acc[i][j][r];
          } else {
            E* C = (E*)g.C + b0 * g.sC0 + b1 * g.sC1;
            double v = g.alpha * (double)acc[i][j][r];
            if (g.beta != 0.0) v += g.beta * to_f64(C[(int64_t)row * g.ldc + col]);
            C[(int64_t)row * g.ldc + col] = from_f64<E>(v);
          }
        }
      }
}

constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 1024;

int sumsq_blocks(int M, int N) {
  int64_t mn = (int64_t)M * N;
  return (int)std::min<int64_t>(RED_MAX_BLOCKS, std::max<int64_t>(1, cdiv(mn, RED_THREADS * 4)));
}

// C = alpha * sum_s W[s] + beta * C, summed in a fixed order; optional
// per-block sums of squares of the result.
template <typename Acc, typename TC>
__global__ __launch_bounds__(RED_THREADS) void splitk_reduce(const Acc* __restrict__ W, int S, int M,
                                                          int N, TC* C, int64_t ldc, double alpha,
                                                          double beta, double* sumsq) {
  const int64_t mn = (int64_t)M * N;
  constexpr int SB = 8;  // partials loaded per batch (summed in order, s = 0, 1, ...)
  double ss = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < mn;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s0 = 0; s0 < S; s0 += SB) {
      Acc p[SB];
#pragma unroll
      for (int j = 0; j < SB; ++j) p[j] = s0 + j < S ? W[(int64_t)(s0 + j) * mn + idx] : Acc(0);
#pragma unroll
      for (int j = 0; j < SB; ++j)
        if (s0 + j < S) v += (double)p[j];
    }
    const int64_t row = idx / N, col = idx % N;
    TC* dst = C + row * ldc + col;
    v *= alpha;
    if (beta != 0.0) v += beta * to_f64(*dst);
    *dst = from_f64<TC>(v);
    ss += v * v;
  }
  if (sumsq) {
    __shared__ double red[RED_THREADS / 64];
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
      sumsq[blockIdx.x] = t;
    }
  }
}

namespace {

struct TileCfg {
  int BM, BN;
};
constexpr int NCFG = 4;
constexpr TileCfg CFGS[NCFG] = {{64, 64}, {64, 48}, {48, 64}, {32, 32}};

template <typename E, bool AT, bool BT, bool SPLIT, bool VEC>
void launch_cfg(int cfg, dim3 grid, hipStream_t s, const GemmArgs& a) {
  switch (cfg) {
    case 0: gemm_kernel<E, AT, BT, 64, 64, 2, 2, SPLIT, VEC><<<grid, 256, 0, s>>>(a); break;
    case 1: gemm_kernel<E, AT, BT, 64, 48, 4, 1, SPLIT, VEC><<<grid, 256, 0, s>>>(a); break;
    case 2: gemm_kernel<E, AT, BT, 48, 64, 1, 4, SPLIT, VEC><<<grid, 256, 0, s>>>(a); break;
    default: gemm_kernel<E, AT, BT, 32, 32, 2, 2, SPLIT, VEC><<<grid, 256, 0, s>>>(a); break;
  }
}

template <typename E, bool SPLIT, bool VEC>
void launch_trans(bool at, bool bt, int cfg, dim3 grid, hipStream_t s, const GemmArgs& a) {
  if (!at && !bt) launch_cfg<E, false, false, SPLIT, VEC>(cfg, grid, s, a);
  else if (!at && bt) launch_cfg<E, false, true, SPLIT, VEC>(cfg, grid, s, a);
  else if (at && !bt) launch_cfg<E, true, false, SPLIT, VEC>(cfg, grid, s, a);
  else launch_cfg<E, true, true, SPLIT, VEC>(cfg, grid, s, a);
}

template <typename E>
void launch_any(bool split, bool vec, bool at, bool bt, int cfg, dim3 grid, hipStream_t s,
                const GemmArgs& a) {
  if (split) {
    if (vec) launch_trans<E, true, true>(at, bt, cfg, grid, s, a);
    else launch_trans<E, true, false>(at, bt, cfg, grid, s, a);
  } else {
    if (vec) launch_trans<E, false, true>(at, bt, cfg, grid, s, a);
    else launch_trans<E, false, false>(at, bt, cfg, grid, s, a);
  }
}

// 16-byte loads are legal for an operand whose base, leading dimension and
// batch offsets are multiples of 16 bytes (tile origins along the
// contiguous dimension are multiples of 16 bytes by construction).
bool vec_ok(const Operand& o, size_t es) {
  const int64_t v = 16 / (int64_t)es;
  return ((uintptr_t)o.p % 16) == 0 && o.ld % v == 0 && o.s0 % v == 0 && o.s1 % v == 0;
}

template <typename Acc>
void launch_reduce(DType out, const Acc* W, int S, int M, int N, void* C, int64_t ldc,
                   double alpha, double beta, double* sumsq, hipStream_t s) {
  // with norm partials the block count is sumsq_blocks(); without, one
  // element per thread
  const int blocks = sumsq ? sumsq_blocks(M, N)
                           : (int)std::min<int64_t>(65536, cdiv((int64_t)M * N, RED_THREADS));
  switch (out) {
    case DType::F64:
      splitk_reduce<Acc, double><<<blocks, RED_THREADS, 0, s>>>(W, S, M, N, (double*)C, ldc, alpha,
                                                                beta, sumsq);
      break;
    case DType::F32:
      splitk_reduce<Acc, float><<<blocks, RED_THREADS, 0, s>>>(W, S, M, N, (float*)C, ldc, alpha,
                                                               beta, sumsq);
      break;
    case DType::BF16:
      splitk_reduce<Acc, bf16><<<blocks, RED_THREADS, 0, s>>>(W, S, M, N, (bf16*)C, ldc, alpha,
                                                              beta, sumsq);
      break;
  }
}

// Tile of least padded area; the 32x32 tile re-reads its operands twice as
// often, so it is charged a third more area.
int pick_cfg(int M, int N) {
  int best = 0;
  int64_t best_area = INT64_MAX;
  for (int c = 0; c < NCFG; ++c) {
    int64_t area = cdiv(M, CFGS[c].BM) * CFGS[c].BM * cdiv(N, CFGS[c].BN) * CFGS[c].BN;
    if (CFGS[c].BM * CFGS[c].BN < 64 * 48) area += area / 3;
    if (area < best_area) {
      best_area = area;
      best = c;
    }
  }
  return best;
}

}  // namespace

// Batches of small products (the pair contractions of the enlarged corner:
// chi D^2 batches of chi x D^2 x D^2): C[b0,b1] = A[b0] B[b1] with K, N <= 64
// and A independent of b1.  A workgroup holds a row tile of A[b0] in LDS
// ([m][k], k contiguous) and runs over a group of b1: it stages B[b1] in LDS
// ([n][k]) and its four wavefronts each take 16-row tiles of the output,
// all 16-column tiles of a row tile at once, over the whole (short) k
// range.  Each output element is written once, straight from the
// accumulators.
constexpr int SB_KMAX = 64, SB_NMAX = 64;
constexpr int SB_LDS = 64 * 1024;

struct SmallBatchArgs {
  int M, N, K;
  const void* A;
  int64_t lda, sA0;
  bool at;
  const void* B;
  int64_t ldb, sB1;
  bool bt;
  void* C;
  int64_t ldc, sC0, sC1;
  int nb0, nb1;
  int mt;      // rows of A per workgroup (multiple of 16)
  int mtiles;  // row tiles per b0
  int group;   // b1 values per workgroup
  int kp;      // LDS row length (elements)
};

template <typename E, int KS, int NT>
__global__ __launch_bounds__(256) void small_batch_kernel(SmallBatchArgs g) {
  using MF = Mfma<E>;
  using accv = typename MF::accv;
  constexpr int KPL = MF::KPL;
  constexpr int KSTEP = 4 * KPL;      // k per MFMA
  constexpr int KPAD = KS * KSTEP;    // k range held in LDS (zero beyond K)
  extern __shared__ __attribute__((aligned(16))) unsigned char sb_lds[];
  E* As = (E*)sb_lds;  // [mt][kp]

  const int b0 = blockIdx.x / g.mtiles, m0 = (blockIdx.x % g.mtiles) * g.mt;
  const int rows = min(g.mt, g.M - m0);
  const E* __restrict__ A = (const E*)g.A + (int64_t)b0 * g.sA0;

  // A tile [m][k], zero beyond the data.  The source is walked in its own
  // storage order (k-major when transposed) with the (outer, inner) position
  // advanced incrementally; loads are issued in batches of LB per thread
  // before their LDS stores.
  {
    constexpr int LB = 16;
    const int outer = g.at ? KPAD : g.mt, inner = g.at ? g.mt : KPAD;
    const int so = 256 / inner, si = 256 % inner;
    int o = threadIdx.x / inner, in = threadIdx.x % inner;
    while (o < outer) {
      E v[LB];
      int om[LB], im[LB];
#pragma unroll
      for (int j = 0; j < LB; ++j) {
        om[j] = o;
        im[j] = in;
        const int m = g.at ? in : o, k = g.at ? o : in;
        v[j] = zero_of<E>();
        if (o < outer && m < rows && k < g.K)
          v[j] = g.at ? A[(int64_t)k * g.lda + m0 + m] : A[(int64_t)(m0 + m) * g.lda + k];
        in += si;
        o += so;
        if (in >= inner) {
          in -= inner;
          ++o;
        }
      }
#pragma unroll
      for (int j = 0; j < LB; ++j) {
        const int m = g.at ? im[j] : om[j], k = g.at ? om[j] : im[j];
        if (om[j] < outer) As[m * g.kp + k] = v[j];
      }
    }
  }
  __syncthreads();

  // Each wavefront takes its own batches b1 = first + wid + 4 i and sweeps
  // every row tile of the A tile with them: no barrier after the A tile.
  // The B fragments come straight from memory, one batch ahead of use.
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r16 = lane & 15, grp = lane >> 4;
  const int b1first = blockIdx.y * g.group, b1end = min(g.nb1, b1first + g.group);
  E bf[NT][KS][KPL], bn[NT][KS][KPL];
  auto load_b = [&](int b1, E (&dst)[NT][KS][KPL]) {
    const E* __restrict__ B = (const E*)g.B + (int64_t)b1 * g.sB1;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int u = 0; u < KPL; ++u) {
          const int n = t * 16 + r16, k = s * KSTEP + grp * KPL + u;
          dst[t][s][u] = zero_of<E>();
          if (n < g.N && k < g.K) dst[t][s][u] = g.bt ? B[(int64_t)n * g.ldb + k] : B[(int64_t)k * g.ldb + n];
        }
  };
  int b1 = b1first + wid;
  if (b1 < b1end) load_b(b1, bf);
  for (; b1 < b1end; b1 += 4) {
    if (b1 + 4 < b1end) load_b(b1 + 4, bn);
    E* __restrict__ C = (E*)g.C + (int64_t)b0 * g.sC0 + (int64_t)b1 * g.sC1;
    for (int tm = 0; tm * 16 < rows; ++tm) {
      E af[KS][KPL];
#pragma unroll
      for (int s = 0; s < KS; ++s)
        __builtin_memcpy(&af[s][0], &As[(tm * 16 + r16) * g.kp + s * KSTEP + grp * KPL],
                         KPL * sizeof(E));
      accv acc[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = accv{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = MF::mma(&af[s][0], &bf[t][s][0], acc[t]);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = MF::ROWS_INTERLEAVED ? r * 4 + grp : grp * 4 + r;
          const int row = tm * 16 + rr, col = t * 16 + r16;
          if (row < rows && col < g.N)
            C[(int64_t)(m0 + row) * g.ldc + col] = from_f64<E>((double)acc[t][r]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int u = 0; u < KPL; ++u) bf[t][s][u] = bn[t][s][u];
  }
}

// The same batches when A is stored with its rows contiguous
// (A[b0](row, k) = A[b0 sA0 + k lda + row]) and the output rows take whole
// 16-byte groups of columns (FP64, FP32).  A workgroup holds in LDS the
// 16-row slices of AG consecutive batches b0 ([b0][k][row], filled with
// 16-byte loads); each of its four wavefronts keeps one B[b1] in registers
// and sweeps those AG batches, reading the next batch's fragments from LDS
// while the products of the current one run.  The MFMA computes the
// transposed 16 x 16 tile (rows = output columns, columns = output rows),
// so a lane ends with four adjacent columns of one output row and writes
// them with one vector store; the FP64 result interleaves rows across the
// lane groups, which the row order of the B fragment undoes.  For the V3
// product the outputs of consecutive b0 are adjacent in a row, so a
// wavefront writes whole row segments of AG*N elements.
struct SmallBatchRowsArgs {
  int M, N, K;
  const void* A;
  int64_t lda, sA0;
  const void* B;
  int64_t ldb, sB1;
  bool bt;
  void* C;
  int64_t ldc, sC0, sC1;
  int nb0, nb1;
  int ag;      // batches b0 per workgroup
  int mtiles;  // 16-row tiles
};

template <typename E, int KS, int NT>
__global__ __launch_bounds__(256) void small_batch_rows_kernel(SmallBatchRowsArgs g) {
  using MF = Mfma<E>;
  using accv = typename MF::accv;
  typedef E v4 __attribute__((ext_vector_type(4)));
  constexpr int KPAD = KS * 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char sbr_lds[];
  v4* As4 = (v4*)sbr_lds;  // [ag][KPAD][16] elements
  const E* As = (const E*)sbr_lds;

  const int r0 = (blockIdx.x % g.mtiles) * 16, a0 = (blockIdx.x / g.mtiles) * g.ag;
  const int na = min(g.ag, g.nb0 - a0);
  {
    // row (a, k) of the tile = 16 elements = 4 vectors; M is a multiple of 4
    constexpr int LB = 8;
    const E* __restrict__ A = (const E*)g.A;
    const int tot4 = g.ag * KPAD * 4;
    for (int base = 0; base < tot4; base += 256 * LB) {
      v4 v[LB];
#pragma unroll
      for (int j = 0; j < LB; ++j) {
        const int i4 = base + threadIdx.x + 256 * j, row = i4 >> 2, q = i4 & 3;
        const int k = row % KPAD, a = row / KPAD;
        v[j] = v4{0, 0, 0, 0};
        if (i4 < tot4 && a < na && k < g.K && r0 + 4 * q < g.M)
          v[j] = *(const v4*)(A + (int64_t)(a0 + a) * g.sA0 + (int64_t)k * g.lda + r0 + 4 * q);
      }
#pragma unroll
      for (int j = 0; j < LB; ++j) {
        const int i4 = base + threadIdx.x + 256 * j;
        if (i4 < tot4) As4[i4] = v[j];
      }
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r16 = lane & 15, grp = lane >> 4;
  const int b1 = blockIdx.y * 4 + wid;
  if (b1 >= g.nb1) return;
  // fragment row r16 of column tile t holds output column t*16 + prow
  const int prow = MF::ROWS_INTERLEAVED ? 4 * (r16 & 3) + (r16 >> 2) : r16;
  E bf[NT][KS];
  {
    const E* __restrict__ B = (const E*)g.B + (int64_t)b1 * g.sB1;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int n = t * 16 + prow, k = s * 4 + grp;
        bf[t][s] = zero_of<E>();
        if (n < g.N && k < g.K) bf[t][s] = g.bt ? B[(int64_t)n * g.ldb + k] : B[(int64_t)k * g.ldb + n];
      }
  }
  const bool rowok = r0 + r16 < g.M;
  E* __restrict__ Cl =
      (E*)g.C + (int64_t)b1 * g.sC1 + (int64_t)(r0 + r16) * g.ldc + 4 * grp;
  E af[KS], an[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) af[s] = As[(s * 4 + grp) * 16 + r16];
  for (int a = 0; a < na; ++a) {
    const int a1 = a + 1 < na ? a + 1 : a;
#pragma unroll
    for (int s = 0; s < KS; ++s) an[s] = As[(a1 * KPAD + s * 4 + grp) * 16 + r16];
    accv acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = accv{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = MF::mma(&bf[t][s], &af[s], acc[t]);
    E* __restrict__ Ca = Cl + (int64_t)(a0 + a) * g.sC0;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (rowok && t * 16 + 4 * grp < g.N)
        *(v4*)(Ca + t * 16) = v4{acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
#pragma unroll
    for (int s = 0; s < KS; ++s) af[s] = an[s];
  }
}

namespace {

// Launches the row-layout small-batch kernel if the operands allow it.
bool small_batch_rows(hipStream_t s, DType e, int M, int N, int K, const Operand& A,
                      const Operand& B, const Output& C, int nb0, int nb1, int ks, int nt) {
  const int es = (int)dtype_size(e);
  auto al = [&](const void* p) { return ((uintptr_t)p % (4 * (uintptr_t)es)) == 0; };
  if (e == DType::BF16 || !A.trans || M % 4 || N % 4 || A.ld % 4 || A.s0 % 4 || C.ld % 4 ||
      C.s0 % 4 || C.s1 % 4 || !al(A.p) || !al(C.p))
    return false;
  const int kpad = ks * 4;
  const int64_t per_batch = (int64_t)kpad * 16 * es;  // LDS bytes per batch b0
  SmallBatchRowsArgs g{};
  g.ag = (int)std::min<int64_t>({e == DType::F32 ? 16 : 8, SB_LDS / per_batch, nb0});
  g.mtiles = (int)cdiv(M, 16);
  g.M = M; g.N = N; g.K = K;
  g.A = A.p; g.lda = A.ld; g.sA0 = A.s0;
  g.B = B.p; g.ldb = B.ld; g.sB1 = B.s1; g.bt = B.trans;
  g.C = C.p; g.ldc = C.ld; g.sC0 = C.s0; g.sC1 = C.s1;
  g.nb0 = nb0; g.nb1 = nb1;
  const dim3 grid((unsigned)(g.mtiles * cdiv(nb0, g.ag)), (unsigned)cdiv(nb1, 4));
  const size_t lds = (size_t)g.ag * per_batch;
#define CTM_SBR(T, KS_, NT_) small_batch_rows_kernel<T, KS_, NT_><<<grid, 256, lds, s>>>(g)
  if (e == DType::F32) {
    if (ks == 1) CTM_SBR(float, 1, 1);
    else if (ks == 4) CTM_SBR(float, 4, 1);
    else if (ks == 9) CTM_SBR(float, 9, 3);
    else CTM_SBR(float, 16, 4);
  } else {
    if (ks == 1) CTM_SBR(double, 1, 1);
    else if (ks == 4) CTM_SBR(double, 4, 1);
    else if (ks == 9) CTM_SBR(double, 9, 3);
    else CTM_SBR(double, 16, 4);
  }
#undef CTM_SBR
  CTM_LAUNCHED();
  return true;
}

// Launches the small-batch kernel if the product has its shape; false if
// not (the caller then uses the general kernel).
bool small_batch(hipStream_t s, DType e, int M, int N, int K, const Operand& A, const Operand& B,
                 const Output& C, int nb0, int nb1, double alpha, double beta) {
  if (nb0 * (int64_t)nb1 <= 1 || K > SB_KMAX || N > SB_NMAX || A.s1 != 0 || B.s0 != 0 ||
      alpha != 1.0 || beta != 0.0 || C.t != e)
    return false;
  const int es = (int)dtype_size(e);
  const int kstep = e == DType::BF16 ? 32 : 4;
  // instances: k steps x column tiles, the smallest that covers (K, N)
  int ks = (int)cdiv(std::max(K, 1), kstep), nt = (int)cdiv(N, 16);
  if (e == DType::BF16) {
    ks = 2;
    nt = nt <= 1 ? 1 : 4;
  } else if (ks <= 1 && nt <= 1) {
    ks = 1;
    nt = 1;
  } else if (ks <= 4 && nt <= 1) {
    ks = 4;
    nt = 1;
  } else if (ks <= 9 && nt <= 3) {
    ks = 9;
    nt = 3;
  } else {
    ks = 16;
    nt = 4;
  }
  if (small_batch_rows(s, e, M, N, K, A, B, C, nb0, nb1, ks, nt)) return true;
  const int kpad = ks * kstep;
  const int kp = kpad + 16 / es;  // 16 bytes of row padding
  const int64_t mt_fit = SB_LDS / ((int64_t)kp * es) / 16 * 16;
  if (mt_fit < 16) return false;
  SmallBatchArgs g{};
  // row tiles of (nearly) equal height
  g.mtiles = (int)cdiv(M, mt_fit);
  g.mt = (int)(cdiv(cdiv(M, g.mtiles), 16) * 16);
  g.M = M; g.N = N; g.K = K;
  g.A = A.p; g.lda = A.ld; g.sA0 = A.s0; g.at = A.trans;
  g.B = B.p; g.ldb = B.ld; g.sB1 = B.s1; g.bt = B.trans;
  g.C = C.p; g.ldc = C.ld; g.sC0 = C.s0; g.sC1 = C.s1;
  g.nb0 = nb0; g.nb1 = nb1;
  g.kp = kp;
  // each workgroup reuses its A tile over `group` batches of B, a multiple
  // of the four wavefronts (one batch each at a time), sized for about four
  // thousand wavefronts' worth of batches in flight
  const int64_t base = (int64_t)nb0 * g.mtiles;
  g.group = (int)std::min<int64_t>(4 * cdiv(nb1, 4), 4 * std::max<int64_t>(1, cdiv(base * nb1, 4096)));
  const dim3 grid((unsigned)base, (unsigned)cdiv(nb1, g.group));
  const size_t lds = (size_t)g.mt * kp * es;
#define CTM_SB(T, KS_, NT_) small_batch_kernel<T, KS_, NT_><<<grid, 256, lds, s>>>(g)
  // (ks, nt) is exactly one of the instances below
  if (e == DType::BF16) {
    if (nt == 1) CTM_SB(bf16, 2, 1);
    else CTM_SB(bf16, 2, 4);
  } else if (e == DType::F32) {
    if (ks == 1) CTM_SB(float, 1, 1);
    else if (ks == 4) CTM_SB(float, 4, 1);
    else if (ks == 9) CTM_SB(float, 9, 3);
    else CTM_SB(float, 16, 4);
  } else {
    if (ks == 1) CTM_SB(double, 1, 1);
    else if (ks == 4) CTM_SB(double, 4, 1);
    else if (ks == 9) CTM_SB(double, 9, 3);
    else CTM_SB(double, 16, 4);
  }
#undef CTM_SB
  CTM_LAUNCHED();
  return true;
}

}  // namespace

constexpr int MAX_SPLIT = 16;

size_t gemm_scratch_bytes(DType e, int M, int N) {
  const size_t acc = e == DType::F64 ? 8 : 4;
  return (size_t)MAX_SPLIT * M * N * acc;
}

void gemm(hipStream_t s, DType e, int M, int N, int K, const Operand& A, const Operand& B,
          const Output& C, int nb0, int nb1, double alpha, double beta, const Scratch& ws,
          int ksplit, double* sumsq, const KernelEvents* ev) {
  if (M <= 0 || N <= 0 || nb0 <= 0 || nb1 <= 0) return;
  if (ksplit == 0 && sumsq == nullptr && ev == nullptr &&
      small_batch(s, e, M, N, K, A, B, C, nb0, nb1, alpha, beta))
    return;
  const int cfg = pick_cfg(M, N);
  const int BM = CFGS[cfg].BM, BN = CFGS[cfg].BN;
  const int BK = 128 / (int)dtype_size(e);
  GemmArgs a{};
  a.M = M;
  a.N = N;
  a.K = K;
  a.A = A.p;
  a.lda = A.ld;
  a.sA0 = A.s0;
  a.sA1 = A.s1;
  a.B = B.p;
  a.ldb = B.ld;
  a.sB0 = B.s0;
  a.sB1 = B.s1;
  a.C = C.p;
  a.ldc = C.ld;
  a.sC0 = C.s0;
  a.sC1 = C.s1;
  a.nb1 = nb1;
  a.tiles_m = (int)cdiv(M, BM);
  a.tiles_n = (int)cdiv(N, BN);
  a.alpha = alpha;
  a.beta = beta;
  const int64_t tiles = (int64_t)a.tiles_m * a.tiles_n;
  const int64_t nbatch = (int64_t)nb0 * nb1;
  const bool batched = nbatch > 1;
  const DType acc_t = e == DType::F64 ? DType::F64 : DType::F32;
  bool split = ksplit > 1 || C.t != e || sumsq != nullptr;
  if (!batched && ksplit == 0 && tiles < 1024) {
    // small outputs (Gram matrices) take up to 64 k-splits when the scratch
    // holds them
    const int cap = (int64_t)M * N <= 65536 ? 64 : MAX_SPLIT;
    const int want = (int)std::min<int64_t>(cap, std::max<int64_t>(1, 1024 / tiles));
    const int maxk = (int)std::max<int64_t>(1, cdiv(K, 4 * BK));
    const int fit = (int)std::max<int64_t>(
        1, (int64_t)(ws.bytes / ((size_t)M * N * dtype_size(acc_t))));
    ksplit = std::min(std::min(want, maxk), fit);
    if (ksplit > 1) split = true;
  }
  if (ksplit < 1) ksplit = 1;
  if (split && batched)
    throw std::invalid_argument("gemm: split-K output or a foreign output type needs an unbatched product");
  if (split) {
    const size_t need = (size_t)ksplit * M * N * dtype_size(acc_t);
    if (need > ws.bytes) throw std::invalid_argument("gemm: scratch too small");
  }
  a.kchunk = split ? (int)std::max<int64_t>(BK, cdiv(cdiv(K, ksplit), BK) * BK) : std::max(K, 1);
  if (split) {
    ksplit = (int)std::max<int64_t>(1, cdiv(K, a.kchunk));
    a.C = ws.p;
  }
  dim3 grid((unsigned)(tiles * nbatch), split ? ksplit : 1);
  if (ev) CTM_HIP(hipEventRecord(ev->begin, s));
  const bool vec = vec_ok(A, dtype_size(e)) && vec_ok(B, dtype_size(e));
  switch (e) {
    case DType::F64: launch_any<double>(split, vec, A.trans, B.trans, cfg, grid, s, a); break;
    case DType::F32: launch_any<float>(split, vec, A.trans, B.trans, cfg, grid, s, a); break;
    case DType::BF16: launch_any<bf16>(split, vec, A.trans, B.trans, cfg, grid, s, a); break;
  }
  CTM_LAUNCHED();
  if (ev) CTM_HIP(hipEventRecord(ev->end, s));
  if (split) {
    if (acc_t == DType::F64)
      launch_reduce<double>(C.t, (const double*)ws.p, ksplit, M, N, C.p, C.ld, alpha, beta, sumsq, s);
    else
      launch_reduce<float>(C.t, (const float*)ws.p, ksplit, M, N, C.p, C.ld, alpha, beta, sumsq, s);
    CTM_LAUNCHED();
  }
}

}  // namespace ctm
