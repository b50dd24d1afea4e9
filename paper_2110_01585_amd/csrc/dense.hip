// Gaussian i.i.d. compressive sensing: Woodbury moments of the likelihood site
// (see dense.h).  FP64 throughout; the three large products (S = H D^-1 H^T,
// the Cholesky trailing updates, the blocked triangular solve for Z^T) run on
// one GEMM kernel built on v_mfma_f64_16x16x4f64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.h"

namespace eptv {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kDT = 64;   // Cholesky block size (and the small GEMM tile)
constexpr int kDK = 32;   // K depth staged in LDS per GEMM round

// C = beta C + alpha A diag(w) B^T (+ diag on the main diagonal): A is M x K
// and B is N x K, both with k contiguous; w (length K) may be null.  With
// `lower`, only the elements n <= m are written (tiles above the diagonal are
// skipped).  One 64 x 64 output tile per workgroup, 4 waves of 32 x 32, each
// as 2 x 2 blocks of 16 x 16 MFMA outputs.  MFMA operand layout (16x16x4
// f64): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] (k = l / 16); the
// result element (4 r + l / 16, l % 16) is register r of lane l.  The next K
// round's operands are loaded into registers while the current one is
// multiplied.  A workgroup reads all of A's rows of its tile before it writes
// C, so C may alias A when the output has a single tile column (N <= 64).
// The staged tiles are k-major with a swizzle: element (row, k) sits at
// [k][(row + 16 ((k / 8) % 4)) % 64] of a row of 80, so the MFMA operand reads
// (16 rows x 4 k per wave) and the staging writes (16 rows x 4 groups of 8 k
// per wave) both touch each bank pair at most twice, the minimum for 8-byte
// accesses of 64 lanes.  Operand rows are read as 16-byte words where the
// leading dimensions and base addresses allow it (`vec`).
template <class TA, class TB>
struct GemmArgs {
  const TA* A;
  long long lda;
  const TB* B;
  long long ldb;
  const double* w;
  double* C;
  long long ldc;
  int M, N, K;
  double alpha, beta, diag;
  int lower;
  int nt_n;   // tiles along n
  int vec;    // rows of A, B (and w) may be read as 16-byte words
};

__device__ __forceinline__ int swz(int row, int k) { return (row + 16 * ((k >> 3) & 3)) & (kDT - 1); }

// eight consecutive elements as doubles, from a 16-byte aligned address
__device__ __forceinline__ void load8(const float* p, double (&v)[8]) {
  const float4 x = *reinterpret_cast<const float4*>(p);
  const float4 y = *reinterpret_cast<const float4*>(p + 4);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
}
__device__ __forceinline__ void load8(const double* p, double (&v)[8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 x = *reinterpret_cast<const double2*>(p + 2 * i);
    v[2 * i] = x.x;
    v[2 * i + 1] = x.y;
  }
}

template <class TA, class TB>
__global__ __launch_bounds__(256) void k_dgemm_nt(GemmArgs<TA, TB> g) {
  constexpr int BT = kDT, KD = kDK;
  constexpr int NB = 2;                       // 16 x 16 MFMA blocks per wave and direction
  constexpr int kRow = BT + 16;
  __shared__ double As[KD][kRow];
  __shared__ double Bs[KD][kRow];
  const int tm = blockIdx.x / g.nt_n, tn = blockIdx.x % g.nt_n;
  const int m0 = tm * BT, n0 = tn * BT;
  if (g.lower && n0 > m0 + BT - 1) return;    // whole tile above the diagonal
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * (BT / 2), wn = (wave & 1) * (BT / 2);
  d4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = d4{0, 0, 0, 0};
  constexpr int kPer = BT * KD / 256;         // staged elements per thread and operand
  constexpr int kTpr = KD / kPer;             // threads per staged row
  const int lr = t / kTpr, lk = (t % kTpr) * kPer;
  const int am = m0 + lr, bn = n0 + lr;
  const TA* arow = g.A + (long long)am * g.lda;
  const TB* brow = g.B + (long long)bn * g.ldb;
  static_assert(kPer == 8, "the staging reads eight consecutive k per thread");
  double av[kPer], bv[kPer];
  auto fetch = [&](int k0) {
    if (g.vec && k0 + lk + kPer <= g.K) {
      if (am < g.M) {
        load8(arow + k0 + lk, av);
      } else {
#pragma unroll
        for (int u = 0; u < kPer; ++u) av[u] = 0.0;
      }
      if (bn < g.N) {
        load8(brow + k0 + lk, bv);
        if (g.w) {
          double wv[kPer];
          load8(g.w + k0 + lk, wv);
#pragma unroll
          for (int u = 0; u < kPer; ++u) bv[u] *= wv[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < kPer; ++u) bv[u] = 0.0;
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = k0 + lk + u;
      const bool kin = k < g.K;
      av[u] = (am < g.M && kin) ? (double)arow[k] : 0.0;
      bv[u] = (bn < g.N && kin) ? (double)brow[k] * (g.w ? g.w[k] : 1.0) : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < g.K; k0 += KD) {
    __syncthreads();   // the previous round's LDS reads are done
    const int sc = swz(lr, lk);   // (lk + u) / 8 == lk / 8
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      As[lk + u][sc] = av[u];
      Bs[lk + u][sc] = bv[u];
    }
    __syncthreads();
    if (k0 + KD < g.K) fetch(k0 + KD);
#pragma unroll
    for (int kk = 0; kk < KD; kk += 4) {
      const int r = lane & 15, c = kk + (lane >> 4);
      double a[NB], b[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        a[i] = As[c][swz(wm + 16 * i + r, c)];
        b[i] = Bs[c][swz(wn + 16 * i + r, c)];
      }
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();   // every wave's reads of A are done before C (which may alias A) is written
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = 0; bj < NB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * bi + 4 * r + (lane >> 4);
        const int n = n0 + wn + 16 * bj + (lane & 15);
        if (m < g.M && n < g.N && (!g.lower || n <= m)) {
          double v = g.alpha * acc[bi][bj][r];
          if (g.beta != 0.0) v += g.beta * g.C[(long long)m * g.ldc + n];
          if (m == n) v += g.diag;
          g.C[(long long)m * g.ldc + n] = v;
        }
      }
}

template <class TA, class TB>
static hipError_t dgemm(const TA* A, long long lda, const TB* B, long long ldb, const double* w,
                        double* C, long long ldc, int M, int N, int K, double alpha, double beta,
                        double diag, bool lower, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  GemmArgs<TA, TB> g;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.w = w; g.C = C; g.ldc = ldc;
  g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.beta = beta; g.diag = diag;
  g.lower = lower ? 1 : 0;
  // 16-byte words: every row start aligned (base and leading dimension)
  auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  constexpr long long va = 16 / sizeof(TA), vb = 16 / sizeof(TB);
  g.vec = al(A) && al(B) && lda % va == 0 && ldb % vb == 0 && (!w || al(w)) ? 1 : 0;
  const int nt_m = (M + kDT - 1) / kDT;
  g.nt_n = (N + kDT - 1) / kDT;
  hipLaunchKernelGGL((k_dgemm_nt<TA, TB>), dim3(nt_m * g.nt_n), dim3(256), 0, s, g);
  return hipGetLastError();
}

// Cholesky factor of the nb x nb diagonal block at (j0, j0) of S, in place
// (lower triangle), and the inverse of the factor (64 x 64, lower triangular,
// row-major) into Linv, so that the triangular solves with the block become
// GEMMs; rows and columns past nb act as the identity.
// Right-looking on unscaled columns: with A = U D U^T (U unit lower, D the
// pivots), step c subtracts A[r][c] A[k][c] / D_c from A[r][k] (k > c, r >= k),
// and the same step eliminates column c from X, the running inverse of U (X = I
// at the start; X[r][j] -= U[r][c] X[c][j] for r > c, U[r][c] = A[r][c] / D_c).
// Both read only what steps before c have finished, so one barrier per step
// suffices: column c + 1 of A and row c + 1 of X are published in LDS (double
// buffered) by the threads that own them.  At the end L = U D^(1/2), i.e.
// L[r][k] = A[r][k] / sqrt(D_k), and L^-1 = D^(-1/2) X.  Thread t owns column
// t % 64, rows t / 64 + 4 q (q < 16), of both A and X, in registers.  A
// non-positive pivot gives NaN, which the sweep then reports as a non-finite
// state.
__global__ __launch_bounds__(256) void k_chol_diag(double* S, long long lds, int j0, int nb, double* Linv) {
  constexpr int kQ = kDT / 4;
  __shared__ double col[2][kDT];   // column c of A (unscaled)
  __shared__ double row[2][kDT];   // row c of X
  __shared__ double piv[kDT];
  const int t = threadIdx.x, k = t % kDT, g = t / kDT;
  double a[kQ], x[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int r = g + 4 * q;
    a[q] = (r < nb && k < nb) ? (r >= k ? S[(long long)(j0 + r) * lds + j0 + k] : 0.0)
                              : (r == k ? 1.0 : 0.0);
    x[q] = r == k ? 1.0 : 0.0;
    if (k == 0) col[0][r] = a[q];
    if (r == 0) row[0][k] = x[q];
  }
  __syncthreads();
  for (int c = 0; c < kDT; ++c) {
    const int b = c & 1;
    // every LDS read of the step before its first LDS write (the writes go to
    // the other buffer, which the compiler cannot tell from these), so the
    // reads are in flight together
    double arc[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) arc[q] = col[b][g + 4 * q];
    const double d = col[b][c];
    const double ck = col[b][k];
    const double xck = row[b][k];        // X[c][k]
    const double rd = 1.0 / d;
    const double akc = ck * rd;          // U[k][c]
    if (t == c) piv[c] = d;
    const bool kc = k > c;
    double xn = 0.0;                     // this thread's X[c + 1][k], if it holds row c + 1
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int r = g + 4 * q;
      if (kc && r >= k) a[q] = __builtin_fma(-arc[q], akc, a[q]);
      if (r > c) x[q] = __builtin_fma(-arc[q] * rd, xck, x[q]);
      xn = r == c + 1 ? x[q] : xn;
    }
    // column c + 1 of A and row c + 1 of X, published by their owners
    if (k == c + 1) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) col[b ^ 1][g + 4 * q] = a[q];
    }
    if (c + 1 < kDT && ((c + 1 - g) & 3) == 0) row[b ^ 1][k] = xn;
    __syncthreads();
  }
  const double sk = 1.0 / sqrt(piv[k]);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int r = g + 4 * q;
    if (r < nb && k < nb && r >= k) S[(long long)(j0 + r) * lds + j0 + k] = a[q] * sk;
    Linv[r * kDT + k] = x[q] / sqrt(piv[r]);
  }
}

// 32 x 32 tiles through LDS: out (cols x rows) = in^T (rows x cols), float.
__global__ __launch_bounds__(256) void k_transpose_f32(const float* __restrict__ in, float* __restrict__ out,
                                                       int rows, int cols) {
  __shared__ float tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int r = by + j, c = bx + tx;
    if (r < rows && c < cols) tile[j][tx] = in[(long long)r * cols + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = bx + j, c = by + tx;   // out row = in column
    if (r < cols && c < rows) out[(long long)r * rows + c] = tile[tx][j];
  }
}

// rows x cols float (contiguous) -> double with leading dimension ld >= cols
__global__ __launch_bounds__(256) void k_f32_to_f64(const float* __restrict__ in, double* __restrict__ out,
                                                    int rows, int cols, int ld) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)rows * cols) return;
  out[(i / cols) * ld + i % cols] = (double)in[i];
}

// Wave-level FP64 sum, the same bits on every lane (butterfly).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// H^T y: one wave per pixel (row of H^T), FP64 sum; into the H^T y plane and
// the pixel-space observation (both pitched).
__global__ __launch_bounds__(256) void k_gauss_hty(const float* __restrict__ HT, const float* __restrict__ y,
                                                   int M, int N, int W, int pitch, long long off,
                                                   float* __restrict__ hty, float* __restrict__ ypix) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= N) return;
  const float* h = HT + (long long)row * M;
  double acc = 0.0;
  for (int a = lane; a < M; a += kWave) acc += (double)h[a] * (double)y[a];
  acc = wave_sum(acc);
  if (lane == 0) {
    const long long p = off + (long long)(row / W) * pitch + row % W;
    hty[p] = (float)acc;
    ypix[p] = (float)acc;
  }
}

// Cavity precisions and right-hand side from the pitched planes into flat
// FP64 vectors; w = 1 / d.
__global__ __launch_bounds__(256) void k_gauss_gather(const float* __restrict__ tauc,
                                                      const float* __restrict__ bpl, int N, int W,
                                                      int pitch, long long off, double* __restrict__ d,
                                                      double* __restrict__ w, double* __restrict__ b) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const long long p = off + (long long)(i / W) * pitch + i % W;
  const double dv = (double)tauc[p];
  d[i] = dv;
  w[i] = 1.0 / dv;
  b[i] = (double)bpl[p];
}

// Partial sums of t = Z (b / d) = sum_i Z^T[i, :] b_i / d_i over chunks of
// kGaussChunk rows: one thread per column a of one chunk.
__global__ __launch_bounds__(256) void k_gauss_tpart(const double* __restrict__ ZT, int ld,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ w, int M, int N,
                                                     double* __restrict__ tpart) {
  const int a = blockIdx.x * 256 + threadIdx.x, chunk = blockIdx.y;
  if (a >= M) return;
  const int i0 = chunk * kGaussChunk, i1 = min(i0 + kGaussChunk, N);
  double acc = 0.0;
  for (int i = i0; i < i1; ++i) acc += ZT[(long long)i * ld + a] * (b[i] * w[i]);
  tpart[(long long)chunk * M + a] = acc;
}

__global__ __launch_bounds__(256) void k_gauss_tsum(const double* __restrict__ tpart, int M, int nchunk,
                                                    double* __restrict__ t) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= M) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += tpart[(long long)c * M + a];
  t[a] = acc;
}

// Per pixel (one wave per row of Z^T): v_i = 1/d_i - |z_i|^2 / d_i^2 and
// E_i = (b_i - z_i . t) / d_i, into the pitched variance and x planes.
__global__ __launch_bounds__(256) void k_gauss_moments(const double* __restrict__ ZT, int ld,
                                                       const double* __restrict__ t,
                                                       const double* __restrict__ d, const double* __restrict__ b,
                                                       int M, int N, int W, int pitch, long long off,
                                                       float* __restrict__ var, float* __restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= N) return;
  const double* z = ZT + (long long)row * ld;
  double zz = 0.0, zt = 0.0;
  for (int a = lane; a < M; a += kWave) {
    const double v = z[a];
    zz += v * v;
    zt += v * t[a];
  }
  zz = wave_sum(zz);
  zt = wave_sum(zt);
  if (lane == 0) {
    const double dv = d[row];
    const long long p = off + (long long)(row / W) * pitch + row % W;
    var[p] = (float)(1.0 / dv - zz / (dv * dv));
    x[p] = (float)((b[row] - zt) / dv);
  }
}

// ---------------------------------------------------------------------------
// host side

hipError_t gauss_setup(LikCtx& lc, const LikInstInfo* li, int n, hipStream_t s, std::string& err) {
  lc.gauss.clear();
  char* cur = lc.gaussbuf;
  auto take = [&](size_t bytes) {
    char* at = cur;
    cur += (bytes + 255) / 256 * 256;
    return at;
  };
  for (int i = 0; i < n; ++i) {
    if (li[i].op != OP_GAUSS) continue;
    GaussPlan P;
    for (int k = 0; k < (int)lc.hinst.size(); ++k)
      if (lc.hinst[k].inst == i) P.li = k;
    P.M = li[i].sense_rows;
    P.N = li[i].H * li[i].W;
    const size_t m = (size_t)P.M, nn = (size_t)P.N;
    P.nchunk = (P.N + kGaussChunk - 1) / kGaussChunk;
    P.Hm = reinterpret_cast<float*>(take(m * nn * 4));
    P.HT = reinterpret_cast<float*>(take(m * nn * 4));
    P.ld = gauss_ld(P.M);
    P.S = reinterpret_cast<double*>(take(m * (size_t)P.ld * 8));
    P.ZT = reinterpret_cast<double*>(take(nn * (size_t)P.ld * 8));
    P.d = reinterpret_cast<double*>(take(nn * 8));
    P.w = reinterpret_cast<double*>(take(nn * 8));
    P.b = reinterpret_cast<double*>(take(nn * 8));
    P.t = reinterpret_cast<double*>(take(m * 8));
    P.tpart = reinterpret_cast<double*>(take((size_t)P.nchunk * m * 8));
    P.Linv = reinterpret_cast<double*>(take((m + 63) / 64 * 64 * 64 * 8));
    P.y = reinterpret_cast<float*>(take(m * 4));
    hipError_t e = hipMemcpyAsync(P.Hm, li[i].sense, m * nn * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      err = "copy of the sensing matrix";
      return e;
    }
    hipLaunchKernelGGL(k_transpose_f32, dim3((P.N + 31) / 32, (P.M + 31) / 32), dim3(256), 0, s, P.Hm,
                       P.HT, P.M, P.N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    lc.gauss.push_back(P);
  }
  // the host matrix may go out of scope when ep_tv_create returns
  return lc.gauss.empty() ? hipSuccess : hipStreamSynchronize(s);
}

hipError_t gauss_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s) {
  for (GaussPlan& P : lc.gauss) {
    const LikInst& L = lc.hinst[P.li];
    hipError_t e = hipMemcpyAsync(P.y, d_y[L.inst], sizeof(float) * P.M, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gauss_hty, dim3((P.N + 3) / 4), dim3(256), 0, s, P.HT, P.y, P.M, P.N, L.W,
                       L.pitch, L.off, lc.planes[LP_HTY], lc.ypix);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Z^T[:, blocks lo..hi) L[lo..hi, lo..hi)^T = R in place (R: the current
// contents of those columns, already reduced by the columns before lo):
// split at the middle block, solve the left half, subtract its contribution
// from the right half (one GEMM over all rows), solve the right half; a single
// block is one GEMM with the inverse of its diagonal Cholesky block.
static hipError_t trsm_right(LikCtx& lc, GaussPlan& P, int lo, int hi, hipStream_t s) {
  const int M = P.M, N = P.N, ld = P.ld;
  const int c_lo = lo * kDT, c_hi = std::min(M, hi * kDT);
  if (hi - lo == 1) {
    const int bj = c_hi - c_lo;
    const double* Linv = P.Linv + (long long)lo * kDT * kDT;
    hipError_t e = lik_timed(lc, KT_DGEMM, s, [&]() {
      return dgemm<double, double>(P.ZT + c_lo, ld, Linv, kDT, nullptr, P.ZT + c_lo, ld, N, bj, bj, 1.0, 0.0,
                                   0.0, false, s);
    });
    lc.dgemm_flops += 2.0 * (double)N * (double)bj * (double)bj;
    return e;
  }
  const int mid = (lo + hi) / 2, c_mid = mid * kDT;
  hipError_t e = trsm_right(lc, P, lo, mid, s);
  if (e != hipSuccess) return e;
  // Z^T[:, mid..hi) -= Z^T[:, lo..mid) L[mid..hi, lo..mid)^T
  e = lik_timed(lc, KT_DGEMM, s, [&]() {
    return dgemm<double, double>(P.ZT + c_lo, ld, P.S + (long long)c_mid * ld + c_lo, ld, nullptr, P.ZT + c_mid,
                                 ld, N, c_hi - c_mid, c_mid - c_lo, -1.0, 1.0, 0.0, false, s);
  });
  if (e != hipSuccess) return e;
  lc.dgemm_flops += 2.0 * (double)N * (double)(c_hi - c_mid) * (double)(c_mid - c_lo);
  return trsm_right(lc, P, mid, hi, s);
}

hipError_t gauss_update(LikCtx& lc, const InstState* hst, hipStream_t s) {
  hipError_t e;
  for (GaussPlan& P : lc.gauss) {
    const LikInst& L = lc.hinst[P.li];
    const InstState& st = hst[L.inst];
    if (!(st.active && (st.sweeps > 0 || st.warm))) continue;
    const int M = P.M, N = P.N, ld = P.ld, nb = (M + kDT - 1) / kDT;
    const double xi = 1.0 / (double)L.inv_xi;
    hipLaunchKernelGGL(k_gauss_gather, dim3((N + 255) / 256), dim3(256), 0, s, lc.planes[LP_TAUC],
                       lc.planes[LP_B], N, L.W, L.pitch, L.off, P.d, P.w, P.b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // S = xi I + H D^-1 H^T (lower triangle), then its Cholesky factor in place
    e = lik_timed(lc, KT_DGEMM, s, [&]() {
      return dgemm<float, float>(P.Hm, N, P.Hm, N, P.w, P.S, ld, M, M, N, 1.0, 0.0, xi, true, s);
    });
    if (e != hipSuccess) return e;
    lc.dgemm_flops += (double)M * (double)(M + kDT) * (double)N;
    for (int j = 0; j < nb; ++j) {
      const int j0 = j * kDT, bj = std::min(kDT, M - j0), rest = M - j0 - bj;
      double* Linv = P.Linv + (long long)j * kDT * kDT;
      hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, P.S, (long long)ld, j0, bj, Linv);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (rest <= 0) break;
      // panel L_ij = S_ij L_jj^-T, in place
      double* panel = P.S + (long long)(j0 + bj) * ld + j0;
      e = lik_timed(lc, KT_DGEMM, s, [&]() {
        return dgemm<double, double>(panel, ld, Linv, kDT, nullptr, panel, ld, rest, bj, bj, 1.0, 0.0, 0.0,
                                     false, s);
      });
      if (e != hipSuccess) return e;
      lc.dgemm_flops += 2.0 * (double)rest * (double)bj * (double)bj;
      double* trail = P.S + (long long)(j0 + bj) * ld + (j0 + bj);
      e = lik_timed(lc, KT_DGEMM, s, [&]() {
        return dgemm<double, double>(panel, ld, panel, ld, nullptr, trail, ld, rest, rest, bj, -1.0, 1.0, 0.0,
                                     true, s);
      });
      if (e != hipSuccess) return e;
      lc.dgemm_flops += (double)rest * (double)(rest + kDT) * (double)bj;
    }
    // Z^T = H^T L^-T (Z^T L^T = H^T), recursively over column blocks so that
    // the large updates are single wide GEMMs
    hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)(((long long)N * M + 255) / 256)), dim3(256), 0, s, P.HT,
                       P.ZT, N, M, ld);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = trsm_right(lc, P, 0, nb, s)) != hipSuccess) return e;
    // t = Z (b / d), then v and E per pixel
    hipLaunchKernelGGL(k_gauss_tpart, dim3((M + 255) / 256, P.nchunk), dim3(256), 0, s, P.ZT, ld, P.b, P.w, M,
                       N, P.tpart);
    hipLaunchKernelGGL(k_gauss_tsum, dim3((M + 255) / 256), dim3(256), 0, s, P.tpart, M, P.nchunk, P.t);
    hipLaunchKernelGGL(k_gauss_moments, dim3((N + 3) / 4), dim3(256), 0, s, P.ZT, ld, P.t, P.d, P.b, M, N, L.W,
                       L.pitch, L.off, lc.planes[LP_VAR], lc.planes[LP_X]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace eptv
