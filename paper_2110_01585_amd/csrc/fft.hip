// Masked orthonormal 2-D DFT operator for compressive sensing, on a
// hand-written FFT.
//
// Observation model (Sec. II-A, Eq. (1), with H = a subset of the orthonormal
// 2-D DFT coefficients): y_w = (F x)_w + n_w for w in the mask, complex noise of
// variance xi per real component.  Treating (Re, Im) as two real observations,
//   H^T H v = Re(F^H diag(mask) F v),   H^T y = Re(F^H diag(mask) y),
// and H^T H is circulant with eigenvalues (mask(w) + mask(-w)) / 2.
//
// FFT: power-of-two lengths up to 4096.  A 2-D transform is a batch of row
// FFTs (whole rows in LDS, up to 4096 points per workgroup; Stockham auto-sort
// passes of radix 16, then 8, 4 or 2, each work item doing its radix-R DFT in
// registers; twiddles from a full-circle table), a tiled transpose, and a
// second batch of row FFTs; the spectrum-domain products are applied in that
// transposed layout (element (c, r) holds frequency (r, c)), and the inverse
// transform undoes the transpose.  Loads and stores of every pass are
// contiguous per row.  Element-wise work before and after the transform
// (building the search direction, scaling, the final q = H^T H p / xi +
// tau_c p) is fused into the first and last passes.
#include <cmath>
#include <cstring>

#include "fft.h"

namespace eptv {

enum {
  PRE_COMPLEX = 0,   // load the complex row from `src`
  PRE_REAL,          // load a real plane (pitched), imaginary part 0
  PRE_DIRECTION,     // p = z + beta p_in (or x in mode 0) from the CG planes; store p_out
  PRE_OBS            // observed coefficients (user array, interleaved) times the mask
};
enum {
  POST_COMPLEX = 0,  // store the complex row to `dst`
  POST_SCALE,        // multiply by `mul` (transposed layout, real) then store
  POST_Q,            // q = Re(v) * scale / xi + tau_c * p  (real plane), store q
  POST_REAL,         // real part * scale -> real plane
  POST_PRECOND       // multiply by scale / (mul / xi + d_bar) (transposed layout), store
};

struct FftArgs {
  const float2* src;
  float2* dst;
  const float2* tw;          // e^{-2 pi i t / L}, t < L/2
  int nrows, L, logL;
  int pre, post, inverse;
  // real planes (pitched) for PRE_REAL / PRE_DIRECTION / POST_Q / POST_REAL
  long long off;
  int pitch;
  const float* real_in;      // PRE_REAL
  float* real_out;           // POST_REAL, POST_Q
  const float* mul;          // POST_SCALE: per-element real factor (transposed layout, dense)
  float scale;
  // CG planes
  const float* r; const float* tauc; const float* x; const float* p_in; float* p_out;
  const float* pvec;         // POST_Q: the vector whose product is formed
  const float* zpl;          // PRE_DIRECTION with a stored preconditioned residual (else null)
  float diagA, inv_xi;
  const InstState* st;       // PRE_DIRECTION: beta and the iteration count of this instance
  int inst;
  int mode0;                 // PRE_DIRECTION: use x (the product A x for the CG start)
  const float* obs;          // PRE_OBS: interleaved complex observations (user), dense
  const uint8_t* mask;       // PRE_OBS
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// LDS index with one pad element per 16: the radix-16 pass writes 16
// consecutive outputs per work item, which without padding puts the lanes of a
// wave 128 bytes apart and onto the same few LDS banks.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
template <int N>
struct Padded {
  static constexpr int value = N + N / 16;
};

// ---- in-register DFTs of size 2..16 (radix-2 decimation in time) ----
// cos(2 pi t / 16); the argument is a compile-time constant once the butterfly
// loops are unrolled, so the value folds into the instruction
__device__ constexpr float cos16(int t) {
  switch (t & 15) {
    case 0: return 1.0f;
    case 1: case 15: return 0.92387953251128674f;
    case 2: case 14: return 0.70710678118654752f;
    case 3: case 13: return 0.38268343236508977f;
    case 4: case 12: return 0.0f;
    case 5: case 11: return -0.38268343236508977f;
    case 6: case 10: return -0.70710678118654752f;
    case 7: case 9: return -0.92387953251128674f;
    default: return -1.0f;
  }
}

__device__ constexpr int bitrev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

// b e^{s 2 pi i t / 16}, s = +1 for the inverse transform and -1 for the
// forward one; t < 8.  t = 0 and t = 4 (a multiplication by s i) cost nothing.
template <bool INV>
__device__ __forceinline__ float2 rot16(float2 b, int t) {
  constexpr float sg = INV ? 1.f : -1.f;
  if (t == 0) return b;
  if (t == 4) return make_float2(-sg * b.y, sg * b.x);
  const float c = cos16(t), sn = sg * cos16(t + 12);   // sin(x) = cos(x - pi/2)
  return make_float2(c * b.x - sn * b.y, c * b.y + sn * b.x);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2 (&v)[R]) {
  constexpr int bits = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bitrev_c(i, bits);
    if (j > i) {
      const float2 t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
#pragma unroll
  for (int m = 2; m <= R; m <<= 1) {
#pragma unroll
    for (int k = 0; k < R; k += m) {
#pragma unroll
      for (int j = 0; j < m / 2; ++j) {
        // w = e^{s 2 pi i j / m}, index j * 16 / m of the 16-point circle
        const float2 tw = rot16<INV>(v[k + j + m / 2], j * (16 / m));
        const float2 u = v[k + j];
        v[k + j] = make_float2(u.x + tw.x, u.y + tw.y);
        v[k + j + m / 2] = make_float2(u.x - tw.x, u.y - tw.y);
      }
    }
  }
}

// One radix-R Stockham pass over `rows` rows of length L held in LDS, in place:
// every work item reads its R inputs into registers before the barrier and
// writes its R outputs after it.  Work item j of a row (j < L/R), k = j mod Ns:
//   in:  X[j + r L/R],  twiddled by e^{s 2 pi i r k / (R Ns)}
//   out: X[(j - k) R + k + r Ns]
// R, Ns and L are compile-time, so the index arithmetic is shifts and masks.
// In the padded index, the r-th input and output of an item sit at fixed
// offsets from its first ones whenever the unpadded stride is a multiple of 16
// (or, for the outputs of the first pass, the R outputs lie in one group of
// 16), so those accesses take immediate offsets.
template <int R, int Ns, int L, bool INV, int NP>
__device__ __forceinline__ void stockham_pass(float2* X, int rows, const float2* __restrict__ tw) {
  // work items per thread for NP points in the workgroup (NP <= 4096)
  constexpr int kItems = NP / R > 256 ? NP / R / 256 : 1;
  constexpr int per_row = L / R;
  constexpr int step = L / (R * Ns);
  constexpr bool kInFold = per_row % 16 == 0;
  constexpr int kInStride = per_row + per_row / 16;
  constexpr bool kOutFold = Ns == 1 || Ns % 16 == 0;
  constexpr int kOutStride = Ns == 1 ? 1 : Ns + Ns / 16;
  const int total = rows * per_row;
  float2 v[kItems][R];
  int base[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int w = threadIdx.x + it * 256;
    base[it] = -1;
    if (w < total) {
      const int row = w / per_row, j = w % per_row;
      const int k = j & (Ns - 1);
      const int rbase = row * L + j;
      const int pin = pidx(rbase);
      const int ks = k * step;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 x = X[kInFold ? pin + r * kInStride : pidx(rbase + r * per_row)];
        if (Ns > 1 && r > 0) {
          const float2 t = tw[r * ks];   // e^{-2 pi i r k / (R Ns)}
          x = INV ? make_float2(x.x * t.x + x.y * t.y, x.y * t.x - x.x * t.y)
                  : make_float2(x.x * t.x - x.y * t.y, x.y * t.x + x.x * t.y);
        }
        v[it][r] = x;
      }
      base[it] = row * L + (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    if (base[it] >= 0) {
      dft_reg<R, INV>(v[it]);
      const int pout = pidx(base[it]);
#pragma unroll
      for (int r = 0; r < R; ++r)
        X[kOutFold ? pout + r * kOutStride : pidx(base[it] + r * Ns)] = v[it][r];
    }
  }
  __syncthreads();
}

// All passes of a length-L transform in a workgroup of NP points: radix 16
// while at least 16 points per butterfly remain, then one pass of the remaining
// radix.  (Radix-8 passes, which keep all four waves busy in a 2048-point
// workgroup where radix-16 passes occupy two, measured slower: one more LDS
// round trip and barrier per transform.)
template <int L, int Ns, bool INV, int NP>
__device__ __forceinline__ void fft_passes(float2* X, int rows, const float2* __restrict__ tw) {
  if constexpr (Ns < L) {
    constexpr int R = (L / Ns) >= 16 ? 16 : (L / Ns);
    stockham_pass<R, Ns, L, INV, NP>(X, rows, tw);
    fft_passes<L, Ns * R, INV, NP>(X, rows, tw);
  }
}

// Complex rows per workgroup of the row-transform kernels for length L: 2048
// points, at most 16 rows (4096-point blocks, one radix-16 item per thread,
// halve the workgroups in flight and run slower).  The kernels' LDS arrays,
// their launch grids and the RF_INV partial counts all follow from this one
// definition.
// Entries of the twiddle table the passes of a length-L transform read: one
// more than the largest index r k L / (R Ns) over the passes' radix R, stride Ns,
// r < R and k < Ns.
constexpr int tw_span(int L) {
  int m = 0;
  for (int Ns = 1; Ns < L;) {
    const int R = L / Ns >= 16 ? 16 : L / Ns;
    const int v = (R - 1) * (Ns - 1) * (L / (R * Ns));
    m = v > m ? v : m;
    Ns *= R;
  }
  return m + 1;
}

constexpr int rows_per_block(int L) { return L >= 2048 ? 1 : (2048 / L > 16 ? 16 : 2048 / L); }

template <int L>
__global__ __launch_bounds__(256) void k_fft_rows(FftArgs a) {
  constexpr int kRows = rows_per_block(L);
  __shared__ float2 X[Padded<kRows * L>::value];
  const int row0 = blockIdx.x * kRows;
  const int rows = min(kRows, a.nrows - row0);
  // ---- load (pre-op) ----
  #pragma unroll
  for (int u_ = 0; u_ < (kRows * L + 255) / 256; ++u_) {
    const int i = threadIdx.x + u_ * 256;
    if (i >= rows * L) continue;
    const int row = row0 + i / L, c = i % L;
    float2 v;
    if (a.pre == PRE_COMPLEX) {
      v = a.src[(long long)row * L + c];
    } else if (a.pre == PRE_REAL) {
      v = make_float2(a.real_in[a.off + (long long)row * a.pitch + c], 0.f);
    } else if (a.pre == PRE_DIRECTION) {
      const long long p = a.off + (long long)row * a.pitch + c;
      float pv;
      if (a.mode0) {
        pv = a.x[p];
      } else {
        const InstState& st = a.st[a.inst];
        const float z = a.zpl ? a.zpl[p] : a.r[p] / (a.diagA + a.tauc[p]);
        pv = st.cg_it == 0 ? z : z + (float)st.cg_beta * a.p_in[p];
        a.p_out[p] = pv;
      }
      v = make_float2(pv, 0.f);
    } else {   // PRE_OBS
      const long long q = (long long)row * L + c;
      v = a.mask[q] ? make_float2(a.obs[2 * q], a.obs[2 * q + 1]) : make_float2(0.f, 0.f);
    }
    X[pidx(i)] = v;
  }
  __syncthreads();
  // ---- Stockham passes: radix 16 while possible, then 8, 4, 2 ----
  if (a.logL > 0) {
    if (a.inverse)
      fft_passes<L, 1, true, kRows * L>(X, rows, a.tw);
    else
      fft_passes<L, 1, false, kRows * L>(X, rows, a.tw);
  }
  // ---- store (post-op) ----
  #pragma unroll
  for (int u_ = 0; u_ < (kRows * L + 255) / 256; ++u_) {
    const int i = threadIdx.x + u_ * 256;
    if (i >= rows * L) continue;
    const int row = row0 + i / L, c = i % L;
    const float2 v = X[pidx(i)];
    if (a.post == POST_COMPLEX) {
      a.dst[(long long)row * L + c] = v;
    } else if (a.post == POST_SCALE) {
      const float m = a.mul[(long long)row * L + c] * a.scale;
      a.dst[(long long)row * L + c] = make_float2(v.x * m, v.y * m);
    } else if (a.post == POST_Q) {
      const long long p = a.off + (long long)row * a.pitch + c;
      a.real_out[p] = v.x * a.scale * a.inv_xi + a.tauc[p] * a.pvec[p];
    } else if (a.post == POST_REAL) {
      a.real_out[a.off + (long long)row * a.pitch + c] = v.x * a.scale;
    } else {   // POST_PRECOND
      const float dbar = (float)a.st[a.inst].dbar;
      const float m = a.scale / (a.mul[(long long)row * L + c] * a.inv_xi + dbar);
      a.dst[(long long)row * L + c] = make_float2(v.x * m, v.y * m);
    }
  }
}

// ---------------------------------------------------------------------------
// Real-input 2-D transforms for the fast CG of circulant-preconditioned
// instances: z = M^{-1} r with M = H^T H / xi + d_bar I, and the exact product
// q = (H^T H / xi + diag tau_c) p, both through three row kernels and two
// transposes on half spectra (the input is real, the spectra are even).
//   RF_FWD:  complex row j = v[2j] + i v[2j+1] (two real rows), forward FFT, split
//            into the half spectra of both rows, k = 0..W/2:
//              V_a(k) = (Z(k) + conj Z(W-k)) / 2,  V_b(k) = (Z(k) - conj Z(W-k)) / 2i;
//            stored as rows 2j, 2j+1 of an H x (W/2+1) array.  v = r, or the new
//            search direction p = z + beta p (written back) for the product;
//   RF_FILT: (after a transpose) rows of length H, one per k: forward FFT,
//            multiply by scale / (spec / xi + d_bar) or by scale * spec / xi,
//            inverse FFT;
//   RF_INV:  (after the transpose back) rebuild Z(k) = V_a(k) + i V_b(k) for all k
//            (V(W-k) = conj V(k)), inverse FFT, Re -> row 2j, Im -> row 2j+1:
//            z with partials of r.z and r.r, or q = result + tau_c p with
//            partials of p.q.
enum { RF_FWD = 0, RF_FILT, RF_INV };
enum { RFM_PRECOND = 0, RFM_PRODUCT = 1 };

struct RfftArgs {
  const float2* src;         // RF_FILT / RF_INV input (dense complex rows)
  float2* dst;               // RF_FWD / RF_FILT output (dense complex rows)
  const float2* tw;
  int nrows;                 // complex rows processed (RF_FWD / RF_INV: H / 2; RF_FILT: W/2 + 1)
  int logL;
  int ld;                    // row stride of the half-spectrum array (W/2 + 1)
  int tld;                   // RF_FWD output / RF_INV input: the half spectrum transposed,
                             // element (row, k) at [k tld + row] (tld = H)
  int mode;                  // RFM_PRECOND or RFM_PRODUCT
  int update;                // RF_FWD precondition: first x += alpha p, r -= alpha q
  const double* apart;       // RF_FWD update: the p.q partials alpha is formed from
  int acount;
  long long off;             // real planes (pitched)
  int pitch;
  float* r;                  // residual
  float* x;                  // CG iterate (RF_FWD precondition with update)
  const float* q;            // A p (RF_FWD precondition with update)
  const float* z;            // preconditioned residual (RF_FWD, product: direction update)
  const float* p_in;         // previous search direction (RF_FWD product)
  float* p;                  // current direction (RF_FWD product: written; RF_INV product and
                             // RF_FWD precondition update: read)
  const float* tauc;
  float* out;                // RF_INV: z (precondition) or q (product)
  const float* specT;        // eigenvalues of H^T H, transposed dense (W x H)
  float inv_xi, scale;
  float diagA;               // diagonal of H^T H / xi (the scaled preconditioner's a_0)
  const InstState* st;
  InstState* st_w;           // RF_FWD update: block 0 records alpha
  int inst;
  double* part0;             // RF_INV partials at [part_base + row block]
  double* part1;
  int part_base;
};

// alpha = r.z / p.q of a CG step (Hestenes-Stiefel), from the p.q partials of
// the product, summed exactly as the per-instance finishing kernel sums them:
// each thread in ascending order, a butterfly over each wave, then the four
// wave totals in a fixed order.  Every workgroup of the pass forms the same
// value.  Called by all 256 threads.
__device__ __forceinline__ double cg_alpha(const double* __restrict__ part, int cnt, double rz) {
  double s = 0.0;
  constexpr int kU = 16;
  for (int t0 = threadIdx.x; t0 < cnt; t0 += kU * 256) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * 256;
      v[u] = t < cnt ? part[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) s += v[u];
  }
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
  __shared__ double w[4];
  if (threadIdx.x % kWave == 0) w[threadIdx.x / kWave] = s;
  __syncthreads();
  const double pq = (w[0] + w[1]) + (w[2] + w[3]);
  return pq != 0.0 ? rz / pq : 0.0;
}

// What one thread loads for its workgroup's rows in each stage, all of it
// before the first LDS store.
template <int L, int STAGE>
struct RfftRegs {
  static constexpr int kPts = rows_per_block(L) * L;
  static constexpr int N4 = (kPts / 4 + 255) / 256;                          // 4-column words
  static constexpr int N2 = (kPts / 2 + 255) / 256;                          // complex pairs
  static constexpr int NH = (rows_per_block(L) * (L / 2 + 1) + 255) / 256;   // half spectrum
  // RF_FWD: r or z (v), q or p_in (w), x, p of rows 2j (a) and 2j+1 (b)
  float4 va[STAGE == RF_FWD ? N4 : 1], vb[STAGE == RF_FWD ? N4 : 1];
  float4 wa[STAGE == RF_FWD ? N4 : 1], wb[STAGE == RF_FWD ? N4 : 1];
  float4 xa[STAGE == RF_FWD ? N4 : 1], xb[STAGE == RF_FWD ? N4 : 1];
  float4 pa[STAGE == RF_FWD ? N4 : 1], pb[STAGE == RF_FWD ? N4 : 1];
  float4 ca[STAGE == RF_FWD ? N4 : 1], cb[STAGE == RF_FWD ? N4 : 1];   // tau_c (scaled preconditioner)
  // RF_FILT: two complex values and their two eigenvalues
  float4 lv[STAGE == RF_FILT ? N2 : 1];
  float2 sp[STAGE == RF_FILT ? N2 : 1];
  // RF_INV: (V_a(k), V_b(k))
  float4 ab[STAGE == RF_INV ? NH : 1];
};

template <int L, int STAGE>
__global__ __launch_bounds__(256) void k_rfft(RfftArgs a) {
  constexpr int kRows = rows_per_block(L);
  constexpr int kPts = kRows * L;
  using Regs = RfftRegs<L, STAGE>;
  constexpr int N4 = Regs::N4, N2 = Regs::N2, NH = Regs::NH;
  __shared__ float2 X[Padded<kPts>::value];
  const int half = L / 2;
  // neighbouring row blocks (which share the cache lines of the transposed
  // half spectrum) run on one XCD
  const int u = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = u * kRows, rows = min(kRows, a.nrows - row0);
  const InstState& st = a.st[a.inst];
  if (st.cg_done != 0) {   // uniform per launch (one instance)
    if (STAGE == RF_INV && threadIdx.x == 0) {
      a.part0[a.part_base + u] = 0.0;
      a.part1[a.part_base + u] = 0.0;
    }
    return;
  }
  // The part of the twiddle table the passes read, in LDS: the passes then
  // issue no global loads, and the table's one load per workgroup overlaps
  // with the data loads.
  constexpr int kTw = (tw_span(L) + 1) / 2 * 2;
  __shared__ float2 T[kTw];
  for (int i = threadIdx.x; 2 * i < kTw; i += 256)
    reinterpret_cast<float4*>(T)[i] = reinterpret_cast<const float4*>(a.tw)[i];

  const bool first = st.cg_it == 0;
  const bool upd = a.mode == RFM_PRECOND && a.update;
  // diagonally scaled circulant S C^{-1} S, s_i^2 = (a_0 + d_bar) / (a_0 + tau_c,i),
  // which gives the preconditioner A's diagonal (set per solve; uniform per launch)
  const bool scaled = a.mode == RFM_PRECOND && st.pc_scaled != 0;
  // RF_FWD: the transformed plane v (r, or z for the new direction), the plane
  // w it is combined with (q for the update of r, p_in for p = z + beta p_in);
  // RF_INV: the plane e the result is dotted with (r, or p for q = result + tau_c p)
  const float* vsrc = a.mode == RFM_PRECOND ? a.r : a.z;
  const float* wsrc = a.mode == RFM_PRECOND ? a.q : a.p_in;
  const bool wload = a.mode == RFM_PRECOND ? upd : !first;
  const float* esrc = a.mode == RFM_PRECOND ? a.r : a.p;
  // plane index of column i % L of real row 2 (row0 + i / L)
  auto plane = [&](int i) __attribute__((always_inline)) {
    return a.off + (long long)(2 * (row0 + i / L)) * a.pitch + i % L;
  };
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);

  // ---- global loads ----
  Regs R;
  {
    if (STAGE == RF_FWD) {
      // the two real rows 2j, 2j+1 of each complex row, as 16-byte words of
      // four columns (planes and pitches are 64-float aligned, L is a multiple of 4)
#pragma unroll
      for (int q = 0; q < N4; ++q) {
        const int i = 4 * ((int)threadIdx.x + 256 * q);
        R.va[q] = R.vb[q] = R.wa[q] = R.wb[q] = R.xa[q] = R.xb[q] = R.pa[q] = R.pb[q] = zero4;
        R.ca[q] = R.cb[q] = zero4;
        if (i >= rows * L) continue;
        const long long p = plane(i), p1 = p + a.pitch;
        R.va[q] = *reinterpret_cast<const float4*>(vsrc + p);
        R.vb[q] = *reinterpret_cast<const float4*>(vsrc + p1);
        if (wload) {
          R.wa[q] = *reinterpret_cast<const float4*>(wsrc + p);
          R.wb[q] = *reinterpret_cast<const float4*>(wsrc + p1);
        }
        if (upd) {
          R.xa[q] = *reinterpret_cast<const float4*>(a.x + p);
          R.xb[q] = *reinterpret_cast<const float4*>(a.x + p1);
          R.pa[q] = *reinterpret_cast<const float4*>(a.p + p);
          R.pb[q] = *reinterpret_cast<const float4*>(a.p + p1);
        }
        if (scaled) {
          R.ca[q] = *reinterpret_cast<const float4*>(a.tauc + p);
          R.cb[q] = *reinterpret_cast<const float4*>(a.tauc + p1);
        }
      }
    } else if (STAGE == RF_FILT) {
      // two complex values (16 bytes) per load, rows contiguous, and the
      // filter's eigenvalues for use after the forward transform
#pragma unroll
      for (int q = 0; q < N2; ++q) {
        const int i = 2 * ((int)threadIdx.x + 256 * q);
        R.lv[q] = zero4;
        R.sp[q] = make_float2(0.f, 0.f);
        if (i >= rows * L) continue;
        const long long e = (long long)(row0 + i / L) * L + i % L;
        R.lv[q] = *reinterpret_cast<const float4*>(a.src + e);
        R.sp[q] = *reinterpret_cast<const float2*>(a.specT + e);
      }
    } else {
      // each stored k <= W/2 once (it fills Z(k) and Z(W-k))
#pragma unroll
      for (int q = 0; q < NH; ++q) {
        const int i = threadIdx.x + 256 * q;
        R.ab[q] = zero4;
        if (i >= rows * (half + 1)) continue;
        const int j = row0 + i / (half + 1), kk = i % (half + 1);
        R.ab[q] = *reinterpret_cast<const float4*>(a.src + (long long)kk * a.tld + 2 * j);
      }
    }
  }
  float alpha = 0.f;
  const float beta = (float)st.cg_beta;
  if (STAGE == RF_FWD && upd) {
    // after the data loads are issued, so their latency overlaps
    const double al = cg_alpha(a.apart, a.acount, st.cg_rz);
    alpha = (float)al;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st_w[a.inst].cg_alpha = al;
  }

  {
    // ---- element-wise work and the row data into LDS ----
    if (STAGE == RF_FWD) {
#pragma unroll
      for (int q = 0; q < N4; ++q) {
        const int i = 4 * ((int)threadIdx.x + 256 * q);
        if (i >= rows * L) continue;
        const long long p = plane(i), p1 = p + a.pitch;
        const float ra[4] = {R.va[q].x, R.va[q].y, R.va[q].z, R.va[q].w};
        const float rb[4] = {R.vb[q].x, R.vb[q].y, R.vb[q].z, R.vb[q].w};
        const float sa[4] = {R.wa[q].x, R.wa[q].y, R.wa[q].z, R.wa[q].w};
        const float sb[4] = {R.wb[q].x, R.wb[q].y, R.wb[q].z, R.wb[q].w};
        float oa[4], ob[4];
        if (a.mode == RFM_PRECOND) {
          if (upd) {
            const float xa4[4] = {R.xa[q].x, R.xa[q].y, R.xa[q].z, R.xa[q].w};
            const float xb4[4] = {R.xb[q].x, R.xb[q].y, R.xb[q].z, R.xb[q].w};
            const float pa4[4] = {R.pa[q].x, R.pa[q].y, R.pa[q].z, R.pa[q].w};
            const float pb4[4] = {R.pb[q].x, R.pb[q].y, R.pb[q].z, R.pb[q].w};
            float na[4], nb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              oa[k] = ra[k] - alpha * sa[k];
              ob[k] = rb[k] - alpha * sb[k];
              na[k] = xa4[k] + alpha * pa4[k];
              nb[k] = xb4[k] + alpha * pb4[k];
            }
            *reinterpret_cast<float4*>(a.x + p) = make_float4(na[0], na[1], na[2], na[3]);
            *reinterpret_cast<float4*>(a.x + p1) = make_float4(nb[0], nb[1], nb[2], nb[3]);
            *reinterpret_cast<float4*>(a.r + p) = make_float4(oa[0], oa[1], oa[2], oa[3]);
            *reinterpret_cast<float4*>(a.r + p1) = make_float4(ob[0], ob[1], ob[2], ob[3]);
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              oa[k] = ra[k];
              ob[k] = rb[k];
            }
          }
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            oa[k] = first ? ra[k] : ra[k] + beta * sa[k];
            ob[k] = first ? rb[k] : rb[k] + beta * sb[k];
          }
          *reinterpret_cast<float4*>(a.p + p) = make_float4(oa[0], oa[1], oa[2], oa[3]);
          *reinterpret_cast<float4*>(a.p + p1) = make_float4(ob[0], ob[1], ob[2], ob[3]);
        }
        if (scaled) {
          const float a0 = a.diagA, num = a0 + (float)st.dbar;
          const float ca4[4] = {R.ca[q].x, R.ca[q].y, R.ca[q].z, R.ca[q].w};
          const float cb4[4] = {R.cb[q].x, R.cb[q].y, R.cb[q].z, R.cb[q].w};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            oa[k] *= __builtin_sqrtf(num / (a0 + ca4[k]));
            ob[k] *= __builtin_sqrtf(num / (a0 + cb4[k]));
          }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) X[pidx(i + k)] = make_float2(oa[k], ob[k]);
      }
    } else if (STAGE == RF_FILT) {
#pragma unroll
      for (int q = 0; q < N2; ++q) {
        const int i = 2 * ((int)threadIdx.x + 256 * q);
        if (i >= rows * L) continue;
        X[pidx(i)] = make_float2(R.lv[q].x, R.lv[q].y);
        X[pidx(i + 1)] = make_float2(R.lv[q].z, R.lv[q].w);
      }
    } else {
#pragma unroll
      for (int q = 0; q < NH; ++q) {
        const int i = threadIdx.x + 256 * q;
        if (i >= rows * (half + 1)) continue;
        const int jr = i / (half + 1), kk = i % (half + 1);
        const float4 v = R.ab[q];   // V_a(k) = (v.x, v.y), V_b(k) = (v.z, v.w)
        X[pidx(jr * L + kk)] = make_float2(v.x - v.w, v.y + v.z);
        if (kk > 0 && kk < half) X[pidx(jr * L + L - kk)] = make_float2(v.x + v.w, v.z - v.y);
      }
    }
    __syncthreads();

    // ---- passes ----
    if (STAGE == RF_FWD) {
      fft_passes<L, 1, false, kPts>(X, rows, T);
    } else if (STAGE == RF_FILT) {
      fft_passes<L, 1, false, kPts>(X, rows, T);
      const float dbar = (float)st.dbar;
#pragma unroll
      for (int q = 0; q < N2; ++q) {
        const int i = 2 * ((int)threadIdx.x + 256 * q);
        if (i >= rows * L) continue;
        const float spv[2] = {R.sp[q].x, R.sp[q].y};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const float sp = spv[k] * a.inv_xi;
          // the preconditioner's filter needs no correctly rounded division
          const float m = a.mode == RFM_PRECOND ? a.scale * __builtin_amdgcn_rcpf(sp + dbar)
                                                : a.scale * sp;
          X[pidx(i + k)] = make_float2(X[pidx(i + k)].x * m, X[pidx(i + k)].y * m);
        }
      }
      __syncthreads();
      fft_passes<L, 1, true, kPts>(X, rows, T);
    } else {
      fft_passes<L, 1, true, kPts>(X, rows, T);
    }

    // ---- stores ----
    if (STAGE == RF_FWD) {
#pragma unroll
      for (int q = 0; q < (kRows * (L / 2 + 1) + 255) / 256; ++q) {
        const int i = threadIdx.x + q * 256;
        if (i >= rows * (half + 1)) continue;
        const int jr = i / (half + 1), k = i % (half + 1);
        const float2 zk = X[pidx(jr * L + k)];
        float2 zm = X[pidx(jr * L + ((L - k) & (L - 1)))];
        zm.y = -zm.y;                                   // conj Z(W - k)
        const float2 sa = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
        const float2 sb = make_float2(0.5f * (zk.y - zm.y), -0.5f * (zk.x - zm.x));   // (Z - conj) / 2i
        const int j = row0 + jr;
        *reinterpret_cast<float4*>(a.dst + (long long)k * a.tld + 2 * j) =
            make_float4(sa.x, sa.y, sb.x, sb.y);
      }
    } else if (STAGE == RF_FILT) {
#pragma unroll
      for (int q = 0; q < N2; ++q) {
        const int i = 2 * ((int)threadIdx.x + q * 256);
        if (i >= rows * L) continue;
        const float2 v0 = X[pidx(i)], v1 = X[pidx(i + 1)];
        *reinterpret_cast<float4*>(a.dst + (long long)(row0 + i / L) * L + i % L) =
            make_float4(v0.x, v0.y, v1.x, v1.y);
      }
    } else {
      // r (precondition) or p and tau_c (product), rows 2j and 2j+1 as 16-byte
      // words of four columns, all loaded before the first store (loaded here,
      // after the transform: issued with the spectrum they delay its passes)
      float4 ea[N4], eb[N4], ta[N4], tb[N4];
#pragma unroll
      for (int q = 0; q < N4; ++q) {
        const int i = 4 * ((int)threadIdx.x + 256 * q);
        ea[q] = eb[q] = ta[q] = tb[q] = zero4;
        if (i >= rows * L) continue;
        const long long p = plane(i), p1 = p + a.pitch;
        ea[q] = *reinterpret_cast<const float4*>(esrc + p);
        eb[q] = *reinterpret_cast<const float4*>(esrc + p1);
        if (a.mode != RFM_PRECOND || scaled) {
          ta[q] = *reinterpret_cast<const float4*>(a.tauc + p);
          tb[q] = *reinterpret_cast<const float4*>(a.tauc + p1);
        }
      }
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int q = 0; q < N4; ++q) {
        const int i = 4 * ((int)threadIdx.x + 256 * q);
        if (i >= rows * L) continue;
        const long long p = plane(i), p1 = p + a.pitch;
        const float va[4] = {ea[q].x, ea[q].y, ea[q].z, ea[q].w};
        const float vb[4] = {eb[q].x, eb[q].y, eb[q].z, eb[q].w};
        const float ua[4] = {ta[q].x, ta[q].y, ta[q].z, ta[q].w};
        const float ub[4] = {tb[q].x, tb[q].y, tb[q].z, tb[q].w};
        float oa[4], ob[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float2 zz = X[pidx(i + k)];
          if (a.mode == RFM_PRECOND) {
            oa[k] = zz.x;
            ob[k] = zz.y;
            if (scaled) {
              const float a0 = a.diagA, num = a0 + (float)st.dbar;
              oa[k] *= __builtin_sqrtf(num / (a0 + ua[k]));
              ob[k] *= __builtin_sqrtf(num / (a0 + ub[k]));
            }
            s0 += (double)va[k] * oa[k] + (double)vb[k] * ob[k];
            s1 += (double)va[k] * va[k] + (double)vb[k] * vb[k];
          } else {
            oa[k] = zz.x + ua[k] * va[k];
            ob[k] = zz.y + ub[k] * vb[k];
            s0 += (double)va[k] * oa[k] + (double)vb[k] * ob[k];
          }
        }
        *reinterpret_cast<float4*>(a.out + p) = make_float4(oa[0], oa[1], oa[2], oa[3]);
        *reinterpret_cast<float4*>(a.out + p1) = make_float4(ob[0], ob[1], ob[2], ob[3]);
      }
      // deterministic block sum: butterfly over each wave, then the four wave
      // totals in a fixed order
#pragma unroll
      for (int off = kWave / 2; off >= 1; off >>= 1) {
        s0 += __shfl_xor(s0, off, kWave);
        s1 += __shfl_xor(s1, off, kWave);
      }
      __shared__ double sa[4], sb[4];
      if (threadIdx.x % kWave == 0) {
        sa[threadIdx.x / kWave] = s0;
        sb[threadIdx.x / kWave] = s1;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        a.part0[a.part_base + u] = (sa[0] + sa[1]) + (sa[2] + sa[3]);
        a.part1[a.part_base + u] = (sb[0] + sb[1]) + (sb[2] + sb[3]);
      }
    }
  }
}

// out (W x H) = transpose of in (H x W), kTrT x kTrT tiles through padded LDS
constexpr int kTrT = 32;
__global__ __launch_bounds__(256) void k_transpose(const float2* __restrict__ in,
                                                   float2* __restrict__ out, int H, int W,
                                                   const InstState* __restrict__ st, int inst) {
  constexpr int kRowsPer = 256 / kTrT;
  if (st && st[inst].cg_done) return;   // a finished CG's passes are skipped, so is this
  __shared__ float2 tile[kTrT][kTrT + 1];
  const int bx = blockIdx.x * kTrT, by = blockIdx.y * kTrT;
  const int tx = threadIdx.x % kTrT, ty = threadIdx.x / kTrT;
  // compile-time trip counts, so all loads of a thread are in flight at once
#pragma unroll
  for (int k = 0; k < kTrT / kRowsPer; ++k) {
    const int r = ty + kRowsPer * k;
    const int gr = by + r, gc = bx + tx;
    if (gr < H && gc < W) tile[r][tx] = in[(long long)gr * W + gc];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTrT / kRowsPer; ++k) {
    const int r = ty + kRowsPer * k;
    const int gc = bx + r, gr = by + tx;   // output row = input column
    if (gc < W && gr < H) out[(long long)gc * H + gr] = tile[tx][r];
  }
}

__global__ void k_twiddles(float2* tw, int L) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L) return;
  double s, c;
  sincos(-6.283185307179586476925 * (double)t / (double)L, &s, &c);
  tw[t] = make_float2((float)c, (float)s);
}

// eigenvalues of H^T H: (mask(w) + mask(-w)) / 2, in the plane layout (for the
// spectral estimator) and in the transposed dense layout (for the products)
__global__ void k_dft_spectrum(const uint8_t* __restrict__ mask, float* __restrict__ spec_plane,
                               long long off, int pitch, float* __restrict__ specT, int H, int W) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)H * W) return;
  const int r = (int)(i / W), c = (int)(i % W);
  const int rn = (H - r) % H, cn = (W - c) % W;
  const float v = 0.5f * ((mask[i] ? 1.f : 0.f) + (mask[(long long)rn * W + cn] ? 1.f : 0.f));
  spec_plane[off + (long long)r * pitch + c] = v;
  specT[(long long)c * H + r] = v;
}

// transposed dense copy of a spectrum plane
__global__ void k_spec_to_T(const float* __restrict__ spec_plane, long long off, int pitch,
                            float* __restrict__ specT, int H, int W) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)H * W) return;
  const int r = (int)(i / W), c = (int)(i % W);
  specT[(long long)c * H + r] = spec_plane[off + (long long)r * pitch + c];
}

// per-tile partial sums of p.q for DFT instances (the FFT passes work on rows)
__global__ __launch_bounds__(256) void k_dot_tiles(const LikInst* __restrict__ inst,
                                                   const int4* __restrict__ tiles, int tile0,
                                                   int ntiles, const float* __restrict__ pv,
                                                   const float* __restrict__ q,
                                                   double* __restrict__ part0,
                                                   double* __restrict__ part1,
                                                   const InstState* __restrict__ st) {
  __shared__ double sa[256];
  const int tile = tile0 + blockIdx.x;
  const int4 td = tiles[tile];
  const LikInst L = inst[td.x];
  double acc = 0.0;
  if (!st[L.inst].cg_done) {
    const int c0 = td.y * kLikTW, r0 = td.z * kLikTH;
    const int c1 = min(c0 + kLikTW, L.W), r1 = min(r0 + kLikTH, L.H);
    const int cols = c1 - c0, n = cols * (r1 - r0);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const long long p = L.off + (long long)(r0 + i / cols) * L.pitch + (c0 + i % cols);
      acc += (double)pv[p] * (double)q[p];
    }
  }
  sa[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sa[threadIdx.x] += sa[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part0[tile] = sa[0];
    part1[tile] = 0.0;
  }
  (void)ntiles;
}

// ---------------------------------------------------------------------------
// host side

static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

template <int L>
static void launch_rows(const FftArgs& a, hipStream_t s) {
  constexpr int kRows = rows_per_block(L);
  hipLaunchKernelGGL(k_fft_rows<L>, dim3((a.nrows + kRows - 1) / kRows), dim3(256), 0, s, a);
}

static hipError_t rows(const FftArgs& a, hipStream_t s) {
  switch (a.L) {
    case 4: launch_rows<4>(a, s); break;
    case 8: launch_rows<8>(a, s); break;
    case 16: launch_rows<16>(a, s); break;
    case 32: launch_rows<32>(a, s); break;
    case 64: launch_rows<64>(a, s); break;
    case 128: launch_rows<128>(a, s); break;
    case 256: launch_rows<256>(a, s); break;
    case 512: launch_rows<512>(a, s); break;
    case 1024: launch_rows<1024>(a, s); break;
    case 2048: launch_rows<2048>(a, s); break;
    case 4096: launch_rows<4096>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L, int STAGE>
static void launch_rfft_t(const RfftArgs& a, hipStream_t s) {
  constexpr int kRows = rows_per_block(L);
  hipLaunchKernelGGL((k_rfft<L, STAGE>), dim3((a.nrows + kRows - 1) / kRows), dim3(256), 0, s, a);
}

template <int STAGE>
static hipError_t launch_rfft(int L, const RfftArgs& a, hipStream_t s) {
  switch (L) {
    case 4: launch_rfft_t<4, STAGE>(a, s); break;
    case 8: launch_rfft_t<8, STAGE>(a, s); break;
    case 16: launch_rfft_t<16, STAGE>(a, s); break;
    case 32: launch_rfft_t<32, STAGE>(a, s); break;
    case 64: launch_rfft_t<64, STAGE>(a, s); break;
    case 128: launch_rfft_t<128, STAGE>(a, s); break;
    case 256: launch_rfft_t<256, STAGE>(a, s); break;
    case 512: launch_rfft_t<512, STAGE>(a, s); break;
    case 1024: launch_rfft_t<1024, STAGE>(a, s); break;
    case 2048: launch_rfft_t<2048, STAGE>(a, s); break;
    case 4096: launch_rfft_t<4096, STAGE>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Number of partial-sum slots the RF_INV stage of an H x W instance writes
// (one per row block).
int rfft_partials(int H, int W) {
  const int kRows = rows_per_block(W);
  return (H / 2 + kRows - 1) / kRows;
}

static FftArgs base_args(const LikCtx& lc, const LikInst& L) {
  FftArgs a;
  std::memset(&a, 0, sizeof(a));
  a.st = lc.d_st;
  a.inst = L.inst;
  a.off = L.off;
  a.pitch = L.pitch;
  a.scale = 1.f;
  a.inv_xi = L.inv_xi;
  a.diagA = L.diagA;
  a.tauc = lc.planes[LP_TAUC];
  return a;
}

hipError_t dft_setup(LikCtx& lc, const LikInstInfo* li, int n, size_t fft_bytes, hipStream_t s,
                     std::string& err) {
  auto& list = lc.dft;
  list.clear();
  // workspace: per DFT instance A, B (complex N each), twiddles, transposed spectrum, mask
  char* cur = reinterpret_cast<char*>(lc.fft);
  size_t used = 0;
  for (size_t k = 0; k < lc.hinst.size(); ++k) {
    const LikInst& L = lc.hinst[k];
    if (L.op == OP_HAD || (L.op != OP_DFT && L.precond != PRECOND_CIRCULANT)) continue;
    const LikInstInfo& I = li[L.inst];
    DftPlan d;
    d.li = (int)k;
    d.H = L.H; d.W = L.W; d.logH = ilog2(L.H); d.logW = ilog2(L.W);
    const size_t N = (size_t)L.H * L.W;
    auto take = [&](size_t bytes) {
      char* p = cur + used;
      used += (bytes + 255) / 256 * 256;
      return p;
    };
    d.A = reinterpret_cast<float2*>(take(N * sizeof(float2)));
    d.B = reinterpret_cast<float2*>(take(N * sizeof(float2)));
    d.twW = reinterpret_cast<float2*>(take(sizeof(float2) * L.W));
    d.twH = reinterpret_cast<float2*>(take(sizeof(float2) * L.H));
    d.specT = reinterpret_cast<float*>(take(N * sizeof(float)));
    d.mask = reinterpret_cast<uint8_t*>(take(N));
    if (used > fft_bytes) {
      err = "FFT workspace layout mismatch";
      return hipErrorInvalidValue;
    }
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_twiddles, dim3((L.W + 255) / 256), dim3(256), 0, s, d.twW, L.W);
    hipLaunchKernelGGL(k_twiddles, dim3((L.H + 255) / 256), dim3(256), 0, s, d.twH, L.H);
    if (L.op == OP_DFT) {
      if ((e = hipMemcpyAsync(d.mask, I.mask, N, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_dft_spectrum, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, d.mask,
                         lc.planes[LP_SPEC], L.off, L.pitch, d.specT, L.H, L.W);
    } else {
      // the blur spectrum plane was written by the setup kernel already
      hipLaunchKernelGGL(k_spec_to_T, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                         lc.planes[LP_SPEC], L.off, L.pitch, d.specT, L.H, L.W);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    list.push_back(d);
  }
  (void)n;
  (void)err;
  return hipStreamSynchronize(s);   // the host mask copies must finish before they go away
}

// Forward 2-D DFT (unnormalised) of the A rows prepared by `pre`, result in B
// (transposed layout), multiplied by mul * scale.
static hipError_t forward_into_B(DftPlan& d, FftArgs pre, const float* mul, float scale,
                                 hipStream_t s, int post_mode = POST_SCALE) {
  pre.dst = d.A; pre.tw = d.twW; pre.nrows = d.H; pre.L = d.W; pre.logL = d.logW;
  pre.post = POST_COMPLEX; pre.inverse = 0;
  hipError_t e = rows(pre, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose, dim3((d.W + kTrT - 1) / kTrT, (d.H + kTrT - 1) / kTrT), dim3(256), 0, s, d.A,
                     d.B, d.H, d.W, nullptr, 0);
  FftArgs c = pre;
  c.pre = PRE_COMPLEX; c.src = d.B; c.dst = d.B; c.tw = d.twH; c.nrows = d.W; c.L = d.H;
  c.logL = d.logH; c.post = post_mode; c.mul = mul; c.scale = scale;
  return rows(c, s);
}

// Inverse 2-D DFT (unnormalised) of B (transposed layout); the last row pass
// applies `post` (real result times scale).
static hipError_t inverse_from_B(DftPlan& d, FftArgs post, hipStream_t s) {
  FftArgs c = post;
  c.pre = PRE_COMPLEX; c.src = d.B; c.dst = d.B; c.tw = d.twH; c.nrows = d.W; c.L = d.H;
  c.logL = d.logH; c.post = POST_COMPLEX; c.inverse = 1;
  hipError_t e = rows(c, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose, dim3((d.H + kTrT - 1) / kTrT, (d.W + kTrT - 1) / kTrT), dim3(256), 0, s, d.B,
                     d.A, d.W, d.H, nullptr, 0);
  FftArgs r = post;
  r.pre = PRE_COMPLEX; r.src = d.A; r.tw = d.twW; r.nrows = d.H; r.L = d.W; r.logL = d.logW;
  r.inverse = 1;
  return rows(r, s);
}

// H^T v = Re(F^H diag(mask) v) = Re(IDFT(mask v)) / sqrt(N) of a complex
// observation-space array v (interleaved re, im) into the pixel plane `out`.
// The masked array is copied into A (a row pass without stages is a plain
// copy), transposed into B and inverse-transformed.
static hipError_t dft_back_project(LikCtx& lc, DftPlan& d, const float* v, float* out, hipStream_t s) {
  const LikInst& L = lc.hinst[d.li];
  const double N = (double)d.H * d.W;
  FftArgs a = base_args(lc, L);
  a.pre = PRE_OBS; a.obs = v; a.mask = d.mask;
  a.dst = d.A; a.tw = d.twW; a.nrows = d.H; a.L = d.W; a.logL = 0; a.post = POST_COMPLEX;
  hipError_t e = rows(a, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose, dim3((d.W + kTrT - 1) / kTrT, (d.H + kTrT - 1) / kTrT), dim3(256), 0, s, d.A,
                     d.B, d.H, d.W, nullptr, 0);
  FftArgs post = base_args(lc, L);
  post.post = POST_REAL;
  post.real_out = out;
  post.scale = (float)(1.0 / std::sqrt(N));
  return inverse_from_B(d, post, s);
}

hipError_t dft_back_project_inst(LikCtx& lc, int li, const float* v, float* out, hipStream_t s) {
  for (DftPlan& d : lc.dft)
    if (d.li == li) return dft_back_project(lc, d, v, out, s);
  return hipErrorInvalidValue;
}

hipError_t dft_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s) {
  for (DftPlan& d : lc.dft) {
    const LikInst& L = lc.hinst[d.li];
    if (L.op != OP_DFT) continue;
    // H^T y, then y_pix = H^T y
    hipError_t e = dft_back_project(lc, d, d_y[L.inst], lc.planes[LP_HTY], s);
    if (e != hipSuccess) return e;
    // the cold start and the observation range use H^T y as the pixel-space observation
    e = hipMemcpy2DAsync(lc.ypix + L.off, sizeof(float) * L.pitch, lc.planes[LP_HTY] + L.off,
                         sizeof(float) * L.pitch, sizeof(float) * L.W, L.H,
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t dft_apply(LikCtx& lc, int mode, hipStream_t s) {
  for (DftPlan& d : lc.dft) {
    const LikInst& L = lc.hinst[d.li];
    if (L.op != OP_DFT) continue;
    const double N = (double)d.H * d.W;
    float* p_in = lc.planes[lc.pcur ? LP_P1 : LP_P0];
    float* p_out = lc.planes[lc.pcur ? LP_P0 : LP_P1];
    // the CG kernels skip converged instances on the device; the transform
    // itself always runs (its cost is independent of the values)
    FftArgs pre = base_args(lc, L);
    pre.pre = PRE_DIRECTION;
    pre.r = lc.planes[LP_R]; pre.x = lc.planes[LP_X]; pre.p_in = p_in; pre.p_out = p_out;
    pre.mode0 = mode == 0;
    pre.zpl = lc.planes[LP_Z];
    hipError_t e = forward_into_B(d, pre, d.specT, (float)(1.0 / N), s);
    if (e != hipSuccess) return e;
    FftArgs post = base_args(lc, L);
    post.post = POST_Q;
    post.real_out = lc.planes[LP_Q];
    post.pvec = mode == 0 ? lc.planes[LP_X] : p_out;
    post.scale = 1.f;
    if ((e = inverse_from_B(d, post, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dot_tiles, dim3(L.ntiles), dim3(256), 0, s, lc.d_inst, lc.d_tiles, L.tile0,
                       L.ntiles, post.pvec, lc.planes[LP_Q], lc.part0, lc.part1, lc.d_st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fft_precondition(LikCtx& lc, hipStream_t s) {
  for (DftPlan& d : lc.dft) {
    const LikInst& L = lc.hinst[d.li];
    if (L.precond != PRECOND_CIRCULANT) continue;
    const double N = (double)d.H * d.W;
    FftArgs pre = base_args(lc, L);
    pre.pre = PRE_REAL;
    pre.real_in = lc.planes[LP_R];
    hipError_t e = forward_into_B(d, pre, d.specT, (float)(1.0 / N), s, POST_PRECOND);
    if (e != hipSuccess) return e;
    FftArgs post = base_args(lc, L);
    post.post = POST_REAL;
    post.real_out = lc.planes[LP_Z];
    post.scale = 1.f;
    if ((e = inverse_from_B(d, post, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Fast-CG transforms (RF_FWD, transpose, RF_FILT, transpose, RF_INV).
// RFM_PRECOND, every circulant-preconditioned instance: z = M^{-1} r with r.z,
// r.r partials (update = 1: first x += alpha p, r -= alpha q).  RFM_PRODUCT,
// masked-DFT instances: p = z + beta p_in, q = (H^T H / xi + diag tau_c) p with
// p.q partials.  Partials go to [tile0, tile0 + npart).
hipError_t rfft_cg(LikCtx& lc, int mode, int update, hipStream_t s) {
  for (DftPlan& d : lc.dft) {
    const LikInst& L = lc.hinst[d.li];
    if (L.precond != PRECOND_CIRCULANT) continue;
    if (mode == RFM_PRODUCT && L.op != OP_DFT) continue;   // blur products: direct kernel
    const int Wh = d.W / 2 + 1;
    RfftArgs a;
    std::memset(&a, 0, sizeof(a));
    a.off = L.off; a.pitch = L.pitch; a.inv_xi = L.inv_xi; a.st = lc.d_st; a.st_w = lc.d_st;
    a.diagA = L.diagA;
    a.inst = L.inst;
    a.ld = Wh; a.mode = mode; a.update = update;
    a.r = lc.planes[LP_R]; a.z = lc.planes[LP_Z]; a.tauc = lc.planes[LP_TAUC];
    a.p_in = lc.planes[lc.pcur ? LP_P1 : LP_P0];     // same ping-pong as the CG kernels
    a.p = lc.planes[lc.pcur ? LP_P0 : LP_P1];
    a.x = lc.planes[LP_X]; a.q = lc.planes[LP_Q];
    // the row passes write and read the half spectrum transposed (W/2+1 rows of
    // length H), which is the layout the column pass works in: no transposes
    a.tld = d.H;
    RfftArgs f = a;
    f.dst = d.B; f.tw = d.twW; f.nrows = d.H / 2; f.logL = d.logW;
    f.apart = lc.part0 + L.tile0; f.acount = L.fin_count[FIN_ALPHA];
    hipError_t e = lik_timed(lc, KT_RF_FWD, s, [&]() { return launch_rfft<RF_FWD>(d.W, f, s); });
    if (e != hipSuccess) return e;
    RfftArgs g = a;
    g.src = d.B; g.dst = d.B; g.tw = d.twH; g.nrows = Wh; g.logL = d.logH; g.specT = d.specT;
    g.scale = (float)(1.0 / ((double)d.H * d.W));
    if ((e = lik_timed(lc, KT_RF_FILT, s, [&]() { return launch_rfft<RF_FILT>(d.H, g, s); })) !=
        hipSuccess)
      return e;
    RfftArgs v = a;
    v.src = d.B; v.tw = d.twW; v.nrows = d.H / 2; v.logL = d.logW;
    v.out = lc.planes[mode == RFM_PRECOND ? LP_Z : LP_Q];
    v.part0 = lc.part0; v.part1 = lc.part1; v.part_base = L.tile0;
    if ((e = lik_timed(lc, KT_RF_INV, s, [&]() { return launch_rfft<RF_INV>(d.W, v, s); })) !=
        hipSuccess)
      return e;
  }
  return hipSuccess;
}

hipError_t rfft_precondition(LikCtx& lc, int update, hipStream_t s) {
  return rfft_cg(lc, RFM_PRECOND, update, s);
}
hipError_t rfft_product(LikCtx& lc, hipStream_t s) { return rfft_cg(lc, RFM_PRODUCT, 0, s); }

void dft_destroy(LikCtx& lc) {
  lc.dft.clear();
  lc.wht.clear();
}

}  // namespace eptv
