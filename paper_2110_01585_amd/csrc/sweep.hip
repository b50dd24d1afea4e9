// Fused EP sweep over the four colour classes of pixel pairs (Algorithm 1,
// inner loop over k = 1..4, with all pairs of a class in parallel).
//
// Dependency structure used for the fusion.  V1 (horizontal, left column even)
// and V2 (horizontal, left column odd) only couple pixels of one row; V3
// (vertical, top row even) and V4 (vertical, top row odd) only pixels of one
// column.  The state of a pixel after the four classes therefore depends on
// pixels at most 2 columns and 2 rows away.  One wave owns a vertical strip of
// 128 columns (2 per lane; lane l holds columns c0-2+2l and c0-1+2l, so every V1
// pair is inside a lane) of which the middle 124 are written, and marches through
// a chunk of rows two at a time (downwards shown; odd chunks march down, even
// chunks up, the mirror image of this order):
//
//   load rows (r, r+1)  ->  V1 on both rows (lane-local)
//                       ->  V2 on both rows (pair = lane's right pixel and the
//                           next lane's left pixel; cavities and results cross
//                           lanes by shuffles)
//                       ->  V3 on (r, r+1) (lane-local)
//                       ->  V4 on (r-1, r) with row r-1 carried from the
//                           previous step, after which rows r-1 and r are final
//                           and are stored.
//
// A chunk of rows [R0, R1) loads rows R0-2 .. R1+1; halo pixels are recomputed,
// never stored, so every pixel is written by exactly one wave; all reads come
// from the previous sweep's buffer and all writes go to the other one.  Each edge's
// E|u| (for EM) and each clamp are counted by the wave that stores the edge's
// first (left/top) pixel.  HBM traffic per sweep: 5 sites read (40 B/px) and 4
// written (32 B/px).
#include <algorithm>

#include "ep_tv_internal.h"
#include "tilted.h"

namespace eptv {

struct Px {
  float t[5];
  float e[5];
};

template <int K>
__device__ __forceinline__ void cavity(const Px& p, float& c, float& m) {
  // Leave-one-out sums of the other four sites' natural parameters (Q / q_k,
  // Sec. III-B), accumulated in FP64 so the mean's numerator cannot cancel.
  double t = 0.0, e = 0.0;
#pragma unroll
  for (int l = 0; l < 5; ++l) {
    if (l != K) {
      t += (double)p.t[l];
      e += (double)p.e[l];
    }
  }
  c = frcp((float)t);
  m = (float)e * c;
}

struct PairOut {
  float ti, ei, tj, ej;  // new site (tau, eta) for the two endpoints, clamped
  bool ki, kj;           // clamped?
  float eabs;
};

// Tilted moments of u = x_i - x_j, Gehre-Jin projection onto (x_i, x_j) and
// the site update of Eq. (update_qk_x) in the equivalent cancellation-free
// form tau_i = rho / (s - rho c_i), eta_i = tau_i E_i + delta / s (and i<->j,
// delta -> -delta); variance clamp of Sec. III-C at 1e8.
template <class PR>
__device__ __forceinline__ PairOut pair_core(float ci, float mi, float cj, float mj, const PR& lam) {
  // no contraction into fused multiply-adds: the update of (i, j) must be the
  // exact mirror of the update of (j, i).  The fused multiply-adds written out
  // map onto each other under the exchange (delta changes sign, s and rho do
  // not), so they keep the mirror exact.
#pragma clang fp contract(off)
  const float s = ci + cj;
  const Tilt T = lam.tilt(mi - mj, s);
  const float dels = T.dels;
  const float Ei = __builtin_fmaf(dels, ci, mi);
  const float Ej = __builtin_fmaf(-dels, cj, mj);
  PairOut o;
  o.ti = T.rho * frcp(lam.den(T, s, ci, cj));
  o.tj = T.rho * frcp(lam.den(T, s, cj, ci));
  o.ki = o.ti < kPrecFloor;
  o.kj = o.tj < kPrecFloor;
  o.ti = o.ki ? kPrecFloor : o.ti;
  o.tj = o.kj ? kPrecFloor : o.tj;
  o.ei = __builtin_fmaf(o.ti, Ei, dels);
  o.ej = __builtin_fmaf(o.tj, Ej, -dels);
  o.eabs = T.eabs;
  return o;
}

template <int K>
__device__ __forceinline__ void damp(Px& p, float tn, float en, float alpha) {
  p.t[K] = alpha * tn + (1.0f - alpha) * p.t[K];
  p.e[K] = alpha * en + (1.0f - alpha) * p.e[K];
}

struct Acc {
  double eabs;
  unsigned clamps;
};

// Pair inside one lane (V1 on a row, V3/V4 on a column).
template <int K, class PR>
__device__ __forceinline__ void pair_local(Px& P, Px& Q, bool exists, bool cnt_edge, bool cnt_p,
                                           bool cnt_q, const PR& lam, float alpha, Acc& acc) {
  float ci, mi, cj, mj;
  cavity<K>(P, ci, mi);
  cavity<K>(Q, cj, mj);
  const PairOut o = pair_core(ci, mi, cj, mj, lam);
  if (exists) {
    damp<K>(P, o.ti, o.ei, alpha);
    damp<K>(Q, o.tj, o.ej, alpha);
    if (cnt_edge) acc.eabs += (double)o.eabs;
    acc.clamps += (cnt_p && o.ki ? 1u : 0u) + (cnt_q && o.kj ? 1u : 0u);
  }
}

// Neighbouring lanes' values by DPP wave shifts (one VALU move, no LDS round
// trip); the lane without a neighbour gets its own value, as with __shfl_down /
// __shfl_up of one lane.  Called with every lane of the wave active.
__device__ __forceinline__ int from_next_lane(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ int from_prev_lane(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ float from_next_lane(float v) {
  return __builtin_bit_cast(float, from_next_lane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float from_prev_lane(float v) {
  return __builtin_bit_cast(float, from_prev_lane(__builtin_bit_cast(int, v)));
}

// V2 pair: this lane's right pixel R with the next lane's left pixel.
// exists: the pair (R, next L) exists (evaluated by the owning lane).
template <class PR>
__device__ __forceinline__ void pair_v2(Px& L, Px& R, bool exists, bool cnt_edge, bool cnt_r,
                                        bool cnt_l, const PR& lam, float alpha, Acc& acc, int lane) {
  float cl, ml;
  cavity<2>(L, cl, ml);
  const float cj = from_next_lane(cl);
  const float mj = from_next_lane(ml);
  float ci, mi;
  cavity<2>(R, ci, mi);
  const PairOut o = pair_core(ci, mi, cj, mj, lam);
  // hand the partner's new site back to the lane that owns it
  const float tj = from_prev_lane(o.tj);
  const float ej = from_prev_lane(o.ej);
  const int bits = from_prev_lane((exists ? 1 : 0) | (o.kj ? 2 : 0));
  if (exists) {
    damp<2>(R, o.ti, o.ei, alpha);
    if (cnt_edge) acc.eabs += (double)o.eabs;
    acc.clamps += (cnt_r && o.ki) ? 1u : 0u;
  }
  if (lane > 0 && (bits & 1)) {
    damp<2>(L, tj, ej, alpha);
    acc.clamps += (cnt_l && (bits & 2)) ? 1u : 0u;
  }
}

struct Raw {
  float4 v[5];  // the five sites of a lane's pixel pair, as loaded
};

// The five sites of a lane's pixel pair.  idx is always inside the planes: rows
// and columns beyond a free boundary are read at a clamped position.  Such
// pixels (and the column right of an odd-width image, read from the row's
// padding) take part only in pairs that do not exist and are never stored, so
// what they hold never reaches a result; loading them anyway keeps the loads
// unconditional and spares a select per value.
__device__ __forceinline__ void fetch(const SweepArgs& a, long long idx, Raw& R) {
  const float2* S[5] = {a.S0, a.I1, a.I2, a.I3, a.I4};
#pragma unroll
  for (int l = 0; l < 5; ++l) R.v[l] = *reinterpret_cast<const float4*>(S[l] + idx);
}

__device__ __forceinline__ void unpack(const Raw& R, Px& L, Px& Rt) {
#pragma unroll
  for (int l = 0; l < 5; ++l) {
    L.t[l] = R.v[l].x;
    L.e[l] = R.v[l].y;
    Rt.t[l] = R.v[l].z;
    Rt.e[l] = R.v[l].w;
  }
}

__device__ __forceinline__ void store_row(const SweepArgs& a, long long idx, bool wL, bool wR,
                                          const Px& L, const Px& R) {
  float2* S[4] = {a.O1, a.O2, a.O3, a.O4};
  if (wL && wR) {
#pragma unroll
    for (int l = 0; l < 4; ++l)
      *reinterpret_cast<float4*>(S[l] + idx) =
          make_float4(L.t[l + 1], L.e[l + 1], R.t[l + 1], R.e[l + 1]);
  } else if (wL) {
#pragma unroll
    for (int l = 0; l < 4; ++l) S[l][idx] = make_float2(L.t[l + 1], L.e[l + 1]);
  } else if (wR) {
#pragma unroll
    for (int l = 0; l < 4; ++l) S[l][idx + 1] = make_float2(R.t[l + 1], R.e[l + 1]);
  }
}

__device__ __forceinline__ void totals(const Px& p, float& mu, float& v) {
  float t = p.t[0], e = p.e[0];
#pragma unroll
  for (int l = 1; l < 5; ++l) {
    t += p.t[l];
    e += p.e[l];
  }
  v = frcp(t);
  mu = e * v;
}

__device__ __forceinline__ int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// V4 pair across a boundary shared with a neighbouring wave of the block: both
// waves publish the class-4 cavity (c, m) of their boundary pixels in LDS, then
// each evaluates the pair (top, bottom) from the same inputs and keeps the
// update of its own pixel.  Every wave of the block calls this at the same two
// points (after its first and after its last row pair), shared boundary or not,
// so the barriers match.  X: LDS, [2 phases][kWavesPerBlock][kWave].
template <class PR>
__device__ __forceinline__ void pair_x4_one(Px& own, bool own_top, float co, float mo, float cp,
                                            float mp, bool exists, bool own_int, const PR& lam,
                                            float alpha, Acc& acc) {
  const float ci = own_top ? co : cp, mi = own_top ? mo : mp;
  const float cj = own_top ? cp : co, mj = own_top ? mp : mo;
  const PairOut o = pair_core(ci, mi, cj, mj, lam);
  if (exists) {
    damp<4>(own, own_top ? o.ti : o.tj, own_top ? o.ei : o.ej, alpha);
    if (own_top && own_int) acc.eabs += (double)o.eabs;   // the top pixel's wave counts the edge
    acc.clamps += (own_int && (own_top ? o.ki : o.kj)) ? 1u : 0u;
  }
}

template <class PR>
__device__ __forceinline__ void exchange_v4(float4* X, int phase, int wave, int partner, int lane,
                                            bool shared, Px& oL, Px& oR, bool own_top, bool vL,
                                            bool vR, bool wL, bool wR, const PR& lam, float alpha,
                                            Acc& acc) {
  float cL = 0.f, mL = 0.f, cR = 0.f, mR = 0.f;
  if (shared) {
    cavity<4>(oL, cL, mL);
    cavity<4>(oR, cR, mR);
    X[(phase * kWavesPerBlock + wave) * kWave + lane] = make_float4(cL, mL, cR, mR);
  }
  __syncthreads();
  if (shared) {
    const float4 q = X[(phase * kWavesPerBlock + partner) * kWave + lane];
    pair_x4_one(oL, own_top, cL, mL, q.x, q.y, vL, wL, lam, alpha, acc);
    pair_x4_one(oR, own_top, cR, mR, q.z, q.w, vR, wR, lam, alpha, acc);
  }
}

// Store a final row of the strip and fold its change into the convergence
// measures (DELTA): largest |mu - mu_old| and |v / v_old - 1| over stored pixels.
template <bool DELTA>
__device__ __forceinline__ void finish_row(const SweepArgs& a, long long idx, bool wL, bool wR,
                                           const Px& L, const Px& R, float omL, float ovL,
                                           float omR, float ovR, float& dmu, float& dv,
                                           unsigned& flags) {
  store_row(a, idx, wL, wR, L, R);
  if (DELTA) {
    float m1, v1;
    if (wL) {
      totals(L, m1, v1);
      dmu = fmaxf(dmu, fabsf(m1 - omL));
      dv = fmaxf(dv, fabsf((v1 - ovL) * frcp(ovL)));
      if (!(fabsf(m1) < 3.0e38f) || !(v1 > 0.f && v1 < 3.0e38f)) flags |= FLAG_NONFINITE;
    }
    if (wR) {
      totals(R, m1, v1);
      dmu = fmaxf(dmu, fabsf(m1 - omR));
      dv = fmaxf(dv, fabsf((v1 - ovR) * frcp(ovR)));
      if (!(fabsf(m1) < 3.0e38f) || !(v1 > 0.f && v1 < 3.0e38f)) flags |= FLAG_NONFINITE;
    }
  }
}

// One tile (strip x chunk) of one instance; `tile` and every value derived from
// the tile descriptor are wave-uniform (scalar registers).
//
// The tile's row pairs (r, r+1), r = R0-2, R0, ..., are visited downwards
// (UP = false) or upwards (UP = true); the result is the same either way, since
// every update of a class reads only the previous classes' results.  Even
// chunks march up and odd chunks down, so the halo rows two neighbouring chunks
// share are read by both at about the same time (both start there, or both end
// there) and the second read is served by L2.
//   down: pair (r, r+1), then V4 on (r-1, r) with row r-1 carried; rows r-1, r
//         are final; row r+1 is carried;
//   up:   pair (r, r+1), then V4 on (r+1, r+2) with row r+2 carried; rows
//         r+1, r+2 are final; row r is carried.
// The factor of an instance: lambda for l1 (it moves under EM), the mixture
// constants for MoG2 / BG (fixed).
__device__ __forceinline__ void make_factor(const InstDev&, const InstState& st, L1Factor& f) {
  f.lam = (float)st.lam;
}
__device__ __forceinline__ void make_factor(const InstDev&, const InstState& st, L1FactorQu& f) {
  f.lam = (float)st.lam;
}
__device__ __forceinline__ void make_factor(const InstDev& I, const InstState&, MixtureFactor& f) {
  f.f.dla = I.mix_dla;
  f.f.dv = I.mix_dv;
  f.f.v1 = I.mix_v1;
  f.f.v2 = I.mix_v2;
}

template <bool DELTA, bool UP, class PR>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, int tile, int wave, int lane,
                                           bool x_start, bool x_end, float4* X) {
  const int4 td = a.tiles[tile];
  const InstDev I = a.inst[td.x];
  const InstState& ST = a.st[td.x];
  PR lam;
  make_factor(I, ST, lam);
  const float alpha = I.alpha;
  const bool per = I.bnd == BND_PERIODIC;
  const int W = I.W, H = I.H;
  const int c0 = td.y * kStripInt;
  const int cl = c0 - 2 + 2 * lane;
  const int cr = cl + 1;
  bool vL, vR, vN;
  int gcl;
  if (per) {
    vL = vR = vN = true;
    gcl = wrap(cl, W);
  } else {
    vL = cl >= 0 && cl < W;
    vR = cr >= 0 && cr < W;
    vN = cl + 2 >= 0 && cl + 2 < W;
    // lanes outside the image read the nearest even column inside it (every
    // lane that stores has vL, so its column is its own)
    gcl = vL ? cl : (cl < 0 ? 0 : (W - 1) & ~1);
  }
  const bool wL = vL && cl >= c0 && cl < c0 + kStripInt && cl < W;
  const bool wR = vR && cr >= c0 && cr < c0 + kStripInt && cr < W;
  const bool v1col = vL && vR;
  const bool v2col = vR && vN && lane < kWave - 1;

  const int R0 = td.z * I.chunk_rows;
  const int R1 = min(R0 + I.chunk_rows, H);
  // row pairs (r, r+1), r = lo, lo+2, ..., hi: two halo rows beyond each boundary
  // that is not shared with a neighbouring wave of the block (x_start: the
  // boundary where the march starts, x_end: where it ends)
  const bool sh_top = UP ? x_end : x_start;
  const bool sh_bot = UP ? x_start : x_end;
  const int lo = sh_top ? R0 : R0 - 2;
  const int hi = sh_bot ? R1 - 2 : R0 - 2 + 2 * ((R1 - R0 + 2) / 2);
  const int npairs = (hi - lo) / 2 + 1;
  const int rfirst = UP ? hi : lo;
  constexpr int kStep = UP ? -2 : 2;

  Acc acc{0.0, 0u};
  float dmu = 0.f, dv = 0.f;
  unsigned flags = 0u;
  Px aL, aR;                    // carried row after V3
  float aomL = 0.f, aovL = 1.f, aomR = 0.f, aovR = 1.f;

  auto row_ok = [&](int r) { return per || (r >= 0 && r < H); };
  auto row_in = [&](int r) { return r >= R0 && r < R1; };
  // rows beyond a free boundary are read at the nearest row inside (and never
  // stored: only rows of the chunk are)
  auto row_idx = [&](int r) {
    const int g = per ? wrap(r, H) : min(max(r, 0), H - 1);
    return I.off + (long long)g * I.pitch + gcl;
  };
  // Each row pair is loaded when its turn comes: the kernel is held to 168
  // registers so three waves share a SIMD, and the other waves' tilted-moment
  // work covers a wave's load latency.  (Requesting the next pair one
  // iteration ahead needs 40 more registers and leaves two waves per SIMD,
  // which is slower.)
  for (int it = 0; it < npairs; ++it) {
    const int r = rfirst + it * kStep;
    const bool bv = row_ok(r);
    const bool cv = row_ok(r + 1);
    const bool bint = row_in(r);
    const bool cint = row_in(r + 1);
    Raw nb, nc;
    fetch(a, row_idx(r), nb);
    fetch(a, row_idx(r + 1), nc);
    Px bL, bR, cL, cR;
    unpack(nb, bL, bR);
    unpack(nc, cL, cR);
    float bomL = 0.f, bovL = 1.f, bomR = 0.f, bovR = 1.f, comL = 0.f, covL = 1.f, comR = 0.f,
          covR = 1.f;
    if (DELTA) {
      totals(bL, bomL, bovL);
      totals(bR, bomR, bovR);
      totals(cL, comL, covL);
      totals(cR, comR, covR);
    }
    // V1 on both rows
    pair_local<1>(bL, bR, bv && v1col, bint && wL, bint && wL, bint && wR, lam, alpha, acc);
    pair_local<1>(cL, cR, cv && v1col, cint && wL, cint && wL, cint && wR, lam, alpha, acc);
    // V2 on both rows
    pair_v2(bL, bR, bv && v2col, bint && wR, bint && wR, bint && wL, lam, alpha, acc, lane);
    pair_v2(cL, cR, cv && v2col, cint && wR, cint && wR, cint && wL, lam, alpha, acc, lane);
    // V3 on (r, r+1)
    {
      const bool ex = bv && cv && (per || r + 1 < H);
      pair_local<3>(bL, cL, ex && vL, bint && wL, bint && wL, cint && wL, lam, alpha, acc);
      pair_local<3>(bR, cR, ex && vR, bint && wR, bint && wR, cint && wR, lam, alpha, acc);
    }
    if (!UP) {
      // V4 on (r-1, r), then rows r-1 and r are final
      if (it > 0) {
        const bool aint = row_in(r - 1);
        const bool ex = row_ok(r - 1) && bv;
        pair_local<4>(aL, bL, ex && vL, aint && wL, aint && wL, bint && wL, lam, alpha, acc);
        pair_local<4>(aR, bR, ex && vR, aint && wR, aint && wR, bint && wR, lam, alpha, acc);
        if (aint)
          finish_row<DELTA>(a, row_idx(r - 1), wL, wR, aL, aR, aomL, aovL, aomR, aovR, dmu, dv,
                            flags);
      } else {
        // shared top boundary: row R0 pairs with the wave above's row R0-1
        exchange_v4(X, 0, wave, wave - 1, lane, x_start, bL, bR, false, vL, vR, wL, wR, lam, alpha,
                    acc);
      }
      if (bint)
        finish_row<DELTA>(a, row_idx(r), wL, wR, bL, bR, bomL, bovL, bomR, bovR, dmu, dv, flags);
      aL = cL;
      aR = cR;
      aomL = comL; aovL = covL; aomR = comR; aovR = covR;
    } else {
      // V4 on (r+1, r+2), then rows r+1 and r+2 are final
      if (it > 0) {
        const bool aint = row_in(r + 2);
        const bool ex = cv && row_ok(r + 2);
        pair_local<4>(cL, aL, ex && vL, cint && wL, cint && wL, aint && wL, lam, alpha, acc);
        pair_local<4>(cR, aR, ex && vR, cint && wR, cint && wR, aint && wR, lam, alpha, acc);
        if (aint)
          finish_row<DELTA>(a, row_idx(r + 2), wL, wR, aL, aR, aomL, aovL, aomR, aovR, dmu, dv,
                            flags);
      } else {
        // shared bottom boundary: row R1-1 pairs with the wave below's row R1
        exchange_v4(X, 0, wave, wave + 1, lane, x_start, cL, cR, true, vL, vR, wL, wR, lam, alpha,
                    acc);
      }
      if (cint)
        finish_row<DELTA>(a, row_idx(r + 1), wL, wR, cL, cR, comL, covL, comR, covR, dmu, dv,
                          flags);
      aL = bL;
      aR = bR;
      aomL = bomL; aovL = bovL; aomR = bomR; aovR = bovR;
    }
  }
  // the boundary where the march ends: the carried row pairs with the
  // neighbouring wave's row and is final after that
  if (!UP) {
    exchange_v4(X, 1, wave, wave + 1, lane, x_end, aL, aR, true, vL, vR, wL, wR, lam, alpha, acc);
    if (x_end)
      finish_row<DELTA>(a, row_idx(R1 - 1), wL, wR, aL, aR, aomL, aovL, aomR, aovR, dmu, dv, flags);
  } else {
    exchange_v4(X, 1, wave, wave - 1, lane, x_end, aL, aR, false, vL, vR, wL, wR, lam, alpha, acc);
    if (x_end)
      finish_row<DELTA>(a, row_idx(R0), wL, wR, aL, aR, aomL, aovL, aomR, aovR, dmu, dv, flags);
  }

  // wave reductions (fixed order -> deterministic)
  double e = acc.eabs;
  unsigned ncl = acc.clamps;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    e += __shfl_xor(e, off, kWave);
    ncl += __shfl_xor(ncl, off, kWave);
    dmu = fmaxf(dmu, __shfl_xor(dmu, off, kWave));
    dv = fmaxf(dv, __shfl_xor(dv, off, kWave));
    flags |= __shfl_xor(flags, off, kWave);
  }
  if (lane == 0) {
    a.part_eabs[tile] = e;
    a.part_clamp[tile] = ncl;
    a.part_dmu[tile] = dmu;
    a.part_dv[tile] = dv;
    a.part_flags[tile] = flags;
  }
}

// One wave per tile; consecutive tiles (vertically adjacent chunks of a strip)
// form a block, whose shared boundaries exchange cavities in LDS instead of
// recomputing halo rows; neighbouring blocks are mapped to the same XCD.
// Every path through one tile block passes exactly two barriers.
template <bool DELTA, class PR>
__device__ __forceinline__ void sweep_block(const SweepArgs& a, int blk, int wave, int lane,
                                            float4* X) {
  const int tile = blk * kWavesPerBlock + wave;
  const bool has = tile < a.ntiles;
  const int4 td = has ? a.tiles[tile] : make_int4(0, 0, 0, 0);
  if (!has || !a.st[td.x].active) {
    if (has) {
      // A frozen instance (converged, diverged or non-finite) keeps its sites:
      // they are carried into the output buffer, so the buffer the context
      // reads next holds the instance's final state whatever the parity of the
      // sweeps that run after it froze.
      const InstDev I = a.inst[td.x];
      const int c0 = td.y * kStripInt;
      const int R0 = td.z * I.chunk_rows;
      const int R1 = min(R0 + I.chunk_rows, I.H);
      for (int r = R0; r < R1; ++r) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int c = c0 - 2 + 2 * lane + k;
          if (c < c0 || c >= c0 + kStripInt || c >= I.W) continue;
          const long long p = I.off + (long long)r * I.pitch + c;
          a.O1[p] = a.I1[p];
          a.O2[p] = a.I2[p];
          a.O3[p] = a.I3[p];
          a.O4[p] = a.I4[p];
        }
      }
      if (lane == 0) {
        a.part_eabs[tile] = 0.0;
        a.part_dmu[tile] = 0.f;
        a.part_dv[tile] = 0.f;
        a.part_clamp[tile] = 0u;
        a.part_flags[tile] = 0u;
      }
    }
    __syncthreads();   // the two exchange points of the other waves
    __syncthreads();
    return;
  }
  bool sh_up = false, sh_dn = false;
  if (wave > 0) {
    const int4 t = a.tiles[tile - 1];
    sh_up = t.x == td.x && t.y == td.y && t.z == td.z - 1;
  }
  if (wave < kWavesPerBlock - 1 && tile + 1 < a.ntiles) {
    const int4 t = a.tiles[tile + 1];
    sh_dn = t.x == td.x && t.y == td.y && t.z == td.z + 1;
  }
  if (td.z & 1)
    sweep_tile<DELTA, false, PR>(a, tile, wave, lane, sh_up, sh_dn, X);
  else
    sweep_tile<DELTA, true, PR>(a, tile, wave, lane, sh_dn, sh_up, X);
}

// One block per tile block, or (persistent launch) a resident grid whose
// blocks take the tile blocks h = blockIdx.x, blockIdx.x + gridDim.x, ...: a
// static schedule with no dependence between blocks.  With gridDim.x a multiple
// of 8, block h stays on the XCD that block-index order h would have given it,
// so the XCD remap keeps neighbouring tile blocks in one L2 either way.  At
// least three waves per SIMD (at most 168 registers per lane).
template <bool DELTA, class PR>
__global__ __launch_bounds__(kWavesPerBlock * kWave, 3) void k_tv_sweep(SweepArgs a) {
  __shared__ float4 X[2 * kWavesPerBlock * kWave];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int nblk = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  for (int h = blockIdx.x; h < nblk; h += gridDim.x)
    sweep_block<DELTA, PR>(a, xcd_remap(h, nblk), wave, lane, X);
}

template <class PR>
__global__ __launch_bounds__(256) void k_tilted(int n, const float* __restrict__ m,
                                                const float* __restrict__ s, PR f,
                                                float* __restrict__ rho, float* __restrict__ del,
                                                float* __restrict__ eabs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Tilt T = f.tilt(m[i], s[i]);
  rho[i] = T.rho;
  del[i] = T.delta;
  eabs[i] = T.eabs;
}

hipError_t launch_tilted(int n, const float* m, const float* s, float lam, float* rho, float* del,
                         float* eabs, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  L1Factor f;
  f.lam = lam;
  hipLaunchKernelGGL(k_tilted<L1Factor>, dim3((n + 255) / 256), dim3(256), 0, st, n, m, s, f, rho,
                     del, eabs);
  return hipGetLastError();
}

hipError_t launch_tilted_mixture(int n, const float* m, const float* s, float dla, float dv,
                                 float v1, float v2, float* rho, float* del, float* eabs,
                                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  MixtureFactor f;
  f.f.dla = dla;
  f.f.dv = dv;
  f.f.v1 = v1;
  f.f.v2 = v2;
  hipLaunchKernelGGL(k_tilted<MixtureFactor>, dim3((n + 255) / 256), dim3(256), 0, st, n, m, s, f,
                     rho, del, eabs);
  return hipGetLastError();
}

// Grid of one launch: a block per tile block, or for the persistent launch the
// blocks the device holds at once (occupancy of this kernel variant times the
// compute units, a multiple of 8), if fewer.
template <bool DELTA, class PR>
static hipError_t launch_sweep_t(const SweepArgs& a, int blocks, hipStream_t s) {
  int grid = blocks;
  if (a.persistent) {
    constexpr int kMaxDev = 64;
    static int resident[kMaxDev] = {};   // per device and kernel variant, looked up once
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    if (resident[dev] == 0) {
      int per_cu = 0, cus = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tv_sweep<DELTA, PR>,
                                                       kWavesPerBlock * kWave, 0);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      resident[dev] = std::max(8, per_cu * cus / 8 * 8);
    }
    grid = std::min(blocks, resident[dev]);
  }
  hipLaunchKernelGGL((k_tv_sweep<DELTA, PR>), dim3(grid), dim3(kWavesPerBlock * kWave), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tv_sweep(const SweepArgs& a, bool want_delta, hipStream_t s) {
  const int blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0) return hipSuccess;
  if (a.prior == PRIOR_L1 && a.em_opt == 2) {
    // EM with option 2: the sweep accumulates E|u| under Q(u) instead
    return want_delta ? launch_sweep_t<true, L1FactorQu>(a, blocks, s)
                      : launch_sweep_t<false, L1FactorQu>(a, blocks, s);
  }
  if (a.prior == PRIOR_L1)
    return want_delta ? launch_sweep_t<true, L1Factor>(a, blocks, s)
                      : launch_sweep_t<false, L1Factor>(a, blocks, s);
  return want_delta ? launch_sweep_t<true, MixtureFactor>(a, blocks, s)
                    : launch_sweep_t<false, MixtureFactor>(a, blocks, s);
}

}  // namespace eptv

