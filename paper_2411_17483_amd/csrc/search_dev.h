// search_dev.h -- device helpers shared by the search kernels (internal).
#pragma once

#include "search.h"

namespace sofa {

// ----------------------------------------------------------------------------
__device__ __forceinline__ uint32_t byte_of(const uint4& w, int j) {
  uint32_t v = (j < 4) ? w.x : (j < 8) ? w.y : (j < 12) ? w.z : w.w;
  return (v >> (8 * (j & 3))) & 255u;
}

__device__ __forceinline__ float lb_word(const float* T, const uint4& w) {
  // positions 0..15 in order: bytes 0..3 of w.x, then w.y, w.z, w.w
  float s = 0.0f;
  const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int j = 0; j < 16; j++) s += T[j * kAlphaMax + ((wv[j >> 2] >> (8 * (j & 3))) & 255u)];
  return s;
}

__device__ __forceinline__ float lb_leaf(const float* T, const uint4& sq, const uint4& lo,
                                         const uint4& hi) {
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 16; j++) {
    uint32_t q = byte_of(sq, j), a = byte_of(lo, j), b = byte_of(hi, j);
    // clamp(q, a, b) for a <= b, as a min and a max (byte operands select
    // straight from the envelope words)
    uint32_t c = max(min(q, b), a);
    s += T[j * kAlphaMax + c];
  }
  return s;
}

// FP16 code of a non-negative bound, rounded down; +inf stays +inf, finite
// values above the largest code clamp to it
__device__ __forceinline__ uint16_t f16_down(float x) {
  const uint32_t f = __float_as_uint(x);
  if (f & 0x80000000u) return 0;                // cannot occur; 0 keeps the leaf
  if (f >= 0x7F800000u) return 0x7C00u;         // +inf
  const int e = (int)(f >> 23) - 127 + 15;
  if (e >= 31) return 0x7BFFu;
  if (e <= 0) return (uint16_t)(x * 0x1p24f);   // subnormal: floor(x / 2^-24), exact scaling
  return (uint16_t)((e << 10) | ((f >> 13) & 0x3FFu));
}

// the FP16 code a stored envelope bound must not exceed for its leaf to
// survive U: U widened by the slack of the FP32 bound sum, rounded down (the
// codes of non-negative values order like the values)
__device__ __forceinline__ uint32_t u_code(const SearchArgs& a, int q) {
  return f16_down(__uint_as_float(a.U[q]) * (1.0f + 0x1p-16f));
}

__device__ __forceinline__ unsigned long long* stat_ptr(const SearchArgs& a, int slot) {
  const unsigned shard = (blockIdx.x + 13u * blockIdx.y) % (unsigned)kStatShards;
  return a.stats + shard * kStatSlots + slot;
}
__device__ __forceinline__ void stat_add(const SearchArgs& a, int slot, unsigned long long v) {
  if (a.stats && v) atomicAdd(stat_ptr(a, slot), v);
}
__device__ __forceinline__ void stat_max(const SearchArgs& a, int slot, unsigned long long v) {
  if (!a.stats) return;
  unsigned long long* p = stat_ptr(a, slot);
  if (v > __atomic_load_n(p, __ATOMIC_RELAXED)) atomicMax(p, v);
}

__device__ __forceinline__ float key_d(uint64_t key) { return __uint_as_float((uint32_t)(key >> 32)); }
constexpr uint64_t kEmpty = ~0ull;

// Sorted per-wave candidate list: rank r lives in register r/64, lane r%64.
// `evicted` keeps the smallest key ever pushed out of the list (or refused
// when the list was full); the search is exact as long as that key lies
// outside the final error band, which k_finalize checks.
template <int R>
struct WaveList {
  uint64_t e[R];
  uint64_t evicted;
  __device__ void reset() {
#pragma unroll
    for (int r = 0; r < R; r++) e[r] = kEmpty;
    evicted = kEmpty;
  }
  __device__ uint64_t at(int rank) const {
    uint64_t v = kEmpty;
#pragma unroll
    for (int r = 0; r < R; r++)
      if (rank / 64 == r) v = __shfl(e[r], rank & 63);
    return v;
  }
  __device__ void insert(uint64_t key, int lane) {
    int pos = 0;
    uint64_t top[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      pos += __popcll(__ballot(e[r] < key));
      top[r] = __shfl(e[r], 63);
    }
    if (pos >= 64 * R) {
      evicted = key < evicted ? key : evicted;
      return;
    }
    const uint64_t last = top[R - 1];
    evicted = last < evicted ? last : evicted;
#pragma unroll
    for (int r = 0; r < R; r++) {
      uint64_t up = __shfl_up(e[r], 1);
      if (lane == 0) up = (r > 0) ? top[r - 1] : e[r];
      int rank = lane + 64 * r;
      e[r] = rank < pos ? e[r] : (rank == pos ? key : up);
    }
  }
};

// FP32 squared distance of 4 rows at once: lane group g = lane/16 handles the
// row at xrow (when active); lane li = lane%16 owns elements li*4 + 64*it.
// Partial sums are checked every 64 CHK elements against `abandon`; a group
// whose partial exceeds it stops loading.  Returns the group's sum (all 16
// lanes) or +inf when abandoned/inactive.
template <int NIT, int CHK = 4>
__device__ __forceinline__ float dist4(const float* __restrict__ xrow, bool active,
                                       const float4 (&q)[NIT], int li, float abandon) {
  float acc = 0.0f;
  bool live = active;
#pragma unroll
  for (int it = 0; it < NIT; it++) {
    if (live) {
      float4 x = *reinterpret_cast<const float4*>(xrow + li * 4 + 64 * it);
      float d0 = q[it].x - x.x, d1 = q[it].y - x.y, d2 = q[it].z - x.z, d3 = q[it].w - x.w;
      acc = fmaf(d0, d0, acc);
      acc = fmaf(d1, d1, acc);
      acc = fmaf(d2, d2, acc);
      acc = fmaf(d3, d3, acc);
    }
    if (it % CHK == CHK - 1 && it + 1 < NIT) {
      float p = acc;
      p += __shfl_xor(p, 8);
      p += __shfl_xor(p, 4);
      p += __shfl_xor(p, 2);
      p += __shfl_xor(p, 1);
      if (p > abandon) live = false;
    }
  }
  acc += __shfl_xor(acc, 8);
  acc += __shfl_xor(acc, 4);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 1);
  return live ? acc : INFINITY;
}

constexpr int kRefRows = 4;  // rows per 16-lane group and step: 16 rows of a wave in flight

// FP32 squared distances of kRefRows rows per 16-lane group (lane li owns
// elements li*4 + 64*it), the loads of every row issued before any sum.
// Past the first 256 elements a row continues only while its partial sum
// stays within `abandon`; abandoned and inactive rows return +inf.
template <int NIT>
__device__ __forceinline__ void dist_rows(const float* __restrict__ X, int n_pad,
                                          const uint32_t (&pos)[kRefRows], const bool (&act)[kRefRows],
                                          const float4 (&q)[NIT], int li, float abandon,
                                          float (&d)[kRefRows]) {
  constexpr int H = NIT < 4 ? NIT : 4;  // float4 steps per lane loaded together
  float acc[kRefRows];
  bool live[kRefRows];
#pragma unroll
  for (int r = 0; r < kRefRows; r++) {
    acc[r] = 0.0f;
    live[r] = act[r];
  }
#pragma unroll
  for (int h0 = 0; h0 < NIT; h0 += H) {
    float4 x[kRefRows][H];
#pragma unroll
    for (int r = 0; r < kRefRows; r++)
      if (live[r]) {
#pragma unroll
        for (int it = 0; it < H; it++)
          x[r][it] = *reinterpret_cast<const float4*>(X + (int64_t)pos[r] * n_pad + li * 4 + 64 * (h0 + it));
      }
#pragma unroll
    for (int r = 0; r < kRefRows; r++)
      if (live[r]) {
#pragma unroll
        for (int it = 0; it < H; it++) {
          const float4 qv = q[h0 + it];
          const float d0 = qv.x - x[r][it].x, d1 = qv.y - x[r][it].y;
          const float d2 = qv.z - x[r][it].z, d3 = qv.w - x[r][it].w;
          acc[r] = fmaf(d0, d0, acc[r]);
          acc[r] = fmaf(d1, d1, acc[r]);
          acc[r] = fmaf(d2, d2, acc[r]);
          acc[r] = fmaf(d3, d3, acc[r]);
        }
      }
    if (h0 + H < NIT) {
#pragma unroll
      for (int r = 0; r < kRefRows; r++) {
        float p = acc[r];
        p += __shfl_xor(p, 8);
        p += __shfl_xor(p, 4);
        p += __shfl_xor(p, 2);
        p += __shfl_xor(p, 1);
        live[r] = live[r] && p <= abandon;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRefRows; r++) {
    float p = acc[r];
    p += __shfl_xor(p, 8);
    p += __shfl_xor(p, 4);
    p += __shfl_xor(p, 2);
    p += __shfl_xor(p, 1);
    d[r] = live[r] ? p : INFINITY;
  }
}

// q row of a query held in registers by lane li of every 16-lane group
template <int NIT>
__device__ __forceinline__ void load_q(const float* qrow, int li, float4 (&q)[NIT]) {
#pragma unroll
  for (int it = 0; it < NIT; it++) q[it] = *reinterpret_cast<const float4*>(qrow + li * 4 + 64 * it);
}

// FP64 squared distance in time order with no contraction: the same
// arithmetic as the ranking key of record.
// q and x 16-byte aligned, n a multiple of 4.  The sum runs over t in order
// (no contraction); the loads are issued kExactU float4 pairs at a time, so
// that one thread's 2n loads do not wait one by one.
constexpr int kExactU = 8;
__device__ inline double exact_d2(const float* __restrict__ q, const float* __restrict__ x, int n) {
#pragma clang fp contract(off)
  const float4* qv = reinterpret_cast<const float4*>(q);
  const float4* xv = reinterpret_cast<const float4*>(x);
  double s = 0.0;
  for (int t0 = 0; t0 < n; t0 += 4 * kExactU) {
    float4 a[kExactU], b[kExactU];
#pragma unroll
    for (int u = 0; u < kExactU; u++) {
      const bool in = t0 + 4 * u < n;
      a[u] = in ? qv[t0 / 4 + u] : make_float4(0.f, 0.f, 0.f, 0.f);
      b[u] = in ? xv[t0 / 4 + u] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kExactU; u++) {
      if (t0 + 4 * u >= n) break;
      const float qs[4] = {a[u].x, a[u].y, a[u].z, a[u].w};
      const float xs[4] = {b[u].x, b[u].y, b[u].z, b[u].w};
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const double d = (double)qs[e] - (double)xs[e];
        const double sq = d * d;
        s = s + sq;
      }
    }
  }
  return s;
}


constexpr int kHistBins = 256;                 // per-query histogram of flushed distances

// Flush a wave's in-band candidates into the query's result buffer, record
// the smallest key that was evicted or could not be stored, and tighten the
// query's bound from the histogram of everything flushed so far.
template <int R>
__device__ void flush_wave_list(const SearchArgs& a, const int q, WaveList<R>& wl, float& Umin,
                                const int lane) {

      const float ug = __uint_as_float(__atomic_load_n(a.U + q, __ATOMIC_RELAXED));
      Umin = ug < Umin ? ug : Umin;
      const float band = Umin * a.band_f;
      uint64_t evk = wl.evicted;
      int cnt = 0;
      uint64_t bals[R];
#pragma unroll
      for (int r = 0; r < R; r++) {
        bals[r] = __ballot(wl.e[r] != kEmpty && key_d(wl.e[r]) <= band);
        cnt += __popcll(bals[r]);
      }
      if (cnt > 0) {
        uint32_t b0 = 0;
        if (lane == 0) b0 = atomicAdd(a.rescnt + q, (uint32_t)cnt);
        b0 = __shfl(b0, 0);
        int off = 0;
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        uint64_t lost = kEmpty;
        const float hb = a.hbase[q];
        const bool hist_on = hb > 0.0f && hb < INFINITY;
#pragma unroll
        for (int r = 0; r < R; r++) {
          if ((bals[r] >> lane) & 1ull) {
            const uint32_t slot = b0 + off + __popcll(bals[r] & lt);
            if (slot < (uint32_t)a.cap) a.res[(int64_t)q * a.cap + slot] = wl.e[r];
            else lost = wl.e[r] < lost ? wl.e[r] : lost;
            if (hist_on) {
              int bk = (int)(key_d(wl.e[r]) / hb * (float)kHistBins);
              bk = bk < 0 ? 0 : (bk >= kHistBins ? kHistBins - 1 : bk);
              atomicAdd(a.hist + (int64_t)q * kHistBins + bk, 1u);
            }
          }
          off += __popcll(bals[r]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          uint64_t t = __shfl_xor(lost, o);
          lost = t < lost ? t : lost;
        }
        evk = lost < evk ? lost : evk;
        if (hist_on) {
          // the first bucket edge below which at least k candidates lie is a
          // bound on the k-th distance (one bucket of slack for rounding)
          uint32_t c4[kHistBins / 64];
          uint32_t cs = 0;
#pragma unroll
          for (int i = 0; i < kHistBins / 64; i++) {
            c4[i] = __atomic_load_n(a.hist + (int64_t)q * kHistBins + lane * (kHistBins / 64) + i,
                                    __ATOMIC_RELAXED);
            cs += c4[i];
          }
          uint32_t incl = cs;
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            uint32_t t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
          }
          const uint64_t hit = __ballot(incl >= (uint32_t)a.k);
          if (hit) {
            const int hl = __builtin_ctzll(hit);
            uint32_t run = __shfl(incl - cs, hl);
            int bk = hl * (kHistBins / 64) + kHistBins / 64 - 1;
            for (int i = 0; i < kHistBins / 64; i++) {
              run += __shfl(c4[i], hl);
              if (run >= (uint32_t)a.k) {
                bk = hl * (kHistBins / 64) + i;
                break;
              }
            }
            const float uh = hb * ((float)(bk + 2) / (float)kHistBins) * a.upd_f;
            if (uh < Umin) {
              Umin = uh;
              if (lane == 0) atomicMin(a.U + q, __float_as_uint(uh));
            }
          }
        }
      }
      if (lane == 0 && evk != kEmpty && key_d(evk) <= band)
        atomicMin(reinterpret_cast<unsigned long long*>(a.evmin) + q, evk);
    }

}  // namespace sofa
