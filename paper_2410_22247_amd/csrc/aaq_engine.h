// Device engine (gfx950) of the p-layer MaxCut QAOA statevector estimator: the tile
// engine and the sweep kernels, templated on the amplitude type R (float: complex64,
// double: complex128) and the tile size LT (a tile of 2^LT amplitudes held by a
// workgroup of 2^(LT-4) threads, 16 amplitudes per thread).
//
// The tile's register bits are switched between "arrangements" through an LDS
// transpose so that every mixer butterfly is a register-to-register operation:
// arrangement k keeps tile bits [b0(k), b0(k)+4) in registers and spreads the other
// tile bits over the threads.  The last arrangement (high tile bits in registers) is
// the one used for global loads and stores: consecutive lanes then touch consecutive
// amplitudes.  The one before it is the "phase" arrangement.
//
// A sweep = load (or synthesise |+>) -> ops at the load arrangement -> mixer A
// through the arrangements -> ops at the phase arrangement -> mixer B back -> store.
// The ops are the cost phase exp(-i gamma C(z)) (QAOA section, U_P), its inverse,
// the energy / lambda step and the gradient accumulations of the adjoint method.
// C(z) and h(z) are exact integers recomputed per amplitude from uint64 adjacency
// masks and the term lists.
//
// Included by one translation unit per (R, LT) instantiation and by the common one.
#pragma once
#include <hip/hip_runtime.h>

#include "aaq_internal.h"
#include "aaq_launch.h"

namespace aaq {

// Read-only uniform data (graph masks, term lists, per-sweep scale records) is read
// through the constant address space: with a uniform address such a load is one scalar
// load for the whole wave (no vector registers, no wait on the vector memory counter).
// No kernel writes the data it reads this way; it comes from host uploads or from an
// earlier kernel of the stream.
// (The host compilation pass sees these device functions too; address spaces exist only
// in the device pass.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> using cptr = const __attribute__((address_space(4))) T*;
#else
template <class T> using cptr = const T*;
#endif
template <class T> __device__ __forceinline__ cptr<T> cst(const T* p) { return (cptr<T>)p; }

template <class R> struct Cx;
template <> struct Cx<float> {
  using V = float2;
};
template <> struct Cx<double> {
  using V = double2;
};

template <class R, int LT> struct Geo {
  using V = typename Cx<R>::V;
  static constexpr int L = LT, RB = kRegBits, NR = 1 << RB;
  static constexpr int NA = geo_na(L);
  static constexpr int LAST = NA - 1, P = NA - 2;
  static constexpr int TILE = 1 << L;
  static constexpr int LB = L - RB;  // thread bits
  static constexpr int NT = 1 << LB; // threads per workgroup
  __host__ __device__ static constexpr int b0(int k) { return geo_b0(k, L); }
  static_assert(NA >= 3, "a tile needs a load, a phase and a third arrangement");
};

template <class R> __device__ __forceinline__ typename Cx<R>::V mkv(R x, R y) {
  typename Cx<R>::V v;
  v.x = x;
  v.y = y;
  return v;
}

// the default deferred-table hook of Tile::run: nothing to load
struct NoTabs {
  __device__ __forceinline__ void operator()() const {}
};

// tile index of register r of thread t in an arrangement whose register bits start at B0
template <int B0, int RB> __device__ __forceinline__ uint32_t tidx(uint32_t t, uint32_t r) {
  return (t & ((1u << B0) - 1u)) | (r << B0) | ((t >> B0) << (B0 + RB));
}
// LDS slot of tile index j: one padding slot per 16 entries.  P is additive over
// disjoint bit sets, P(a | b) = P(a) + P(b), so the slot of (thread part | register
// part) is a per-thread base plus a compile-time offset.
__host__ __device__ constexpr uint32_t lds_slot(uint32_t j) { return j + (j >> 4); }
// the tile index without its bit 3 (the half-tile exchange below); additive over
// disjoint bit sets that do not hold bit 3, like lds_slot
__host__ __device__ constexpr uint32_t drop_bit3(uint32_t j) { return (j & 7u) | ((j >> 4) << 3); }
// thread part of the tile index in an arrangement whose register bits start at B0
template <int B0, int RB> __device__ __forceinline__ uint32_t tpart(uint32_t t) {
  return (t & ((1u << B0) - 1u)) | ((t >> B0) << (B0 + RB));
}

// e^{-i theta X} on an amplitude pair with c = cos(theta), s = sin(theta):
// (x, y) -> (c x - i s y, -i s x + c y)
template <class V, class R> __device__ __forceinline__ void bfly(V& x, V& y, R c, R s) {
  const V x0 = x, y0 = y;
  x.x = c * x0.x + s * y0.y;
  x.y = c * x0.y - s * y0.x;
  y.x = c * y0.x + s * x0.y;
  y.y = c * y0.y - s * x0.x;
}
// (I - i k X) on a pair: (x, y) -> (x - i k y, y - i k x)
template <class V, class R> __device__ __forceinline__ void bflyk(V& x, V& y, R k) {
  const V x0 = x, y0 = y;
  x.x = x0.x + k * y0.y;
  x.y = x0.y - k * y0.x;
  y.x = y0.x + k * x0.y;
  y.y = y0.y - k * x0.x;
}
// Im(conj(u) v)
template <class V> __device__ __forceinline__ auto imcm(const V& u, const V& v) { return u.x * v.y - u.y * v.x; }
// a * b + c, one rounding
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ uint64_t pdep64(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t bit = 1; mask; bit <<= 1) {
    const uint64_t low = mask & (~mask + 1);
    if (x & bit) r |= low;
    mask &= mask - 1;
  }
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------
// Per-sweep context (all uniform across the workgroup).
template <class R> struct Ctx {
  using V = typename Cx<R>::V;
  const GraphDev* g;
  const int4* terms;
  const V* tab;    // [p][cmax+1]
  V* psi;          // global state (nullptr when the tile never leaves registers)
  V* lam;
  R amp;           // 2^{-n/2}
  int T;
  int cmax;
  uint64_t N = 0;  // amplitudes per state (stride between checkpoint buffers)
  bool off32 = false;  // every byte offset inside one state buffer fits in 32 bits
  bool nt = false;     // non-temporal state loads: set for single-instance evaluations that
                       // stream more state than the last-level cache holds (the batched
                       // units and small energy-only evaluations keep their state cached)
  // Centre of h and C for the adjoint sums: cmax / 2, the mean of both under |+>.  lambda
  // is made as (h - cen) psi and the gamma gradient sums (C - cen) Im(conj(lambda) psi).
  // Neither changes a gradient: <psi|G|psi> is real for a Hermitian generator G, and
  // <lambda|psi> = <psi_f|H|psi_f> is real at every position (both states are moved by
  // the same unitaries), so the shifts drop out of 2 Im <lambda|G|psi>.  They shrink the
  // magnitudes that cancel in those sums, and with them the float32 rounding.
  R cen = R(0);
};

// Per-thread accumulators for one sweep.
struct Acc {
  double e, nrm, gpre, gmid, ba, bb;
  __device__ void zero() { e = nrm = gpre = gmid = ba = bb = 0.0; }
};

// EN: the energy / lambda step is compiled in (only the last forward sweep needs it)
template <class R, int NS, bool EN, int LT> struct Tile {
  using G = Geo<R, LT>;
  using V = typename G::V;
  static constexpr int NR = G::NR, RB = G::RB, L = G::L, LB = G::LB, NA = G::NA, LAST = G::LAST, P = G::P;

  V a[NS][NR];
  bool lam_live;

  // ------------------------------------------------ compile-time qubit masks of the routes
  // tile bits held in registers by arrangement K
  __host__ __device__ static constexpr uint32_t regmask(int K) { return ((1u << RB) - 1u) << G::b0(K); }
  // first arrangement after the load arrangement on route RT
  __host__ __device__ static constexpr int first_arr(int RT) { return RT == ROUTE_FULL ? 0 : 1; }
  // tile bits a route may mix: all of them, or (sets of high qubits) all but the low
  // kMinContig bits, which such a set always holds passively
  __host__ __device__ static constexpr uint32_t route_bits(int RT) {
    return RT == ROUTE_FULL ? ((1u << L) - 1u) : (((1u << L) - 1u) & ~((1u << kMinContig) - 1u));
  }
  // tile bits mixed at arrangement K when a mixer walks the route forward (LAST, first,
  // ..., P) or backward (P, ..., first, LAST): a qubit is mixed at the first arrangement
  // of the walk that holds it in registers
  __host__ __device__ static constexpr uint32_t fwd_mask(int RT, int K) {
    uint32_t t = route_bits(RT);
    if (K == LAST) return t & regmask(LAST);
    t &= ~regmask(LAST);
    for (int j = first_arr(RT); j < K; ++j) t &= ~regmask(j);
    return t & regmask(K);
  }
  __host__ __device__ static constexpr uint32_t bwd_mask(int RT, int K) {
    uint32_t t = route_bits(RT);
    if (K == LAST) {
      for (int j = first_arr(RT); j <= P; ++j) t &= ~regmask(j);
      return t & regmask(LAST);
    }
    for (int j = K + 1; j <= P; ++j) t &= ~regmask(j);
    return t & regmask(K);
  }
  __host__ __device__ static constexpr bool walks_cover(int RT) {
    uint32_t f = fwd_mask(RT, LAST), b = bwd_mask(RT, LAST);
    for (int j = first_arr(RT); j <= P; ++j) {
      if ((f & fwd_mask(RT, j)) || (b & bwd_mask(RT, j))) return false;  // no bit twice
      f |= fwd_mask(RT, j);
      b |= bwd_mask(RT, j);
    }
    return f == route_bits(RT) && b == route_bits(RT);
  }
  static_assert(walks_cover(ROUTE_FULL) && walks_cover(ROUTE_HIGH), "every route bit is mixed exactly once");

  // -------------------------------------------------------------- LDS transpose
  // HX: the half-tile exchange.  When both arrangements keep tile bit 3 as a thread bit
  // (register bits at 4 and up), it is thread bit 3 on both sides, so the half of the
  // tile with bit 3 = h moves only among the threads with thread bit 3 = h: the two
  // halves take turns in a buffer of half a tile (slots of the index without bit 3).
  // Half the LDS per workgroup lets more workgroups share a compute unit.
  template <int KF, int KT, bool HX = false> __device__ __forceinline__ void xchg1(V (&x)[NR], V* lds) {
    constexpr int BF = G::b0(KF), BT = G::b0(KT);
    const uint32_t t = threadIdx.x;
    if constexpr (HX) {
      static_assert(BF > 3 && BT > 3, "tile bit 3 must be a thread bit in both arrangements");
      const uint32_t h = (t >> 3) & 1u;
      V* wb = lds + lds_slot(drop_bit3(tpart<BF, RB>(t)));
      const V* rb = lds + lds_slot(drop_bit3(tpart<BT, RB>(t)));
#pragma unroll
      for (uint32_t ph = 0; ph < 2; ++ph) {
        if (h == ph) {
#pragma unroll
          for (int r = 0; r < NR; ++r) wb[lds_slot(drop_bit3((uint32_t)r << BF))] = x[r];
        }
        __syncthreads();
        if (h == ph) {
#pragma unroll
          for (int r = 0; r < NR; ++r) x[r] = rb[lds_slot(drop_bit3((uint32_t)r << BT))];
        }
        __syncthreads();
      }
    } else {
      V* wb = lds + lds_slot(tpart<BF, RB>(t));
#pragma unroll
      for (int r = 0; r < NR; ++r) wb[lds_slot((uint32_t)r << BF)] = x[r];
      __syncthreads();
      const V* rb = lds + lds_slot(tpart<BT, RB>(t));
#pragma unroll
      for (int r = 0; r < NR; ++r) x[r] = rb[lds_slot((uint32_t)r << BT)];
      __syncthreads();
    }
  }
  // one-state sweeps of the high-qubit route exchange half tiles (every arrangement of
  // that route has its register bits at 4 and up)
  static constexpr bool half_xchg(int RT) { return NS == 1 && RT == ROUTE_HIGH; }
  // LAM: lambda is live (compile-time, so no per-register branch)
  template <int KF, int KT, bool LAM, bool HX = false> __device__ __forceinline__ void xchg(V* lds) {
    xchg1<KF, KT, HX>(a[0], lds);
    if constexpr (NS == 2 && LAM) xchg1<KF, KT>(a[NS - 1], lds);
  }

  // -------------------------------------------------------------- mixer butterflies
  // (I - i k X_q) on the tile bits of MASK, a compile-time subset of arrangement K's
  // register bits: (x, y) -> (x - i k y, y - i k x), two FMAs per amplitude.  A qubit
  // that the set does not mix (not in `act`) gets k = 0 by a uniform select, so the
  // unrolled butterflies carry no branches.  With LAM, lambda gets the same gates and
  // the mixer's gradient terms Im <lam|X_q|psi> are accumulated.  Every gate (I - i k X)
  // applied to both states multiplies each such term by 1 + k^2 = 1/w (the X's commute),
  // so the terms of the qubits mixed here are evaluated once after this arrangement's
  // butterflies and weighted by wcur = w^(gates of the mixer applied so far): that is
  // the term at the start of the mixer.  Evaluating after the butterflies keeps no
  // pre-gate values alive.
  // PSI: psi gets the gates too (false: only lambda, for a last arrangement after which
  // psi is neither stored nor used; the terms are then formed before the gates)
  template <int K, uint32_t MASK, bool LAM, bool PSI = true>
  __device__ __forceinline__ void mix_at(uint32_t act, R k, R w, R& wcur, R& gsum) {
    static_assert(PSI || (NS == 2 && LAM), "only lambda's gates need psi's to be skipped");
    // terms before the gates carry the scale of the gates applied so far
    if constexpr (!PSI) grad_terms<K, MASK>(act, wcur, gsum);
    constexpr int B0 = G::b0(K);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      if (!((MASK >> (B0 + b)) & 1u)) continue;
      const bool on = ((act >> (B0 + b)) & 1u) != 0;
      const R kk = on ? k : R(0);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r & (1 << b)) continue;
        const int r1 = r | (1 << b);
        if constexpr (NS == 2 && LAM) bflyk(a[NS - 1][r], a[NS - 1][r1], kk);
        if constexpr (PSI) bflyk(a[0][r], a[0][r1], kk);
      }
      wcur *= on ? w : R(1);
      // keep the scheduler from interleaving the butterflies of different qubits, which
      // holds pre- and post-gate values at once (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (PSI && NS == 2 && LAM) grad_terms<K, MASK>(act, wcur, gsum);
  }

  // The mixer's gradient terms of the qubits of MASK held in registers by arrangement K,
  // weighted by wcur and added to gsum.
  template <int K, uint32_t MASK> __device__ __forceinline__ void grad_terms(uint32_t act, R wcur, R& gsum) {
    constexpr int B0 = G::b0(K);
    // The register bits mixed here are taken two at a time where possible: for qubits
    // b1, b2 and the four registers r0 = r, r1 = r ^ b1, r2 = r ^ b2, r3 = r ^ b1 ^ b2 the
    // eight pair terms of both qubits add up to
    //   Im(conj(lam0 + lam3) (psi1 + psi2)) + Im(conj(lam1 + lam2) (psi0 + psi3)),
    // twelve operations where the two qubits' terms one by one take sixteen.  A pair with
    // a qubit the set does not mix (uniform test) takes the single-qubit form.
    constexpr uint32_t MB = (MASK >> B0) & ((1u << RB) - 1u);
    R gt = R(0);
    uint32_t left = MB;
#pragma unroll
    for (int b1 = 0; b1 < RB; ++b1) {
      if (!((left >> b1) & 1u)) continue;
      int b2 = -1;
#pragma unroll
      for (int c = b1 + 1; c < RB; ++c)
        if (b2 < 0 && ((left >> c) & 1u)) b2 = c;
      left &= ~(1u << b1);
      if (b2 >= 0) left &= ~(1u << b2);
      const bool on1 = ((act >> (B0 + b1)) & 1u) != 0;
      const bool on2 = b2 >= 0 && ((act >> (B0 + b2)) & 1u) != 0;
      if (b2 >= 0 && on1 && on2) {
        R g0 = R(0), g1 = R(0);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r & ((1 << b1) | (1 << b2))) continue;
          const int r1 = r | (1 << b1), r2 = r | (1 << b2), r3 = r1 | r2;
          const V la = mkv<R>(a[NS - 1][r].x + a[NS - 1][r3].x, a[NS - 1][r].y + a[NS - 1][r3].y);
          const V lb = mkv<R>(a[NS - 1][r1].x + a[NS - 1][r2].x, a[NS - 1][r1].y + a[NS - 1][r2].y);
          const V pa = mkv<R>(a[0][r1].x + a[0][r2].x, a[0][r1].y + a[0][r2].y);
          const V pb = mkv<R>(a[0][r].x + a[0][r3].x, a[0][r].y + a[0][r3].y);
          g0 = fmar(la.x, pa.y, g0);
          g0 = fmar(-la.y, pa.x, g0);
          g1 = fmar(lb.x, pb.y, g1);
          g1 = fmar(-lb.y, pb.x, g1);
        }
        gt += g0 + g1;
      } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int b = q == 0 ? b1 : b2;
          if (b < 0) continue;
          // sum over pairs of Im(conj(lam_r) psi_r1) + Im(conj(lam_r1) psi_r): two chains
          // of fused multiply-adds (four per pair)
          R g0 = R(0), g1 = R(0);
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            if (r & (1 << b)) continue;
            const int r1 = r | (1 << b);
            const V &l0 = a[NS - 1][r], &l1 = a[NS - 1][r1], &p0 = a[0][r], &p1 = a[0][r1];
            g0 = fmar(l0.x, p1.y, g0);
            g0 = fmar(-l0.y, p1.x, g0);
            g1 = fmar(l1.x, p0.y, g1);
            g1 = fmar(-l1.y, p0.x, g1);
          }
          gt += ((act >> (B0 + b)) & 1u) ? g0 + g1 : R(0);
        }
      }
    }
    gsum += wcur * gt;
    // the terms are formed here, before a following transpose: the empty volatile asm
    // is ordered with the LDS stores, so the pre-transpose values are not kept alive
    asm volatile("" : "+v"(gsum));
  }

  // -------------------------------------------------------------- z of register 0
  // the global bits of this thread's register 0 at arrangement K (the load or the phase
  // arrangement): the thread index scattered by the set's runs (two VALU per run)
  template <int K> __device__ __forceinline__ uint64_t tbits(const SetSpec& S) const {
    static_assert(K == LAST || K == P, "thread-bit runs exist for the load and phase arrangements");
    constexpr int KI = (K == LAST) ? 0 : 1;
    const uint32_t t = threadIdx.x;
    if (!S.tr64) {
      uint32_t z = 0;
#pragma unroll
      for (int i = 0; i < kMaxRuns; ++i) {
        const uint32_t r = S.trun[KI][i];
        z |= __builtin_amdgcn_ubfe(t, r & 0xFFu, (r >> 8) & 0xFFu) << (r >> 16);
      }
      return z;
    }
    uint64_t z = 0;
#pragma unroll
    for (int i = 0; i < kMaxRuns; ++i) {
      const uint32_t r = S.trun[KI][i];
      z |= (uint64_t)__builtin_amdgcn_ubfe(t, r & 0xFFu, (r >> 8) & 0xFFu) << (r >> 16);
    }
    return z;
  }
  // index z of register 0 at arrangement K, XOR the flip mask F: the register-0
  // amplitude is the one of basis state zbase ^ F (register bits set where F has them)
  template <int K> __device__ __forceinline__ uint64_t zbase(const SetSpec& S, uint64_t tile_base, uint64_t F) const {
    return (tile_base | tbits<K>(S)) ^ F;
  }

  // C(z) for every register amplitude at arrangement K.  With base b = zb (register bits
  // at their values in the flip mask F, which is uniform) and m the register bits flipped
  // relative to it: C(b ^ m) = C(b) + sum_{v in m} d_v
  //   + sum_{edges (v, w) inside m} 2 (2 [b_v != b_w] - 1),
  // d_v = deg v - 2 #{neighbours u with b_u != b_v}.  Everything about the register bits is
  // uniform (scalar).  ub = tile_base ^ F, the base without this thread's bits (uniform).
  // n <= 32: C(b) = sum_v [b_v] popc(adj_v & ~b), per vertex a sign-extended bit, a
  // three-input AND and a population count, the masks from scalar loads.
  // n > 32 (64-bit masks, three times the vector work per vertex): the tile's uniform part
  // is computed once per wave with lane v taking vertex v.  Let tm be the thread bits'
  // global positions, o the other vertices, and s this thread's values of b at tm (in
  // thread-bit order: s = t ^ ub there).  Splitting the edges by how many ends lie in tm,
  //   C(b) = 1/2 sum_{v in o} dd_v + sum_{v in tm} (z1_v + s_v c_v) + #{edges in tm cut by s},
  // dd_v = #{u in o, u ~ v: ub_u != ub_v}, z1_v = #{u in o, u ~ v: ub_u = 1},
  // c_v = #{u in o, u ~ v} - 2 z1_v; the last term is sum_{v in tm} s_v popc(ta_v & ~s),
  // ta_v = v's neighbours in tm as thread bits.  The wave's sum comes from ballots of the
  // bits of each lane's share, the per-vertex values from readlane.  The whole wave must
  // make the call (every kernel calling this runs full waves to here).
  template <int K> __device__ __forceinline__ void cuts(const SetSpec& S, uint64_t zb, uint64_t ub, uint64_t F,
                                                        const GraphDev* g0, int (&cv)[NR]) const {
    const cptr<GraphDev> g = cst(g0);
    const int n = g->n;
    constexpr int B0 = G::b0(K);
    int c0 = 0;
    int d[RB];
    if (n <= 32) {
      const uint32_t z = (uint32_t)zb;
      const cptr<uint4> a4 = (cptr<uint4>)&g->adj32[0];
      for (int v = 0; v < n; v += 4) {
        const uint4 a = a4[v >> 2];
        // bit v of z sign-extended to a mask (v_bfe_i32), then one three-input AND
        c0 = __popc(a.x & ~z & (uint32_t)__builtin_amdgcn_sbfe((int)z, v, 1)) + c0;
        c0 = __popc(a.y & ~z & (uint32_t)__builtin_amdgcn_sbfe((int)z, v + 1, 1)) + c0;
        c0 = __popc(a.z & ~z & (uint32_t)__builtin_amdgcn_sbfe((int)z, v + 2, 1)) + c0;
        c0 = __popc(a.w & ~z & (uint32_t)__builtin_amdgcn_sbfe((int)z, v + 3, 1)) + c0;
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const uint32_t v = S.pos[B0 + b];
        d[b] = 0;
        if (v != kDummy) {
          const uint32_t bm = 0u - (uint32_t)((F >> v) & 1ull);  // the base bit of v, uniform
          d[b] = g->deg[v] - 2 * __popc(g->adj32[v] & ((uint32_t)zb ^ bm));
        }
      }
    } else {
      static_assert(2 * kMaxN < 128, "a lane's share fits the seven ballot bits");
      constexpr int KI = (K == LAST) ? 0 : 1;
      const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
      const uint64_t adj = lane < (uint32_t)n ? g->adj[lane] : 0ull;
      uint64_t tm = 0;
      uint32_t ubt = 0, pt = 0;  // ub at tm and adj at tm, as thread bits
#pragma unroll
      for (int i = 0; i < kMaxRuns; ++i) {
        const uint32_t r = S.trun[KI][i], tb = r & 0xFFu, gb = r >> 16;
        const uint64_t mk = (1ull << ((r >> 8) & 0xFFu)) - 1ull;
        tm |= mk << gb;
        ubt |= (uint32_t)((ub >> gb) & mk) << tb;
        pt |= (uint32_t)((adj >> gb) & mk) << tb;
      }
      const uint64_t ao = adj & ~tm;
      const uint64_t uv = 0ull - ((ub >> lane) & 1ull);
      const int dd = __popcll(ao & (ub ^ uv));
      const int z1 = __popcll(ao & ub);
      const int cc = __popcll(ao) - 2 * z1;
      const uint32_t share = ((tm >> lane) & 1ull) ? (uint32_t)(2 * z1) : (uint32_t)dd;
      int a2 = 0;
#pragma unroll
      for (int k = 0; k < 7; ++k) a2 += __popcll(__ballot((share >> k) & 1u)) << k;
      c0 = a2 >> 1;
      const uint32_t s = threadIdx.x ^ ubt, ns = ~s;
#pragma unroll
      for (int i = 0; i < kMaxRuns; ++i) {
        const uint32_t r = S.trun[KI][i], tb = r & 0xFFu, w = (r >> 8) & 0xFFu, gb = r >> 16;
        for (uint32_t j = 0; j < w; ++j) {
          const int v = (int)(gb + j);
          const int sv = (int)((s >> (tb + j)) & 1u);
          const uint32_t ta = (uint32_t)__builtin_amdgcn_readlane((int)pt, v);
          c0 += sv * __builtin_amdgcn_readlane(cc, v);
          if (ta) c0 += sv * __popc(ta & ns);
        }
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const uint32_t v = S.pos[B0 + b];
        d[b] = 0;
        if (v != kDummy) {
          const uint32_t ta = (uint32_t)__builtin_amdgcn_readlane((int)pt, (int)v);
          const int o = __builtin_amdgcn_readlane(dd, (int)v);
          d[b] = g->deg[v] - 2 * (o + __popc(ta & (((ub >> v) & 1ull) ? ns : s)));
        }
      }
    }
    uint32_t rr[RB], df[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const uint32_t v = S.pos[B0 + b];
      rr[b] = 0;
      df[b] = 0;
      if (v != kDummy) {
        const uint64_t av = g->adj[v];
        const uint32_t fv = (uint32_t)((F >> v) & 1ull);
#pragma unroll
        for (int b2 = 0; b2 < RB; ++b2) {
          const uint32_t w = S.pos[B0 + b2];
          if (w != kDummy && ((av >> w) & 1u)) {
            rr[b] |= 1u << b2;
            if ((uint32_t)((F >> w) & 1ull) != fv) df[b] |= 1u << b2;
          }
        }
      }
    }
    cv[0] = c0;
#pragma unroll
    for (int r = 1; r < NR; ++r) {
      const int hb = 31 - __builtin_clz(r);
      const int rest = r ^ (1 << hb);
      const int npair = __popc(rr[hb] & (uint32_t)rest), ndiff = __popc(df[hb] & (uint32_t)rest);
      cv[r] = cv[rest] + d[hb] + 2 * (2 * ndiff - npair);
    }
  }

  // h(z) = sum_t w_t [z_i != z_j] for every register amplitude at arrangement K (the
  // load or the phase arrangement), from the set's term lists sorted by how many
  // endpoints sit in register bits: with base zb (register bits 0) and x_t the term's
  // value there, h(zb ^ m) = h0 + sum_{b in m} dh_b + sum over both-endpoint terms of
  // the pair correction -2 w (1 - 2x) when m holds both endpoints.
  template <int K> __device__ __forceinline__ void hvals(const SetSpec& S, uint64_t zb, const int4* terms, int (&hv)[NR],
                                                         bool n32) const {
    static_assert(K == LAST || K == P, "term lists exist for the load and phase arrangements");
    constexpr int KI = (K == LAST) ? 0 : 1;
    if (n32)
      hsum<uint32_t>(zb, terms + S.toff[KI], S.tcnt[KI], hv);
    else
      hsum<uint64_t>(zb, terms + S.toff[KI], S.tcnt[KI], hv);
  }
  // the weighted cut C(z) = sum_e w_e [z_u != z_v] from the set's cost-term lists
  template <int K> __device__ __forceinline__ void wcuts(const SetSpec& S, uint64_t zb, const int4* terms, int (&hv)[NR],
                                                         bool n32) const {
    static_assert(K == LAST || K == P, "term lists exist for the load and phase arrangements");
    constexpr int KI = (K == LAST) ? 0 : 1;
    if (n32)
      hsum<uint32_t>(zb, terms + S.coff[KI], S.ccnt[KI], hv);
    else
      hsum<uint64_t>(zb, terms + S.coff[KI], S.ccnt[KI], hv);
  }
  // the sum over one grouped term list (counts: the six group sizes)
  // (M: the index mask type, 32 bits when n <= 32)
  template <class M>
  __device__ __forceinline__ void hsum(uint64_t zb64, const int4* tp0, const uint16_t (&cnt)[6], int (&hv)[NR]) const {
    cptr<int4> tp = cst(tp0);
    const M zb = (M)zb64;
    auto xbit = [&](const int4& tm) -> int { return (int)(((uint32_t)(zb >> tm.x) ^ (uint32_t)(zb >> tm.y)) & 1u); };
    int h0 = 0;
    int dh[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) dh[b] = 0;
    {
      const int c = cnt[0];
      for (int t = 0; t < c; ++t) {
        const int4 tm = tp[t];
        h0 += tm.z * xbit(tm);
      }
      tp += c;
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int c = cnt[1 + b];
      for (int t = 0; t < c; ++t) {
        const int4 tm = tp[t];
        const int x = xbit(tm);
        h0 += tm.z * x;
        dh[b] += tm.z - 2 * tm.z * x;
      }
      tp += c;
    }
    int corr[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) corr[r] = 0;
    for (int t = 0, c = cnt[5]; t < c; ++t) {
      const int4 tm = tp[t];
      const int x = xbit(tm);
      const int ri = tm.w & 15, rj = tm.w >> 4;
      const int dv = tm.z - 2 * tm.z * x;
      h0 += tm.z * x;
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if (ri == b || rj == b) dh[b] += dv;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (((r >> ri) & 1) && ((r >> rj) & 1)) corr[r] -= 2 * dv;
    }
    int lin[NR];
    lin[0] = h0;
#pragma unroll
    for (int r = 1; r < NR; ++r) {
      const int hb = 31 - __builtin_clz(r);
      lin[r] = lin[r ^ (1 << hb)] + dh[hb];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) hv[r] = lin[r] + corr[r];
  }

  // -------------------------------------------------------------- ops at one position
  // LAM: lambda is live on entry (compile-time).  Returns with lam_live set when the
  // energy step created lambda.
  // COPS: the ops at this position, a compile-time mask (the program's own ops are
  // passed for reference only).
  // W: integer edge weights, the cut from the set's cost-term lists (compile-time)
  template <int K, bool LAM, uint32_t COPS, bool W = false>
  __device__ __forceinline__ void ops_at(uint8_t /*ops_rt*/, bool make_lam, const SetSpec& S, uint64_t tile_base,
                                         uint64_t F, const Ctx<R>& cx, const V* ltab, double& gacc, Acc& acc,
                                         double* zz_lds) {
    constexpr uint8_t ops = (uint8_t)COPS;
    if constexpr (ops == 0) return;
    uint64_t zb = zbase<K>(S, tile_base, F);
    // opaque here: the integer work below stays at this position instead of being
    // hoisted above the mixer, where its values would add to the register pressure
    asm volatile("" : "+v"(zb));
    if (EN && (ops & OP_ENERGY)) {
      int hv[NR];
      if (cst(cx.g)->h_is_cut)
        cuts<K>(S, zb, tile_base ^ F, F, cx.g, hv);
      else
        hvals<K>(S, zb, cx.terms, hv, cst(cx.g)->n <= 32);
      double e = 0.0, nr = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const R p2 = a[0][r].x * a[0][r].x + a[0][r].y * a[0][r].y;
        e += (double)p2 * (double)hv[r];
        nr += (double)p2;
      }
      // the sums are formed here, before the steps after this position change the state
      asm volatile("" : "+v"(e), "+v"(nr));
      acc.e += e;
      acc.nrm += nr;
      if (ops & OP_PERTERM) perterm<K>(S, zb, cx, zz_lds);
      if (NS == 2 && make_lam) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const R h = (R)hv[r] - cx.cen;
          a[NS - 1][r] = mkv<R>(h * a[0][r].x, h * a[0][r].y);
        }
        lam_live = true;
      }
    }
    if (ops & (OP_GRADG | OP_PHASE | OP_UNPHASE)) {
      int cv[NR];
      if constexpr (W)
        wcuts<K>(S, zb, cx.terms, cv, cst(cx.g)->n <= 32);
      else
        cuts<K>(S, zb, tile_base ^ F, F, cx.g, cv);
      if constexpr (NS == 2 && LAM) {
        if (ops & OP_GRADG) {
          R gs = R(0);
#pragma unroll
          for (int r = 0; r < NR; ++r) gs += ((R)cv[r] - cx.cen) * imcm(a[NS - 1][r], a[0][r]);
          // formed before the phase step below overwrites the states (ordered with its
          // table reads), so the pre-phase values are not kept alive
          asm volatile("" : "+v"(gs));
          gacc += (double)gs;
        }
      }
      if (ops & (OP_PHASE | OP_UNPHASE)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const V tv = ltab[cv[r]];  // exp(-+i gamma C) times the scale correction
          const R tc = tv.x, ts = tv.y;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            if (s == 0 || (NS == 2 && LAM)) {
              const V x = a[s][r];
              a[s][r] = mkv<R>(x.x * tc - x.y * ts, x.x * ts + x.y * tc);
            }
          }
        }
      }
    }
  }

  // <Z_i Z_j> partial sums per term, in a fixed order: each term's wave sum is kept by
  // lane (t mod 64) of the wave, and the waves then add their sums into the workgroup's
  // LDS accumulator one after another (wave 0 first), so repeated runs give identical bits.
  template <int K> __device__ __forceinline__ void perterm(const SetSpec& S, uint64_t zb, const Ctx<R>& cx, double* zz_lds) const {
    constexpr int B0 = G::b0(K);
    constexpr int NC = (kMaxT + 63) / 64;
    R p2[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) p2[r] = a[0][r].x * a[0][r].x + a[0][r].y * a[0][r].y;
    const int lane = threadIdx.x & 63;
    double mine[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      mine[c] = 0.0;
      const int tend = min(cx.T - c * 64, 64);
      for (int j = 0; j < tend; ++j) {
        const int4 tm = cx.terms[c * 64 + j];
        int ri = -1, rj = -1;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          if (S.pos[B0 + b] == (uint32_t)tm.x) ri = b;
          if (S.pos[B0 + b] == (uint32_t)tm.y) rj = b;
        }
        const uint32_t sm = (ri >= 0 ? (1u << ri) : 0u) ^ (rj >= 0 ? (1u << rj) : 0u);
        R acc = R(0);
#pragma unroll
        for (int r = 0; r < NR; ++r) acc += (__popc((uint32_t)r & sm) & 1) ? -p2[r] : p2[r];
        const int odd = (int)(((zb >> tm.x) ^ (zb >> tm.y)) & 1u);
        double v = odd ? -(double)acc : (double)acc;
        v = wave_sum(v);
        if (lane == j) mine[c] = v;
      }
    }
    const int wave = threadIdx.x >> 6;
    for (int w = 0; w < (1 << LB) / 64; ++w) {
      if (wave == w) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int t = c * 64 + lane;
          if (t < cx.T) zz_lds[t] += mine[c];
        }
      }
      __syncthreads();
    }
  }

  // -------------------------------------------------------------- global I/O
  // Loads and stores happen at the load arrangement LAST: the top tile bits in
  // registers, tile bits 0..8 over the threads, so 32 lanes touch >= 32 consecutive
  // amplitudes (>= 256 bytes).  Dummy tile bits (whole state smaller than a tile) have no
  // global position: amplitudes with a dummy bit set are neither loaded (they are zero)
  // nor stored.
  template <int K> __device__ __forceinline__ uint64_t thread_off(const SetSpec& S) const { return tbits<K>(S); }
  template <int K> __device__ __forceinline__ bool is_dummy(const SetSpec& S, int r) const {
    return S.dummy && (tidx<G::b0(K), RB>(threadIdx.x, r) & S.dummy);
  }
  // Global I/O of the tile at the load arrangement: register r of this thread is element
  // toff + roff[r] of the buffer at `base`.  With off32 (every byte offset inside the
  // buffer below 2^32) the address of register r is the uniform base + roff[r] (scalar
  // registers) plus one 32-bit per-thread byte offset shared by all registers, the form
  // the global load and store instructions take directly; otherwise each register gets a
  // 64-bit address on the vector unit.
  // With OFF32 the registers move through raw buffer loads and stores: a descriptor on
  // `base` (stride 0, every offset below 2^32 in range), the thread's byte offset in one
  // vector register and register r's byte offset roff[r] as a scalar offset.
  static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) {
    // the base is the same for every lane; say so, so that the descriptor lives in
    // scalar registers (a descriptor in vector registers makes every access a loop).
    // readfirstlane returns a signed int: each half is widened as unsigned, or a low
    // word with bit 31 set would sign-extend into the high word of the address
    const uint64_t b = (uint64_t)base;
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint64_t u = ((uint64_t)hi << 32) | (uint64_t)lo;
    return __builtin_amdgcn_make_buffer_rsrc((void*)u, (short)0, (int)0xFFFFFFFF, 0x00020000);
  }
  // cache policy of the state loads: a sweep reads every amplitude once and the next
  // sweep reads what this one stores, not what it loaded, so when the evaluation streams
  // more state than the last-level cache holds the loads are marked non-temporal (the nt
  // bit of the gfx950 cache-policy field); the stores keep the default policy, so freshly
  // written state can stay in the last-level cache
  static constexpr int kStreamPolicy = 2;
  // the same non-temporal load through a 64-bit address (states beyond 4 GiB)
  static __device__ __forceinline__ V gload(const V* q) {
    using E = R __attribute__((ext_vector_type(2)));
    const E x = __builtin_nontemporal_load(reinterpret_cast<const E*>(q));
    return mkv<R>(x.x, x.y);
  }
  template <bool NT>
  static __device__ __forceinline__ V buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t vo, uint32_t so) {
    constexpr int pol = NT ? kStreamPolicy : 0;
    if constexpr (sizeof(V) == 8)
      return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)vo, (int)so, pol));
    else
      return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)vo, (int)so, pol));
  }
  static __device__ __forceinline__ void buf_store(V x, __amdgpu_buffer_rsrc_t rs, uint32_t vo, uint32_t so) {
    if constexpr (sizeof(V) == 8)
      __builtin_amdgcn_raw_buffer_store_b64(
          __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0)), x), rs, (int)vo, (int)so, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b128(
          __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0)), x), rs, (int)vo, (int)so, 0);
  }
  // Register r's element is index toff + roff[r] (toff = tile_base + the thread's
  // offset), or, when r is in S.mirror (half state, its index has bit n-1 set), the
  // mirrored index mfull - (toff + roff[r]): the thread part tmax - thread offset and the
  // uniform part mfull - tile_base - roff[r] - tmax, both >= 0 (the parts are disjoint
  // bit fields of the index).
  template <int K, bool OFF32, bool MIR, bool NT>
  __device__ __forceinline__ void load_regs(int s, const V* base, uint64_t tile_base, uint64_t toff, const SetSpec& S) {
    if constexpr (OFF32) {
      const __amdgpu_buffer_rsrc_t rs = rsrc(base);
      const uint32_t bo = (uint32_t)toff * (uint32_t)sizeof(V);
      if (!S.dummy && !(MIR && S.mirror)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) a[s][r] = buf_load<NT>(rs, bo, (uint32_t)S.roff[r] * (uint32_t)sizeof(V));
      } else if (MIR && S.mirror) {
        const uint32_t bm = (uint32_t)(S.tmax - (toff - tile_base)) * (uint32_t)sizeof(V);
        // uniform over the workgroup: the mirrored registers' scalar offsets are su - roff
        const uint32_t su = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((S.mfull - tile_base - S.tmax) * sizeof(V)));
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const uint32_t ro = (uint32_t)S.roff[r] * (uint32_t)sizeof(V);
          const bool m = (S.mirror >> r) & 1u;
          a[s][r] = buf_load<NT>(rs, m ? bm : bo, m ? su - ro : ro);
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          a[s][r] = is_dummy<K>(S, r) ? mkv<R>(R(0), R(0)) : buf_load<NT>(rs, bo, (uint32_t)S.roff[r] * (uint32_t)sizeof(V));
      }
    } else {
      const V* p = base + toff;
      if (!S.dummy && !(MIR && S.mirror)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) a[s][r] = NT ? gload(p + S.roff[r]) : p[S.roff[r]];
      } else if (MIR && S.mirror) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          a[s][r] = ((S.mirror >> r) & 1u) ? base[S.mfull - toff - S.roff[r]] : p[S.roff[r]];
      } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) a[s][r] = is_dummy<K>(S, r) ? mkv<R>(R(0), R(0)) : p[S.roff[r]];
      }
    }
  }
  template <int K, bool OFF32, bool MIR> __device__ __forceinline__ void store_regs(int s, V* base, uint64_t tile_base,
                                                                          uint64_t toff, const SetSpec& S) const {
    if constexpr (OFF32) {
      const __amdgpu_buffer_rsrc_t rs = rsrc(base);
      const uint32_t bo = (uint32_t)toff * (uint32_t)sizeof(V);
      if (!S.dummy && !(MIR && S.mirror)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) buf_store(a[s][r], rs, bo, (uint32_t)S.roff[r] * (uint32_t)sizeof(V));
      } else if (MIR && S.mirror) {
        const uint32_t bm = (uint32_t)(S.tmax - (toff - tile_base)) * (uint32_t)sizeof(V);
        const uint32_t su = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((S.mfull - tile_base - S.tmax) * sizeof(V)));
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const uint32_t ro = (uint32_t)S.roff[r] * (uint32_t)sizeof(V);
          const bool m = (S.mirror >> r) & 1u;
          buf_store(a[s][r], rs, m ? bm : bo, m ? su - ro : ro);
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (!is_dummy<K>(S, r)) buf_store(a[s][r], rs, bo, (uint32_t)S.roff[r] * (uint32_t)sizeof(V));
      }
    } else {
      V* p = base + toff;
      if (!S.dummy && !(MIR && S.mirror)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) p[S.roff[r]] = a[s][r];
      } else if (MIR && S.mirror) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if ((S.mirror >> r) & 1u)
            base[S.mfull - toff - S.roff[r]] = a[s][r];
          else
            p[S.roff[r]] = a[s][r];
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (!is_dummy<K>(S, r)) p[S.roff[r]] = a[s][r];
      }
    }
  }
  // MIR: the route can hold bit n-1 among the tile bits (sets of high qubits), so the
  // half state's mirrored registers are possible; false compiles them out
  template <int K, bool MIR = true>
  __device__ __forceinline__ void load_all(int s, const V* base, uint64_t tile_base, uint64_t toff, const SetSpec& S,
                                           bool off32, bool nt = false) {
    static_assert(K == LAST, "global I/O happens at the load arrangement");
    if (off32) {
      if (nt)
        load_regs<K, true, MIR, true>(s, base, tile_base, toff, S);
      else
        load_regs<K, true, MIR, false>(s, base, tile_base, toff, S);
    } else {
      if (nt)
        load_regs<K, false, MIR, true>(s, base, tile_base, toff, S);
      else
        load_regs<K, false, MIR, false>(s, base, tile_base, toff, S);
    }
  }
  template <int K, bool MIR = true>
  __device__ __forceinline__ void store_all(int s, V* base, uint64_t tile_base, uint64_t toff, const SetSpec& S,
                                            bool off32) const {
    static_assert(K == LAST, "global I/O happens at the load arrangement");
    if (off32)
      store_regs<K, true, MIR>(s, base, tile_base, toff, S);
    else
      store_regs<K, false, MIR>(s, base, tile_base, toff, S);
  }
  template <int K> __device__ __forceinline__ void init_at(const SetSpec& S, R amp) {
#pragma unroll
    for (int r = 0; r < NR; ++r) a[0][r] = mkv<R>(is_dummy<K>(S, r) ? R(0) : amp, R(0));
  }

  // -------------------------------------------------------------- one sweep on one tile
  // Mixer routes (both start at the load arrangement LAST): ROUTE_FULL visits LAST, 0,
  // 1, ..., P; ROUTE_HIGH, for sets whose mixed qubits are all tile bits >= kMinContig,
  // skips arrangement 0.  Mixer A walks the route forward and ends at the phase
  // arrangement P, mixer B walks it back to LAST.  The qubits mixed at each stop are
  // compile-time masks (fwd_mask, bwd_mask).
  // PSI_P: psi gets the gates at the last stop P too (see mix_at)
  template <int RT, int K, int PREV, bool LAM, bool PSI_P = true>
  __device__ __forceinline__ void fwd_steps(uint32_t act, R k, R w, R& wcur, R& gs, V* lds) {
    if constexpr (K <= P) {
      xchg<PREV, K, LAM, half_xchg(RT)>(lds);
      mix_at<K, fwd_mask(RT, K), LAM, (K < P || PSI_P)>(act, k, w, wcur, gs);
      fwd_steps<RT, K + 1, K, LAM, PSI_P>(act, k, w, wcur, gs, lds);
    }
  }
  template <int RT, int K, bool LAM>
  __device__ __forceinline__ void bwd_steps(uint32_t act, R k, R w, R& wcur, R& gs, V* lds) {
    if constexpr (K >= first_arr(RT)) {
      xchg<K + 1, K, LAM, half_xchg(RT)>(lds);
      mix_at<K, bwd_mask(RT, K), LAM>(act, k, w, wcur, gs);
      bwd_steps<RT, K - 1, LAM>(act, k, w, wcur, gs, lds);
    }
  }
  // PSI_LAST = false: psi is neither stored nor used after this mixer, so the gates of
  // its last stop are applied to lambda only
  template <int RT, bool LAM, bool PSI_LAST = true>
  __device__ __forceinline__ void mix_fwd(uint32_t act, R k, R w, R& gs, V* lds) {
    R wcur = R(1);
    mix_at<LAST, fwd_mask(RT, LAST), LAM>(act, k, w, wcur, gs);
    fwd_steps<RT, first_arr(RT), LAST, LAM, PSI_LAST>(act, k, w, wcur, gs, lds);
  }
  template <int RT, bool LAM, bool PSI_LAST = true>
  __device__ __forceinline__ void mix_bwd(uint32_t act, R k, R w, R& gs, V* lds) {
    constexpr int FIRST = first_arr(RT);
    R wcur = R(1);
    mix_at<P, bwd_mask(RT, P), LAM>(act, k, w, wcur, gs);
    bwd_steps<RT, P - 1, LAM>(act, k, w, wcur, gs, lds);
    xchg<(FIRST < P ? FIRST : P), LAST, LAM, half_xchg(RT)>(lds);
    mix_at<LAST, bwd_mask(RT, LAST), LAM, PSI_LAST>(act, k, w, wcur, gs);
  }

  // Executes program `pg` on the tile with id `tile` of set S (whose route is RT), for
  // a sweep of shape KIND (SK_*), known at compile time: no step is a run-time branch
  // around register updates.  The sweep runs in three stages (pre ops, mixer A + mid
  // ops, mixer B + store), each compiled for lambda live or not; lambda becomes live
  // where the energy step makes it.  Stores and buffer indices follow the program.
  // late_tabs: called once the state loads are issued (a shape whose phase tables are
  // first read at the mid position, after the first LDS exchange and its barrier, loads
  // them there so their latency overlaps the state loads')
  template <int RT, uint32_t KIND, class TabLoad = NoTabs>
  __device__ __forceinline__ void run(const SweepProg& pg, const SetSpec& S, const SwScale& sc, uint64_t tile,
                                      const Ctx<R>& cx, V* lds_x, const V* ltab_pre, const V* ltab_mid, Acc& acc,
                                      double* zz_lds, const TabLoad& late_tabs = TabLoad{}) {
    const cptr<SwScale> scp = cst(&sc);  // uniform: scalar loads
    static_assert((KIND & SK_GENERIC) == 0, "generic sweeps take run_rt");
    static_assert(NS == ((KIND & (SK_LAM_IN | SK_MAKE_LAM)) ? 2 : 1), "state count of the shape");
    static_assert(!((KIND & SK_MAKE_LAM) && (sk_pre(KIND) & OP_ENERGY)), "lambda is made at the mid position");
    constexpr int KL = LAST;
    const uint64_t tile_base = pdep64(tile, S.fixmask);
    if constexpr ((KIND & SK_INIT) != 0) {
      init_at<KL>(S, cx.amp);
    } else {
      const uint64_t toff = tile_base + thread_off<KL>(S);
      if constexpr ((KIND & SK_LOAD_PSI) != 0) load_all<KL, RT == ROUTE_HIGH>(0, cx.psi + pg.ld_buf * cx.N, tile_base, toff, S, cx.off32, cx.nt);
      if constexpr (NS == 2 && (KIND & SK_LAM_IN) != 0)
        load_all<KL, RT == ROUTE_HIGH>(NS - 1, cx.lam, tile_base, toff, S, cx.off32, cx.nt);
      late_tabs();
      if constexpr (NS == 2 && (KIND & SK_LAM_IN) != 0) {
        if (scp->fix_lam) {
          const R fr = (R)scp->lam_fix[0], fi = (R)scp->lam_fix[1];
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const V x = a[NS - 1][r];
            a[NS - 1][r] = mkv<R>(x.x * fr - x.y * fi, x.x * fi + x.y * fr);
          }
        }
      }
    }
    constexpr bool LAM0 = NS == 2 && (KIND & SK_LAM_IN) != 0;
    lam_live = LAM0;
    // SK_PSI_DEAD: psi is not stored (lambda is stored alone), so the last stop of the
    // last mixer applies its gates to lambda only
    constexpr bool PSI_DEAD = (KIND & SK_PSI_DEAD) != 0;
    constexpr bool A_LAST = sk_mid(KIND) == 0 && (KIND & SK_MIXB) == 0;  // nothing after mixer A
    static_assert(!PSI_DEAD || NS == 2, "only two-state sweeps leave psi unstored");
    constexpr bool W = (KIND & SK_WEIGHTED) != 0;
    ops_at<KL, LAM0, sk_pre(KIND), W>(pg.pre_ops, false, S, tile_base, scp->F_pre, cx, ltab_pre, acc.gpre, acc, zz_lds);
    bool at_p = false;
    if constexpr ((KIND & SK_MIXA) != 0) {
      R gs = R(0);
      mix_fwd<RT, LAM0, !(PSI_DEAD && A_LAST)>(S.act, (R)scp->kA, (R)scp->wA, gs, lds_x);
      if (pg.mixA_grad) acc.ba += (double)gs;
      at_p = true;
    }
    if constexpr ((sk_mid(KIND) != 0 || (KIND & SK_MIXB) != 0) && (KIND & SK_MIXA) == 0) {
      xchg<LAST, P, LAM0, half_xchg(RT)>(lds_x);
      at_p = true;
    }
    ops_at<P, LAM0, sk_mid(KIND), W>(pg.mid_ops, (KIND & SK_MAKE_LAM) != 0, S, tile_base, scp->F_mid, cx, ltab_mid,
                                  acc.gmid, acc, zz_lds);
    constexpr bool LAM1 = LAM0 || (NS == 2 && (KIND & SK_MAKE_LAM) != 0);
    if constexpr ((KIND & SK_MIXB) != 0) {
      R gs = R(0);
      mix_bwd<RT, LAM1, !PSI_DEAD>(S.act, (R)scp->kB, (R)scp->wB, gs, lds_x);
      if (pg.mixB_grad) acc.bb += (double)gs;
      at_p = false;
    }
    const bool st_psi = !PSI_DEAD && (pg.flags & F_STORE_PSI) && cx.psi;
    const bool st_lam = NS == 2 && LAM1 && (pg.flags & F_STORE_LAM) && cx.lam;
    if ((st_psi || st_lam) && at_p) {
      if constexpr (PSI_DEAD)
        xchg1<P, LAST>(a[NS - 1], lds_x);  // lambda alone goes back to the store layout
      else
        xchg<P, LAST, LAM1, half_xchg(RT)>(lds_x);
    }
    uint64_t toff = tile_base + thread_off<LAST>(S);
    // opaque to the compiler: the store addresses are formed here, not kept in
    // registers from the loads (that would hold 2 VGPRs per register and state)
    asm volatile("" : "+v"(toff));
    if (st_psi) store_all<LAST, RT == ROUTE_HIGH>(0, cx.psi + pg.st_buf * cx.N, tile_base, toff, S, cx.off32);
    if (st_lam) store_all<LAST, RT == ROUTE_HIGH>(NS - 1, cx.lam, tile_base, toff, S, cx.off32);
  }

  // ================================================================ run-time-flag path
  // The generic sweep (batched unit kernels and shapes without a specialization): the
  // same steps as above with every decision taken from the program at run time.  Mixer
  // butterflies follow a run-time set of pending qubits and lambda's liveness, and the
  // mixer's gradient terms are formed pair by pair before each gate.
  template <int KF, int KT> __device__ __forceinline__ void xchg_rt(V* lds) {
    xchg1<KF, KT>(a[0], lds);
    if (NS == 2 && lam_live) xchg1<KF, KT>(a[NS - 1], lds);
  }

  // (I - i k X_q) on every tile bit of `todo` held in registers by arrangement K:
  // (x, y) -> (x - i k y, y - i k x), two FMAs per amplitude.  With `grad`, the pair's
  // Im <lam|X_q|psi> is accumulated with weight wcur, which tracks the scale change of
  // the preceding gates of the same mixer (wcur *= w after every qubit).
  template <int K> __device__ __forceinline__ void mix_at_rt(uint32_t& todo, R k, R w, R& wcur, bool grad, R& gsum) {
    constexpr int B0 = G::b0(K);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      if ((todo >> (B0 + b)) & 1u) {
        R gq = R(0);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r & (1 << b)) continue;
          const int r1 = r | (1 << b);
          if (NS == 2) {
            if (grad) gq += imcm(a[NS - 1][r], a[0][r1]) + imcm(a[NS - 1][r1], a[0][r]);
            if (lam_live) bflyk(a[NS - 1][r], a[NS - 1][r1], k);
          }
          bflyk(a[0][r], a[0][r1], k);
        }
        if (NS == 2 && grad) gsum += wcur * gq;
        wcur *= w;
      }
    }
    todo &= ~(((1u << RB) - 1u) << B0);
  }

  template <int K>
  __device__ __forceinline__ void ops_at_rt(uint8_t ops, bool make_lam, const SetSpec& S, uint64_t tile_base, uint64_t F,
                                         const Ctx<R>& cx, const V* ltab, double& gacc, Acc& acc, double* zz_lds) {
    if (!ops) return;
    const uint64_t zb = zbase<K>(S, tile_base, F);
    if (EN && (ops & OP_ENERGY)) {
      int hv[NR];
      if (cst(cx.g)->h_is_cut)
        cuts<K>(S, zb, tile_base ^ F, F, cx.g, hv);
      else
        hvals<K>(S, zb, cx.terms, hv, cst(cx.g)->n <= 32);
      double e = 0.0, nr = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const R p2 = a[0][r].x * a[0][r].x + a[0][r].y * a[0][r].y;
        e += (double)p2 * (double)hv[r];
        nr += (double)p2;
      }
      asm volatile("" : "+v"(e), "+v"(nr));  // formed here (see ops_at)
      acc.e += e;
      acc.nrm += nr;
      if (ops & OP_PERTERM) perterm<K>(S, zb, cx, zz_lds);
      if (NS == 2 && make_lam) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const R h = (R)hv[r] - cx.cen;
          a[NS - 1][r] = mkv<R>(h * a[0][r].x, h * a[0][r].y);
        }
        lam_live = true;
      }
    }
    if (ops & (OP_GRADG | OP_PHASE | OP_UNPHASE)) {
      int cv[NR];
      if (cst(cx.g)->weighted)
        wcuts<K>(S, zb, cx.terms, cv, cst(cx.g)->n <= 32);
      else
        cuts<K>(S, zb, tile_base ^ F, F, cx.g, cv);
      if (NS == 2 && (ops & OP_GRADG)) {
        R gs = R(0);
#pragma unroll
        for (int r = 0; r < NR; ++r) gs += ((R)cv[r] - cx.cen) * imcm(a[NS - 1][r], a[0][r]);
        asm volatile("" : "+v"(gs));  // formed here (see ops_at)
        gacc += (double)gs;
      }
      if (ops & (OP_PHASE | OP_UNPHASE)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const V tv = ltab[cv[r]];  // exp(-+i gamma C) times the scale correction
          const R tc = tv.x, ts = tv.y;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            if (s == 0 || lam_live) {
              const V x = a[s][r];
              a[s][r] = mkv<R>(x.x * tc - x.y * ts, x.x * ts + x.y * tc);
            }
          }
        }
      }
    }
  }

  // Mixer routes (both start at the load arrangement LAST): ROUTE_FULL visits LAST, 0,
  // 1, ..., P; ROUTE_HIGH, for sets whose active qubits are all tile bits >= 4, skips
  // arrangement 0.  Mixer A walks the route forward and ends at the phase arrangement
  // P, mixer B walks it back to LAST.  A qubit is mixed at the first arrangement of the
  // walk that holds it in registers.
  template <int K, int PREV>
  __device__ __forceinline__ void fwd_steps_rt(uint32_t& todo, R k, R w, R& wcur, bool gr, R& gs, V* lds) {
    if constexpr (K <= P) {
      xchg_rt<PREV, K>(lds);
      mix_at_rt<K>(todo, k, w, wcur, gr, gs);
      fwd_steps_rt<K + 1, K>(todo, k, w, wcur, gr, gs, lds);
    }
  }
  template <int K, int FIRST>
  __device__ __forceinline__ void bwd_steps_rt(uint32_t& todo, R k, R w, R& wcur, bool gr, R& gs, V* lds) {
    if constexpr (K >= FIRST) {
      xchg_rt<K + 1, K>(lds);
      mix_at_rt<K>(todo, k, w, wcur, gr, gs);
      bwd_steps_rt<K - 1, FIRST>(todo, k, w, wcur, gr, gs, lds);
    }
  }
  template <int RT> __device__ __forceinline__ void mix_fwd_rt(uint32_t& todo, R k, R w, R& wcur, bool gr, R& gs, V* lds) {
    mix_at_rt<LAST>(todo, k, w, wcur, gr, gs);
    fwd_steps_rt<(RT == ROUTE_FULL ? 0 : 1), LAST>(todo, k, w, wcur, gr, gs, lds);
  }
  template <int RT> __device__ __forceinline__ void mix_bwd_rt(uint32_t& todo, R k, R w, R& wcur, bool gr, R& gs, V* lds) {
    constexpr int FIRST = (RT == ROUTE_FULL) ? 0 : 1;
    mix_at_rt<P>(todo, k, w, wcur, gr, gs);
    bwd_steps_rt<P - 1, FIRST>(todo, k, w, wcur, gr, gs, lds);
    xchg_rt<(FIRST < P ? FIRST : P), LAST>(lds);
    mix_at_rt<LAST>(todo, k, w, wcur, gr, gs);
  }

  // Executes program `pg` on the tile with id `tile` of set S (whose route is RT).
  // With `io` false the state stays in registers (whole state in one tile); stores still
  // happen when the program asks for them and a destination exists.
  template <int RT>
  __device__ __forceinline__ void run_rt(const SweepProg& pg, const SetSpec& S, const SwScale& sc, uint64_t tile,
                                      const Ctx<R>& cx, bool io, V* lds_x, const V* ltab_pre, const V* ltab_mid, Acc& acc,
                                      double* zz_lds) {
    const cptr<SwScale> scp = cst(&sc);  // uniform: scalar loads
    constexpr int KL = LAST;
    const uint64_t tile_base = pdep64(tile, S.fixmask);
    if (pg.flags & F_INIT) {
      init_at<KL>(S, cx.amp);
      lam_live = false;
    } else if (io) {
      if (pg.flags & F_LOAD_PSI) load_all<KL, RT == ROUTE_HIGH>(0, cx.psi + pg.ld_buf * cx.N, tile_base, tile_base + thread_off<KL>(S), S, cx.off32,
                                                 cx.nt);
      lam_live = (pg.flags & F_LAM_LIVE) != 0;
      if (NS == 2 && (pg.flags & F_LOAD_LAM)) {
        load_all<KL, RT == ROUTE_HIGH>(NS - 1, cx.lam, tile_base, tile_base + thread_off<KL>(S), S, cx.off32, cx.nt);
        if (scp->fix_lam) {
          const R fr = (R)scp->lam_fix[0], fi = (R)scp->lam_fix[1];
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const V x = a[NS - 1][r];
            a[NS - 1][r] = mkv<R>(x.x * fr - x.y * fi, x.x * fi + x.y * fr);
          }
        }
      }
    }
    const bool make_lam = (pg.flags & F_MAKE_LAM) != 0;
    ops_at_rt<KL>(pg.pre_ops, make_lam, S, tile_base, scp->F_pre, cx, ltab_pre, acc.gpre, acc, zz_lds);
    bool at_p = false;
    if (pg.mixA_dir) {
      R wcur = R(1), gs = R(0);
      uint32_t todo = S.act;
      mix_fwd_rt<RT>(todo, (R)scp->kA, (R)scp->wA, wcur, pg.mixA_grad != 0, gs, lds_x);
      acc.ba += (double)gs;
      at_p = true;
    }
    if ((pg.mid_ops || pg.mixB_dir) && !at_p) {
      xchg_rt<KL, P>(lds_x);
      at_p = true;
    }
    ops_at_rt<P>(pg.mid_ops, make_lam, S, tile_base, scp->F_mid, cx, ltab_mid, acc.gmid, acc, zz_lds);
    if (pg.mixB_dir) {
      R wcur = R(1), gs = R(0);
      uint32_t todo = S.act;
      mix_bwd_rt<RT>(todo, (R)scp->kB, (R)scp->wB, wcur, pg.mixB_grad != 0, gs, lds_x);
      acc.bb += (double)gs;
      at_p = false;
    }
    const bool st_psi = (pg.flags & F_STORE_PSI) && cx.psi;
    const bool st_lam = NS == 2 && (pg.flags & F_STORE_LAM) && cx.lam;
    if ((st_psi || st_lam) && at_p) xchg_rt<P, KL>(lds_x);
    if (st_psi) store_all<KL, RT == ROUTE_HIGH>(0, cx.psi + pg.st_buf * cx.N, tile_base, tile_base + thread_off<KL>(S), S, cx.off32);
    if (st_lam) store_all<KL, RT == ROUTE_HIGH>(NS - 1, cx.lam, tile_base, tile_base + thread_off<KL>(S), S, cx.off32);
  }
  __device__ __forceinline__ void run_any(const SweepProg& pg, const SetSpec& S, const SwScale& sc, uint64_t tile,
                                          const Ctx<R>& cx, bool io, V* lds_x, const V* ltab_pre, const V* ltab_mid,
                                          Acc& acc, double* zz_lds) {
    if (S.route == ROUTE_HIGH)
      run_rt<ROUTE_HIGH>(pg, S, sc, tile, cx, io, lds_x, ltab_pre, ltab_mid, acc, zz_lds);
    else
      run_rt<ROUTE_FULL>(pg, S, sc, tile, cx, io, lds_x, ltab_pre, ltab_mid, acc, zz_lds);
  }
};

// ---------------------------------------------------------------------------------
// workgroup reduction of a few doubles; result valid in thread 0
template <int N, int NT> __device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[wave * N + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[w * N + i];
      v[i] = s;
    }
  }
  __syncthreads();
}

// phase-table multipliers of one position into LDS: exp(-i gamma_l c) (conjugated for
// the inverse gate) times the complex scale correction rho
template <class R>
__device__ __forceinline__ void load_tab(typename Cx<R>::V* ltab, const typename Cx<R>::V* tab, int layer, int cmax,
                                         bool conj, const double* rho) {
  if (layer < 0) return;
  const typename Cx<R>::V* src = tab + (size_t)layer * (cmax + 1);
  const double rr = cst(rho)[0], ri = cst(rho)[1];
  for (int c = threadIdx.x; c <= cmax; c += blockDim.x) {
    const double tr = (double)src[c].x, ti = conj ? -(double)src[c].y : (double)src[c].y;
    ltab[c] = mkv<R>((R)(tr * rr - ti * ri), (R)(tr * ri + ti * rr));
  }
}

// apply a sweep's scale corrections to the per-thread sums
__device__ __forceinline__ void scale_acc(Acc& acc, const SweepProg& pg, const SwScale& sc0) {
  const cptr<SwScale> sc = cst(&sc0);
  const double se = (pg.pre_ops & OP_ENERGY) ? sc->s_pre : sc->s_mid;
  acc.e *= se;
  acc.nrm *= se;
  acc.gpre *= sc->s_pre;
  acc.gmid *= sc->s_mid;
  acc.ba *= sc->s_A;
  acc.bb *= sc->s_B;
}

// Walk a unit's sweep programs and record, per sweep, the butterfly coefficients and

// ---------------------------------------------------------------------------------
// One sweep of a large state: one workgroup per tile.
template <class R> struct SweepArgs {
  typename Cx<R>::V* psi;
  typename Cx<R>::V* lam;
  const GraphDev* g;
  const int4* terms;
  const typename Cx<R>::V* tab;
  const SwScale* scale;  // this sweep's scale record
  double* partial;       // [nslot][ntiles]
  int nslot;
  int T;
  int cmax;
  R amp;
  uint64_t N;  // amplitudes per state
  SetSpec set;
  SweepProg prog;
  int nt;  // non-temporal state loads
};

#define AAQ_TILE_BOUNDS __launch_bounds__(1 << (LT - kRegBits))
// Specialized single-instance sweeps: at most 128 VGPRs per lane, i.e. four waves per
// SIMD, the occupancy the tile LDS allows anyway; the generic sweeps are left to the
// compiler.
// the specialised one-state sweeps of the high-qubit route exchange half tiles: half the
// LDS, so six workgroups fit a compute unit (their registers allow six waves per SIMD)
constexpr bool sweep_half_xchg(int ns, int rt, uint32_t kind) {
  return ns == 1 && rt == ROUTE_HIGH && !(kind & SK_GENERIC);
}
constexpr int sweep_waves_per_eu(int ns, int rt, uint32_t kind) {
  // the per-term shape keeps a term sum per lane and chunk of 64 terms: four waves
  return (kind & SK_GENERIC) ? 1 : ((sk_mid(kind) & OP_PERTERM) != 0) ? 4 : sweep_half_xchg(ns, rt, kind) ? 6 : 4;
}
// partial-sum slots a sweep shape can fill (SLOT_* bits; the generic sweeps: all six)
constexpr uint32_t sweep_slots(uint32_t kind) {
  if (kind & SK_GENERIC) return 0x3Fu;
  const uint32_t ops = sk_pre(kind) | sk_mid(kind);
  uint32_t m = 0;
  if (ops & OP_ENERGY) m |= (1u << SLOT_E) | (1u << SLOT_NORM);
  if (sk_pre(kind) & OP_GRADG) m |= 1u << SLOT_GPRE;
  if (sk_mid(kind) & OP_GRADG) m |= 1u << SLOT_GMID;
  if (kind & SK_MIXA) m |= 1u << SLOT_BA;
  if (kind & SK_MIXB) m |= 1u << SLOT_BB;
  return m;
}
#define AAQ_SWEEP_BOUNDS(NS, RT, KIND) \
  __launch_bounds__(1 << (LT - kRegBits)) __attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu(NS, RT, KIND))))

// One workgroup per tile; partial sums per tile: partial[slot][tile].
template <class R, int NS, bool PT, bool EN, int RT, int LT, uint32_t KIND>
__global__ AAQ_SWEEP_BOUNDS(NS, RT, KIND) void k_sweep(SweepArgs<R> A) {
  using G = Geo<R, LT>;
  using V = typename G::V;
  __shared__ V lds_x[lds_slot(sweep_half_xchg(NS, RT, KIND) ? G::TILE / 2 : G::TILE)];
  __shared__ double red[(G::NT / 64) * 6];
  __shared__ double zz[PT ? kMaxT : 1];
  extern __shared__ unsigned char dyn_lds[];  // two phase tables of cmax+1 entries
  V* ltab0 = reinterpret_cast<V*>(dyn_lds);
  V* ltab1 = ltab0 + (A.cmax + 1);
  const SwScale& sc = *A.scale;
  // a specialised shape with no phase before its first mixer loads its mid table once its
  // state loads are issued (Tile::run); the others load the tables here
  constexpr bool LATE_TAB = (KIND & SK_GENERIC) == 0 && !PT && (sk_pre(KIND) & (OP_PHASE | OP_UNPHASE)) == 0;
  auto mid_tab = [&]() {
    if (A.prog.mid_ops & (OP_PHASE | OP_UNPHASE))
      load_tab<R>(ltab1, A.tab, A.prog.mid_layer, A.cmax, (A.prog.mid_ops & OP_UNPHASE) != 0, sc.rho_mid);
  };
  if constexpr (!LATE_TAB) {
    if (A.prog.pre_ops & (OP_PHASE | OP_UNPHASE))
      load_tab<R>(ltab0, A.tab, A.prog.pre_layer, A.cmax, (A.prog.pre_ops & OP_UNPHASE) != 0, sc.rho_pre);
    mid_tab();
    if (PT)
      for (int t = threadIdx.x; t < A.T; t += G::NT) zz[t] = 0.0;
    __syncthreads();
  }
  Ctx<R> cx{A.g, A.terms, A.tab, A.psi, A.lam, A.amp, A.T, A.cmax, A.N, A.N <= ((uint64_t)1 << 32) / sizeof(V), A.nt != 0,
            (R)(0.5 * A.cmax)};
  Tile<R, NS, EN, LT> tl;
  Acc acc;
  acc.zero();
  const uint32_t tile = blockIdx.x;
  if constexpr ((KIND & SK_GENERIC) != 0)
    tl.template run_rt<RT>(A.prog, A.set, sc, tile, cx, true, lds_x, ltab0, ltab1, acc, PT ? zz : nullptr);
  else if constexpr (LATE_TAB)
    tl.template run<RT, KIND>(A.prog, A.set, sc, tile, cx, lds_x, ltab0, ltab1, acc, PT ? zz : nullptr, mid_tab);
  else
    tl.template run<RT, KIND>(A.prog, A.set, sc, tile, cx, lds_x, ltab0, ltab1, acc, PT ? zz : nullptr);
  const uint32_t nt = gridDim.x;  // tiles of this launch (half of the set's with the half state)
  // only sweeps with an accumulating step write partial sums (the reduction reads no
  // others), and a specialised shape only the slots its steps can fill
  if (((A.prog.pre_ops | A.prog.mid_ops) & (OP_ENERGY | OP_GRADG)) || A.prog.mixA_grad || A.prog.mixB_grad) {
    scale_acc(acc, A.prog, sc);
    constexpr uint32_t SLOTS = sweep_slots(KIND);
    constexpr int NV = __builtin_popcount(SLOTS);
    const double all[6] = {acc.e, acc.nrm, acc.gpre, acc.gmid, acc.ba, acc.bb};
    double v[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0, k = 0; i < 6; ++i)
      if ((SLOTS >> i) & 1u) v[k++] = all[i];
    if constexpr (NV > 0) block_sum<NV, G::NT>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0, k = 0; i < 6; ++i)
        if ((SLOTS >> i) & 1u) A.partial[(size_t)i * nt + tile] = v[k++];
    }
  }
  if (PT) {
    __syncthreads();
    const double se = (A.prog.pre_ops & OP_ENERGY) ? sc.s_pre : sc.s_mid;
    for (int t = threadIdx.x; t < A.T; t += G::NT) A.partial[(size_t)(SLOT_TERMS + t) * nt + tile] = se * zz[t];
  }
}

// ---------------------------------------------------------------------------------
// Batched units: each workgroup takes the next unit from a counter and runs all of
// its sweeps.  Units with n <= L keep their state in registers; larger units sweep
// tile by tile over their own slice of the workspace.
template <class R> struct UnitArgs {
  const UnitDesc* units;
  const SweepProg* progs;
  const int32_t* order;      // unit indices in processing order
  unsigned char* ws;         // workspace base (graphs, terms, tables, states)
  const double* params;      // [rows][2p] (only used by the table kernel)
  double* out;               // [rows][2 + 2p]
  int32_t* counter;
  int count;
  int out_stride;
  int tabmax;                 // max cmax+1 over the units (dynamic LDS sizing)
  typename Cx<R>::V* psi_io;  // optional external state for single-unit calls (n <= L): final psi store
};

template <class R> __device__ __forceinline__ const SwScale* unit_scales(const unsigned char* ws, const UnitDesc* D) {
  const size_t amp = sizeof(typename Cx<R>::V);
  return reinterpret_cast<const SwScale*>(ws + D->tab_off + amp * (size_t)D->p * (D->cmax + 1));
}

template <class R, int NS, int LT> __global__ AAQ_TILE_BOUNDS void k_units(UnitArgs<R> A) {
  using G = Geo<R, LT>;
  using V = typename G::V;
  __shared__ V lds_x[lds_slot(G::TILE)];
  __shared__ double red[(G::NT / 64) * 6];
  __shared__ double outacc[2 + 2 * kMaxP];
  __shared__ int s_idx;
  extern __shared__ unsigned char dyn_lds[];  // two phase tables of up to A.tabmax entries
  V* ltab0 = reinterpret_cast<V*>(dyn_lds);
  V* ltab1 = ltab0 + A.tabmax;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(A.counter, 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    if (idx >= A.count) break;
    const int u = __builtin_amdgcn_readfirstlane(A.order[idx]);
    const UnitDesc* D = A.units + u;
    const int p = D->p;
    for (int i = threadIdx.x; i < 2 + 2 * p; i += G::NT) outacc[i] = 0.0;
    const GraphDev* g = reinterpret_cast<const GraphDev*>(A.ws + D->graph_off);
    const int4* terms = reinterpret_cast<const int4*>(A.ws + D->terms_off);
    const V* tab = reinterpret_cast<const V*>(A.ws + D->tab_off);
    const SwScale* scales = unit_scales<R>(A.ws, D);
    const bool big = D->state_off >= 0;
    V* psi = big ? reinterpret_cast<V*>(A.ws + D->state_off) : A.psi_io;
    V* lam = big && D->lam_off >= 0 ? reinterpret_cast<V*>(A.ws + D->lam_off) : nullptr;
    Ctx<R> cx{g, terms, tab, psi, lam, (R)exp2(-0.5 * (double)D->n), D->T, D->cmax};
    cx.cen = (R)(0.5 * D->cmax);
    Tile<R, NS, true, LT> tl;
    tl.lam_live = false;
    const int ns = D->nsweep;
    for (int si = 0; si < ns; ++si) {
      const SweepProg pg = A.progs[D->prog_off + si];
      const SetSpec& S = D->sets[pg.set];
      const SwScale& sc = scales[si];
      __syncthreads();  // previous sweep's table readers are done
      if (pg.pre_ops & (OP_PHASE | OP_UNPHASE))
        load_tab<R>(ltab0, tab, pg.pre_layer, D->cmax, (pg.pre_ops & OP_UNPHASE) != 0, sc.rho_pre);
      if (pg.mid_ops & (OP_PHASE | OP_UNPHASE))
        load_tab<R>(ltab1, tab, pg.mid_layer, D->cmax, (pg.mid_ops & OP_UNPHASE) != 0, sc.rho_mid);
      __syncthreads();
      Acc acc;
      acc.zero();
      const uint32_t nt = big ? S.ntiles : 1u;
      for (uint32_t t = 0; t < nt; ++t) tl.run_any(pg, S, sc, t, cx, big, lds_x, ltab0, ltab1, acc, nullptr);
      scale_acc(acc, pg, sc);
      double v[6] = {acc.e, acc.nrm, acc.gpre, acc.gmid, acc.ba, acc.bb};
      block_sum<6, G::NT>(v, red);
      if (threadIdx.x == 0) {
        if (pg.pre_ops & OP_ENERGY || pg.mid_ops & OP_ENERGY) {
          outacc[0] += v[0];
          outacc[1] += v[1];
        }
        if (NS == 2) {
          if (pg.pre_ops & OP_GRADG) outacc[2 + pg.pre_layer] += 2.0 * v[2];
          if (pg.mid_ops & OP_GRADG) outacc[2 + pg.mid_layer] += 2.0 * v[3];
          if (pg.mixA_grad) outacc[2 + p + pg.mixA_layer] += 2.0 * v[4];
          if (pg.mixB_grad) outacc[2 + p + pg.mixB_layer] += 2.0 * v[5];
        }
      }
    }
    __syncthreads();
    double* o = A.out + (size_t)D->row * A.out_stride;
    for (int i = threadIdx.x; i < 2 + 2 * p; i += G::NT) o[i] = outacc[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------
// Batched sweeps for plan units larger than one tile: one launch per sweep step over
// every tile of every unit of a group (units with the same program structure).  Block
// (x, y) runs tile x of unit list[y]; blocks past the unit's tile count exit.
template <class R> struct BatchArgs {
  const UnitDesc* units;
  const SweepProg* progs;
  const int32_t* list;  // unit indices of the group
  const int2* wgmap;    // (unit, tile) of each workgroup of a sweep step
  unsigned char* ws;
  int step;
  int tabmax;
};

template <class R, int NS, bool EN, int RT, int LT> __global__ AAQ_TILE_BOUNDS void k_bsweep(BatchArgs<R> A) {
  using G = Geo<R, LT>;
  using V = typename G::V;
  __shared__ V lds_x[lds_slot(G::TILE)];
  __shared__ double red[(G::NT / 64) * 6];
  extern __shared__ unsigned char dyn_lds[];
  const int2 wm = A.wgmap[blockIdx.x];
  const int u = __builtin_amdgcn_readfirstlane(wm.x);
  const UnitDesc* D = A.units + u;
  const uint32_t tile = (uint32_t)__builtin_amdgcn_readfirstlane(wm.y);
  if (tile >= (uint32_t)D->ntiles || A.step >= D->nsweep) return;
  V* ltab0 = reinterpret_cast<V*>(dyn_lds);
  V* ltab1 = ltab0 + A.tabmax;
  const int p = D->p;
  const GraphDev* g = reinterpret_cast<const GraphDev*>(A.ws + D->graph_off);
  const int4* terms = reinterpret_cast<const int4*>(A.ws + D->terms_off);
  const V* tab = reinterpret_cast<const V*>(A.ws + D->tab_off);
  const SwScale& sc = unit_scales<R>(A.ws, D)[A.step];
  const SweepProg pg = A.progs[D->prog_off + A.step];
  const SetSpec& S = D->sets[pg.set];
  if (pg.pre_ops & (OP_PHASE | OP_UNPHASE))
    load_tab<R>(ltab0, tab, pg.pre_layer, D->cmax, (pg.pre_ops & OP_UNPHASE) != 0, sc.rho_pre);
  if (pg.mid_ops & (OP_PHASE | OP_UNPHASE))
    load_tab<R>(ltab1, tab, pg.mid_layer, D->cmax, (pg.mid_ops & OP_UNPHASE) != 0, sc.rho_mid);
  __syncthreads();
  V* psi = reinterpret_cast<V*>(A.ws + D->state_off);
  V* lam = reinterpret_cast<V*>(A.ws + D->lam_off);
  Ctx<R> cx{g, terms, tab, psi, NS == 2 ? lam : nullptr, (R)exp2(-0.5 * (double)D->n), D->T, D->cmax};
  cx.N = (uint64_t)1 << (D->n - D->half);  // stored amplitudes: the stride between checkpoint buffers
  cx.cen = (R)(0.5 * D->cmax);
  Tile<R, NS, EN, LT> tl;
  Acc acc;
  acc.zero();
  tl.template run_rt<RT>(pg, S, sc, tile, cx, true, lds_x, ltab0, ltab1, acc, nullptr);
  scale_acc(acc, pg, sc);
  double v[6] = {acc.e, acc.nrm, acc.gpre, acc.gmid, acc.ba, acc.bb};
  block_sum<6, G::NT>(v, red);
  if (threadIdx.x == 0) {
    double* part = reinterpret_cast<double*>(A.ws + D->part_off) + (size_t)A.step * 6 * D->ntiles;
#pragma unroll
    for (int i = 0; i < 6; ++i) part[(size_t)i * D->ntiles + tile] = v[i];
  }
  (void)p;
}

// The same batched sweep step compiled for its sweep shape KIND (every unit of a group runs
// the same program, so the step's shape is uniform over the launch): the specialised tile
// engine of the single-instance sweeps, with 32-bit buffer offsets within each unit's
// state.  The unit's descriptor, set and program are read through the constant address
// space (uploaded by the host, never written by a kernel).
template <class R, int RT, int LT, uint32_t KIND>
__global__ AAQ_SWEEP_BOUNDS(((KIND & (SK_LAM_IN | SK_MAKE_LAM)) ? 2 : 1), RT, KIND) void k_bsweep_k(BatchArgs<R> A) {
  constexpr int NS = (KIND & (SK_LAM_IN | SK_MAKE_LAM)) ? 2 : 1;
  constexpr bool EN = ((sk_pre(KIND) | sk_mid(KIND)) & OP_ENERGY) != 0;
  using G = Geo<R, LT>;
  using V = typename G::V;
  __shared__ V lds_x[lds_slot(sweep_half_xchg(NS, RT, KIND) ? G::TILE / 2 : G::TILE)];
  __shared__ double red[(G::NT / 64) * 6];
  extern __shared__ unsigned char dyn_lds[];
  const int2 wm = cst(A.wgmap)[blockIdx.x];
  const int u = __builtin_amdgcn_readfirstlane(wm.x);
  const cptr<UnitDesc> D = cst(A.units + u);
  const uint32_t tile = (uint32_t)__builtin_amdgcn_readfirstlane(wm.y);
  if (tile >= (uint32_t)D->ntiles || A.step >= D->nsweep) return;
  V* ltab0 = reinterpret_cast<V*>(dyn_lds);
  V* ltab1 = ltab0 + A.tabmax;
  const GraphDev* g = reinterpret_cast<const GraphDev*>(A.ws + D->graph_off);
  const int4* terms = reinterpret_cast<const int4*>(A.ws + D->terms_off);
  const V* tab = reinterpret_cast<const V*>(A.ws + D->tab_off);
  const size_t amp = sizeof(V);
  const SwScale& sc = reinterpret_cast<const SwScale*>(A.ws + D->tab_off + amp * (size_t)D->p * (D->cmax + 1))[A.step];
  const SweepProg pg = cst(A.progs)[D->prog_off + A.step];
  const SetSpec S = D->sets[pg.set];
  // as in k_sweep: a shape with no phase before its first mixer loads its mid table once
  // its state loads are issued
  constexpr bool LATE_TAB = (sk_pre(KIND) & (OP_PHASE | OP_UNPHASE)) == 0;
  auto mid_tab = [&]() {
    if (pg.mid_ops & (OP_PHASE | OP_UNPHASE))
      load_tab<R>(ltab1, tab, pg.mid_layer, D->cmax, (pg.mid_ops & OP_UNPHASE) != 0, sc.rho_mid);
  };
  if constexpr (!LATE_TAB) {
    if (pg.pre_ops & (OP_PHASE | OP_UNPHASE))
      load_tab<R>(ltab0, tab, pg.pre_layer, D->cmax, (pg.pre_ops & OP_UNPHASE) != 0, sc.rho_pre);
    mid_tab();
    __syncthreads();
  }
  V* psi = reinterpret_cast<V*>(A.ws + D->state_off);
  const uint64_t N = (uint64_t)1 << (D->n - D->half);  // stored amplitudes per state
  Ctx<R> cx{g, terms, tab, psi, NS == 2 ? reinterpret_cast<V*>(A.ws + D->lam_off) : nullptr, (R)exp2(-0.5 * (double)D->n),
            D->T, D->cmax, N,
            N <= ((uint64_t)1 << 32) / sizeof(V), false, (R)(0.5 * D->cmax)};
  Tile<R, NS, EN, LT> tl;
  Acc acc;
  acc.zero();
  if constexpr (LATE_TAB)
    tl.template run<RT, KIND>(pg, S, sc, tile, cx, lds_x, ltab0, ltab1, acc, nullptr, mid_tab);
  else
    tl.template run<RT, KIND>(pg, S, sc, tile, cx, lds_x, ltab0, ltab1, acc, nullptr);
  scale_acc(acc, pg, sc);
  constexpr uint32_t SLOTS = sweep_slots(KIND);
  constexpr int NV = __builtin_popcount(SLOTS);
  double* part = reinterpret_cast<double*>(A.ws + D->part_off) + (size_t)A.step * 6 * D->ntiles;
  if constexpr (NV > 0) {
    const double all[6] = {acc.e, acc.nrm, acc.gpre, acc.gmid, acc.ba, acc.bb};
    double v[NV];
#pragma unroll
    for (int i = 0, k = 0; i < 6; ++i)
      if ((SLOTS >> i) & 1u) v[k++] = all[i];
    block_sum<NV, G::NT>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0, k = 0; i < 6; ++i) part[(size_t)i * D->ntiles + tile] = ((SLOTS >> i) & 1u) ? v[k++] : 0.0;
    }
  } else if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) part[(size_t)i * D->ntiles + tile] = 0.0;
  }
}

// per-unit fixed-order sums of the batched sweeps' partials into d_out rows

template <class R, int K, int LT>
__global__ __launch_bounds__(1 << (LT - kRegBits)) void k_cuts(const GraphDev* g, const int4* terms, int T, int use_terms, SetSpec S,
                                                   int32_t* __restrict__ out) {
  using G = Geo<R, LT>;
  constexpr int KK = (K == 0) ? G::LAST : G::P;
  const uint64_t tile_base = pdep64(blockIdx.x, S.fixmask);
  Tile<R, 1, true, LT> tl;
  const uint64_t zb = tl.template zbase<KK>(S, tile_base, 0ull);
  int v[G::NR];
  if (use_terms)
    tl.template hvals<KK>(S, zb, terms, v, cst(g)->n <= 32);
  else
    tl.template cuts<KK>(S, zb, tile_base, 0ull, g, v);
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int r = 0; r < G::NR; ++r) {
    const uint32_t j = tidx<G::b0(KK), G::RB>(t, r);
    if (j & S.dummy) continue;
    uint64_t z = tile_base;
    for (int b = 0; b < G::L; ++b)
      if ((j >> b) & 1u) z |= (uint64_t)1 << S.pos[b];
    out[z] = v[r];
  }
}

// ------------------------------------------------------------------------------------
// Launch templates, instantiated once per (R, LT) by AAQ_INSTANTIATE_* in their own
// translation units (see aaq_launch.h for the host-facing declarations).
// a sweep kernel specialized for shape KIND (states, energy and per-term steps follow from it)
template <class R, int RT, int LT, uint32_t KIND>
static void sweep_launch_kind(const SweepArgs<R>& A, dim3 grid, dim3 blk, size_t dyn, hipStream_t st) {
  constexpr int NS = (KIND & (SK_LAM_IN | SK_MAKE_LAM)) ? 2 : 1;
  constexpr bool EN = ((sk_pre(KIND) | sk_mid(KIND)) & OP_ENERGY) != 0;
  constexpr bool PT = ((sk_pre(KIND) | sk_mid(KIND)) & OP_PERTERM) != 0;
  launch((k_sweep<R, NS, PT, EN, RT, LT, KIND>), grid, blk, dyn, st, A);
}

// the specialised shape of a sweep (WB: SK_WEIGHTED for the weighted copies, which leave
// the per-term shape to the run-time path); false when none applies
template <class R, int RT, int LT, uint32_t WB>
static bool sweep_launch_shape(uint32_t kind, const SweepArgs<R>& A, dim3 grid, dim3 blk, size_t dyn, hipStream_t st) {
  switch (kind) {
    case SK_F_FIRST: sweep_launch_kind<R, RT, LT, SK_F_FIRST | WB>(A, grid, blk, dyn, st); return true;
    case SK_F_PLAIN: sweep_launch_kind<R, RT, LT, SK_F_PLAIN | WB>(A, grid, blk, dyn, st); return true;
    case SK_F_BOUNDARY: sweep_launch_kind<R, RT, LT, SK_F_BOUNDARY | WB>(A, grid, blk, dyn, st); return true;
    case SK_F_ENERGY: sweep_launch_kind<R, RT, LT, SK_F_ENERGY | WB>(A, grid, blk, dyn, st); return true;
    case SK_F_ENERGY_TERMS:
      if constexpr (WB != 0) return false;
      else sweep_launch_kind<R, RT, LT, SK_F_ENERGY_TERMS>(A, grid, blk, dyn, st);
      return true;
    case SK_TURNAROUND: sweep_launch_kind<R, RT, LT, SK_TURNAROUND | WB>(A, grid, blk, dyn, st); return true;
    case SK_B_PLAIN: sweep_launch_kind<R, RT, LT, SK_B_PLAIN | WB>(A, grid, blk, dyn, st); return true;
    case SK_B_BOUNDARY: sweep_launch_kind<R, RT, LT, SK_B_BOUNDARY | WB>(A, grid, blk, dyn, st); return true;
    case SK_B_LAST: sweep_launch_kind<R, RT, LT, SK_B_LAST | WB>(A, grid, blk, dyn, st); return true;
    case SK_B_PLAIN_PD: sweep_launch_kind<R, RT, LT, SK_B_PLAIN_PD | WB>(A, grid, blk, dyn, st); return true;
    // on the full route (set 0, which takes the turnaround and layer boundaries only with
    // two tile sets) the lambda-only last stop spills registers in some instantiations:
    // those sweeps keep psi's gates there
    case SK_TURNAROUND_PD:
      if constexpr (RT == ROUTE_FULL) sweep_launch_kind<R, RT, LT, SK_TURNAROUND | WB>(A, grid, blk, dyn, st);
      else sweep_launch_kind<R, RT, LT, SK_TURNAROUND_PD | WB>(A, grid, blk, dyn, st);
      return true;
    case SK_B_BOUNDARY_PD:
      if constexpr (RT == ROUTE_FULL) sweep_launch_kind<R, RT, LT, SK_B_BOUNDARY | WB>(A, grid, blk, dyn, st);
      else sweep_launch_kind<R, RT, LT, SK_B_BOUNDARY_PD | WB>(A, grid, blk, dyn, st);
      return true;
    default: return false;
  }
}

template <class R, int RT, int LT>
static void sweep_launch_rt(const SweepArgs<R>& A, const LaunchSweep& L, size_t dyn, hipStream_t st) {
  const bool pt = ((L.prog.pre_ops | L.prog.mid_ops) & OP_PERTERM) != 0;
  const bool en = ((L.prog.pre_ops | L.prog.mid_ops) & OP_ENERGY) != 0;
  const dim3 grid(L.set.ntiles >> (L.half ? 1 : 0)), blk(Geo<R, LT>::NT);
  if (!L.generic) {
    const uint32_t kind = sweep_kind(L.prog);
    if (L.weighted ? sweep_launch_shape<R, RT, LT, SK_WEIGHTED>(kind, A, grid, blk, dyn, st)
                   : sweep_launch_shape<R, RT, LT, 0u>(kind, A, grid, blk, dyn, st))
      return;
  }
  if (pt)
    launch((k_sweep<R, 1, true, true, RT, LT, SK_GENERIC>), grid, blk, dyn, st, A);
  else if (L.two_states && en)
    launch((k_sweep<R, 2, false, true, RT, LT, SK_GENERIC>), grid, blk, dyn, st, A);
  else if (L.two_states)
    launch((k_sweep<R, 2, false, false, RT, LT, SK_GENERIC>), grid, blk, dyn, st, A);
  else if (en)
    launch((k_sweep<R, 1, false, true, RT, LT, SK_GENERIC>), grid, blk, dyn, st, A);
  else
    launch((k_sweep<R, 1, false, false, RT, LT, SK_GENERIC>), grid, blk, dyn, st, A);
}

template <class R, int LT> hipError_t sweep_launch_impl(const LaunchSweep& L, hipStream_t st) {
  SweepArgs<R> A;
  A.psi = reinterpret_cast<typename Cx<R>::V*>(L.psi);
  A.lam = reinterpret_cast<typename Cx<R>::V*>(L.lam);
  A.g = L.g;
  A.terms = L.terms;
  A.tab = reinterpret_cast<const typename Cx<R>::V*>(L.tab);
  A.scale = L.scale;
  A.partial = L.partial;
  A.nslot = L.nslot;
  A.T = L.T;
  A.cmax = L.cmax;
  A.amp = (R)L.amp;
  A.N = L.N;
  A.set = L.set;
  A.prog = L.prog;
  A.nt = L.nt ? 1 : 0;
  const size_t dyn = 2 * sizeof(typename Cx<R>::V) * (size_t)(L.cmax + 1);
  if (L.set.route == ROUTE_HIGH)
    sweep_launch_rt<R, ROUTE_HIGH, LT>(A, L, dyn, st);
  else
    sweep_launch_rt<R, ROUTE_FULL, LT>(A, L, dyn, st);
  return hipGetLastError();
}

template <class R> UnitArgs<R> unit_args(const LaunchUnits& L) {
  UnitArgs<R> A;
  A.units = L.units;
  A.progs = L.progs;
  A.order = L.order;
  A.ws = L.ws;
  A.params = L.params;
  A.out = L.out;
  A.counter = L.counter;
  A.count = L.count;
  A.out_stride = L.out_stride;
  A.tabmax = L.tabmax;
  A.psi_io = reinterpret_cast<typename Cx<R>::V*>(L.psi_io);
  return A;
}

template <class R, int LT> hipError_t units_launch_impl(const LaunchUnits& L, bool grad, int blocks, hipStream_t st) {
  auto A = unit_args<R>(L);
  const size_t dyn = 2 * sizeof(typename Cx<R>::V) * (size_t)L.tabmax;
  if (grad)
    launch((k_units<R, 2, LT>), dim3(blocks), dim3(Geo<R, LT>::NT), dyn, st, A);
  else
    launch((k_units<R, 1, LT>), dim3(blocks), dim3(Geo<R, LT>::NT), dyn, st, A);
  return hipGetLastError();
}

template <class R, int NS, bool EN, int LT>
static void bsweep_launch_t(const BatchArgs<R>& A, int route, dim3 grid, size_t dyn, hipStream_t st) {
  if (route == ROUTE_HIGH)
    launch((k_bsweep<R, NS, EN, ROUTE_HIGH, LT>), grid, dim3(Geo<R, LT>::NT), dyn, st, A);
  else
    launch((k_bsweep<R, NS, EN, ROUTE_FULL, LT>), grid, dim3(Geo<R, LT>::NT), dyn, st, A);
}

template <class R, int RT, int LT>
static bool bsweep_launch_kind(const BatchArgs<R>& A, uint32_t kind, dim3 grid, size_t dyn, hipStream_t st) {
  const dim3 blk(Geo<R, LT>::NT);
  switch (kind) {
    case SK_F_FIRST: launch((k_bsweep_k<R, RT, LT, SK_F_FIRST>), grid, blk, dyn, st, A); return true;
    case SK_F_PLAIN: launch((k_bsweep_k<R, RT, LT, SK_F_PLAIN>), grid, blk, dyn, st, A); return true;
    case SK_F_BOUNDARY: launch((k_bsweep_k<R, RT, LT, SK_F_BOUNDARY>), grid, blk, dyn, st, A); return true;
    case SK_F_ENERGY: launch((k_bsweep_k<R, RT, LT, SK_F_ENERGY>), grid, blk, dyn, st, A); return true;
    case SK_TURNAROUND: launch((k_bsweep_k<R, RT, LT, SK_TURNAROUND>), grid, blk, dyn, st, A); return true;
    case SK_B_PLAIN: launch((k_bsweep_k<R, RT, LT, SK_B_PLAIN>), grid, blk, dyn, st, A); return true;
    case SK_B_BOUNDARY: launch((k_bsweep_k<R, RT, LT, SK_B_BOUNDARY>), grid, blk, dyn, st, A); return true;
    case SK_B_LAST: launch((k_bsweep_k<R, RT, LT, SK_B_LAST>), grid, blk, dyn, st, A); return true;
    // the lambda-only shapes of forward-state checkpoints, with the single-instance
    // sweeps' fallbacks on the full route
    case SK_TURNAROUND_PD:
      if constexpr (RT == ROUTE_FULL) launch((k_bsweep_k<R, RT, LT, SK_TURNAROUND>), grid, blk, dyn, st, A);
      else launch((k_bsweep_k<R, RT, LT, SK_TURNAROUND_PD>), grid, blk, dyn, st, A);
      return true;
    case SK_B_PLAIN_PD: launch((k_bsweep_k<R, RT, LT, SK_B_PLAIN_PD>), grid, blk, dyn, st, A); return true;
    case SK_B_BOUNDARY_PD:
      if constexpr (RT == ROUTE_FULL) launch((k_bsweep_k<R, RT, LT, SK_B_BOUNDARY>), grid, blk, dyn, st, A);
      else launch((k_bsweep_k<R, RT, LT, SK_B_BOUNDARY_PD>), grid, blk, dyn, st, A);
      return true;
    default: return false;
  }
}

template <class R, int LT> hipError_t bsweep_launch_impl(const LaunchBatch& L, hipStream_t st) {
  const dim3 grid(L.wg_count);
  BatchArgs<R> A{L.units, L.progs, L.list, L.wgmap, L.ws, L.step, L.tabmax};
  const size_t dyn = 2 * sizeof(typename Cx<R>::V) * (size_t)L.tabmax;
  if (L.kind != SK_GENERIC) {
    const bool done = L.route == ROUTE_HIGH ? bsweep_launch_kind<R, ROUTE_HIGH, LT>(A, L.kind, grid, dyn, st)
                                            : bsweep_launch_kind<R, ROUTE_FULL, LT>(A, L.kind, grid, dyn, st);
    if (done) return hipGetLastError();
  }
  if (L.two_states)
    (L.energy ? bsweep_launch_t<R, 2, true, LT> : bsweep_launch_t<R, 2, false, LT>)(A, L.route, grid, dyn, st);
  else
    (L.energy ? bsweep_launch_t<R, 1, true, LT> : bsweep_launch_t<R, 1, false, LT>)(A, L.route, grid, dyn, st);
  return hipGetLastError();
}

template <class R, int LT>
hipError_t cuts_launch_impl(const GraphDev* g, const int4* terms, int T, int use_terms, const SetSpec& S, int arr,
                            int32_t* out, hipStream_t st) {
  if (arr == 0)
    launch((k_cuts<R, 0, LT>), dim3(S.ntiles), dim3(Geo<R, LT>::NT), 0, st, g, terms, T, use_terms, S, out);
  else
    launch((k_cuts<R, 1, LT>), dim3(S.ntiles), dim3(Geo<R, LT>::NT), 0, st, g, terms, T, use_terms, S, out);
  return hipGetLastError();
}

}  // namespace aaq

#define AAQ_INSTANTIATE_UNITS(R, LT, SUF)                                                                   \
  namespace aaq {                                                                                           \
  hipError_t launch_units_##SUF(const LaunchUnits& L, bool grad, int blocks, hipStream_t st) {              \
    return units_launch_impl<R, LT>(L, grad, blocks, st);                                                   \
  }                                                                                                         \
  }
#define AAQ_INSTANTIATE_SWEEPS(R, LT, SUF)                                                                  \
  namespace aaq {                                                                                           \
  hipError_t launch_sweep_##SUF(const LaunchSweep& L, hipStream_t st) { return sweep_launch_impl<R, LT>(L, st); } \
  hipError_t launch_bsweep_##SUF(const LaunchBatch& L, hipStream_t st) { return bsweep_launch_impl<R, LT>(L, st); } \
  hipError_t launch_cuts_##SUF(const GraphDev* g, const int4* terms, int T, int use_terms, const SetSpec& S, int arr, \
                               int32_t* out, hipStream_t st) {                                              \
    return cuts_launch_impl<R, LT>(g, terms, T, use_terms, S, arr, out, st);                                \
  }                                                                                                         \
  }
