// HIP kernels (gfx950) for the p-layer MaxCut QAOA statevector estimator.
//
// One 512-thread workgroup owns a tile of 2^L = 8192 amplitudes in registers
// (16 per thread), for complex64 and complex128 alike.
// The tile's register bits are switched between "arrangements" through an LDS
// transpose so that every mixer butterfly is a register-to-register operation:
// arrangement k keeps tile bits [b0(k), b0(k)+RB) in registers and spreads the
// other tile bits over the threads.  The last arrangement (high tile bits in
// registers) is the one used for global loads and stores: consecutive lanes then
// touch consecutive amplitudes.
//
// A sweep = load (or synthesise |+>) -> ops at the load arrangement -> mixer A
// through the arrangements in ascending order -> ops at the "phase" arrangement ->
// mixer B in descending order -> store.  The ops are the cost phase
// exp(-i gamma C(z)) (QAOA section, U_P), its inverse, the energy / lambda step
// and the gradient accumulations of the adjoint method.  C(z) and h(z) are exact
// integers recomputed per amplitude from uint64 adjacency masks and the term list.
#include <hip/hip_runtime.h>

#include "aaq_internal.h"

namespace aaq {

template <class R> struct Cx;
template <> struct Cx<float> {
  using V = float2;
  static constexpr int L = 13, RB = 4;
};
template <> struct Cx<double> {
  using V = double2;
  static constexpr int L = 13, RB = 4;
};

template <class R> struct Geo {
  using V = typename Cx<R>::V;
  static constexpr int L = Cx<R>::L, RB = Cx<R>::RB, NR = 1 << RB;
  static constexpr int NA = (L + RB - 1) / RB;
  static constexpr int LAST = NA - 1, P = NA - 2;
  static constexpr int TILE = 1 << L;
  static constexpr int LB = L - RB;  // thread bits: 2^LB = 512 threads
  __host__ __device__ static constexpr int b0(int k) { return (k * RB < L - RB) ? k * RB : L - RB; }
};
static_assert((1 << Geo<float>::LB) == kThreads, "complex64 tile must map to 512 threads");
static_assert((1 << Geo<double>::LB) == kThreads, "complex128 tile must map to 512 threads");


template <class R> __device__ __forceinline__ typename Cx<R>::V mkv(R x, R y) {
  typename Cx<R>::V v;
  v.x = x;
  v.y = y;
  return v;
}

// tile index of register r of thread t in an arrangement whose register bits start at B0
template <int B0, int RB> __device__ __forceinline__ uint32_t tidx(uint32_t t, uint32_t r) {
  return (t & ((1u << B0) - 1u)) | (r << B0) | ((t >> B0) << (B0 + RB));
}
// LDS slot of tile index j: one padding slot per 16 entries.  P is additive over
// disjoint bit sets, P(a | b) = P(a) + P(b), so the slot of (thread part | register
// part) is a per-thread base plus a compile-time offset.
__host__ __device__ constexpr uint32_t lds_slot(uint32_t j) { return j + (j >> 4); }
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
};

// Per-thread accumulators for one sweep.
struct Acc {
  double e, nrm, gpre, gmid, ba, bb;
  __device__ void zero() { e = nrm = gpre = gmid = ba = bb = 0.0; }
};

// EN: the energy / lambda step is compiled in (only the last forward sweep needs it)
template <class R, int NS, bool EN = true> struct Tile {
  using G = Geo<R>;
  using V = typename G::V;
  static constexpr int NR = G::NR, RB = G::RB, L = G::L, LB = G::LB, NA = G::NA, LAST = G::LAST, P = G::P;

  V a[NS][NR];
  bool lam_live;

  // -------------------------------------------------------------- LDS transpose
  template <int KF, int KT> __device__ __forceinline__ void xchg1(V (&x)[NR], V* lds) {
    constexpr int BF = G::b0(KF), BT = G::b0(KT);
    const uint32_t t = threadIdx.x;
    V* wb = lds + lds_slot(tpart<BF, RB>(t));
#pragma unroll
    for (int r = 0; r < NR; ++r) wb[lds_slot((uint32_t)r << BF)] = x[r];
    __syncthreads();
    const V* rb = lds + lds_slot(tpart<BT, RB>(t));
#pragma unroll
    for (int r = 0; r < NR; ++r) x[r] = rb[lds_slot((uint32_t)r << BT)];
    __syncthreads();
  }
  template <int KF, int KT> __device__ __forceinline__ void xchg(V* lds) {
    xchg1<KF, KT>(a[0], lds);
    if (NS == 2 && lam_live) xchg1<KF, KT>(a[NS - 1], lds);
  }

  // -------------------------------------------------------------- mixer butterflies
  // (I - i k X_q) on every tile bit of `todo` held in registers by arrangement K:
  // (x, y) -> (x - i k y, y - i k x), two FMAs per amplitude.  With `grad`, the pair's
  // Im <lam|X_q|psi> is accumulated with weight wcur, which tracks the scale change of
  // the preceding gates of the same mixer (wcur *= w after every qubit).
  template <int K> __device__ __forceinline__ void mix_at(uint32_t& todo, R k, R w, R& wcur, bool grad, R& gsum) {
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

  // -------------------------------------------------------------- z of register 0
  // index z of register 0 at arrangement K, XOR the flip mask F: the register-0
  // amplitude is the one of basis state zbase ^ F (register bits set where F has them)
  template <int K> __device__ __forceinline__ uint64_t zbase(const SetSpec& S, uint64_t tile_base, uint64_t F) const {
    constexpr int B0 = G::b0(K);
    const uint32_t t = threadIdx.x;
    uint64_t z = tile_base;
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int tb = (i < B0) ? i : i + RB;
      const uint32_t p = S.pos[tb];
      if (p != kDummy) z |= (uint64_t)((t >> i) & 1u) << p;
    }
    return z ^ F;
  }

  // C(z) for every register amplitude at arrangement K.  With base b = zb and m the
  // register bits flipped relative to it: C(b ^ m) = C(b) + sum_{v in m} d_v
  //   + sum_{edges (v, w) inside m} 2 (2 [b_v != b_w] - 1),
  // d_v = deg v - 2 #{neighbours u with b_u != b_v}.
  template <int K> __device__ __forceinline__ void cuts(const SetSpec& S, uint64_t zb, const GraphDev* g, int (&cv)[NR]) const {
    constexpr int B0 = G::b0(K);
    const int n = g->n;
    int c0 = 0;
    for (int v = 0; v < n; ++v) {
      const uint64_t av = g->adj[v];
      c0 += (int)((zb >> v) & 1u) * __popcll(av & ~zb);
    }
    int d[RB];
    uint32_t rr[RB], df[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const uint32_t v = S.pos[B0 + b];
      d[b] = 0;
      rr[b] = 0;
      df[b] = 0;
      if (v != kDummy) {
        const uint64_t av = g->adj[v];
        const uint64_t bv = (zb >> v) & 1u;
        d[b] = g->deg[v] - 2 * __popcll(av & (zb ^ (0ull - bv)));
#pragma unroll
        for (int b2 = 0; b2 < RB; ++b2) {
          const uint32_t w = S.pos[B0 + b2];
          if (w != kDummy && ((av >> w) & 1u)) {
            rr[b] |= 1u << b2;
            if (((zb >> w) & 1u) != bv) df[b] |= 1u << b2;  // register bits of zb are uniform
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

  // h(z) = sum_t w_t [z_i != z_j] for every register amplitude at arrangement K
  template <int K> __device__ __forceinline__ void hvals(const SetSpec& S, uint64_t zb, const int4* terms, int T, int (&hv)[NR]) const {
    constexpr int B0 = G::b0(K);
    int h0 = 0;
    int dh[RB];
    int corr[NR];
#pragma unroll
    for (int b = 0; b < RB; ++b) dh[b] = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) corr[r] = 0;
    for (int t = 0; t < T; ++t) {
      const int4 tm = terms[t];
      int ri = -1, rj = -1;
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (S.pos[B0 + b] == (uint32_t)tm.x) ri = b;
        if (S.pos[B0 + b] == (uint32_t)tm.y) rj = b;
      }
      const int bi = (int)((zb >> tm.x) & 1u), bj = (int)((zb >> tm.y) & 1u);
      const int x = bi ^ bj;
      h0 += tm.z * x;
      // flipping one endpoint changes the term by w (1 - 2x); flipping both leaves it
      if (ri >= 0) {
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if (ri == b) dh[b] += tm.z * (1 - 2 * x);
      }
      if (rj >= 0) {
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if (rj == b) dh[b] += tm.z * (1 - 2 * x);
      }
      if (ri >= 0 && rj >= 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (((r >> ri) & 1) && ((r >> rj) & 1)) corr[r] -= 2 * tm.z * (1 - 2 * x);
      }
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
  template <int K>
  __device__ __forceinline__ void ops_at(uint8_t ops, bool make_lam, const SetSpec& S, uint64_t tile_base, uint64_t F,
                                         const Ctx<R>& cx, const V* ltab, double& gacc, Acc& acc, double* zz_lds) {
    if (!ops) return;
    const uint64_t zb = zbase<K>(S, tile_base, F);
    if (EN && (ops & OP_ENERGY)) {
      int hv[NR];
      if (cx.g->h_is_cut)
        cuts<K>(S, zb, cx.g, hv);
      else
        hvals<K>(S, zb, cx.terms, cx.T, hv);
      double e = 0.0, nr = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const R p2 = a[0][r].x * a[0][r].x + a[0][r].y * a[0][r].y;
        e += (double)p2 * (double)hv[r];
        nr += (double)p2;
      }
      acc.e += e;
      acc.nrm += nr;
      if (ops & OP_PERTERM) perterm<K>(S, zb, cx, zz_lds);
      if (NS == 2 && make_lam) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const R h = (R)hv[r];
          a[NS - 1][r] = mkv<R>(h * a[0][r].x, h * a[0][r].y);
        }
        lam_live = true;
      }
    }
    if (ops & (OP_GRADG | OP_PHASE | OP_UNPHASE)) {
      int cv[NR];
      cuts<K>(S, zb, cx.g, cv);
      if (NS == 2 && (ops & OP_GRADG)) {
        R gs = R(0);
#pragma unroll
        for (int r = 0; r < NR; ++r) gs += (R)cv[r] * imcm(a[NS - 1][r], a[0][r]);
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

  // <Z_i Z_j> partial sums per term, reduced per wave and added into LDS
  template <int K> __device__ __forceinline__ void perterm(const SetSpec& S, uint64_t zb, const Ctx<R>& cx, double* zz_lds) const {
    constexpr int B0 = G::b0(K);
    R p2[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) p2[r] = a[0][r].x * a[0][r].x + a[0][r].y * a[0][r].y;
    for (int t = 0; t < cx.T; ++t) {
      const int4 tm = cx.terms[t];
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
      if ((threadIdx.x & 63) == 0) atomicAdd(&zz_lds[t], v);
    }
  }

  // -------------------------------------------------------------- global I/O
  // Loads and stores happen at the load arrangement LAST: the top tile bits in
  // registers, tile bits 0..8 over the threads, so 32 lanes touch >= 32 consecutive
  // amplitudes (>= 256 bytes).  Dummy tile bits (whole state smaller than a tile) have no
  // global position: amplitudes with a dummy bit set are neither loaded (they are zero)
  // nor stored.
  template <int K> __device__ __forceinline__ uint64_t thread_off(const SetSpec& S) const {
    constexpr int B0 = G::b0(K);
    const uint32_t t = threadIdx.x;
    uint64_t toff = 0;
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int tb = (i < B0) ? i : i + RB;
      if (S.pos[tb] != kDummy) toff |= (uint64_t)((t >> i) & 1u) << S.pos[tb];
    }
    return toff;
  }
  // element offset of register r at the load arrangement (host-computed table)
  template <int K, int r> __device__ __forceinline__ static uint64_t reg_off(const SetSpec& S) {
    static_assert(K == LAST, "global I/O happens at the load arrangement");
    return S.roff[r];
  }
  template <int K> __device__ __forceinline__ bool is_dummy(const SetSpec& S, int r) const {
    return S.dummy && (tidx<G::b0(K), RB>(threadIdx.x, r) & S.dummy);
  }
  template <int K, int r = 0> __device__ __forceinline__ void load_all(int s, const V* p, const SetSpec& S) {
    if constexpr (r < NR) {
      a[s][r] = is_dummy<K>(S, r) ? mkv<R>(R(0), R(0)) : p[reg_off<K, r>(S)];
      load_all<K, r + 1>(s, p, S);
    }
  }
  template <int K, int r = 0> __device__ __forceinline__ void store_all(int s, V* p, const SetSpec& S) const {
    if constexpr (r < NR) {
      if (!is_dummy<K>(S, r)) p[reg_off<K, r>(S)] = a[s][r];
      store_all<K, r + 1>(s, p, S);
    }
  }
  template <int K> __device__ __forceinline__ void init_at(const SetSpec& S, R amp) {
#pragma unroll
    for (int r = 0; r < NR; ++r) a[0][r] = mkv<R>(is_dummy<K>(S, r) ? R(0) : amp, R(0));
  }

  // -------------------------------------------------------------- one sweep on one tile
  // Mixer routes (both start at the load arrangement 3): ROUTE_3012 for the set that
  // holds global bits 0..3 actively, ROUTE_312 for the others, whose active bits are all
  // tile bits >= 5.  Mixer A walks the route forward and ends at the phase arrangement 2,
  // mixer B walks it back to the load arrangement.
  template <int RT> __device__ __forceinline__ void mix_fwd(uint32_t& todo, R k, R w, R& wcur, bool gr, R& gs, V* lds) {
    mix_at<3>(todo, k, w, wcur, gr, gs);
    if constexpr (RT == ROUTE_3012) {
      xchg<3, 0>(lds);
      mix_at<0>(todo, k, w, wcur, gr, gs);
      xchg<0, 1>(lds);
    } else {
      xchg<3, 1>(lds);
    }
    mix_at<1>(todo, k, w, wcur, gr, gs);
    xchg<1, 2>(lds);
    mix_at<2>(todo, k, w, wcur, gr, gs);
  }
  template <int RT> __device__ __forceinline__ void mix_bwd(uint32_t& todo, R k, R w, R& wcur, bool gr, R& gs, V* lds) {
    mix_at<2>(todo, k, w, wcur, gr, gs);
    xchg<2, 1>(lds);
    mix_at<1>(todo, k, w, wcur, gr, gs);
    if constexpr (RT == ROUTE_3012) {
      xchg<1, 0>(lds);
      mix_at<0>(todo, k, w, wcur, gr, gs);
      xchg<0, 3>(lds);
    } else {
      xchg<1, 3>(lds);
    }
    mix_at<3>(todo, k, w, wcur, gr, gs);
  }

  // Executes program `pg` on the tile with id `tile` of set S (whose route is RT).
  // With `io` false the state stays in registers (whole state in one tile); stores still
  // happen when the program asks for them and a destination exists.
  template <int RT>
  __device__ __forceinline__ void run(const SweepProg& pg, const SetSpec& S, const SwScale& sc, uint64_t tile,
                                      const Ctx<R>& cx, bool io, V* lds_x, const V* ltab_pre, const V* ltab_mid, Acc& acc,
                                      double* zz_lds) {
    constexpr int KL = LAST;
    const uint64_t tile_base = pdep64(tile, S.fixmask);
    if (pg.flags & F_INIT) {
      init_at<KL>(S, cx.amp);
      lam_live = false;
    } else if (io) {
      if (pg.flags & F_LOAD_PSI) load_all<KL>(0, cx.psi + tile_base + thread_off<KL>(S), S);
      lam_live = (pg.flags & F_LAM_LIVE) != 0;
      if (NS == 2 && (pg.flags & F_LOAD_LAM)) {
        load_all<KL>(NS - 1, cx.lam + tile_base + thread_off<KL>(S), S);
        if (sc.fix_lam) {
          const R fr = (R)sc.lam_fix[0], fi = (R)sc.lam_fix[1];
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const V x = a[NS - 1][r];
            a[NS - 1][r] = mkv<R>(x.x * fr - x.y * fi, x.x * fi + x.y * fr);
          }
        }
      }
    }
    const bool make_lam = (pg.flags & F_MAKE_LAM) != 0;
    ops_at<KL>(pg.pre_ops, make_lam, S, tile_base, sc.F_pre, cx, ltab_pre, acc.gpre, acc, zz_lds);
    bool at_p = false;
    if (pg.mixA_dir) {
      R wcur = R(1), gs = R(0);
      uint32_t todo = S.act;
      mix_fwd<RT>(todo, (R)sc.kA, (R)sc.wA, wcur, pg.mixA_grad != 0, gs, lds_x);
      acc.ba += (double)gs;
      at_p = true;
    }
    if ((pg.mid_ops || pg.mixB_dir) && !at_p) {
      xchg<KL, P>(lds_x);
      at_p = true;
    }
    ops_at<P>(pg.mid_ops, make_lam, S, tile_base, sc.F_mid, cx, ltab_mid, acc.gmid, acc, zz_lds);
    if (pg.mixB_dir) {
      R wcur = R(1), gs = R(0);
      uint32_t todo = S.act;
      mix_bwd<RT>(todo, (R)sc.kB, (R)sc.wB, wcur, pg.mixB_grad != 0, gs, lds_x);
      acc.bb += (double)gs;
      at_p = false;
    }
    const bool st_psi = (pg.flags & F_STORE_PSI) && cx.psi;
    const bool st_lam = NS == 2 && (pg.flags & F_STORE_LAM) && cx.lam;
    if ((st_psi || st_lam) && at_p) xchg<P, KL>(lds_x);
    if (st_psi) store_all<KL>(0, cx.psi + tile_base + thread_off<KL>(S), S);
    if (st_lam) store_all<KL>(NS - 1, cx.lam + tile_base + thread_off<KL>(S), S);
  }
  __device__ __forceinline__ void run_any(const SweepProg& pg, const SetSpec& S, const SwScale& sc, uint64_t tile,
                                          const Ctx<R>& cx, bool io, V* lds_x, const V* ltab_pre, const V* ltab_mid,
                                          Acc& acc, double* zz_lds) {
    if (S.route == ROUTE_312)
      run<ROUTE_312>(pg, S, sc, tile, cx, io, lds_x, ltab_pre, ltab_mid, acc, zz_lds);
    else
      run<ROUTE_3012>(pg, S, sc, tile, cx, io, lds_x, ltab_pre, ltab_mid, acc, zz_lds);
  }
};

// ---------------------------------------------------------------------------------
// workgroup reduction of a few doubles; result valid in thread 0
template <int N> __device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
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
      for (int w = 0; w < kThreads / 64; ++w) s += red[w * N + i];
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
  const double rr = rho[0], ri = rho[1];
  for (int c = threadIdx.x; c <= cmax; c += kThreads) {
    const double tr = (double)src[c].x, ti = conj ? -(double)src[c].y : (double)src[c].y;
    ltab[c] = mkv<R>((R)(tr * rr - ti * ri), (R)(tr * ri + ti * rr));
  }
}

// apply a sweep's scale corrections to the per-thread sums
__device__ __forceinline__ void scale_acc(Acc& acc, const SweepProg& pg, const SwScale& sc) {
  const double se = (pg.pre_ops & OP_ENERGY) ? sc.s_pre : sc.s_mid;
  acc.e *= se;
  acc.nrm *= se;
  acc.gpre *= sc.s_pre;
  acc.gmid *= sc.s_mid;
  acc.ba *= sc.s_A;
  acc.bb *= sc.s_B;
}

// Walk a unit's sweep programs and record, per sweep, the butterfly coefficients and
// the scale corrections (see SwScale).  out[nsweep].s_pre is 1/|sigma|^2 at the end.
__device__ void build_scales(const SweepProg* progs, int nsweep, const SetSpec* sets, const double* beta, SwScale* out) {
  double sr = 1.0, si = 0.0;  // sigma
  auto position = [&](uint8_t ops, double* rho, double& sx) {
    const double a2 = sr * sr + si * si;
    sx = 1.0 / a2;
    rho[0] = 1.0;
    rho[1] = 0.0;
    if (ops & (OP_PHASE | OP_UNPHASE)) {
      rho[0] = sr / a2;
      rho[1] = -si / a2;
      sr = 1.0;
      si = 0.0;
    }
  };
  uint64_t F = 0, mF = 0;  // flip mask in registers / of the buffers in memory
  auto mixer = [&](int layer, int dir, uint32_t act, uint64_t gact, double& k, double& w, double& sx) {
    k = 0.0;
    w = 1.0;
    sx = 1.0 / (sr * sr + si * si);
    if (!dir) return;
    double sn, cs;
    sincos(beta[layer], &sn, &cs);
    double pr, pi;  // phi
    if (fabs(cs) >= fabs(sn)) {
      k = dir * sn / cs;
      pr = cs;
      pi = 0.0;
    } else {
      k = -dir * cs / sn;
      pr = 0.0;
      pi = -dir * sn;
      F ^= gact;
    }
    w = pr * pr + pi * pi;
    // sigma /= phi^m
    double qr = 1.0, qi = 0.0;
    for (int i = __popc(act); i > 0; --i) {
      const double tr = qr * pr - qi * pi;
      qi = qr * pi + qi * pr;
      qr = tr;
    }
    const double q2 = qr * qr + qi * qi;
    const double nr = (sr * qr + si * qi) / q2, ni = (si * qr - sr * qi) / q2;
    sr = nr;
    si = ni;
  };
  // scales of the buffers in memory: psi and lambda differ after a sweep that stores
  // only lambda (the last forward sweep leaves psi untouched in memory)
  double mpr = 1.0, mpi = 0.0, mlr = 1.0, mli = 0.0;
  for (int i = 0; i < nsweep; ++i) {
    const SweepProg pg = progs[i];
    SwScale r;
    r.lam_fix[0] = 1.0;
    r.lam_fix[1] = 0.0;
    r.fix_lam = 0;
    r.pad = 0;
    if (pg.flags & F_INIT) {
      sr = 1.0;
      si = 0.0;
      F = 0;
    } else if (pg.flags & F_LOAD_PSI) {
      sr = mpr;
      si = mpi;
      F = mF;
    }
    if (pg.flags & F_LOAD_LAM) {  // lambda <- lambda * sigma_psi / sigma_lam
      const double d = mlr * mlr + mli * mli;
      const double fr = (sr * mlr + si * mli) / d, fi = (si * mlr - sr * mli) / d;
      r.lam_fix[0] = fr;
      r.lam_fix[1] = fi;
      r.fix_lam = (fr != 1.0 || fi != 0.0) ? 1u : 0u;
    }
    const uint32_t act = sets[pg.set].act;
    const uint64_t gact = sets[pg.set].gact;
    r.F_pre = F;
    position(pg.pre_ops, r.rho_pre, r.s_pre);
    mixer(pg.mixA_layer, pg.mixA_dir, act, gact, r.kA, r.wA, r.s_A);
    r.F_mid = F;
    position(pg.mid_ops, r.rho_mid, r.s_mid);
    mixer(pg.mixB_layer, pg.mixB_dir, act, gact, r.kB, r.wB, r.s_B);
    if (pg.flags & F_STORE_PSI) {
      mpr = sr;
      mpi = si;
      mF = F;
    }
    if (pg.flags & F_STORE_LAM) {
      mlr = sr;
      mli = si;
    }
    out[i] = r;
  }
  SwScale f;
  position(0, f.rho_pre, f.s_pre);
  f.rho_mid[0] = 1.0;
  f.rho_mid[1] = 0.0;
  f.s_mid = f.s_A = f.s_B = 1.0;
  f.kA = f.kB = 0.0;
  f.wA = f.wB = 1.0;
  f.F_pre = f.F_mid = F;
  f.lam_fix[0] = 1.0;
  f.lam_fix[1] = 0.0;
  f.fix_lam = f.pad = 0;
  out[nsweep] = f;
}

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
  SetSpec set;
  SweepProg prog;
};

#define AAQ_TILE_BOUNDS __launch_bounds__(kThreads)

// One workgroup per tile; partial sums per tile: partial[slot][tile].
template <class R, int NS, bool PT, bool EN, int RT> __global__ AAQ_TILE_BOUNDS void k_sweep(SweepArgs<R> A) {
  using G = Geo<R>;
  using V = typename G::V;
  __shared__ V lds_x[lds_slot(G::TILE)];
  __shared__ double red[(kThreads / 64) * 6];
  __shared__ double zz[PT ? kMaxT : 1];
  extern __shared__ unsigned char dyn_lds[];  // two phase tables of cmax+1 entries
  V* ltab0 = reinterpret_cast<V*>(dyn_lds);
  V* ltab1 = ltab0 + (A.cmax + 1);
  const SwScale& sc = *A.scale;
  if (A.prog.pre_ops & (OP_PHASE | OP_UNPHASE))
    load_tab<R>(ltab0, A.tab, A.prog.pre_layer, A.cmax, (A.prog.pre_ops & OP_UNPHASE) != 0, sc.rho_pre);
  if (A.prog.mid_ops & (OP_PHASE | OP_UNPHASE))
    load_tab<R>(ltab1, A.tab, A.prog.mid_layer, A.cmax, (A.prog.mid_ops & OP_UNPHASE) != 0, sc.rho_mid);
  if (PT)
    for (int t = threadIdx.x; t < A.T; t += kThreads) zz[t] = 0.0;
  __syncthreads();
  Ctx<R> cx{A.g, A.terms, A.tab, A.psi, A.lam, A.amp, A.T, A.cmax};
  Tile<R, NS, EN> tl;
  Acc acc;
  acc.zero();
  const uint32_t tile = blockIdx.x;
  tl.template run<RT>(A.prog, A.set, sc, tile, cx, true, lds_x, ltab0, ltab1, acc, PT ? zz : nullptr);
  scale_acc(acc, A.prog, sc);
  double v[6] = {acc.e, acc.nrm, acc.gpre, acc.gmid, acc.ba, acc.bb};
  block_sum<6>(v, red);
  const uint32_t nt = A.set.ntiles;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) A.partial[(size_t)i * nt + tile] = v[i];
  }
  if (PT) {
    __syncthreads();
    const double se = (A.prog.pre_ops & OP_ENERGY) ? sc.s_pre : sc.s_mid;
    for (int t = threadIdx.x; t < A.T; t += kThreads) A.partial[(size_t)(SLOT_TERMS + t) * nt + tile] = se * zz[t];
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

template <class R, int NS> __global__ AAQ_TILE_BOUNDS void k_units(UnitArgs<R> A) {
  using G = Geo<R>;
  using V = typename G::V;
  __shared__ V lds_x[lds_slot(G::TILE)];
  __shared__ double red[(kThreads / 64) * 6];
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
    for (int i = threadIdx.x; i < 2 + 2 * p; i += kThreads) outacc[i] = 0.0;
    const GraphDev* g = reinterpret_cast<const GraphDev*>(A.ws + D->graph_off);
    const int4* terms = reinterpret_cast<const int4*>(A.ws + D->terms_off);
    const V* tab = reinterpret_cast<const V*>(A.ws + D->tab_off);
    const SwScale* scales = unit_scales<R>(A.ws, D);
    const bool big = D->state_off >= 0;
    V* psi = big ? reinterpret_cast<V*>(A.ws + D->state_off) : A.psi_io;
    V* lam = big ? psi + ((size_t)1 << D->n) : nullptr;
    Ctx<R> cx{g, terms, tab, psi, lam, (R)exp2(-0.5 * (double)D->n), D->T, D->cmax};
    Tile<R, NS> tl;
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
      block_sum<6>(v, red);
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
    for (int i = threadIdx.x; i < 2 + 2 * p; i += kThreads) o[i] = outacc[i];
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
  unsigned char* ws;
  int step;
  int tabmax;
};

template <class R, int NS, bool EN, int RT> __global__ AAQ_TILE_BOUNDS void k_bsweep(BatchArgs<R> A) {
  using G = Geo<R>;
  using V = typename G::V;
  __shared__ V lds_x[lds_slot(G::TILE)];
  __shared__ double red[(kThreads / 64) * 6];
  extern __shared__ unsigned char dyn_lds[];
  const int u = A.list[blockIdx.y];
  const UnitDesc* D = A.units + u;
  const uint32_t tile = blockIdx.x;
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
  V* lam = psi + ((size_t)1 << D->n);
  Ctx<R> cx{g, terms, tab, psi, NS == 2 ? lam : nullptr, (R)exp2(-0.5 * (double)D->n), D->T, D->cmax};
  Tile<R, NS, EN> tl;
  Acc acc;
  acc.zero();
  tl.template run<RT>(pg, S, sc, tile, cx, true, lds_x, ltab0, ltab1, acc, nullptr);
  scale_acc(acc, pg, sc);
  double v[6] = {acc.e, acc.nrm, acc.gpre, acc.gmid, acc.ba, acc.bb};
  block_sum<6>(v, red);
  if (threadIdx.x == 0) {
    double* part = reinterpret_cast<double*>(A.ws + D->part_off) + (size_t)A.step * 6 * D->ntiles;
#pragma unroll
    for (int i = 0; i < 6; ++i) part[(size_t)i * D->ntiles + tile] = v[i];
  }
  (void)p;
}

// per-unit fixed-order sums of the batched sweeps' partials into d_out rows
template <class R> __global__ void k_bsweep_out(BatchArgs<R> A, double* out, int out_stride, int grad) {
  __shared__ double red[4];
  const int u = A.list[blockIdx.x];
  const UnitDesc* D = A.units + u;
  const int p = D->p, nt = D->ntiles;
  double* o = out + (size_t)D->row * out_stride;
  const double* part = reinterpret_cast<const double*>(A.ws + D->part_off);
  auto slot_sum = [&](int s, int slot) -> double {
    double v = 0.0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) v += part[((size_t)s * 6 + slot) * nt + t];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return r;
  };
  for (int oi = 0; oi < 2 + 2 * p; ++oi) {
    double tot = 0.0;
    for (int s = 0; s < D->nsweep; ++s) {
      const SweepProg pg = A.progs[D->prog_off + s];
      if (oi < 2) {
        if ((pg.pre_ops | pg.mid_ops) & OP_ENERGY) tot += slot_sum(s, oi);
      } else if (grad && oi < 2 + p) {
        const int l = oi - 2;
        if ((pg.pre_ops & OP_GRADG) && pg.pre_layer == l) tot += 2.0 * slot_sum(s, SLOT_GPRE);
        if ((pg.mid_ops & OP_GRADG) && pg.mid_layer == l) tot += 2.0 * slot_sum(s, SLOT_GMID);
      } else if (grad) {
        const int l = oi - 2 - p;
        if (pg.mixA_grad && pg.mixA_layer == l) tot += 2.0 * slot_sum(s, SLOT_BA);
        if (pg.mixB_grad && pg.mixB_layer == l) tot += 2.0 * slot_sum(s, SLOT_BB);
      }
    }
    if (threadIdx.x == 0) o[oi] = tot;
  }
}

// ---------------------------------------------------------------------------------
// Phase tables exp(-i gamma_l c), c = 0..cmax (gamma_l * c formed and reduced in FP64,
// rounded to R), then the sweep scale records.
template <class R>
__global__ void k_tables(const double* __restrict__ gamma, const double* __restrict__ beta, int p, int cmax,
                         typename Cx<R>::V* __restrict__ tab, const SweepProg* progs, int nsweep, const SetSpec* sets,
                         SwScale* scales) {
  const int tot = p * (cmax + 1);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
    const int l = i / (cmax + 1), c = i % (cmax + 1);
    double sn, cs;
    sincos(gamma[l] * (double)c, &sn, &cs);
    tab[i] = mkv<R>((R)cs, (R)(-sn));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) build_scales(progs, nsweep, sets, beta, scales);
}

// per-unit tables for a plan; block b handles unit b; also resets the work counter
template <class R> __global__ void k_plan_tables(UnitArgs<R> A, int p, int pstride) {
  using V = typename Cx<R>::V;
  if (blockIdx.x == 0 && threadIdx.x == 0) *A.counter = 0;
  const UnitDesc* D = A.units + blockIdx.x;
  const double* prm = A.params + (size_t)D->row * pstride;
  V* tab = reinterpret_cast<V*>(A.ws + D->tab_off);
  const int cm = D->cmax;
  for (int i = threadIdx.x; i < p * (cm + 1); i += blockDim.x) {
    const int l = i / (cm + 1), c = i % (cm + 1);
    double sn, cs;
    sincos(prm[l] * (double)c, &sn, &cs);
    tab[i] = mkv<R>((R)cs, (R)(-sn));
  }
  if (threadIdx.x == 0)
    build_scales(A.progs + D->prog_off, D->nsweep, D->sets, prm + p, const_cast<SwScale*>(unit_scales<R>(A.ws, D)));
}

// fixed-order sums of per-tile partials: out[o] = scale_o * sum_{sources of o} sum_tiles
struct RedSrc {
  int64_t off;   // element offset into the partial buffer
  int32_t count;
  int32_t out;   // output index
  double scale;
};
__global__ void k_reduce(const double* __restrict__ partial, const RedSrc* __restrict__ src, const int32_t* __restrict__ src_begin,
                         double* __restrict__ out) {
  __shared__ double red[kThreads / 64];
  const int o = blockIdx.x;
  double tot = 0.0;
  for (int k = src_begin[o]; k < src_begin[o + 1]; ++k) {
    const RedSrc s = src[k];
    double v = 0.0;
    for (int i = threadIdx.x; i < s.count; i += blockDim.x) v += partial[s.off + i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += red[w];
      tot += s.scale * t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[o] = tot;
}

// one <Z_i Z_j> pass over the final state (per-term estimator structure)
template <class R>
__global__ __launch_bounds__(256) void k_zz_pass(const typename Cx<R>::V* __restrict__ psi, uint64_t N, int i, int j,
                                                 const double* __restrict__ scale, const uint64_t* __restrict__ flips,
                                                 double* __restrict__ partial) {
  // the buffer holds amplitude z ^ F at index z: the sign of the term flips with F_i ^ F_j
  __shared__ double red[4];
  const double sign = (((*flips >> i) ^ (*flips >> j)) & 1u) ? -1.0 : 1.0;
  double acc = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < N; z += stride) {
    const typename Cx<R>::V a = psi[z];
    const double p2 = (double)(a.x * a.x + a.y * a.y);
    acc += (((z >> i) ^ (z >> j)) & 1u) ? -p2 : p2;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sign * *scale * (red[0] + red[1] + red[2] + red[3]);
}

// exact integer diagonal values through the same per-amplitude code as the kernels,
// computed at arrangement K (0: load arrangement, 1: phase arrangement) of set S
template <class R, int K>
__global__ __launch_bounds__(kThreads) void k_cuts(const GraphDev* g, const int4* terms, int T, int use_terms, SetSpec S,
                                                   int32_t* __restrict__ out) {
  using G = Geo<R>;
  constexpr int KK = (K == 0) ? G::LAST : G::P;
  const uint64_t tile_base = pdep64(blockIdx.x, S.fixmask);
  Tile<R, 1> tl;
  const uint64_t zb = tl.template zbase<KK>(S, tile_base, 0ull);
  int v[G::NR];
  if (use_terms)
    tl.template hvals<KK>(S, zb, terms, T, v);
  else
    tl.template cuts<KK>(S, zb, g, v);
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

}  // namespace aaq

// ------------------------------------------------------------------------------------
// launch wrappers used by the host code
#include "aaq_launch.h"

namespace aaq {

template <class R, int RT> static void sweep_launch_rt(const SweepArgs<R>& A, const LaunchSweep& L, size_t dyn,
                                                    hipStream_t st) {
  const bool pt = ((L.prog.pre_ops | L.prog.mid_ops) & OP_PERTERM) != 0;
  const bool en = ((L.prog.pre_ops | L.prog.mid_ops) & OP_ENERGY) != 0;
  const dim3 grid(L.set.ntiles), blk(kThreads);
  if (pt)
    hipLaunchKernelGGL((k_sweep<R, 1, true, true, RT>), grid, blk, dyn, st, A);
  else if (L.two_states && en)
    hipLaunchKernelGGL((k_sweep<R, 2, false, true, RT>), grid, blk, dyn, st, A);
  else if (L.two_states)
    hipLaunchKernelGGL((k_sweep<R, 2, false, false, RT>), grid, blk, dyn, st, A);
  else if (en)
    hipLaunchKernelGGL((k_sweep<R, 1, false, true, RT>), grid, blk, dyn, st, A);
  else
    hipLaunchKernelGGL((k_sweep<R, 1, false, false, RT>), grid, blk, dyn, st, A);
}

template <class R> static hipError_t sweep_launch(const LaunchSweep& L, hipStream_t st) {
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
  A.set = L.set;
  A.prog = L.prog;
  const size_t dyn = 2 * sizeof(typename Cx<R>::V) * (size_t)(L.cmax + 1);
  if (L.set.route == ROUTE_312)
    sweep_launch_rt<R, ROUTE_312>(A, L, dyn, st);
  else
    sweep_launch_rt<R, ROUTE_3012>(A, L, dyn, st);
  return hipGetLastError();
}

hipError_t launch_sweep(const LaunchSweep& L, bool dbl, hipStream_t st) {
  return dbl ? sweep_launch<double>(L, st) : sweep_launch<float>(L, st);
}

hipError_t launch_tables(const double* gamma, const double* beta, int p, int cmax, void* tab, const SweepProg* progs,
                         int nsweep, const SetSpec* sets, SwScale* scales, bool dbl, hipStream_t st) {
  const int tot = p * (cmax + 1);
  const int blocks = (tot + 255) / 256;
  if (dbl)
    hipLaunchKernelGGL(k_tables<double>, dim3(blocks), dim3(256), 0, st, gamma, beta, p, cmax,
                       reinterpret_cast<double2*>(tab), progs, nsweep, sets, scales);
  else
    hipLaunchKernelGGL(k_tables<float>, dim3(blocks), dim3(256), 0, st, gamma, beta, p, cmax,
                       reinterpret_cast<float2*>(tab), progs, nsweep, sets, scales);
  return hipGetLastError();
}

template <class R> static UnitArgs<R> unit_args(const LaunchUnits& L) {
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

hipError_t launch_plan_tables(const LaunchUnits& L, int p, bool dbl, hipStream_t st) {
  if (dbl)
    hipLaunchKernelGGL(k_plan_tables<double>, dim3(L.count), dim3(256), 0, st, unit_args<double>(L), p, 2 * p);
  else
    hipLaunchKernelGGL(k_plan_tables<float>, dim3(L.count), dim3(256), 0, st, unit_args<float>(L), p, 2 * p);
  return hipGetLastError();
}

hipError_t launch_units(const LaunchUnits& L, bool grad, bool dbl, int blocks, hipStream_t st) {
  if (dbl) {
    auto A = unit_args<double>(L);
    const size_t dyn = 2 * sizeof(double2) * (size_t)L.tabmax;
    if (grad)
      hipLaunchKernelGGL((k_units<double, 2>), dim3(blocks), dim3(kThreads), dyn, st, A);
    else
      hipLaunchKernelGGL((k_units<double, 1>), dim3(blocks), dim3(kThreads), dyn, st, A);
  } else {
    auto A = unit_args<float>(L);
    const size_t dyn = 2 * sizeof(float2) * (size_t)L.tabmax;
    if (grad)
      hipLaunchKernelGGL((k_units<float, 2>), dim3(blocks), dim3(kThreads), dyn, st, A);
    else
      hipLaunchKernelGGL((k_units<float, 1>), dim3(blocks), dim3(kThreads), dyn, st, A);
  }
  return hipGetLastError();
}

template <class R, int NS, bool EN>
static void bsweep_launch_t(const BatchArgs<R>& A, int route, dim3 grid, size_t dyn, hipStream_t st) {
  if (route == ROUTE_312)
    hipLaunchKernelGGL((k_bsweep<R, NS, EN, ROUTE_312>), grid, dim3(kThreads), dyn, st, A);
  else
    hipLaunchKernelGGL((k_bsweep<R, NS, EN, ROUTE_3012>), grid, dim3(kThreads), dyn, st, A);
}

hipError_t launch_bsweep(const LaunchBatch& L, bool dbl, hipStream_t st) {
  const dim3 grid(L.max_tiles, L.nlist);
  if (dbl) {
    BatchArgs<double> A{L.units, L.progs, L.list, L.ws, L.step, L.tabmax};
    const size_t dyn = 2 * sizeof(double2) * (size_t)L.tabmax;
    if (L.two_states)
      (L.energy ? bsweep_launch_t<double, 2, true> : bsweep_launch_t<double, 2, false>)(A, L.route, grid, dyn, st);
    else
      (L.energy ? bsweep_launch_t<double, 1, true> : bsweep_launch_t<double, 1, false>)(A, L.route, grid, dyn, st);
  } else {
    BatchArgs<float> A{L.units, L.progs, L.list, L.ws, L.step, L.tabmax};
    const size_t dyn = 2 * sizeof(float2) * (size_t)L.tabmax;
    if (L.two_states)
      (L.energy ? bsweep_launch_t<float, 2, true> : bsweep_launch_t<float, 2, false>)(A, L.route, grid, dyn, st);
    else
      (L.energy ? bsweep_launch_t<float, 1, true> : bsweep_launch_t<float, 1, false>)(A, L.route, grid, dyn, st);
  }
  return hipGetLastError();
}

hipError_t launch_bsweep_out(const LaunchBatch& L, double* out, int out_stride, bool grad, bool dbl, hipStream_t st) {
  if (dbl) {
    BatchArgs<double> A{L.units, L.progs, L.list, L.ws, 0, L.tabmax};
    hipLaunchKernelGGL(k_bsweep_out<double>, dim3(L.nlist), dim3(256), 0, st, A, out, out_stride, (int)grad);
  } else {
    BatchArgs<float> A{L.units, L.progs, L.list, L.ws, 0, L.tabmax};
    hipLaunchKernelGGL(k_bsweep_out<float>, dim3(L.nlist), dim3(256), 0, st, A, out, out_stride, (int)grad);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, const void* src, const int32_t* src_begin, double* out, int nout,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(nout), dim3(256), 0, st, partial, reinterpret_cast<const RedSrc*>(src), src_begin, out);
  return hipGetLastError();
}

hipError_t launch_zz_pass(const void* psi, uint64_t N, int i, int j, const double* scale, const uint64_t* flips,
                          double* partial, int blocks, bool dbl, hipStream_t st) {
  if (dbl)
    hipLaunchKernelGGL(k_zz_pass<double>, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const double2*>(psi), N, i, j,
                       scale, flips, partial);
  else
    hipLaunchKernelGGL(k_zz_pass<float>, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float2*>(psi), N, i, j,
                       scale, flips, partial);
  return hipGetLastError();
}

hipError_t launch_cuts(const GraphDev* g, const int4* terms, int T, int use_terms, const SetSpec& S, int arr, int32_t* out,
                       bool dbl, hipStream_t st) {
  if (dbl) {
    if (arr == 0)
      hipLaunchKernelGGL((k_cuts<double, 0>), dim3(S.ntiles), dim3(kThreads), 0, st, g, terms, T, use_terms, S, out);
    else
      hipLaunchKernelGGL((k_cuts<double, 1>), dim3(S.ntiles), dim3(kThreads), 0, st, g, terms, T, use_terms, S, out);
  } else {
    if (arr == 0)
      hipLaunchKernelGGL((k_cuts<float, 0>), dim3(S.ntiles), dim3(kThreads), 0, st, g, terms, T, use_terms, S, out);
    else
      hipLaunchKernelGGL((k_cuts<float, 1>), dim3(S.ntiles), dim3(kThreads), 0, st, g, terms, T, use_terms, S, out);
  }
  return hipGetLastError();
}

int tile_bits(bool dbl) { return dbl ? Geo<double>::L : Geo<float>::L; }

}  // namespace aaq
