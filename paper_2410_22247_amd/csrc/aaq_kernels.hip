// Common kernels of the estimator (gfx950): phase tables and sweep scale records,
// fixed-order reductions, the pass-per-term <Z_i Z_j> kernel, and the host-facing
// launch functions that dispatch to the per-(precision, tile size) instantiations.
#include "aaq_engine.h"

namespace aaq {

// A unit's sweep programs, set masks and sin/cos(beta) staged in LDS by the whole
// workgroup, so the sequential walk below reads no global memory.
constexpr int kMaxSweeps = 2 * (kMaxP * (kMaxSets - 1) + 1);
struct ScaleStage {
  SweepProg progs[kMaxSweeps];
  uint64_t gact[kMaxSets];
  uint32_t act[kMaxSets];
  double sb[kMaxP], cb[kMaxP];
  // scale and flips each stored psi buffer was written with (indexed by buffer: kept in
  // LDS, so the walk makes no private-memory round trips)
  double mpr[kMaxCkpt], mpi[kMaxCkpt];
  uint64_t mF[kMaxCkpt];
  // per sweep and mixer (2 i + 0: mixer A, 2 i + 1: mixer B), computed by the whole
  // workgroup before the walk: k, w = |phi|^2, the flip flag and u = 1 / phi^m (the
  // factor the walk multiplies sigma by), so the sequential walk does no division or
  // power for a mixer
  struct Mix {
    double k, w, ur, ui;
    uint32_t flip, pad;
  } mix[kMaxSweeps * 2];
};

// the mixer quantities of sweep i's mixer X (0 = A, 1 = B) for a set with m mixed qubits:
// e^{-i beta X} = phi (I - i k X) per qubit, with phi = cos(beta) and k = tan(beta) when
// |cos| >= |sin|, else phi = -i dir sin(beta), k = -dir cot(beta) and a flip of the qubit
__device__ void mixer_factors(ScaleStage& S, int i, int X) {
  const SweepProg& pg = S.progs[i];
  const int layer = X ? pg.mixB_layer : pg.mixA_layer;
  const int dir = X ? pg.mixB_dir : pg.mixA_dir;
  ScaleStage::Mix& o = S.mix[2 * i + X];
  o.k = 0.0;
  o.w = 1.0;
  o.ur = 1.0;
  o.ui = 0.0;
  o.flip = 0;
  o.pad = 0;
  if (!dir) return;
  const double sn = S.sb[layer], cs = S.cb[layer];
  double pr, pi;  // phi
  if (fabs(cs) >= fabs(sn)) {
    o.k = dir * sn / cs;
    pr = cs;
    pi = 0.0;
  } else {
    o.k = -dir * cs / sn;
    pr = 0.0;
    pi = -dir * sn;
    o.flip = 1;
  }
  o.w = pr * pr + pi * pi;
  double qr = 1.0, qi = 0.0;  // phi^m
  for (int j = __popc(S.act[pg.set]); j > 0; --j) {
    const double tr = qr * pr - qi * pi;
    qi = qr * pi + qi * pr;
    qr = tr;
  }
  const double q2 = qr * qr + qi * qi;
  o.ur = qr / q2;  // 1 / q = conj(q) / |q|^2
  o.ui = -qi / q2;
}

// Walk a unit's sweep programs and record, per sweep, the butterfly coefficients and
// the scale corrections (see SwScale).  out[nsweep].s_pre is 1/|sigma|^2 at the end.
__device__ void build_scales(ScaleStage& S, int nsweep, SwScale* out) {
  const SweepProg* progs = S.progs;
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
  uint64_t F = 0;  // flip mask in registers
  auto mixer = [&](const ScaleStage::Mix& m, int dir, uint64_t gact, double& k, double& w, double& sx) {
    k = m.k;
    w = m.w;
    sx = 1.0 / (sr * sr + si * si);
    if (!dir) return;
    if (m.flip) F ^= gact;
    // sigma /= phi^m, as sigma * u
    const double nr = sr * m.ur - si * m.ui, ni = sr * m.ui + si * m.ur;
    sr = nr;
    si = ni;
  };
  // scales of the buffers in memory: psi and lambda differ after a sweep that stores
  // only lambda (the last forward sweep leaves psi untouched in memory); with
  // checkpoints every psi buffer keeps the scale and flips it was stored with
  double* mpr = S.mpr;
  double* mpi = S.mpi;
  uint64_t* mF = S.mF;
  double mlr = 1.0, mli = 0.0;
  for (int b = 0; b < kMaxCkpt; ++b) {
    mpr[b] = 1.0;
    mpi[b] = 0.0;
    mF[b] = 0;
  }
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
      sr = mpr[pg.ld_buf];
      si = mpi[pg.ld_buf];
      F = mF[pg.ld_buf];
    }
    // lambda's scale relative to psi's: rho = sigma_psi / sigma_lam.  Both states take the
    // same gates, and a mixer and its inverse have factors whose product is real and
    // positive (cos^2 or sin^2 of beta), so rho is real and positive; it only drifts in
    // magnitude.  While it stays within 2^+-24 lambda is left as loaded and rho is folded
    // into the sweep's gradient scale factors (its sums carry conj(sigma_lam) sigma_psi =
    // |sigma_psi|^2 / rho; such sweeps have no energy step); otherwise (or if rho were not
    // real) lambda is multiplied by rho on load.
    double gs = 1.0;
    if (pg.flags & F_LOAD_LAM) {
      const double d = mlr * mlr + mli * mli;
      const double fr = (sr * mlr + si * mli) / d, fi = (si * mlr - sr * mli) / d;
      const bool real = fabs(fi) <= 1e-12 * fabs(fr);
      if (real && fr > 0x1p-24 && fr < 0x1p24 && !((pg.pre_ops | pg.mid_ops) & OP_ENERGY)) {
        gs = fr;
      } else {
        r.lam_fix[0] = fr;
        r.lam_fix[1] = fi;
        r.fix_lam = 1u;
      }
    }
    const uint64_t gact = S.gact[pg.set];
    r.F_pre = F;
    position(pg.pre_ops, r.rho_pre, r.s_pre);
    mixer(S.mix[2 * i], pg.mixA_dir, gact, r.kA, r.wA, r.s_A);
    r.F_mid = F;
    position(pg.mid_ops, r.rho_mid, r.s_mid);
    mixer(S.mix[2 * i + 1], pg.mixB_dir, gact, r.kB, r.wB, r.s_B);
    if (gs != 1.0) {  // lambda loaded with scale sigma_psi / gs (no energy step here)
      r.s_pre *= gs;
      r.s_mid *= gs;
      r.s_A *= gs;
      r.s_B *= gs;
    }
    if (pg.flags & F_STORE_PSI) {
      mpr[pg.st_buf] = sr;
      mpi[pg.st_buf] = si;
      mF[pg.st_buf] = F;
    }
    if (pg.flags & F_STORE_LAM) {
      mlr = sr / gs;
      mli = si / gs;
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

// whole-workgroup entry: stage, then thread 0 walks the sweeps
__device__ void stage_and_build_scales(ScaleStage& S, const SweepProg* progs, int nsweep, const SetSpec* sets, int nsets,
                                       const double* beta, int p, SwScale* out) {
  for (int i = threadIdx.x; i < nsweep; i += blockDim.x) S.progs[i] = progs[i];
  for (int s = threadIdx.x; s < nsets; s += blockDim.x) {
    S.act[s] = sets[s].act;
    S.gact[s] = sets[s].gact;
  }
  for (int l = threadIdx.x; l < p; l += blockDim.x) sincos(beta[l], &S.sb[l], &S.cb[l]);
  __syncthreads();
  for (int t = threadIdx.x; t < 2 * nsweep; t += blockDim.x) mixer_factors(S, t >> 1, t & 1);
  __syncthreads();
  if (threadIdx.x == 0) build_scales(S, nsweep, out);
}


// Each wave sums one (sweep, slot) partial of the unit over its tiles (lanes stride the
// tiles, then a fixed butterfly), with no workgroup barrier per sum; thread 0 then adds the
// pair sums into the outputs in (sweep, slot) order, the order of the sweeps for every
// output, so the result does not depend on scheduling.
template <class R> __global__ void k_bsweep_out(BatchArgs<R> A, double* out, int out_stride, int grad) {
  constexpr int kChunk = 64;  // (sweep, slot) pairs per round
  __shared__ double ps[kChunk];
  __shared__ double tot[2 + 2 * kMaxP];
  const int u = A.list[blockIdx.x];
  const UnitDesc* D = A.units + u;
  const int p = D->p, nt = D->ntiles, nout = 2 + 2 * p;
  double* o = out + (size_t)D->row * out_stride;
  const double* part = reinterpret_cast<const double*>(A.ws + D->part_off);
  const SweepProg* progs = A.progs + D->prog_off;
  for (int i = threadIdx.x; i < nout; i += blockDim.x) tot[i] = 0.0;
  // the output a sweep's slot adds to (-1: the sweep does not fill that slot)
  auto target = [&](const SweepProg& pg, int slot) -> int {
    switch (slot) {
      case SLOT_E:
      case SLOT_NORM: return ((pg.pre_ops | pg.mid_ops) & OP_ENERGY) ? slot : -1;
      case SLOT_GPRE: return (grad && (pg.pre_ops & OP_GRADG)) ? 2 + pg.pre_layer : -1;
      case SLOT_GMID: return (grad && (pg.mid_ops & OP_GRADG)) ? 2 + pg.mid_layer : -1;
      case SLOT_BA: return (grad && pg.mixA_grad) ? 2 + p + pg.mixA_layer : -1;
      default: return (grad && pg.mixB_grad) ? 2 + p + pg.mixB_layer : -1;
    }
  };
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int npairs = 6 * D->nsweep;
  for (int c0 = 0; c0 < npairs; c0 += kChunk) {
    for (int q = wave; q < kChunk && c0 + q < npairs; q += nw) {
      const int s = (c0 + q) / 6, slot = (c0 + q) % 6;
      double v = 0.0;
      if (target(progs[s], slot) >= 0) {
        for (int t = lane; t < nt; t += 64) v += part[((size_t)s * 6 + slot) * nt + t];
        v = wave_sum(v);
      }
      if (lane == 0) ps[q] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 0; q < kChunk && c0 + q < npairs; ++q) {
        const int s = (c0 + q) / 6, slot = (c0 + q) % 6;
        const int oi = target(progs[s], slot);
        if (oi >= 0) tot[oi] += (slot >= SLOT_GPRE ? 2.0 : 1.0) * ps[q];
      }
    }
    __syncthreads();
  }
  // with the half state every sum covers one of each pair (z, ~z) of equal terms
  const double hs = D->half ? 2.0 : 1.0;
  for (int i = threadIdx.x; i < nout; i += blockDim.x) o[i] = hs * tot[i];
}


// ---------------------------------------------------------------------------------
// Phase tables exp(-i gamma_l c), c = 0..cmax (gamma_l * c formed and reduced in FP64,
// rounded to R), then the sweep scale records.
template <class R>
__global__ void k_tables(const double* __restrict__ gamma, const double* __restrict__ beta, int p, int cmax,
                         typename Cx<R>::V* __restrict__ tab, const SweepProg* progs, int nsweep, const SetSpec* sets,
                         int nsets, SwScale* scales) {
  __shared__ ScaleStage stage;
  const int tot = p * (cmax + 1);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
    const int l = i / (cmax + 1), c = i % (cmax + 1);
    double sn, cs;
    sincos(gamma[l] * (double)c, &sn, &cs);
    tab[i] = mkv<R>((R)cs, (R)(-sn));
  }
  if (blockIdx.x == 0) stage_and_build_scales(stage, progs, nsweep, sets, nsets, beta, p, scales);
}

// per-unit tables for a plan; block b handles unit b; also resets the work counter
template <class R> __global__ void k_plan_tables(UnitArgs<R> A, int p, int pstride) {
  using V = typename Cx<R>::V;
  __shared__ ScaleStage stage;
  if (blockIdx.x == 0 && threadIdx.x < 4) A.counter[threadIdx.x] = 0;  // one work counter per unit kernel launch
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
  stage_and_build_scales(stage, A.progs + D->prog_off, D->nsweep, D->sets, D->nsets, prm + p, p,
                         const_cast<SwScale*>(unit_scales<R>(A.ws, D)));
}

// fixed-order sums of per-tile partials: out[o] = scale_o * sum_{sources of o} sum_tiles
struct RedSrc {
  int64_t off;   // element offset into the partial buffer
  int32_t count;
  int32_t out;   // output index
  double scale;
};
// Two fixed-order stages: block (o, c) sums chunk c (of kRedChunks equal slices) of
// every source of output o into stage[o][c]; k_reduce_final adds the chunks in order.
constexpr int kRedChunks = kReduceChunks;
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partial, const RedSrc* __restrict__ src,
                                                const int32_t* __restrict__ src_begin, double* __restrict__ stage) {
  __shared__ double red[4];
  const int o = blockIdx.x, c = blockIdx.y;
  double tot = 0.0;
  for (int k = src_begin[o]; k < src_begin[o + 1]; ++k) {
    const RedSrc s = src[k];
    const int64_t lo = (int64_t)s.count * c / kRedChunks, hi = (int64_t)s.count * (c + 1) / kRedChunks;
    double v = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) v += partial[s.off + i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) tot += s.scale * (red[0] + red[1] + red[2] + red[3]);
    __syncthreads();
  }
  if (threadIdx.x == 0) stage[(size_t)o * kRedChunks + c] = tot;
}
__global__ __launch_bounds__(64) void k_reduce_final(const double* __restrict__ stage, double* __restrict__ out) {
  const int o = blockIdx.x;
  double v = threadIdx.x < kRedChunks ? stage[(size_t)o * kRedChunks + threadIdx.x] : 0.0;
  v = wave_sum(v);
  if (threadIdx.x == 0) out[o] = v;
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

// ---------------------------------------------------------------- final-state sampling
// The buffer holds sigma psi(z ^ F) at index z (uniform scale sigma, flip mask F), so the
// probability of bitstring z is |buf[z ^ F]|^2 / sum |buf|^2.  Bitstrings are drawn by
// inverse CDF in bitstring order, in three levels: FP64 sums over sub-blocks of 2^ls = 64
// indices and over blocks of 2^lb indices (index block c holds bitstring block c ^ (F >> lb),
// index sub-block s of a block holds bitstring sub-block s ^ ((F >> ls) mod 2^(lb - ls))),
// the blocks' inclusive prefix in bitstring-block order, then per shot a binary search over
// the blocks, a wave-wide prefix scan over the chosen block's sub-block sums and one over the
// chosen sub-block's amplitudes.
__host__ __device__ constexpr int samp_sub_bits(int lb) { return lb < 6 ? lb : 6; }

template <class R>
__global__ __launch_bounds__(256) void k_samp_blocksum(const typename Cx<R>::V* __restrict__ psi, int lb,
                                                       double* __restrict__ bsum, double* __restrict__ ssum) {
  // sub-block sums (one wave-wide sum per 64 consecutive indices), then the block sum as
  // their sum in index order
  __shared__ double sub[128];
  const uint64_t base = (uint64_t)blockIdx.x << lb;
  const int B = 1 << lb, ls = samp_sub_bits(lb), nsub = B >> ls;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = wave * 64; c < B; c += 256) {
    double pz = 0.0;
    if (c + lane < B) {
      const typename Cx<R>::V a = psi[base + c + lane];
      pz = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    }
    pz = wave_sum(pz);
    if (lane == 0) sub[c >> ls] = pz;
  }
  __syncthreads();
  if (threadIdx.x < nsub) ssum[((uint64_t)blockIdx.x << (lb - ls)) + threadIdx.x] = sub[threadIdx.x];
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int s2 = 0; s2 < nsub; ++s2) t += sub[s2];
    bsum[blockIdx.x] = t;
  }
}

// one workgroup: cum[b] = sum_{c <= b} bsum[c ^ fhi], in a fixed order
__global__ __launch_bounds__(1024) void k_samp_scan(const double* __restrict__ bsum, uint64_t nb,
                                                    const uint64_t* __restrict__ flips, int lb, double* __restrict__ cum) {
  __shared__ double part[1024];
  const uint64_t fhi = (*flips >> lb) & (nb - 1);
  const uint64_t chunk = (nb + 1023) / 1024;
  const uint64_t lo = min(nb, (uint64_t)threadIdx.x * chunk), hi = min(nb, lo + chunk);
  double s = 0.0;
  for (uint64_t b = lo; b < hi; ++b) s += bsum[b ^ fhi];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int t = 0; t < 1024; ++t) {
      const double v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  double run = part[threadIdx.x];
  for (uint64_t b = lo; b < hi; ++b) {
    run += bsum[b ^ fhi];
    cum[b] = run;
  }
}

// one wave per shot (four shots per workgroup)
template <class R>
__global__ __launch_bounds__(256) void k_sample(const typename Cx<R>::V* __restrict__ psi, int lb, uint64_t nb,
                                                const double* __restrict__ cum, const double* __restrict__ ssum,
                                                const uint64_t* __restrict__ flips, const double* __restrict__ uniform,
                                                int shots, const GraphDev* g, const int4* __restrict__ cost_terms,
                                                uint64_t* __restrict__ samples, int32_t* __restrict__ cuts) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= shots) return;  // uniform over the wave
  const uint64_t F = *flips;
  const double total = cum[nb - 1];
  const double u = fmin(fmax(uniform[k], 0.0), 0x1.fffffffffffffp-1);  // into [0, 1); NaN -> 0
  const double t = u * total;
  uint64_t lo = 0, hi = nb - 1;  // smallest block with cum > t
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (cum[mid] > t) hi = mid;
    else lo = mid + 1;
  }
  const uint64_t b = lo;
  double r = t - (b ? cum[b - 1] : 0.0);
  // the chosen block's sub-block sums in bitstring order, two per lane (at most 128)
  const int ls = samp_sub_bits(lb), nsub = 1 << (lb - ls);
  const uint64_t fhi = (F >> lb) & (nb - 1);
  const int fsub = (int)((F >> ls) & (uint64_t)(nsub - 1));
  const double* ms = ssum + ((b ^ fhi) << (lb - ls));
  const int s0 = 2 * lane, s1 = s0 + 1;
  const double v0 = s0 < nsub ? ms[s0 ^ fsub] : 0.0, v1 = s1 < nsub ? ms[s1 ^ fsub] : 0.0;
  double sc = v0 + v1;  // inclusive prefix over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double v = __shfl_up(sc, o, 64);
    if (lane >= o) sc += v;
  }
  const uint64_t hit = __ballot(sc > r);
  int sel;
  bool exact = true;
  if (hit) {
    const int L = __builtin_ctzll(hit);
    const double before = L ? __shfl(sc, L - 1, 64) : 0.0;
    const double first = __shfl(v0, L, 64);
    sel = (before + first > r) ? 2 * L : 2 * L + 1;
    r -= (sel == 2 * L) ? before : before + first;
  } else {
    // rounding left the residual above the block's sub-block mass: the last sub-block
    // with mass, and in it the last amplitude with mass
    const uint64_t nz = __ballot(v0 > 0.0 || v1 > 0.0);
    const int L = nz ? 63 - __builtin_clzll(nz) : 0;
    sel = (__shfl(v1, L, 64) > 0.0) ? 2 * L + 1 : 2 * L;
    exact = false;
  }
  // the chosen sub-block's amplitudes in bitstring order, one per lane
  const int S = 1 << ls;
  const uint64_t z0 = (b << lb) | ((uint64_t)sel << ls);
  double pz = 0.0;
  if (lane < S) {
    const typename Cx<R>::V a = psi[(z0 | (uint64_t)lane) ^ F];
    pz = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
  }
  double se = pz;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double v = __shfl_up(se, o, 64);
    if (lane >= o) se += v;
  }
  const uint64_t eh = exact ? __ballot(se > r) : 0ull;
  const uint64_t enz = __ballot(pz > 0.0);
  uint64_t zsel;
  if (eh)
    zsel = z0 | (uint64_t)__builtin_ctzll(eh);
  else  // rounding again: the sub-block's last amplitude with mass
    zsel = z0 | (uint64_t)(enz ? 63 - __builtin_clzll(enz) : 0);
  int cut = 0;
  if (g->weighted) {  // the weighted cut: the H_C term list holds every edge with its weight
    for (int t = 0; t < g->T; ++t) {
      const int4 tm = cost_terms[t];
      cut += tm.z * (int)(((zsel >> tm.x) ^ (zsel >> tm.y)) & 1u);
    }
  } else {
    for (int v = 0; v < g->n; ++v) cut += (int)((zsel >> v) & 1u) * __popcll(g->adj[v] & ~zsel);
  }
  if (lane == 0) {
    samples[k] = zsel;
    cuts[k] = cut;
  }
}

// best and mean cut of the shots
__global__ __launch_bounds__(256) void k_samp_stats(const int32_t* __restrict__ cuts, int shots, double* __restrict__ stats) {
  __shared__ long long smax[256], ssum[256];
  long long mx = -1, sm = 0;
  for (int k = threadIdx.x; k < shots; k += 256) {
    mx = max(mx, (long long)cuts[k]);
    sm += cuts[k];
  }
  smax[threadIdx.x] = mx;
  ssum[threadIdx.x] = sm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + o]);
      ssum[threadIdx.x] += ssum[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = (double)smax[0];
    stats[1] = (double)ssum[0] / (double)shots;
  }
}

// light-cone units: the shared (gamma, beta) into every unit's parameter row, and the
// fixed-order sum of the unit outputs (energy and gradients summed, norm averaged)
__global__ __launch_bounds__(256) void k_lc_bcast(const double* __restrict__ params, int np, double* __restrict__ rows,
                                                  int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count * np) rows[i] = params[i % np];
}
__global__ __launch_bounds__(256) void k_lc_sum(const double* __restrict__ rows, int count, int stride,
                                                double* __restrict__ out) {
  const int o = threadIdx.x;
  if (o >= stride) return;
  double s = 0.0;
  for (int u = 0; u < count; ++u) s += rows[(size_t)u * stride + o];
  out[o] = (o == 1) ? s / count : s;
}

// ------------------------------------------------------------------------------------
// launch functions used by the host code
hipError_t launch_tables(const double* gamma, const double* beta, int p, int cmax, void* tab, const SweepProg* progs,
                         int nsweep, const SetSpec* sets, int nsets, SwScale* scales, bool dbl, hipStream_t st) {
  const int tot = p * (cmax + 1);
  const int blocks = (tot + 255) / 256;
  if (dbl)
    launch(k_tables<double>, dim3(blocks), dim3(256), 0, st, gamma, beta, p, cmax,
                       reinterpret_cast<double2*>(tab), progs, nsweep, sets, nsets, scales);
  else
    launch(k_tables<float>, dim3(blocks), dim3(256), 0, st, gamma, beta, p, cmax,
                       reinterpret_cast<float2*>(tab), progs, nsweep, sets, nsets, scales);
  return hipGetLastError();
}

hipError_t launch_sample(const void* psi, int n, int lb, double* bsum, double* cum, double* ssum, const uint64_t* flips,
                         const double* uniform, int shots, const GraphDev* g, const int4* cost_terms, uint64_t* samples,
                         int32_t* cuts, double* stats, bool dbl, hipStream_t st) {
  if (lb > 13 || lb > n) return hipErrorInvalidValue;  // at most 128 sub-blocks of 64 per block
  const uint64_t nb = (uint64_t)1 << (n - lb);
  const dim3 gs((unsigned)((shots + 3) / 4));
  if (dbl) {
    launch(k_samp_blocksum<double>, dim3((unsigned)nb), dim3(256), 0, st, (const double2*)psi, lb, bsum, ssum);
    launch(k_samp_scan, dim3(1), dim3(1024), 0, st, bsum, nb, flips, lb, cum);
    launch(k_sample<double>, gs, dim3(256), 0, st, (const double2*)psi, lb, nb, cum, ssum, flips, uniform, shots,
                       g, cost_terms, samples, cuts);
  } else {
    launch(k_samp_blocksum<float>, dim3((unsigned)nb), dim3(256), 0, st, (const float2*)psi, lb, bsum, ssum);
    launch(k_samp_scan, dim3(1), dim3(1024), 0, st, bsum, nb, flips, lb, cum);
    launch(k_sample<float>, gs, dim3(256), 0, st, (const float2*)psi, lb, nb, cum, ssum, flips, uniform, shots, g,
                       cost_terms, samples, cuts);
  }
  launch(k_samp_stats, dim3(1), dim3(256), 0, st, cuts, shots, stats);
  return hipGetLastError();
}

hipError_t launch_lc_bcast(const double* params, int np, double* rows, int count, hipStream_t st) {
  const int tot = count * np;
  launch(k_lc_bcast, dim3((tot + 255) / 256), dim3(256), 0, st, params, np, rows, count);
  return hipGetLastError();
}

hipError_t launch_lc_sum(const double* rows, int count, int stride, double* out, hipStream_t st) {
  if (stride > 256) return hipErrorInvalidValue;
  launch(k_lc_sum, dim3(1), dim3(256), 0, st, rows, count, stride, out);
  return hipGetLastError();
}

hipError_t launch_plan_tables(const LaunchUnits& L, int p, bool dbl, hipStream_t st) {
  if (dbl)
    launch(k_plan_tables<double>, dim3(L.count), dim3(256), 0, st, unit_args<double>(L), p, 2 * p);
  else
    launch(k_plan_tables<float>, dim3(L.count), dim3(256), 0, st, unit_args<float>(L), p, 2 * p);
  return hipGetLastError();
}

hipError_t launch_bsweep_out(const LaunchBatch& L, double* out, int out_stride, bool grad, bool dbl, hipStream_t st) {
  if (dbl) {
    BatchArgs<double> A{L.units, L.progs, L.list, L.wgmap, L.ws, 0, L.tabmax};
    launch(k_bsweep_out<double>, dim3(L.nlist), dim3(256), 0, st, A, out, out_stride, (int)grad);
  } else {
    BatchArgs<float> A{L.units, L.progs, L.list, L.wgmap, L.ws, 0, L.tabmax};
    launch(k_bsweep_out<float>, dim3(L.nlist), dim3(256), 0, st, A, out, out_stride, (int)grad);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, const void* src, const int32_t* src_begin, double* stage, double* out,
                         int nout, hipStream_t st) {
  launch(k_reduce, dim3(nout, kRedChunks), dim3(256), 0, st, partial, reinterpret_cast<const RedSrc*>(src),
                     src_begin, stage);
  launch(k_reduce_final, dim3(nout), dim3(64), 0, st, stage, out);
  return hipGetLastError();
}

hipError_t launch_zz_pass(const void* psi, uint64_t N, int i, int j, const double* scale, const uint64_t* flips,
                          double* partial, int blocks, bool dbl, hipStream_t st) {
  if (dbl)
    launch(k_zz_pass<double>, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const double2*>(psi), N, i, j,
                       scale, flips, partial);
  else
    launch(k_zz_pass<float>, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float2*>(psi), N, i, j,
                       scale, flips, partial);
  return hipGetLastError();
}

hipError_t launch_sweep(const LaunchSweep& L, bool dbl, int tile_bits, hipStream_t st) {
  switch (tile_bits) {
    case 12: return dbl ? launch_sweep_d12(L, st) : launch_sweep_f12(L, st);
    case 13: return dbl ? launch_sweep_d13(L, st) : launch_sweep_f13(L, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bsweep(const LaunchBatch& L, bool dbl, int tile_bits, hipStream_t st) {
  switch (tile_bits) {
    case 12: return dbl ? launch_bsweep_d12(L, st) : launch_bsweep_f12(L, st);
    case 13: return dbl ? launch_bsweep_d13(L, st) : launch_bsweep_f13(L, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_units(const LaunchUnits& L, bool grad, bool dbl, int tile_bits, int blocks, hipStream_t st) {
  switch (tile_bits) {
    case 10: return dbl ? launch_units_d10(L, grad, blocks, st) : launch_units_f10(L, grad, blocks, st);
    case 12: return dbl ? launch_units_d12(L, grad, blocks, st) : launch_units_f12(L, grad, blocks, st);
    case 13: return dbl ? launch_units_d13(L, grad, blocks, st) : launch_units_f13(L, grad, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cuts(const GraphDev* g, const int4* terms, int T, int use_terms, const SetSpec& S, int arr, int32_t* out,
                       bool dbl, int tile_bits, hipStream_t st) {
  switch (tile_bits) {
    case 12:
      return dbl ? launch_cuts_d12(g, terms, T, use_terms, S, arr, out, st) : launch_cuts_f12(g, terms, T, use_terms, S, arr, out, st);
    case 13:
      return dbl ? launch_cuts_d13(g, terms, T, use_terms, S, arr, out, st) : launch_cuts_f13(g, terms, T, use_terms, S, arr, out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace aaq
