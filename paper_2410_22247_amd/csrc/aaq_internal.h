// Internal data structures shared by the host planner and the HIP kernels.
//
// State layout: amplitude z (vertex v = bit v of z) at element z of a flat array of
// complex64 (float2) or complex128 (double2).  A "tile" is 2^L amplitudes that one
// workgroup of 2^(L-4) threads holds in registers (L = 10, 12 or 13): tile bit j is
// global index bit pos[j]; the remaining global bits are enumerated by the tile id
// (ascending).  Tile bits always include global bits 0..4 so that every
// global load/store touches >= 256 contiguous bytes.
#pragma once
#include <stdint.h>

#include <initializer_list>

namespace aaq {

constexpr int kMaxN = 34;
constexpr int kMaxP = 64;
constexpr int kMaxT = 34 * 33 / 2;  // max terms (complete graph on 34 vertices)
constexpr int kMaxSets = 5;
constexpr int kMinContig = 5;       // low global bits every tile must contain
constexpr uint8_t kDummy = 0xFF;    // tile bit without a vertex (n < L)
constexpr int kRegBits = 4;         // register bits per thread: 16 amplitudes

// Register arrangements of a tile of L bits: arrangement k keeps tile bits
// [geo_b0(k), geo_b0(k) + 4) in registers; geo_na(L) arrangements, the last one (top
// tile bits in registers) is used for global loads and stores, the one before it is
// where phases and the energy are applied.
constexpr int geo_na(int L) { return (L + kRegBits - 1) / kRegBits; }
constexpr int geo_b0(int k, int L) { return (k * kRegBits < L - kRegBits) ? k * kRegBits : L - kRegBits; }

// mixer routes through the register arrangements, from the load arrangement to the
// phase arrangement: every arrangement, or all but arrangement 0 (sets whose active
// qubits are all tile bits >= 4)
enum : uint8_t { ROUTE_FULL = 0, ROUTE_HIGH = 1 };

// per-position operations inside a sweep
enum : uint8_t {
  OP_PHASE = 1,    // multiply live states by exp(-i gamma_l C(z))
  OP_UNPHASE = 2,  // multiply live states by exp(+i gamma_l C(z))
  OP_GRADG = 4,    // accumulate 2 Im sum conj(lam) C psi  (d/dgamma_l)
  OP_ENERGY = 8,   // accumulate sum |psi|^2 h(z) and |psi|^2; with F_MAKE_LAM: lam = h psi
  OP_PERTERM = 16  // with OP_ENERGY: accumulate <Z_i Z_j> per term
};

// sweep flags
enum : uint8_t {
  F_LOAD_PSI = 1,
  F_LOAD_LAM = 2,
  F_STORE_PSI = 4,
  F_STORE_LAM = 8,
  F_INIT = 16,      // synthesize |+> instead of loading psi
  F_LAM_LIVE = 32,  // lambda is live at sweep start
  F_MAKE_LAM = 64   // OP_ENERGY creates lambda = h psi
};

// Compile-time shape of a sweep (the steps it has), used to specialize the sweep
// kernels so that no step is a run-time branch around register updates.  Bits 0-7:
// structure; bits 8-15: the ops at the load position; bits 16-23: the ops at the
// phase position.  SK_GENERIC: every decision is taken from the SweepProg at run time.
enum : uint32_t {
  SK_INIT = 1u << 0,      // synthesise |+>
  SK_LOAD_PSI = 1u << 1,  // load psi
  SK_LAM_IN = 1u << 2,    // load lambda, live from the start
  SK_MIXA = 1u << 3,
  SK_MIXB = 1u << 4,
  SK_MAKE_LAM = 1u << 5,  // the energy step creates lambda
  SK_PSI_DEAD = 1u << 6,  // psi is not stored after the last mixer (lambda alone is)
  SK_WEIGHTED = 1u << 7,  // integer edge weights: the cut from the set's cost-term lists
  SK_GENERIC = 1u << 31
};
constexpr uint32_t sk_pre(uint32_t kind) { return (kind >> 8) & 0xFFu; }
constexpr uint32_t sk_mid(uint32_t kind) { return (kind >> 16) & 0xFFu; }
constexpr uint32_t sk_make(uint32_t bits, uint32_t pre_ops, uint32_t mid_ops) {
  return bits | (pre_ops << 8) | (mid_ops << 16);
}
// the shapes of the multi-set sweep programs (first, plain, layer-boundary and last
// forward sweeps; the turnaround; plain, layer-boundary and last backward sweeps)
constexpr uint32_t SK_F_FIRST = sk_make(SK_INIT | SK_MIXA, OP_PHASE, 0);
constexpr uint32_t SK_F_PLAIN = sk_make(SK_LOAD_PSI | SK_MIXA, 0, 0);
constexpr uint32_t SK_F_BOUNDARY = sk_make(SK_LOAD_PSI | SK_MIXA | SK_MIXB, 0, OP_PHASE);
constexpr uint32_t SK_F_ENERGY = sk_make(SK_LOAD_PSI | SK_MIXA, 0, OP_ENERGY);
constexpr uint32_t SK_F_ENERGY_TERMS = sk_make(SK_LOAD_PSI | SK_MIXA, 0, OP_ENERGY | OP_PERTERM);
constexpr uint32_t SK_TURNAROUND = sk_make(SK_LOAD_PSI | SK_MIXA | SK_MIXB | SK_MAKE_LAM, 0, OP_ENERGY);
constexpr uint32_t SK_B_PLAIN = sk_make(SK_LOAD_PSI | SK_LAM_IN | SK_MIXA, 0, 0);
constexpr uint32_t SK_B_BOUNDARY = sk_make(SK_LOAD_PSI | SK_LAM_IN | SK_MIXA | SK_MIXB, 0, OP_GRADG | OP_UNPHASE);
constexpr uint32_t SK_B_LAST = sk_make(SK_LOAD_PSI | SK_LAM_IN | SK_MIXA, 0, OP_GRADG);
// the turnaround and the backward sweeps when psi is not stored (the turnaround of every
// gradient evaluation; the backward sweeps with forward-state checkpoints)
constexpr uint32_t SK_TURNAROUND_PD = SK_TURNAROUND | SK_PSI_DEAD;
constexpr uint32_t SK_B_PLAIN_PD = SK_B_PLAIN | SK_PSI_DEAD;
constexpr uint32_t SK_B_BOUNDARY_PD = SK_B_BOUNDARY | SK_PSI_DEAD;

// partial-sum slots written per sweep and tile
enum : int { SLOT_E = 0, SLOT_NORM = 1, SLOT_GPRE = 2, SLOT_GMID = 3, SLOT_BA = 4, SLOT_BB = 5, SLOT_TERMS = 6 };

struct SetSpec {
  uint8_t pos[16];   // global bit of tile bit j, kDummy if none
  uint32_t act;      // tile-bit mask mixed in this set
  uint32_t dummy;    // tile-bit mask of dummy bits
  uint64_t fixmask;  // global bits enumerated by the tile id
  uint32_t ntiles;
  uint8_t kl;         // load/store arrangement (the last one: register bits = the top tile bits)
  uint8_t route;      // mixer route: ROUTE_FULL or ROUTE_HIGH (arrangements visited)
  uint8_t pad[6];
  uint64_t gact;      // global bits of the active (mixed) qubits
  uint64_t roff[16];  // element offset of register r at the load/store arrangement
  // Observable terms sorted for the two arrangements where h(z) is evaluated (index 0:
  // load arrangement, 1: phase arrangement): first the terms with no endpoint among the
  // register bits, then those with one endpoint at register bit 0, 1, 2, 3, then those
  // with both endpoints in registers (int4 .w = ri | rj << 4).  toff is the offset in
  // int4 entries from the start of the unit's term array, tcnt the six group sizes.
  uint16_t toff[2];
  uint16_t tcnt[2][6];
  // The weighted cut's terms (every edge with its weight) in the same grouping, for the
  // cost phase and the gamma gradient of weighted instances (empty otherwise).
  uint16_t coff[2];
  uint16_t ccnt[2][6];
  // Half state (the global spin-flip symmetry psi(~z) = psi(z)): only indices below
  // 2^(n-1) are stored.  Registers whose index has bit n-1 set (mask `mirror`) live at
  // the mirrored index mfull - index (mfull = 2^n - 1); tmax is the largest thread offset
  // at the load arrangement.  mirror = 0 outside half mode and for sets that hold bit
  // n-1 in the tile id (their processed tiles are all below 2^(n-1)).
  uint16_t mirror;
  uint16_t pad2[3];
  uint64_t tmax;
  uint64_t mfull;
  // The thread bits of the load (index 0) and phase (index 1) arrangements scattered to
  // their global bits, as at most kMaxRuns runs of consecutive thread bits that land on
  // consecutive global bits (tile positions ascend, so a set has two or three): run i is
  // packed as (first thread bit) | (width << 8) | (first global bit << 16); unused runs
  // are 0 (width 0 contributes nothing).  tr64: some run reaches bit 32 or above.
  uint32_t trun[2][4];
  uint32_t tr64;
  uint32_t pad3;
};
constexpr int kMaxRuns = 4;

struct SweepProg {
  int8_t set;
  uint8_t flags;
  uint8_t pre_ops;
  int8_t pre_layer;
  int8_t mixA_layer;
  int8_t mixA_dir;  // +1 apply e^{-i beta X}, -1 apply its inverse, 0 none
  uint8_t mixA_grad;
  uint8_t mid_ops;
  int8_t mid_layer;
  int8_t mixB_layer;
  int8_t mixB_dir;
  uint8_t mixB_grad;
  uint8_t ld_buf;  // psi buffer (in units of one state) loaded / stored: 0 except with
  uint8_t st_buf;  // forward-state checkpoints, where sweep i stores buffer i
};
constexpr int kMaxCkpt = 32;  // max psi buffers of a checkpointed program

// shape of a sweep program (stores and buffer indices stay run-time values)
inline uint32_t sweep_kind(const SweepProg& s) {
  uint32_t b = 0;
  if (s.flags & F_INIT) b |= SK_INIT;
  if (s.flags & F_LOAD_PSI) b |= SK_LOAD_PSI;
  if ((s.flags & F_LOAD_LAM) && (s.flags & F_LAM_LIVE)) b |= SK_LAM_IN;
  else if (s.flags & (F_LOAD_LAM | F_LAM_LIVE)) return SK_GENERIC;
  if (s.mixA_dir) b |= SK_MIXA;
  if (s.mixB_dir) b |= SK_MIXB;
  if (s.flags & F_MAKE_LAM) b |= SK_MAKE_LAM;
  const uint32_t k = sk_make(b, s.pre_ops, s.mid_ops);
  for (uint32_t known : {SK_F_FIRST, SK_F_PLAIN, SK_F_BOUNDARY, SK_F_ENERGY, SK_F_ENERGY_TERMS, SK_TURNAROUND,
                         SK_B_PLAIN, SK_B_BOUNDARY, SK_B_LAST})
    if (k == known) {
      const bool dead = (s.flags & F_STORE_LAM) && !(s.flags & F_STORE_PSI);
      if (dead && (k == SK_TURNAROUND || k == SK_B_PLAIN || k == SK_B_BOUNDARY)) return k | SK_PSI_DEAD;
      return k;
    }
  return SK_GENERIC;
}

// Per-sweep scale record.  Mixer gates are applied as (I - i k X) per qubit, with
// |k| <= 1; the dropped scalar factor phi per qubit (cos b, or +-i sin b together with
// a bit flip X) accumulates into a uniform complex scale sigma = stored / true, and the
// bit flips into a uniform global mask F (the buffers hold the amplitude of z ^ F at
// index z; flips are never moved in memory).  The device tracks sigma and F along the
// sweep sequence, cancels sigma in the phase tables (rho = 1/sigma), the energy and
// the gradient sums (s = 1/|sigma|^2), and evaluates C and h at z ^ F.
struct SwScale {
  double rho_pre[2];  // complex multiplier folded into the pre-position phase table
  double rho_mid[2];
  double s_pre, s_mid;  // 1/|sigma|^2 at the pre / mid position
  double s_A, s_B;      // 1/|sigma|^2 at the start of mixer A / B
  double kA, wA, kB, wB;  // butterfly coefficient, per-qubit |phi|^2 of mixer A / B
  uint64_t F_pre, F_mid;  // flip mask at the pre / mid position: the buffers hold amplitude z ^ F at index z
  double lam_fix[2];      // multiplier for lambda when loaded (equalises the scales of psi and lambda)
  uint32_t fix_lam, pad;  // nonzero when lam_fix != 1
};

// graph block in device memory (uniform and read-only for the kernels that read it:
// scalar loads through the constant address space)
constexpr int kAdjPad = (kMaxN + 3) / 4 * 4;  // masks padded with zeros to a multiple of 4
struct GraphDev {
  int32_t n, m, T, cmax;   // cmax = |E| = last phase-table index
  int32_t h_is_cut;        // the observable is H_C: h(z) = C(z), computed from the adjacency masks
  int32_t weighted;        // integer edge weights: C(z) comes from the sets' cost-term lists
  uint64_t adj[kAdjPad];   // adjacency bitmasks
  uint32_t adj32[kAdjPad]; // their low 32 bits (all of them when n <= 32)
  int32_t deg[kAdjPad];
};

// one batched unit (instance x parameter point)
struct UnitDesc {
  int32_t n, p, nsweep, nsets;
  int64_t graph_off;   // byte offset of GraphDev in the workspace
  int64_t terms_off;   // byte offset of int4 terms (i, j, w, 0)
  int64_t tab_off;     // byte offset of this unit's phase tables [p][cmax+1], then SwScale[nsweep+1]
  int64_t state_off;   // byte offset of psi (lambda follows), -1 when n <= L
  int32_t prog_off;    // index of the first SweepProg
  int32_t row;         // row in d_params / d_out
  int32_t T, cmax;
  int64_t part_off;    // byte offset of the per-tile partial sums [nsweep][6][ntiles] (n > L units)
  int64_t lam_off;     // byte offset of lambda, after the psi buffers (n > L units with gradients)
  int32_t ntiles;      // tiles per sweep (of the stored half with the half state)
  int32_t L;           // tile size (log2 amplitudes) of the unit's kernels
  int32_t half;        // 1: the unit stores and sweeps the half state (n > L units only)
  int32_t pad_;
  SetSpec sets[kMaxSets];
};

}  // namespace aaq
