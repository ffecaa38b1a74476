// Device-side helpers of libtbsma: constants, Philox4x32-10, wave
// reductions, XCD-aware block numbering and the kernel argument bundles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tbsma {

constexpr int kTile = 64;   // slots per tile = one wavefront
constexpr int kBlock = 256; // threads of every per-atom kernel
constexpr int kSortCells = 16;  // cells per block of the cell sort
constexpr int kNPart = 8;   // FP64 partial sums per tile
constexpr int kStage = 1536;  // neighbour positions a pair-pass block stages
                              // in LDS (24 KB), at most
constexpr int kGatherSpan = 65536;  // widest slot window of gather staging

// Launch shapes of the mixed pair passes, chosen per replica (tbsma_system
// shape): tiles per block (1, 2 or 4) and the stage class, the LDS the block
// reserves for staged positions (class 0: 1152 entries, 18 KB, which leaves
// room for the density pass's full occupancy; class 1: kStage).  The block
// map holds the blocks of class 0 first, then those of class 1, and each
// class is one launch of its own kernel variant.
constexpr int kStageClasses = 2;
__host__ __device__ constexpr int stage_of_class(int c) {
  return c == 0 ? 1152 : kStage;
}
constexpr int32_t kShapeDefault = 4 | (1 << 4);  // 4 tiles, class 1
__host__ __device__ inline int shape_tpb(int32_t s) { return s & 15; }
__host__ __device__ inline int shape_cls(int32_t s) { return (s >> 4) & 15; }

// per-tile partial sums
constexpr int kPartE = 0;   // sum of E_i
constexpr int kPartW = 1;   // sum of w_i = 1/2 sum_j E'_ij dz^2 / r
constexpr int kPartK = 2;   // sum over dynamic atoms of m |v - u|^2
constexpr int kPartKz = 3;  // sum over dynamic atoms of m (v_z - u_z)^2
constexpr int kPartA = 4;   // init: sum v_x, v_y, v_z, count (4..7)
constexpr int kPartQ = 4;   // steps: barostat force sum_top F_z - sum_bottom F_z

// Physical constants: k_B (eV/K) and 1 eV/(A amu) in A/ps^2, from the SI
// values of the electronvolt and the atomic mass unit.
constexpr double kBoltz = 8.617333262e-5;
constexpr double kAccel = 1.602176634e-19 / 1.66053906660e-27 * 1.0e-4;
constexpr double kEvA3ToGPa = 1.602176634e-19 * 1.0e21;

// Float constants of the mixed-precision pair kernels.  Distances are in
// position quanta (2^-qbits A); every scale is folded into the constants.
struct PotF {
  float rc2;        // r_cut^2 in quanta^2
  float rt;         // r_tail in quanta
  float aP, bP;     // (2q/r0) phi(r) = exp2(aP r + bP)
  float aF, bF;     // phi(r) = exp2(aF r + bF)
  float aV, bV;     // V(r)   = exp2(aV r + bV)
  float bW;         // -2 V'(r) = (2p/r0) V(r) = exp2(aV r + bW)
  // The cubic tails on (r_tail, r_cut] in u = (r_cut - r)/(r_cut - r_tail),
  // which vanish with their slope at u = 0; u is clamped at 0 beyond r_cut,
  // so the tail expressions give exactly 0 there and need no cut-off test.
  float uS, uB;     // u = uS r + uB
  float fa, fb;     // phi    = u^2 (fa + fb u)
  float va, vb;     // V      = u^2 (va + vb u)
  float dv0, dv1;   // 2 V'(r) = u (dv0 + dv1 u)
  float dp0, dp1;   // -phi'(r) = u (dp0 + dp1 u)
  float wscale;     // 2^-qbits / 2: converts the virial accumulator to eV
};

// Double constants of the FP64 pair kernels (Angstrom units).
struct PotD {
  double rc, rc2, rt, r0, xi2, A, k2q, kp, w;
  double f0, f1, f2, f3;  // phi tail cubic in t = (r - rt)/w
  double v0, v1, v2, v3;  // V tail cubic in t
};

// Device view of the system (plain pointers, passed by value).
struct Dev {
  int32_t R, max_zbins;
  int64_t N, C;
  const int64_t *rep_off, *cell_off;
  const int32_t *tile_rep, *grid_dim, *rep_id;
  const int32_t *tag;           // [N] tag of each slot, or NULL: slot - rep_off
  const double *grid_lo;
  double *x, *y, *z, *vx, *vy, *vz, *z0;
  uint8_t *flag;
  int4 *qpos;
  // cells and lists
  int32_t *cell_start, *cell_atoms;
  int32_t *nl, *nn;
  int32_t *nact;                // pairs within r_cut per atom: core, tail
  int2 *win;                    // [N/64] slot window [lo, hi) of a tile's lists
  int2 *bmap;                   // list-build blocks: first tile, tiles
  int4 *cbmap;                  // cell-sort blocks: replica, first cell, cells
  int32_t ncbmap;               // number of cell-sort blocks
  uint8_t *lane_atom;           // [N] pair-pass lane order within a block
  int32_t *nn_lane;             // [N] list lengths in lane order
  int32_t *nl_lane;             // lists in lane order (CL8 layout), or NULL
  // pruning of the lane-ordered lists (mixed precision)
  int32_t pruning;              // 1 when enabled
  int32_t rebuild_bound;        // 1: rebuild test by the pruning bound
  float prune_r2q;              // (r_cut + 2d)^2 + margin, quanta^2
  float prune_d2q;              // d^2, quanta^2
  float skin_half_q;            // skin/2 less one quantum, in quanta
  int4 *qprune;                 // [N] quantised positions at the last pruning;
                                // .w: the displacement since the list build
                                // then (float, quanta, rounded up)
  uint8_t *atom_lane;           // [N] row of each atom in its block's lane order
  int32_t *ncore;               // [N] leading entries of each full row (mixed)
                                // within the core radius at the build
  float core_r2q;               // core radius^2, quanta^2 (0: no core)
  unsigned long long *stats;    // [2] list-length sums (diagnostics)
  int32_t nbmap;                // number of list-build blocks
  const int32_t *shape;         // [R] launch shape of each replica, or NULL
                                // (kShapeDefault)
  int32_t *boff;                // [R] first block of each replica in bmap
  int32_t cls_off[kStageClasses + 1];  // first block of each stage class
  // gather staging of the pair passes (mixed precision): blocks whose slot
  // window exceeds LDS stage the exact set of their neighbours
  int32_t gather;               // 1 when enabled
  int32_t *gcnt;                // [nbmap] staged neighbours, 0: not staged
  uint16_t *glist;              // [nbmap * kStage] their offsets from the
                                // block's window start, ascending
  int32_t *wl;                  // work lists of a step (see work_lists)
  int64_t *callb;               // first step and end step of the current
                                // step-loop call, the step flags of the
                                // current step (kStepLog, kStepKick,
                                // kStepPend), and the step-loop counters
                                // (kCallRebuilds, kCallPrunes)
  // when the mixed force pass computes energies and the virial: 1 always,
  // 0 never, -1 when the step being completed is logged ((*step + 1) %
  // n_log == 0, the step loops)
  int32_t energies;
  int32_t n_log;
  const int64_t *step;
  // step loops only: per-replica status; retired replicas are skipped
  const uint32_t *rstatus;
  int32_t k_cap;
  double *xr, *yr, *zr;
  // workspace
  uint32_t *rflag;              // [R] bit 0: some atom moved more than skin/2
                                // since the list build; bit 1: more than the
                                // pruning half-width since the last pruning
  int32_t *cnt;                 // [C]
  double *part;                 // [N/64 * kNPart]
  unsigned long long *zbmin, *zbmax;  // [R * max_zbins] ordered keys of z
  uint32_t *wstatus;            // [R]
  int32_t *nnmax;               // [1]
  double *rsum;                 // [R * 8] per-replica scratch sums
  double *nhw;                  // [R * 5] Nose-Hoover step state (kNh*)
  double *baw;                  // [R * 2] barostat step state (kBa*)
  // parameters used on the device
  double cell, inv_cell, skin_half2, qscale, inv_qscale, mass;
  int32_t all;                  // 1: rebuild every replica
};

struct DevMD {
  double dt, gamma, c1, r_cut;
  int32_t lab_frame, n_log, n_slots;
  // 1: the second half kick of a step is left to the next step's first
  // kernel unless the step is logged or ends the call (mixed precision
  // without Nose-Hoover and barostat, whose sums need the velocities of
  // every step)
  int32_t defer;
  const double *T, *v_pull, *z_lo, *z_hi, *vol, *L0;
  const uint64_t *seed;
  const int32_t *dof;
  int64_t *step;
  double *obs;
  uint32_t *status;
  double retire;   // grip travel after rupture before retiring (<= 0: never)
  double *dfail;   // [R] grip displacement at the first rupture (-1: none)
  double nh_tau;   // Nose-Hoover relaxation time (ps); 0: not used
  double *nh_xi;   // [R] thermostat friction zeta (1/ps) at the current step
  double *nh_eta;  // [R] its time integral, or NULL
  double grip_step;   // stepwise grips: move of each grip per hold (A)
  int64_t grip_hold;  // steps per hold; 0: continuous pulling at v_pull
  const double *T_start;  // [R] temperature ramp: T_start at ramp_begin,
  int64_t ramp_begin;     //   rising linearly to T over ramp_steps steps
  int64_t ramp_steps;     //   (0: the target is T throughout)
  double baro_mass;       // axial barostat on the grip separation (amu; 0: off)
  double baro_load;       // outward pull on each grip (eV/A)
  double baro_damp;       // friction on the barostat coordinate (1/ps)
  double *baro_s;         // [2R] grip travel s (A) and ds/dt (A/ps)
};

// Per-replica barostat state in the workspace (DevMD::baro_mass > 0), at
// Dev::baw + 2 r: the grip travel the next step places the grips at, and
// ds/dt after that step's first half kick.
constexpr int kBaS = 0;
constexpr int kBaV = 1;

// Per-replica Nose-Hoover state in the workspace (DevMD::nh_tau > 0), at
// offsets of Dev::nhw + 5 r:
constexpr int kNhPend = 0;  // velocity scale the next first half kick applies
constexpr int kNhEnd = 1;   // scale of the last end-of-step half step, still
                            // to be applied when the call ends (1: none)
constexpr int kNhZeta = 2;  // zeta and eta after the next step's first
constexpr int kNhEta = 3;   //   thermostat half step
constexpr int kNhTop = 4;   // top-grip travel at which kNhEnd was taken

// Grips.  Continuous pulling (grip_hold = 0): the bottom grip rests and the
// top one moves at v_pull.  Stepwise symmetric grips (Simulation details):
// each hold of grip_hold steps begins with both grips moving grip_step
// outwards.  Travel after n steps of the top grip (+z) and the bottom grip
// (-z); their sum is the elongation D of eq 4.
__device__ __forceinline__ double grip_top(const DevMD &M, int r, int64_t n) {
  if (M.grip_hold > 0)
    return M.grip_step * (double)((n + M.grip_hold - 1) / M.grip_hold);
  return M.v_pull[r] * (double)n * M.dt;
}
__device__ __forceinline__ double grip_bottom(const DevMD &M, int64_t n) {
  if (M.grip_hold > 0)
    return M.grip_step * (double)((n + M.grip_hold - 1) / M.grip_hold);
  return 0.0;
}
__device__ __forceinline__ double elongation(const DevMD &M, int r,
                                             int64_t n) {
  return grip_top(M, r, n) + grip_bottom(M, n);
}

// Streaming velocity of the affine stretch at axial position z when the top
// grip has travelled D; zero in the lab frame, when the grip rests, and with
// stepwise grips.
__device__ __forceinline__ double stream_u(const DevMD &M, int r, double z,
                                           double D) {
  double vp = M.v_pull[r];
  if (M.lab_frame || vp == 0.0 || M.grip_hold > 0 || M.baro_mass > 0.0)
    return 0.0;
  return vp * (z - M.z_lo[r]) / (M.z_hi[r] - M.z_lo[r] + D);
}

// Target temperature of replica r at time t (in steps): linear from
// T_start at ramp_begin to T at ramp_begin + ramp_steps, constant outside
// (the equilibration ramp of Simulation details); T without a ramp.
__device__ __forceinline__ double target_T(const DevMD &M, int r, double t) {
  if (M.ramp_steps <= 0) return M.T[r];
  double f = (t - (double)M.ramp_begin) / (double)M.ramp_steps;
  if (f < 0.0) f = 0.0;
  if (f > 1.0) f = 1.0;
  return M.T_start[r] + (M.T[r] - M.T_start[r]) * f;
}

// Axial barostat (Simulation details: zero pressure along [100] during the
// equilibration).  The grip separation is the coordinate it controls: both
// grips move outwards by s, an extended coordinate of mass W with
// W d2s/dt2 = Q + 2 F_load, Q = sum_top F_z - sum_bottom F_z = -dE/ds, and an
// optional friction gamma_b applied as exp(-gamma_b dt/2) before the first
// and after the second half kick of ds/dt in each step (velocity Verlet).
// Half kick of ds/dt for the grip force Q:
__device__ __forceinline__ double baro_kick(const DevMD &M, double sdot,
                                            double Q) {
  return sdot + 0.5 * M.dt * (kAccel / M.baro_mass) * (Q + 2.0 * M.baro_load);
}

// One Nose-Hoover thermostat half step (dt/2) of replica r for the kinetic
// energy K (eV) of its peculiar velocities at target temperature Tt:
// zeta += dt/4 G(K); eta += dt/2 zeta; scale s = exp(-zeta dt/2); K *= s^2;
// zeta += dt/4 G(K), with G(K) = (2K / (g kB Tt) - 1) / tau^2.  Returns s
// (1 when g kB Tt <= 0: such a replica is left unthermostatted).
__device__ __forceinline__ double nh_half(const DevMD &M, int r, double Tt,
                                          double &zeta, double &eta,
                                          double &K) {
  const double gkT = (double)M.dof[r] * kBoltz * Tt;
  if (!(gkT > 0.0)) return 1.0;
  const double tau2 = M.nh_tau * M.nh_tau;
  zeta += 0.25 * M.dt * (2.0 * K / gkT - 1.0) / tau2;
  eta += 0.5 * M.dt * zeta;
  const double s = exp(-0.5 * M.dt * zeta);
  K *= s * s;
  zeta += 0.25 * M.dt * (2.0 * K / gkT - 1.0) / tau2;
  return s;
}

// Tag of the atom in slot i of replica r (the counter word of its random
// numbers): the system's tag array when it has one, else the slot offset.
__device__ __forceinline__ uint32_t atom_tag(const Dev &S, int r, int64_t i) {
  return S.tag != nullptr ? (uint32_t)S.tag[i] : (uint32_t)(i - S.rep_off[r]);
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
// that each XCD works on one contiguous range of tiles, which keeps the
// neighbours' positions in that XCD's L2.
__device__ __forceinline__ int64_t xcd_block() {
  int64_t nb = gridDim.x, b = blockIdx.x;
  int64_t q = nb / 8, rem = nb % 8, xc = b % 8, k = b / 8;
  int64_t start = xc < rem ? xc * (q + 1) : rem * (q + 1) + (xc - rem) * q;
  return start + k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

__device__ __forceinline__ uint4 rng_words(uint64_t seed, uint32_t rep,
                                           uint32_t tag, uint64_t step,
                                           uint32_t stream) {
  return philox4x32_10(make_uint4(tag, (uint32_t)step, rep, stream),
                       make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
}

__device__ __forceinline__ double u01(uint32_t w) {
  return ((double)w + 0.5) * 0x1p-32;
}

// Three standard normals of one counter (Box-Muller, FP64).
__device__ __forceinline__ void gauss3(uint64_t seed, uint32_t rep,
                                       uint32_t tag, uint64_t step,
                                       uint32_t stream, double &n0,
                                       double &n1, double &n2) {
  uint4 o = rng_words(seed, rep, tag, step, stream);
  const double twopi = 6.283185307179586476925286766559;
  double a = sqrt(-2.0 * log(u01(o.x)));
  double b = sqrt(-2.0 * log(u01(o.z)));
  double s, c;
  sincos(twopi * u01(o.y), &s, &c);
  n0 = a * c;
  n1 = a * s;
  n2 = b * cos(twopi * u01(o.w));
}

// -2 ln u for the uniform u = (w + 1/2) 2^-32 of a Philox word, in FP32 with
// a relative error of a few ulp over the whole of (0, 1).  Below 1/2, u is
// formed from 2w + 1 with one rounding.  From 1/2 on, v = 1 - u = (~w + 1/2)
// 2^-32 is formed the same way (exactly, before that rounding) and
// ln u = ln(1 - v) is taken as ln(y) (-v) / (y - 1) with y = 1 - v rounded,
// Goldberg's correction for log(1 + x) (y - 1 is exact for y in [1/2, 1]),
// so that draws next to 1 keep their relative precision instead of being
// cancelled to the ulp of 1.
__device__ __forceinline__ float m2ln_u01f(uint32_t w) {
  const float m2ln2 = -1.3862943611198906f;  // -2 ln 2
  const bool low = w < 0x80000000u;
  const uint32_t h = low ? w : ~w;  // below 2^31 either way
  const float t = (float)(2u * h + 1u) * 0x1p-33f;  // u (low) or v = 1 - u
  if (low) return m2ln2 * __builtin_amdgcn_logf(t);
  const float y = 1.0f - t;
  const float d = y - 1.0f;
  return d == 0.0f ? 2.0f * t : m2ln2 * __builtin_amdgcn_logf(y) * (-t / d);
}

// The angle 2 pi u of a Philox word as the revolution count u - [u >= 1/2] in
// [-1/2, 1/2): the same sine and cosine, with the argument's rounding error
// bounded by 2^-25 of a revolution.
__device__ __forceinline__ float rev_u01f(uint32_t w) {
  return fmaf((float)(int32_t)w, 0x1p-32f, 0x1p-33f);
}

// The same three normals as gauss3 in FP32 (mixed precision), from the same
// Philox words: sqrt(-2 ln u) with u of full relative precision (m2ln_u01f),
// and the sine and cosine of pi (2 t) for the revolution count t of rev_u01f
// (sincospif, cospif), so that each normal is within a few FP32 ulp of the
// FP64 value.
__device__ __forceinline__ void gauss3f(uint64_t seed, uint32_t rep,
                                        uint32_t tag, uint64_t step,
                                        uint32_t stream, float &n0, float &n1,
                                        float &n2) {
  uint4 o = rng_words(seed, rep, tag, step, stream);
  const float a = __builtin_amdgcn_sqrtf(m2ln_u01f(o.x));
  const float b = __builtin_amdgcn_sqrtf(m2ln_u01f(o.z));
  float s1, c1;
  sincospif(2.0f * rev_u01f(o.y), &s1, &c1);
  n0 = a * c1;
  n1 = a * s1;
  n2 = b * cospif(2.0f * rev_u01f(o.w));
}

// Order-preserving map of a double to an unsigned key (for atomic min/max).
__device__ __forceinline__ unsigned long long dkey(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

// Flags of the current step of a step-loop call (callb[2]), set once per
// step so that kernels need no 64-bit division by n_log: the step is logged;
// the force pass does its second half kick; the position update first
// applies the previous step's deferred kick (DevMD::defer).
constexpr int64_t kStepLog = 1, kStepKick = 2, kStepPend = 4;

// Counters in callb, advanced by the step loops' work-list kernel since the
// workspace was initialised: replica list rebuilds, and replica prunings
// without a rebuild.
constexpr int kCallRebuilds = 3, kCallPrunes = 4;

// The flags of step m of the call recorded in callb (see kStepLog).
__device__ __forceinline__ int64_t step_flags(const DevMD &M,
                                              const int64_t *callb,
                                              int64_t m) {
  const bool log = (m + 1) % M.n_log == 0;
  const bool kick = !M.defer || log || m + 1 == callb[1];
  const bool pend = M.defer && m != callb[0] && m % M.n_log != 0;
  return (log ? kStepLog : 0) | (kick ? kStepKick : 0) |
         (pend ? kStepPend : 0);
}

// Work lists of a step, written by k_worklist from the rebuild and pruning
// flags, so that the cell, list-build and pruning kernels launch a fixed,
// small grid whatever the number of replicas that rebuild or prune.
// Replicas come in order in each list.
struct WorkLists {
  int32_t *count;    // [4] entries of the four lists
  int32_t *tiles;    // tiles of the replicas that rebuild
  int32_t *blocks;   // list-build blocks (bmap entries) of the replicas that
                     // rebuild or prune
  int32_t *reps;     // the replicas that rebuild
  int32_t *cblocks;  // cell-sort blocks (cbmap entries) of those replicas
};
// Capacities: N/64 tiles, N/64 + R + 1 list-build blocks (one tile per block
// at the least), R replicas, C/kSortCells + R + 1 cell-sort blocks.
__host__ __device__ inline int64_t work_lists_size(int64_t N, int64_t R,
                                                   int64_t C) {
  return 4 + N / kTile + (N / kTile + R + 1) + R + (C / kSortCells + R + 1);
}
__device__ __forceinline__ WorkLists work_lists(const Dev &S) {
  WorkLists W;
  W.count = S.wl;
  W.tiles = S.wl + 4;
  W.blocks = W.tiles + S.N / kTile;
  W.reps = W.blocks + (S.N / kTile + S.R + 1);
  W.cblocks = W.reps + S.R;
  return W;
}

__device__ __forceinline__ int32_t rep_shape(const Dev &S, int r) {
  return S.shape != nullptr ? S.shape[r] : kShapeDefault;
}

// Stage (LDS entries) of the pair-pass block at index blk of the block map.
__device__ __forceinline__ int block_stage(const Dev &S, int64_t blk) {
  return blk < S.cls_off[1] ? stage_of_class(0) : stage_of_class(1);
}

__device__ __forceinline__ bool rebuilds(const Dev &S, int r) {
  return S.all || (S.rflag[r] & 1u);
}

// Whether replica r has been retired (step loops only).
__device__ __forceinline__ bool retired(const Dev &S, int r) {
  return S.rstatus != nullptr && (S.rstatus[r] & 32u);
}

// Whether replica r's pruned lists must be pruned again this step.
__device__ __forceinline__ bool prunes(const Dev &S, int r) {
  return S.pruning && (S.rflag[r] & 2u);
}

// Cell coordinate along one axis, clamped to the grid (clamping keeps the
// 27-cell search exact); *out set when clamped.
__device__ __forceinline__ int cell_coord(double v, double lo, double inv_h,
                                          int dim, bool &out) {
  double t = floor((v - lo) * inv_h);
  if (!(t >= 0.0)) {
    out = true;
    return 0;
  }
  if (t > (double)(dim - 1)) {
    out = true;
    return dim - 1;
  }
  return (int)t;
}

}  // namespace tbsma
