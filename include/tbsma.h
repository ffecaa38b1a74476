/*
 * tbsma.h - C ABI of libtbsma: TB-SMA (second-moment tight-binding,
 * Cleri-Rosato) molecular dynamics of gold nanowires under elongation on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow the method of French, Pervaje, Santos, Iacovella and
 * Cummings, "Probing the Statistical Validity of the Ductile-to-Brittle
 * Transition in Metallic Nanowires using GPU Computing":
 *   - energy: eqs 1-3 (band term, repulsive term, total) with the Au
 *     parameters of Table 1 (r0 read as the nearest-neighbour distance
 *     2.884 A, the value that reproduces the fitted cohesive energy);
 *   - forces: the two-stage evaluation of Methods ("TB-SMA potential"): a
 *     first loop over neighbours for the density rho_i, a global
 *     synchronisation, a second loop for the forces, which depend on rho of
 *     both atoms of a pair;
 *   - dynamics: velocity Verlet with dt = 2 fs and two rigid grip layers at
 *     each end of a [100] wire (Simulation details, Figure 1), here with a
 *     Langevin thermostat and a continuously pulled top grip;
 *   - observables: engineering strain (eq 4) and virial stress (eq 5).
 *
 * Conventions common to every call
 * --------------------------------
 * Units: Angstrom, eV, amu, ps, K.  The wire axis [100] is z.
 * Memory: every buffer is owned by the caller.  Pointers documented "device"
 *   are HIP device memory of the current device; "host" pointers are ordinary
 *   host memory read during the call.  The library allocates no device memory
 *   in any call; its scratch lives in the caller's workspace (see
 *   tbsma_workspace_query).
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the default
 *   stream.  Calls enqueue work and return without waiting, except where a
 *   call says it synchronises.
 * Layout: R replicas (independent wires) share one index space of N atom
 *   slots.  Replica r owns slots [rep_off[r], rep_off[r+1]); every offset is a
 *   multiple of TBSMA_TILE, and the slots after a replica's real atoms are
 *   padding (flag TBSMA_PAD).  Per-atom arrays are structure-of-arrays.
 *   Atoms keep their slot for the whole run.  An atom's tag (the counter
 *   word of its random numbers) is tag[slot] when the system has a tag array
 *   (tbsma_system.tag), else the slot minus rep_off[r]; so a replica may
 *   hold its atoms in any fixed order, for instance blocked by space so
 *   that the pair passes can stage the neighbours of each block of slots in
 *   LDS.
 * Errors: calls return TBSMA_OK (0) or a negative code; the message of the
 *   last failure on the calling thread is returned by tbsma_last_error().
 *   Conditions found on the device while running (neighbour-list overflow,
 *   non-finite values, atoms outside their grid, rupture) are per-replica
 *   status bits, not return codes; tbsma_step and tbsma_run_batch also turn
 *   an overflow into TBSMA_ECAPACITY when they return.
 *   No C++ exception crosses this interface.
 */
#ifndef TBSMA_H
#define TBSMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TBSMA_TILE 64 /* atom-slot granularity of a replica (one wavefront) */
#define TBSMA_NOBS 10 /* doubles per observable record */

/* return codes */
#define TBSMA_OK 0
#define TBSMA_EINVAL (-1)    /* invalid argument or inconsistent sizes */
#define TBSMA_ECAPACITY (-2) /* neighbour-list rows too short */
#define TBSMA_EHIP (-3)      /* a HIP runtime call failed */
#define TBSMA_EDEVICE (-4)   /* current device is not gfx950 */

/* precision of the pair arithmetic */
#define TBSMA_FP64 0  /* everything in FP64 */
#define TBSMA_MIXED 1 /* FP32 pair math and forces; FP64 x, v, sums, grips */

/* per-atom flags */
#define TBSMA_DYN 0        /* integrated */
#define TBSMA_GRIP_FIXED 1 /* rigid bottom grip, held at its reference */
#define TBSMA_GRIP_PULL 2  /* rigid top grip, moved along +z at v_pull */
#define TBSMA_PAD 3        /* padding slot, no atom */

/* per-replica status bits (tbsma_md.status) */
#define TBSMA_ST_OVERFLOW 1u   /* a neighbour-list row exceeded k_cap */
#define TBSMA_ST_NONFINITE 2u  /* NaN/Inf in energy or kinetic energy (logged
                                  steps; every step with Nose-Hoover or the
                                  barostat) */
#define TBSMA_ST_OUTSIDE 4u    /* an atom left its cell grid (still exact) */
#define TBSMA_ST_RUPTURED 8u   /* axial gap >= r_cut found at a logged step */
#define TBSMA_ST_REBUILT 16u   /* neighbour list rebuilt at some step */
#define TBSMA_ST_DONE 32u      /* retired: the pulled grip moved `retire` A
                                  past the rupture; the replica is frozen */

/* observable record (tbsma_md.obs), TBSMA_NOBS doubles */
#define TBSMA_OBS_STEP 0    /* step index of the state */
#define TBSMA_OBS_EPOT 1    /* potential energy, eq 3 (eV) */
#define TBSMA_OBS_KE 2      /* kinetic energy of dynamic atoms, peculiar (eV) */
#define TBSMA_OBS_T 3       /* temperature, 3 N_dyn - 3 degrees of freedom */
#define TBSMA_OBS_WZZ 4     /* 1/2 sum_i sum_j E'_ij dz^2 / r (eV) */
#define TBSMA_OBS_SZZ 5     /* virial stress sigma_zz of eq 5 (GPa) */
#define TBSMA_OBS_STRAIN 6  /* engineering strain of eq 4 */
#define TBSMA_OBS_GAP 7     /* largest empty axial gap, exact when >= cell/2 */
#define TBSMA_OBS_D 8       /* displacement of the pulled grip (A) */
#define TBSMA_OBS_STATUS 9  /* status bits of the replica at that step */

/*
 * Potential and list parameters (Methods, Table 1).
 *  A, xi, p, q, r0  Table 1 (Au: 0.2061 eV, 1.790 eV, 10.229, 4.036, 2.884 A).
 *  r_tail, r_cut    each radial function is the exponential of eq 1 / eq 2 up
 *                   to r_tail and a cubic Hermite tail reaching value and slope
 *                   zero at r_cut; r_tail == r_cut is the paper's hard cut.
 *  skin             Verlet skin; lists hold pairs with r < r_cut + skin.
 *  cell             cell edge (>= r_cut + skin, and cell/2 <= r_cut).
 *  mass             atomic mass (amu).
 *  precision        TBSMA_FP64 or TBSMA_MIXED.
 *  qbits            MIXED only: positions are quantised to 2^-qbits A about
 *                   the centre of each replica's grid (16 <= qbits <= 24);
 *                   the grid half-extent must stay below 2^(31-qbits) A.
 *  prune            MIXED only: half-width d (A) of the pruned lists the pair
 *                   passes read, 0 <= d <= skin/2 (0: no pruning).  Each list
 *                   is pruned to the pairs within r_cut + 2d, and pruned again
 *                   from the full list whenever some atom of the replica has
 *                   moved more than d since the last pruning, so no pair
 *                   within r_cut is ever left out.  The pairs within
 *                   r_cut - m at the last build, m = min(skin/2, 0.8 A), are
 *                   kept without a test until the next one (such a pair
 *                   leaves r_cut + 2d only when stretched by more than
 *                   m + 2d, and contributes nothing beyond r_cut).
 *  gather           MIXED only, 0 or 1: 1 lets a block of the pair passes
 *                   whose slot window is too wide for LDS (thick wires)
 *                   stage the exact set of its neighbours instead, through
 *                   a list of up to 1536 neighbour offsets kept in the
 *                   workspace (about 12 bytes per slot more workspace).
 *                   Results do not depend on it: the pair arithmetic is the
 *                   same whichever way positions reach it.
 *  rebuild_exact    0 or 1.  A replica's lists are rebuilt once some atom
 *                   may have moved more than skin/2 since the last build.
 *                   With pruning (MIXED, prune > 0) and 0, the position
 *                   update bounds each atom's displacement since the build
 *                   by its displacement since the last pruning plus the one
 *                   since the build recorded at that pruning, and does not
 *                   read the build positions; lists then rebuild a little
 *                   sooner.  With 1, or without pruning, it tests the FP64
 *                   distance from the build positions (x_ref, y_ref, z_ref),
 *                   so that runs with and without pruning rebuild on the
 *                   same steps.
 */
typedef struct {
  double A, xi, p, q, r0;
  double r_tail, r_cut;
  double skin;
  double cell;
  double mass;
  int32_t precision;
  int32_t qbits;
  double prune;
  int32_t gather;
  int32_t rebuild_exact;
} tbsma_params;

/*
 * Atoms and the replica layout.
 *  R, N          replicas, atom slots (N = rep_off_h[R], multiple of TILE).
 *  C             cells of all replica grids (C = cell_off_h[R]).
 *  max_zbins     axial bins per replica for the rupture gap (>= 2 gz of every
 *                replica).
 *  rep_off_h     host [R+1] slot offsets (non-decreasing multiples of TILE).
 *  cell_off_h    host [R+1] cell offsets, cell_off_h[r+1]-cell_off_h[r] =
 *                gx*gy*gz of replica r.
 *  rep_off, cell_off   device copies of the two arrays above.
 *  tile_rep      device [N/TILE]: replica of each tile of TILE slots.
 *  grid_dim      device [3R] int: cells along x, y, z of each replica.
 *  grid_lo       device [3R] double: lower corner of each replica's grid.
 *  rep_id        device [R]: persistent replica id (random-counter word).
 *  x, y, z       device [N] FP64 positions.
 *  vx, vy, vz    device [N] FP64 velocities (A/ps).
 *  z0            device [N] FP64 reference z of grip atoms (set by
 *                tbsma_init_state).
 *  flag          device [N] TBSMA_DYN / GRIP_FIXED / GRIP_PULL / PAD.
 *  qpos          device [4N] int32 (MIXED; NULL for FP64): quantised x, y, z
 *                and, after the density pass, the bits of FP32 g_i.
 *  tag           device [N] int32 or NULL: tag of the atom in each slot,
 *                0 <= tag < atoms of its replica, distinct within a replica
 *                (NULL: slot minus rep_off[r]).
 *  shape_h, shape  host and device copies of [R] int32, or both NULL: the
 *                launch shape of each replica's pair-pass blocks,
 *                TBSMA_SHAPE(tiles_per_block, stage_class) with
 *                tiles_per_block 1, 2 or 4 and stage_class 0 (1152 staged
 *                neighbour positions per block) or 1 (1536).  NULL means
 *                TBSMA_SHAPE(4, 1) for every replica.  Shapes change how
 *                work is laid out on the GPU, never a result bit: per-bucket
 *                choices of an autotuner coexist in one batch.  A workspace
 *                belongs to the shapes it was sized and initialised for.
 */
#define TBSMA_SHAPE(tiles_per_block, stage_class) \
  ((tiles_per_block) | ((stage_class) << 4))
typedef struct {
  int32_t R;
  int32_t max_zbins;
  int64_t N;
  int64_t C;
  const int64_t *rep_off_h;
  const int64_t *cell_off_h;
  const int64_t *rep_off;
  const int64_t *cell_off;
  const int32_t *tile_rep;
  const int32_t *grid_dim;
  const double *grid_lo;
  const int32_t *rep_id;
  double *x, *y, *z;
  double *vx, *vy, *vz;
  double *z0;
  uint8_t *flag;
  int32_t *qpos;
  const int32_t *tag;
  const int32_t *shape_h;
  const int32_t *shape;
} tbsma_system;

/*
 * Cell lists.  cell_start: device [C + R] int32.  For replica r and local
 * cell c (c = (cz*gy + cy)*gx + cx), the slots of its atoms are
 * cell_atoms[cell_start[cell_off[r]+r+c] .. cell_start[cell_off[r]+r+c+1]),
 * in ascending slot order.  cell_atoms: device [N] int32, the permutation
 * of each replica's slots sorted by cell (the atom arrays themselves are not
 * reordered by a build: their slot order is fixed when the system is laid
 * out, see Layout above).
 */
typedef struct {
  int32_t *cell_start;
  int32_t *cell_atoms;
} tbsma_cells;

/*
 * Verlet lists (full: both i->j and j->i), stored in chunks of 8 entries:
 * entry k of atom i is nl[((k/8)*N + i)*8 + k%8], k < nn[i] <= k_cap, in
 * an order fixed by the positions alone: cell-scan order (cells by z, y, x;
 * slots ascending within a cell) in FP64; in MIXED, the pairs within
 * r_cut - min(skin/2, 0.8 A) first, then the others, each part in that order within each of eight
 * interleaved shares of the candidate scan (groups of 8 candidates, or
 * every eighth of the 27 cells when a tile's candidates exceed LDS),
 * shares in turn.  The entries nn[i] <= k < 8*ceil(nn[i]/8) of an atom's last chunk
 * hold 0x7fffffff.
 * nl: device [k_cap*N] int32; k_cap must be a multiple of 8.
 * x_ref, y_ref, z_ref: device [N] positions at the last build.
 * nact (optional, MIXED only; NULL to skip): device [2N] int32, rewritten
 * by every density pass when given: the numbers of list entries of atom i
 * with 0 < r <= r_tail (nact[2i]) and r_tail < r < r_cut (nact[2i+1]) at
 * the current positions.  A diagnostic: the passes are faster without it.
 * nl_lane (MIXED; NULL for FP64): device [k_cap*N] int32, the lists as the
 * mixed pair passes read them: within each block of up to four tiles of one
 * replica, atoms by descending list length (ties by slot), the p-th atom's
 * list as row (block start + p) of the same chunked layout, pruned to the
 * pairs within r_cut + 2 prune and those kept without a test (see
 * tbsma_params.prune), in the order of nl, each entry encoded as
 * the byte offset 16 (j - lo) of neighbour j from the start lo of the
 * block's slot window, or, in a block staged through its gather list
 * (tbsma_params.gather), 16 times the neighbour's rank in that list.
 * Written by the list build and by the pruning in the step loops; opaque to
 * the caller (save and restore it as a whole, with the workspace, which
 * holds the lane order, the gather lists and the positions at the last
 * pruning).
 */
typedef struct {
  int32_t *nl;
  int32_t *nn;
  int32_t k_cap;
  int32_t reserved;
  double *x_ref, *y_ref, *z_ref;
  int32_t *nact;
  int32_t *nl_lane;
} tbsma_nlist;

/*
 * Force-pass outputs.  fx, fy, fz, e_atom: device [N], float for MIXED and
 * double for FP64.  g: device [N] double, FP64 only (1/sqrt(rho_i), 0 when
 * rho_i = 0); NULL for MIXED.  rep_energy, rep_wzz: device [R] double, written
 * by tbsma_forces: sum of E_i (eq 3) and 1/2 sum_i sum_j E'_ij dz^2/r.
 */
typedef struct {
  void *fx, *fy, *fz;
  void *e_atom;
  double *g;
  double *rep_energy;
  double *rep_wzz;
} tbsma_forces_out;

/*
 * Dynamics settings and observables.
 *  dt, gamma     time step (ps) and Langevin friction (1/ps; 0 = no Langevin
 *                thermostat).
 *  lab_frame     0: the thermostat acts on the velocity relative to the
 *                affine stretching profile u(z) = v_pull (z - z_lo) /
 *                (z_hi - z_lo + D); 1: on the lab-frame velocity.
 *  n_log         observables are recorded when the new step index is a
 *                multiple of n_log (>= 1);  n_slots: ring slots per replica.
 *  T, v_pull, z_lo, z_hi, vol, L0: device [R] double: target temperature,
 *                grip speed, inner faces of the fixed and pulled grips at
 *                t = 0, constant hard-sphere volume (eq 5), initial length
 *                (eq 4).
 *  seed          device [R] uint64: Philox key of each replica.
 *  dof           device [R] int32: kinetic degrees of freedom (3 N_dyn - 3).
 *  step          device [1] int64: index of the current state; advanced by
 *                one per step on the device.
 *  obs           device [n_slots * R * TBSMA_NOBS]: record of replica r at
 *                logged step s is at ((s / n_log) % n_slots) * R + r.
 *  status        device [R] uint32 status bits (OR-accumulated).
 *  retire        grip travel (A) after the first logged step at which the
 *                replica is ruptured, beyond which it is retired: status
 *                TBSMA_ST_DONE, and the step loops leave its atoms, lists and
 *                forces untouched (its record repeats at later logged steps).
 *                0 or less: never retire.
 *  dfail         device [R] double: grip displacement D at the first logged
 *                step at which the replica was ruptured (its failure point;
 *                strain D/L0, eq 4), -1 before that.  Set it to -1 when the
 *                run starts.  May be NULL when retire <= 0.
 *  nh_tau        Nose-Hoover thermostat (Simulation details) when > 0 (ps;
 *                needs gamma = 0): one friction zeta per replica acting on
 *                the peculiar velocities of the dynamic atoms,
 *                dzeta/dt = (2K / (g kB T) - 1) / nh_tau^2 (g = dof[r]),
 *                integrated by the symmetric Trotter splitting: a thermostat
 *                half step before and after each velocity Verlet step.
 *                Replicas with T <= 0 or dof <= 0 are not thermostatted.
 *  nh_xi         device [R] double: zeta (1/ps) at the current step, read
 *                and updated by the step loops (zero it to start).  Needed
 *                when nh_tau > 0.
 *  nh_eta        device [R] double or NULL: the time integral of zeta, with
 *                which E_pot + K + Q zeta^2/2 + g kB T eta (Q = g kB T
 *                nh_tau^2) is conserved while the grips rest.
 *                Each step-loop call starts from the velocities as they are
 *                (it sums the kinetic energy afresh), so runs split into
 *                different calls agree to rounding, not bit for bit.
 *  grip_step, grip_hold
 *                grip_hold > 0 selects the stepwise symmetric grips of
 *                Simulation details: each hold of grip_hold steps begins with
 *                the TBSMA_GRIP_FIXED atoms moving grip_step (A) along -z and
 *                the TBSMA_GRIP_PULL atoms grip_step along +z; grips rest in
 *                between and v_pull is not used.  grip_hold = 0: the bottom
 *                grip rests and the top one moves at v_pull.  The elongation
 *                D of eq 4 is the sum of both grips' travel.
 *  T_start, ramp_begin, ramp_steps
 *                temperature ramp of the equilibration (Simulation details):
 *                when ramp_steps > 0 the target temperature of replica r at
 *                time t (in steps) is T_start[r] + (T[r] - T_start[r]) *
 *                clamp((t - ramp_begin) / ramp_steps, 0, 1) (T_start: device
 *                [R] double); otherwise it is T[r].  The Langevin O step takes
 *                it at mid-step, the Nose-Hoover half steps at the start and
 *                end of the step, tbsma_init_state at step 0.
 *  baro_mass, baro_load, baro_damp, baro_s
 *                axial barostat of the equilibration (Simulation details:
 *                zero pressure along [100]), on the grip separation: when
 *                baro_mass > 0 (amu; needs grip_hold = 0; v_pull is not
 *                used) both grips move outwards by s[r], an extended
 *                coordinate with baro_mass d2s/dt2 = Q + 2 baro_load, where
 *                Q = sum_top F_z - sum_bottom F_z = -dE/ds and baro_load
 *                (eV/A) is the outward pull on each grip (0: zero axial
 *                load), integrated by velocity Verlet with the atoms; ds/dt
 *                is multiplied by exp(-baro_damp dt/2) (baro_damp in 1/ps)
 *                before its first and after its second half kick of each
 *                step.  baro_s: device [2R] double, s and ds/dt of each
 *                replica, read and updated (zero them to start; the grips
 *                must then sit at z0).  The elongation D is 2 s.
 */
typedef struct {
  double dt, gamma;
  int32_t lab_frame;
  int32_t n_log;
  int32_t n_slots;
  int32_t reserved;
  const double *T, *v_pull, *z_lo, *z_hi, *vol, *L0;
  const uint64_t *seed;
  const int32_t *dof;
  int64_t *step;
  double *obs;
  uint32_t *status;
  double retire;
  double *dfail;
  double nh_tau;
  double *nh_xi;
  double *nh_eta;
  double grip_step;
  int64_t grip_hold;
  const double *T_start;
  int64_t ramp_begin;
  int64_t ramp_steps;
  double baro_mass;
  double baro_load;
  double baro_damp;
  double *baro_s;
} tbsma_md;

/*
 * Bytes of device workspace that every call below takes as `work` for this
 * system (per-replica displacement maxima, cell counters, per-tile partial
 * sums, axial bins).  Host-only; returns TBSMA_EINVAL on bad sizes.
 */
int tbsma_workspace_query(const tbsma_params *prm, const tbsma_system *sys,
                          size_t *bytes);

/*
 * Puts a freshly allocated workspace into its initial state (enqueued on
 * stream).  Call once after allocating it, before any other call uses it.
 */
int tbsma_workspace_init(const tbsma_params *prm, const tbsma_system *sys,
                         void *work, void *stream);

/*
 * Host-side wire builder (Simulation details, Figure 1): the [100] FCC
 * cylinder of lattice constant a, diameter D and length L with the axis
 * through an atom column; sites (i, j, k) a/2 with i+j+k even,
 * i^2 + j^2 <= (D/a)^2 and 0 <= k a/2 < L, in (k, j, i) order (planes along
 * the axis, then rows, then columns); the n_grip lowest planes get
 * TBSMA_GRIP_FIXED and the n_grip highest TBSMA_GRIP_PULL.
 * Ring notch (Figure 1: three atoms wide, two deep): of the K planes, planes
 * K/2 - notch_layers/2 ... K/2 - notch_layers/2 + notch_layers - 1 (integer
 * division) lose every site farther than D/2 - notch_depth (A) from the
 * axis; notch_layers = 0 builds no notch.
 * x, y, z, flag are host arrays of capacity cap (may be NULL when cap = 0).
 * *n_out receives the atom count; TBSMA_ECAPACITY if it exceeds cap.
 */
int tbsma_build_wire(double a, double D, double L, int32_t n_grip,
                     int32_t notch_layers, double notch_depth, double *x,
                     double *y, double *z, uint8_t *flag, int64_t cap,
                     int64_t *n_out);

/*
 * Initial state (Simulation details: random Gaussian velocities): every
 * real atom's position gets a uniform jitter of +-jitter per component
 * (Philox stream 2); dynamic atoms get Maxwell-Boltzmann velocities at T[r]
 * (stream 1), minus their centre-of-mass velocity, rescaled to exactly T[r]
 * over dof[r], plus the stretching profile at t = 0; fixed grips are at rest
 * and pulled grips move at v_pull (rest with stepwise grips).  Sets z0 = z
 * and *step = 0.  Synchronises the stream.
 */
int tbsma_init_state(const tbsma_params *prm, tbsma_system *sys,
                     const tbsma_md *md, void *work, double jitter,
                     void *stream);

/*
 * Per-replica constants of the dynamics and observables, from the atoms in
 * their current slots (flags and z; call it before tbsma_init_state's jitter
 * to take them from the lattice sites), written to device arrays [R]:
 *  dof   3 N_dyn - 3, the kinetic degrees of freedom of the temperature
 *        (N_dyn dynamic atoms; 0 when N_dyn <= 1; Simulation details'
 *        thermostat, the temperature in the observables);
 *  vol   eq 5's constant volume N (4/3) pi (r0/2)^3 over the replica's N
 *        atoms (hard spheres of radius r0/2: the paper leaves the radius
 *        unstated);
 *  z_lo, z_hi  the inner faces of the fixed and pulled grips at this state
 *        (largest z of the TBSMA_GRIP_FIXED atoms, smallest z of the
 *        TBSMA_GRIP_PULL atoms; the replica's lowest / highest z when it has
 *        no such grip), which anchor the stretching profile of tbsma_md.
 * They are tbsma_md's dof, vol, z_lo and z_hi.  Counts, minima and maxima
 * are exact, so results do not depend on the device's reduction order.
 */
int tbsma_replica_constants(const tbsma_params *prm, const tbsma_system *sys,
                            int32_t *dof, double *vol, double *z_lo,
                            double *z_hi, void *stream);

/*
 * The current state as the start of a new stretch (after equilibration,
 * Simulation details): every atom's grip reference z0 = z, and for each
 * replica the initial length of eq 4 grows by the barostat's elongation,
 * L0[r] += 2 s[r], with s[r] and ds/dt then zeroed (baro_s: device [2R] as in
 * tbsma_md, or NULL to leave L0 as it is).  L0: device [R].  The step index,
 * status and records are the caller's to reset.
 */
int tbsma_rebase(const tbsma_params *prm, tbsma_system *sys, double *L0,
                 double *baro_s, void *stream);

/*
 * Cell binning (the cell list behind the Verlet list): bins every real atom
 * of every replica into its grid (atoms outside are clamped to the border
 * cells, which keeps the list exact, and raise TBSMA_ST_OUTSIDE in the
 * workspace only) and writes cell_start / cell_atoms.
 */
int tbsma_build_cells(const tbsma_params *prm, const tbsma_system *sys,
                      tbsma_cells *cells, void *work, void *stream);

/*
 * Verlet lists of every replica from its cells: all j != i of the same
 * replica with |r_j - r_i| < r_cut + skin; stores the positions as x_ref.
 * When need_cap is non-NULL the call synchronises and, if a row exceeded
 * k_cap, writes the longest row length to *need_cap and returns
 * TBSMA_ECAPACITY (rows are then truncated and must be rebuilt).
 */
int tbsma_neighbors(const tbsma_params *prm, const tbsma_system *sys,
                    const tbsma_cells *cells, tbsma_nlist *nl, void *work,
                    int32_t *need_cap, void *stream);

/*
 * Energies and forces of eqs 1-3 in two passes over the Verlet list:
 * pass 1 rho_i -> g_i = 1/sqrt(rho_i); pass 2
 * F_i = sum_j E'_ij (r_j - r_i)/r_ij with E'_ij = 2V'(r) - (g_i+g_j)phi'(r)/2,
 * E_i = -sqrt(rho_i) + sum_j V(r_ij), and per-replica sums of E_i and of the
 * zz virial into out->rep_energy / out->rep_wzz.
 */
int tbsma_forces(const tbsma_params *prm, const tbsma_system *sys,
                 const tbsma_nlist *nl, tbsma_forces_out *out, void *work,
                 void *stream);

/*
 * One of the two passes of tbsma_forces on its own, for timing and for
 * callers that keep g: pass 1 is the density pass (writes g_i), pass 2 the
 * force pass (reads the g_i of pass 1, writes forces, energies and the
 * per-tile sums; no per-replica reduction), pass 3 the force pass as the
 * MIXED step loops run it on steps that are not logged (forces only; e_atom
 * and the tile sums untouched; in FP64 the same as pass 2).  In MIXED
 * precision all read the quantised positions in qpos as last written by the
 * library (every call that moves atoms or builds lists keeps them current).
 * TBSMA_EINVAL for any other pass number.
 */
int tbsma_forces_pass(const tbsma_params *prm, const tbsma_system *sys,
                      const tbsma_nlist *nl, tbsma_forces_out *out, void *work,
                      int32_t pass, void *stream);

/*
 * n_steps MD steps of every replica, one launch per kernel per step (the
 * plain path; with R = 1 it is one replica per launch).  Each step:
 * [Nose-Hoover half step], half kick, half drift, Langevin O step (noise
 * counter (tag, step, rep_id, 0)), half drift, grips placed at z0 minus the
 * bottom grip's travel (TBSMA_GRIP_FIXED) or z0 plus the top grip's travel
 * (TBSMA_GRIP_PULL) after step+1 steps;
 * per-replica rebuild of cells and lists where some atom moved more than
 * skin/2 since the last build; both force passes; half kick; per-replica
 * reductions and observables.  Forces in `out` must hold F at the current
 * state on entry (tbsma_forces).  With Nose-Hoover, the half step that ends
 * one step and the one that begins the next act as one velocity scale, and
 * the last end-of-step half step is applied when the call ends.  Forces are
 * rewritten every step; in MIXED
 * precision the per-atom energies e_atom (and the energy and virial behind
 * the observables) are evaluated only on logged steps ((step+1) % n_log ==
 * 0), so after a call e_atom belongs to the last logged step.  Synchronises
 * at the end and returns TBSMA_ECAPACITY if any list overflowed during the
 * call.
 */
int tbsma_step(const tbsma_params *prm, tbsma_system *sys, tbsma_cells *cells,
               tbsma_nlist *nl, tbsma_forces_out *out, const tbsma_md *md,
               void *work, int64_t n_steps, void *stream);

/*
 * The same n_steps as tbsma_step for all replicas, captured once as a HIP
 * graph of steps_per_graph steps and replayed (the last partial chunk is
 * launched directly).  Every decision (rebuilds, logging, step index) is
 * taken on the device, so replays need no host work.  The instantiated graph
 * is cached for identical arguments.  Synchronises at the end and returns
 * TBSMA_ECAPACITY if any list overflowed.
 */
int tbsma_run_batch(const tbsma_params *prm, tbsma_system *sys,
                    tbsma_cells *cells, tbsma_nlist *nl,
                    tbsma_forces_out *out, const tbsma_md *md, void *work,
                    int64_t n_steps, int32_t steps_per_graph, void *stream);

/*
 * For callers that cannot allocate device memory or hold a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): tbsma_step with the library's own device scratch of
 * TBSMA_NOALLOC_SCRATCH_BYTES in place of `work`.  The scratch is a static
 * array of the library, one per device, held until the process ends; the
 * call allocates nothing.
 * Because the scratch keeps whatever the previous call on the device left
 * there, each call first puts it into its initial state (as
 * tbsma_workspace_init), bins and lists every replica afresh at the current
 * positions (tbsma_build_cells, tbsma_neighbors), evaluates the forces there
 * (tbsma_forces: out, including rep_energy and rep_wzz, is written), then
 * runs the n_steps steps of tbsma_step.  The result equals that sequence on a
 * freshly initialised workspace.  n_steps = 0 does nothing.
 * Errors: TBSMA_ECAPACITY when the system's workspace
 * (tbsma_workspace_query) exceeds TBSMA_NOALLOC_SCRATCH_BYTES, before any
 * work is enqueued; TBSMA_ECAPACITY after the steps if a list row exceeded
 * k_cap (as tbsma_step).  Synchronises at the end.
 * Every call on one device shares the same scratch: calls that overlap on a
 * device (different streams or host threads) race and must be serialised.
 */
#define TBSMA_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int tbsma_step_noalloc(const tbsma_params *prm, tbsma_system *sys,
                       tbsma_cells *cells, tbsma_nlist *nl,
                       tbsma_forces_out *out, const tbsma_md *md,
                       int64_t n_steps, void *stream);

/*
 * Diagnostics of the lists, out_host[6]: [0] sum over atoms of nn (the
 * Verlet lists), [1] sum of the lengths of the lists the mixed pair passes
 * read (pruned; equal to [0] in FP64); MIXED only (0 in FP64): how the pair
 * passes reach each block's neighbours: [2] blocks whose slot window fits in
 * LDS, [3] blocks staged through a gather list (tbsma_params.gather), [4]
 * blocks that gather from global memory, [5] neighbours listed by the
 * gather-staged blocks.  Synchronises.
 */
int tbsma_list_stats(const tbsma_params *prm, const tbsma_system *sys,
                     const tbsma_nlist *nl, void *work, int64_t *out_host,
                     void *stream);

/*
 * Diagnostics of the random numbers: for tag = 0 .. n-1 writes the four
 * Philox4x32-10 words of counter (tag, lo32(step), rep_id, stream_id) under
 * key (lo32(seed), hi32(seed)) to out_u32[4 tag ..] and the three Box-Muller
 * normals to out_gauss[3 tag ..] (device buffers; either may be NULL).
 */
int tbsma_rng_fill(uint64_t seed, uint32_t rep_id, uint64_t step,
                   uint32_t stream_id, int64_t n, uint32_t *out_u32,
                   double *out_gauss, void *stream);

/*
 * The three FP32 normals that the MIXED Langevin O step draws for counter
 * (tag, lo32(step), rep_id, stream_id) and key (lo32(seed), hi32(seed)),
 * tag = 0 .. n-1, written to out_gauss[3 tag ..] (device buffer): the same
 * Philox words and Box-Muller form as tbsma_rng_fill, in FP32, each within
 * a few FP32 ulp of the FP64 normal (the noise of Simulation details'
 * thermostat, replayable from its counter).
 */
int tbsma_rng_normals_f32(uint64_t seed, uint32_t rep_id, uint64_t step,
                          uint32_t stream_id, int64_t n, float *out_gauss,
                          void *stream);

/*
 * Counters of the step loops (tbsma_step, tbsma_run_batch) since the
 * workspace was initialised: out_host[0] = replica neighbour-list rebuilds,
 * out_host[1] = replica prunings of the pair-pass lists without a rebuild.
 * Diagnostics; synchronises.
 */
int tbsma_event_counts(const tbsma_params *prm, const tbsma_system *sys,
                   void *work, int64_t *out_host, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *tbsma_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TBSMA_H */
