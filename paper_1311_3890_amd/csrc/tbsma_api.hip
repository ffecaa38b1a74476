// C ABI of libtbsma (declared in include/tbsma.h): argument checks,
// workspace layout, constant folding for the kernels, the plain step loop
// and the graph-captured batched loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <algorithm>
#include <vector>

#include "tbsma.h"
#include "tbsma_device.hpp"
#include "tbsma_kernels.hpp"

using namespace tbsma;

// Device scratch of tbsma_step_noalloc, in place of a caller's workspace.
// In host code `scratch` names a host-side stand-in, not device memory:
// kernels and copies get the address that hipGetSymbolAddress returns for
// the current device (each device holds its own copy of the array).
static_assert(TBSMA_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
constexpr size_t kScratchBytes = TBSMA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(TBSMA_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

// The kernels are built for gfx950 only.
int check_device() {
  static std::mutex mu;
  static int known[64] = {0};  // 0 unknown, 1 ok, 2 bad
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(TBSMA_EDEVICE, "device %d", dev);
  std::lock_guard<std::mutex> lk(mu);
  if (known[dev] == 0) {
    hipDeviceProp_t p;
    HIPCHK(hipGetDeviceProperties(&p, dev));
    known[dev] = strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  if (known[dev] != 1)
    return fail(TBSMA_EDEVICE, "libtbsma is built for gfx950 only");
  return TBSMA_OK;
}

int check_params(const tbsma_params *p) {
  if (!p) return fail(TBSMA_EINVAL, "params is NULL");
  if (!(p->r0 > 0 && p->A > 0 && p->xi > 0 && p->p > 0 && p->q > 0))
    return fail(TBSMA_EINVAL, "potential parameters must be positive");
  if (!(p->r_tail > 0 && p->r_tail <= p->r_cut))
    return fail(TBSMA_EINVAL, "need 0 < r_tail <= r_cut");
  if (!(p->skin >= 0)) return fail(TBSMA_EINVAL, "skin must be >= 0");
  if (!(p->cell >= p->r_cut + p->skin))
    return fail(TBSMA_EINVAL, "cell edge %g < r_cut + skin", p->cell);
  if (!(0.5 * p->cell <= p->r_cut))
    return fail(TBSMA_EINVAL, "cell/2 must not exceed r_cut");
  if (!(p->mass > 0)) return fail(TBSMA_EINVAL, "mass must be positive");
  if (p->precision != TBSMA_FP64 && p->precision != TBSMA_MIXED)
    return fail(TBSMA_EINVAL, "unknown precision %d", p->precision);
  if (p->precision == TBSMA_MIXED && (p->qbits < 16 || p->qbits > 24))
    return fail(TBSMA_EINVAL, "qbits %d outside 16..24", p->qbits);
  if (!(p->prune >= 0 && p->prune <= 0.5 * p->skin))
    return fail(TBSMA_EINVAL, "prune must be in [0, skin/2]");
  if (p->gather != 0 && p->gather != 1)
    return fail(TBSMA_EINVAL, "gather must be 0 or 1");
  if (p->rebuild_exact != 0 && p->rebuild_exact != 1)
    return fail(TBSMA_EINVAL, "rebuild_exact must be 0 or 1");
  return TBSMA_OK;
}

int check_system(const tbsma_params *p, const tbsma_system *s) {
  if (!s) return fail(TBSMA_EINVAL, "system is NULL");
  if (s->R < 0 || s->N < 0 || s->C < 0)
    return fail(TBSMA_EINVAL, "negative sizes");
  if (s->R == 0) return TBSMA_OK;
  if (s->N % TBSMA_TILE) return fail(TBSMA_EINVAL, "N not a multiple of 64");
  if (s->N >= (int64_t)1 << 31) return fail(TBSMA_EINVAL, "N >= 2^31");
  if (!s->rep_off_h || !s->cell_off_h)
    return fail(TBSMA_EINVAL, "host offsets missing");
  if (s->rep_off_h[0] != 0 || s->rep_off_h[s->R] != s->N)
    return fail(TBSMA_EINVAL, "rep_off must run from 0 to N");
  if (s->cell_off_h[0] != 0 || s->cell_off_h[s->R] != s->C)
    return fail(TBSMA_EINVAL, "cell_off must run from 0 to C");
  for (int r = 0; r < s->R; ++r) {
    if (s->rep_off_h[r + 1] < s->rep_off_h[r] ||
        s->rep_off_h[r] % TBSMA_TILE)
      return fail(TBSMA_EINVAL, "rep_off[%d] not a non-decreasing "
                  "multiple of 64", r);
    if (s->cell_off_h[r + 1] <= s->cell_off_h[r])
      return fail(TBSMA_EINVAL, "replica %d has no cells", r);
  }
  if (s->C + s->R >= (int64_t)1 << 31)
    return fail(TBSMA_EINVAL, "too many cells");
  if ((s->shape_h == nullptr) != (s->shape == nullptr))
    return fail(TBSMA_EINVAL, "shape_h and shape must both be given or both NULL");
  if (s->shape_h)
    for (int r = 0; r < s->R; ++r) {
      const int32_t sh = s->shape_h[r];
      const int tpb = shape_tpb(sh), cls = shape_cls(sh);
      if ((tpb != 1 && tpb != 2 && tpb != 4) || cls >= kStageClasses ||
          (sh & ~0xff) != 0)
        return fail(TBSMA_EINVAL, "shape of replica %d (%d) is not a valid "
                    "launch shape", r, sh);
    }
  if (s->max_zbins < 2) return fail(TBSMA_EINVAL, "max_zbins < 2");
  if (!s->rep_off || !s->cell_off || !s->tile_rep || !s->grid_dim ||
      !s->grid_lo || !s->rep_id || !s->x || !s->y || !s->z || !s->vx ||
      !s->vy || !s->vz || !s->z0 || !s->flag)
    return fail(TBSMA_EINVAL, "a device array of the system is NULL");
  if (p && p->precision == TBSMA_MIXED && !s->qpos)
    return fail(TBSMA_EINVAL, "mixed precision needs qpos");
  if (p && p->precision == TBSMA_MIXED && s->N >= (int64_t)1 << 28)
    return fail(TBSMA_EINVAL, "mixed precision needs N < 2^28");
  return TBSMA_OK;
}

struct Layout {
  size_t rflag, cnt, part, zbmin, zbmax, wstatus, nnmax, rsum, win,
      bmap, boff, cbmap, lane_atom, nn_lane, qprune, atom_lane, ncore, stats, nhw,
      baw, wl, callb, gcnt, glist, total;
};

// Blocks of the cell sort: ceil(cells/kSortCells) per replica.
int32_t cell_map_size(const tbsma_system *s) {
  int64_t nb = 0;
  for (int r = 0; r < s->R; ++r)
    nb += (s->cell_off_h[r + 1] - s->cell_off_h[r] + kSortCells - 1) /
          kSortCells;
  return (int32_t)nb;
}

int32_t host_shape(const tbsma_system *s, int r) {
  return s->shape_h ? s->shape_h[r] : kShapeDefault;
}

// Blocks of the list build and pair passes: ceil(tiles / tpb) per replica;
// per stage class when cls is given (cls[c] = blocks of class c).
int32_t block_map_size(const tbsma_system *s, int64_t *cls = nullptr) {
  int64_t nb = 0;
  if (cls)
    for (int c = 0; c < kStageClasses; ++c) cls[c] = 0;
  for (int r = 0; r < s->R; ++r) {
    const int64_t nt = (s->rep_off_h[r + 1] - s->rep_off_h[r]) / TBSMA_TILE;
    const int32_t sh = host_shape(s, r);
    const int64_t v = (nt + shape_tpb(sh) - 1) / shape_tpb(sh);
    nb += v;
    if (cls) cls[shape_cls(sh)] += v;
  }
  return (int32_t)nb;
}

size_t up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout layout(const tbsma_params *p, const tbsma_system *s) {
  Layout L;
  size_t o = 0;
  int64_t R = s->R, nt = s->N / TBSMA_TILE;
  L.rflag = o;
  o += up(4 * (size_t)R);
  L.cnt = o;
  o += up(4 * (size_t)s->C);
  L.part = o;
  o += up(8 * (size_t)kNPart * nt);
  L.zbmin = o;
  o += up(8 * (size_t)R * s->max_zbins);
  L.zbmax = o;
  o += up(8 * (size_t)R * s->max_zbins);
  L.wstatus = o;
  o += up(4 * (size_t)R);
  L.nnmax = o;
  o += 256;
  L.rsum = o;
  o += up(8 * 8 * (size_t)R);
  L.win = o;
  o += up(8 * (size_t)nt);
  L.bmap = o;
  o += up(8 * ((size_t)block_map_size(s) + 1));
  L.boff = o;
  o += up(4 * (size_t)R);
  L.cbmap = o;
  o += up(16 * (size_t)(s->C / kSortCells + R + 1));
  L.lane_atom = o;
  o += up((size_t)s->N);
  L.nn_lane = o;
  o += up(4 * (size_t)s->N);
  L.qprune = o;
  o += up(16 * (size_t)s->N);
  L.atom_lane = o;
  o += up((size_t)s->N);
  L.ncore = o;
  o += up(4 * (size_t)s->N);
  L.stats = o;
  o += 256;
  L.nhw = o;
  o += up(8 * 5 * (size_t)R);
  L.baw = o;
  o += up(8 * 2 * (size_t)R);
  L.wl = o;
  o += up(4 * (size_t)work_lists_size(s->N, R, s->C));
  L.callb = o;
  o += 256;
  // gather staging of the pair passes (mixed precision)
  const bool gather = p->precision == TBSMA_MIXED && p->gather;
  const size_t nbm = s->R > 0 ? (size_t)block_map_size(s) : 0;
  L.gcnt = o;
  o += gather ? up(4 * nbm) : 0;
  L.glist = o;
  o += gather ? up(2 * (size_t)kStage * nbm) : 0;

  L.total = o;
  return L;
}

Dev make_dev(const tbsma_params *p, const tbsma_system *s, void *work) {
  Dev d;
  memset(&d, 0, sizeof(d));
  d.R = s->R;
  d.max_zbins = s->max_zbins;
  d.N = s->N;
  d.C = s->C;
  d.rep_off = s->rep_off;
  d.cell_off = s->cell_off;
  d.tile_rep = s->tile_rep;
  d.grid_dim = s->grid_dim;
  d.rep_id = s->rep_id;
  d.grid_lo = s->grid_lo;
  d.x = s->x;
  d.y = s->y;
  d.z = s->z;
  d.vx = s->vx;
  d.vy = s->vy;
  d.vz = s->vz;
  d.z0 = s->z0;
  d.flag = s->flag;
  d.qpos = reinterpret_cast<int4 *>(s->qpos);
  Layout L = layout(p, s);
  char *w = static_cast<char *>(work);
  d.rflag = reinterpret_cast<uint32_t *>(w + L.rflag);
  d.cnt = reinterpret_cast<int32_t *>(w + L.cnt);
  d.part = reinterpret_cast<double *>(w + L.part);
  d.zbmin = reinterpret_cast<unsigned long long *>(w + L.zbmin);
  d.zbmax = reinterpret_cast<unsigned long long *>(w + L.zbmax);
  d.wstatus = reinterpret_cast<uint32_t *>(w + L.wstatus);
  d.nnmax = reinterpret_cast<int32_t *>(w + L.nnmax);
  d.rsum = reinterpret_cast<double *>(w + L.rsum);
  d.win = reinterpret_cast<int2 *>(w + L.win);
  d.bmap = reinterpret_cast<int2 *>(w + L.bmap);
  d.cbmap = reinterpret_cast<int4 *>(w + L.cbmap);
  d.ncbmap = s->R > 0 ? cell_map_size(s) : 0;
  d.lane_atom = reinterpret_cast<uint8_t *>(w + L.lane_atom);
  d.nn_lane = reinterpret_cast<int32_t *>(w + L.nn_lane);
  d.qprune = reinterpret_cast<int4 *>(w + L.qprune);
  d.atom_lane = reinterpret_cast<uint8_t *>(w + L.atom_lane);
  d.ncore = reinterpret_cast<int32_t *>(w + L.ncore);
  d.stats = reinterpret_cast<unsigned long long *>(w + L.stats);
  d.nhw = reinterpret_cast<double *>(w + L.nhw);
  d.baw = reinterpret_cast<double *>(w + L.baw);
  d.wl = reinterpret_cast<int32_t *>(w + L.wl);
  d.callb = reinterpret_cast<int64_t *>(w + L.callb);
  d.tag = s->tag;
  d.shape = s->shape;
  d.boff = reinterpret_cast<int32_t *>(w + L.boff);
  {
    int64_t cls[kStageClasses];
    block_map_size(s, cls);
    d.cls_off[0] = 0;
    for (int c = 0; c < kStageClasses; ++c)
      d.cls_off[c + 1] = d.cls_off[c] + (int32_t)cls[c];
  }
  d.gather = p->precision == TBSMA_MIXED && p->gather ? 1 : 0;
  d.gcnt = d.gather ? reinterpret_cast<int32_t *>(w + L.gcnt) : nullptr;
  d.glist = d.gather ? reinterpret_cast<uint16_t *>(w + L.glist) : nullptr;

  if (p->precision == TBSMA_MIXED) {
    // a pair is kept when its quantised distance is below r_cut + 2d, with
    // a margin of 1e-5 A for rounding of positions to quanta and of r^2 to
    // FP32; without pruning every listed pair is kept
    const double q = ldexp(1.0, p->qbits);
    const double rp = p->prune > 0 ? p->r_cut + 2.0 * p->prune + 1e-5
                                   : p->r_cut + p->skin + 1.0;
    d.pruning = p->prune > 0 ? 1 : 0;
    d.rebuild_bound = d.pruning && !p->rebuild_exact ? 1 : 0;
    // the core of the full lists: pairs within r_cut - min(skin/2, 0.8 A) at
    // the build, listed first and kept by every pruning until the next build.
    // They leave the pruning radius only when stretched by more than that
    // margin plus 2d, and a pair beyond r_cut contributes nothing.  The
    // radius does not depend on d, so runs with and without pruning list
    // pairs alike.
    const double rcore = p->r_cut - std::min(0.5 * p->skin, 0.8);
    d.core_r2q = rcore > 0 ? (float)(rcore * rcore * q * q) : 0.0f;
    d.prune_r2q = (float)(rp * rp * q * q);
    d.prune_d2q = (float)(p->prune * p->prune * q * q);
    d.skin_half_q = (float)(0.5 * p->skin * q) - 1.0f;
  }
  d.nbmap = s->R > 0 ? block_map_size(s) : 0;
  d.cell = p->cell;
  d.inv_cell = 1.0 / p->cell;
  d.skin_half2 = 0.25 * p->skin * p->skin;
  d.qscale = ldexp(1.0, p->precision == TBSMA_MIXED ? p->qbits : 0);
  d.inv_qscale = 1.0 / d.qscale;
  d.mass = p->mass;
  d.all = 0;
  d.energies = 1;
  return d;
}

void attach_lists(Dev &d, const tbsma_cells *c, const tbsma_nlist *n) {
  if (c) {
    d.cell_start = c->cell_start;
    d.cell_atoms = c->cell_atoms;
  }
  if (n) {
    d.nl = n->nl;
    d.nn = n->nn;
    d.k_cap = n->k_cap;
    d.xr = n->x_ref;
    d.yr = n->y_ref;
    d.zr = n->z_ref;
    d.nact = n->nact;
    d.nl_lane = n->nl_lane;
  }
}

// Cubic Hermite tail of f = pre exp(-k (r/r0 - 1)) on (r_tail, r_cut], as
// coefficients of t = (r - r_tail)/(r_cut - r_tail).
void hermite(double pre, double k, const tbsma_params *p, double c[4]) {
  double w = p->r_cut - p->r_tail;
  double fs = pre * exp(-k * (p->r_tail / p->r0 - 1.0));
  double ms = -(k / p->r0) * fs * w;
  c[0] = fs;
  c[1] = ms;
  c[2] = -3.0 * fs - 2.0 * ms;
  c[3] = 2.0 * fs + ms;
}

PotD make_potd(const tbsma_params *p) {
  PotD P;
  P.rc = p->r_cut;
  P.rc2 = p->r_cut * p->r_cut;
  P.rt = p->r_tail;
  P.r0 = p->r0;
  P.xi2 = p->xi * p->xi;
  P.A = p->A;
  P.k2q = 2.0 * p->q;
  P.kp = p->p;
  double w = p->r_cut - p->r_tail;
  P.w = w > 0 ? w : 1.0;
  double cf[4], cv[4];
  hermite(P.xi2, P.k2q, p, cf);
  hermite(P.A, P.kp, p, cv);
  P.f0 = cf[0];
  P.f1 = cf[1];
  P.f2 = cf[2];
  P.f3 = cf[3];
  P.v0 = cv[0];
  P.v1 = cv[1];
  P.v2 = cv[2];
  P.v3 = cv[3];
  return P;
}

PotF make_potf(const tbsma_params *p) {
  PotF P;
  const double log2e = 1.4426950408889634074;
  double s = ldexp(1.0, -p->qbits);  // Angstrom per quantum
  double xi2 = p->xi * p->xi;
  P.rc2 = (float)((p->r_cut / s) * (p->r_cut / s));
  P.rt = (float)(p->r_tail / s);
  P.aF = (float)(-2.0 * p->q * log2e * s / p->r0);
  P.bF = (float)(log2(xi2) + 2.0 * p->q * log2e);
  P.aP = P.aF;
  P.bP = (float)(log2(xi2 * 2.0 * p->q / p->r0) + 2.0 * p->q * log2e);
  P.aV = (float)(-p->p * log2e * s / p->r0);
  P.bV = (float)(log2(p->A) + p->p * log2e);
  P.bW = (float)(log2(p->A * 2.0 * p->p / p->r0) + p->p * log2e);
  double w = p->r_cut - p->r_tail;
  double wi = w > 0 ? 1.0 / w : 0.0;
  P.uS = (float)(-s * wi);
  P.uB = (float)(p->r_cut * wi);
  // With t = 1 - u, the Hermite cubic c0 + c1 t + c2 t^2 + c3 t^3 that meets
  // (value c0, slope c1 per unit t) at r_tail and (0, 0) at r_cut equals
  // u^2 (a + b u) with a = 3 c0 + c1 and b = -2 c0 - c1; its r-derivative
  // is -u (2a + 3b u) / w.
  double cf[4], cv[4];
  hermite(xi2, 2.0 * p->q, p, cf);
  hermite(p->A, p->p, p, cv);
  const double fa = 3.0 * cf[0] + cf[1], fb = -2.0 * cf[0] - cf[1];
  const double va = 3.0 * cv[0] + cv[1], vb = -2.0 * cv[0] - cv[1];
  P.fa = (float)fa;
  P.fb = (float)fb;
  P.va = (float)va;
  P.vb = (float)vb;
  P.dv0 = (float)(-4.0 * va * wi);
  P.dv1 = (float)(-6.0 * vb * wi);
  P.dp0 = (float)(2.0 * fa * wi);
  P.dp1 = (float)(3.0 * fb * wi);
  P.wscale = (float)(0.5 * s);
  return P;
}

int check_md(const tbsma_md *m, int R) {
  if (!m) return fail(TBSMA_EINVAL, "md is NULL");
  if (!(m->dt > 0) || !(m->gamma >= 0))
    return fail(TBSMA_EINVAL, "need dt > 0 and gamma >= 0");
  if (m->n_log < 1 || m->n_slots < 1)
    return fail(TBSMA_EINVAL, "n_log and n_slots must be >= 1");
  if (R > 0 && (!m->T || !m->v_pull || !m->z_lo || !m->z_hi || !m->vol ||
                !m->L0 || !m->seed || !m->dof || !m->step || !m->obs ||
                !m->status))
    return fail(TBSMA_EINVAL, "a device array of md is NULL");
  if (!(m->nh_tau >= 0) || !std::isfinite(m->nh_tau))
    return fail(TBSMA_EINVAL, "nh_tau must be finite and >= 0");
  if (m->nh_tau > 0 && m->gamma > 0)
    return fail(TBSMA_EINVAL, "Langevin (gamma > 0) and Nose-Hoover "
                "(nh_tau > 0) exclude each other");
  if (m->nh_tau > 0 && R > 0 && !m->nh_xi)
    return fail(TBSMA_EINVAL, "Nose-Hoover needs nh_xi");
  if (m->grip_hold < 0 || !std::isfinite(m->grip_step))
    return fail(TBSMA_EINVAL, "need grip_hold >= 0 and a finite grip_step");
  if (m->ramp_steps < 0)
    return fail(TBSMA_EINVAL, "ramp_steps must be >= 0");
  if (m->ramp_steps > 0 && R > 0 && !m->T_start)
    return fail(TBSMA_EINVAL, "a temperature ramp needs T_start");
  if (!(m->baro_mass >= 0) || !std::isfinite(m->baro_mass) ||
      !std::isfinite(m->baro_load) || !(m->baro_damp >= 0) ||
      !std::isfinite(m->baro_damp))
    return fail(TBSMA_EINVAL, "need finite baro_mass >= 0, baro_load and "
                "baro_damp >= 0");
  if (m->baro_mass > 0 && m->grip_hold > 0)
    return fail(TBSMA_EINVAL, "the barostat and stepwise grips exclude each "
                "other");
  if (m->baro_mass > 0 && R > 0 && !m->baro_s)
    return fail(TBSMA_EINVAL, "the barostat needs baro_s");
  return TBSMA_OK;
}

DevMD make_devmd(const tbsma_params *p, const tbsma_md *m) {
  DevMD M;
  memset(&M, 0, sizeof(M));
  M.dt = m->dt;
  M.gamma = m->gamma;
  M.c1 = exp(-m->gamma * m->dt);
  M.r_cut = p->r_cut;
  M.lab_frame = m->lab_frame;
  M.n_log = m->n_log;
  M.n_slots = m->n_slots;
  M.T = m->T;
  M.v_pull = m->v_pull;
  M.z_lo = m->z_lo;
  M.z_hi = m->z_hi;
  M.vol = m->vol;
  M.L0 = m->L0;
  M.seed = m->seed;
  M.dof = m->dof;
  M.step = m->step;
  M.obs = m->obs;
  M.status = m->status;
  M.retire = m->dfail ? m->retire : 0.0;
  M.dfail = m->dfail;
  M.nh_tau = m->nh_tau;
  M.nh_xi = m->nh_xi;
  M.nh_eta = m->nh_eta;
  M.grip_step = m->grip_hold > 0 ? m->grip_step : 0.0;
  M.grip_hold = m->grip_hold;
  M.T_start = m->T_start;
  M.ramp_begin = m->ramp_begin;
  M.ramp_steps = m->T_start ? m->ramp_steps : 0;
  M.baro_mass = m->baro_s ? m->baro_mass : 0.0;
  M.baro_load = m->baro_load;
  M.baro_damp = m->baro_damp;
  M.defer = (p->precision == TBSMA_MIXED && M.nh_tau <= 0.0 &&
             M.baro_mass <= 0.0)
                ? 1
                : 0;
  M.baro_s = m->baro_s;
  return M;
}

int check_out(const tbsma_params *p, const tbsma_forces_out *o) {
  if (!o || !o->fx || !o->fy || !o->fz || !o->e_atom)
    return fail(TBSMA_EINVAL, "force outputs missing");
  if (p->precision == TBSMA_FP64 && !o->g)
    return fail(TBSMA_EINVAL, "FP64 precision needs the g array");
  return TBSMA_OK;
}

int check_lists(const tbsma_params *p, const tbsma_cells *c,
                const tbsma_nlist *n) {
  if (c && (!c->cell_start || !c->cell_atoms))
    return fail(TBSMA_EINVAL, "cell arrays missing");
  if (n && (!n->nl || !n->nn || !n->x_ref || !n->y_ref || !n->z_ref ||
            n->k_cap < 8 || n->k_cap % 8))
    return fail(TBSMA_EINVAL,
                "neighbour-list arrays missing or k_cap not a multiple of 8");
  if (n && p->precision == TBSMA_MIXED && !n->nl_lane)
    return fail(TBSMA_EINVAL, "mixed precision needs nl_lane");
  return TBSMA_OK;
}

#define TRY(expr)             \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ != TBSMA_OK)      \
      return rc_;             \
  } while (0)

// One MD step (see tbsma_step) enqueued on s.
void enqueue_step(const tbsma_params *p, const Dev &d0, const DevMD &M0,
                  const tbsma_forces_out *o, const PotF &PF, const PotD &PD,
                  hipStream_t s) {
  bool mixed = p->precision == TBSMA_MIXED;
  double rl = p->r_cut + p->skin;
  Dev d = d0;
  d.rstatus = M0.status;
  const DevMD &M = M0;
  launch_integrate_a(d, M, mixed, o->fx, o->fy, o->fz, s);
  launch_worklist(d, s);
  launch_cells(d, s);
  launch_nlist(d, mixed, rl, s);
  Dev df = d;
  df.energies = -1;
  df.step = M.step;
  df.n_log = M.n_log;
  if (mixed) {
    launch_forces_kick(df, M, PF, o->fx, o->fy, o->fz, o->e_atom, s);
  } else {
    launch_forces(df, mixed, PF, PD, o->fx, o->fy, o->fz, o->e_atom, o->g, s);
    launch_integrate_b(d, M, mixed, o->fx, o->fy, o->fz, s);
  }
  launch_reduce_step(d, M, s);
}

int finish_run(const Dev &d, const tbsma_md *m, hipStream_t s) {
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  int32_t nnmax = 0;
  HIPCHK(hipMemcpy(&nnmax, d.nnmax, 4, hipMemcpyDeviceToHost));
  // status words read in chunks into a stack buffer (no host allocation)
  uint32_t st[256];
  for (int r0 = 0; r0 < d.R; r0 += 256) {
    const int n = std::min(256, d.R - r0);
    HIPCHK(hipMemcpy(st, m->status + r0, 4 * (size_t)n,
                     hipMemcpyDeviceToHost));
    for (int k = 0; k < n; ++k)
      if (st[k] & TBSMA_ST_OVERFLOW)
        return fail(TBSMA_ECAPACITY,
                    "neighbour list overflow in replica %d (longest row %d, "
                    "k_cap %d)", r0 + k, nnmax, d.k_cap);
  }
  return TBSMA_OK;
}

// Bodies of the entry points below, after their argument checks, on an
// explicit workspace (the caller's, or the library's static scratch).
int workspace_init_on(const tbsma_params *prm, const tbsma_system *sys,
                      void *work, hipStream_t s) {
  Layout L = layout(prm, sys);
  char *w = static_cast<char *>(work);
  // zero everything (as 32-bit words), then the min-bins to the empty key
  launch_fill_u32(reinterpret_cast<uint32_t *>(w), (int64_t)(L.total / 4), 0u,
                  s);
  launch_fill_u64(reinterpret_cast<unsigned long long *>(w + L.zbmin),
                  (int64_t)sys->R * sys->max_zbins, ~0ull, s);
  launch_block_map(make_dev(prm, sys, work), s);
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int build_cells_on(const tbsma_params *prm, const tbsma_system *sys,
                   const tbsma_cells *cells, void *work, hipStream_t s) {
  Dev d = make_dev(prm, sys, work);
  attach_lists(d, cells, nullptr);
  d.all = 1;
  launch_fill_u32(reinterpret_cast<uint32_t *>(d.cnt), sys->C, 0u, s);
  launch_worklist(d, s);
  launch_cells(d, s);
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int neighbors_on(const tbsma_params *prm, const tbsma_system *sys,
                 const tbsma_cells *cells, const tbsma_nlist *nl, void *work,
                 int32_t *need_cap, hipStream_t s) {
  Dev d = make_dev(prm, sys, work);
  attach_lists(d, cells, nl);
  d.all = 1;
  double rl = prm->r_cut + prm->skin;
  launch_fill_u32(reinterpret_cast<uint32_t *>(d.nnmax), 1, 0u, s);
  const bool mixed = prm->precision == TBSMA_MIXED;
  if (mixed) launch_quantise(d, s);
  launch_worklist(d, s);
  launch_nlist(d, mixed, rl, s);
  HIPCHK(hipGetLastError());
  if (need_cap) {
    HIPCHK(hipStreamSynchronize(s));
    int32_t mx = 0;
    HIPCHK(hipMemcpy(&mx, d.nnmax, 4, hipMemcpyDeviceToHost));
    *need_cap = mx > nl->k_cap ? mx : nl->k_cap;
    if (mx > nl->k_cap)
      return fail(TBSMA_ECAPACITY, "longest row %d exceeds k_cap %d", mx,
                  nl->k_cap);
  }
  return TBSMA_OK;
}

int forces_on(const tbsma_params *prm, const tbsma_system *sys,
              const tbsma_nlist *nl, const tbsma_forces_out *out, void *work,
              hipStream_t s) {
  Dev d = make_dev(prm, sys, work);
  attach_lists(d, nullptr, nl);
  bool mixed = prm->precision == TBSMA_MIXED;
  if (mixed) launch_quantise(d, s);
  launch_forces(d, mixed, make_potf(prm), make_potd(prm), out->fx, out->fy,
                out->fz, out->e_atom, out->g, s);
  launch_reduce_forces(d, out->rep_energy, out->rep_wzz, s);
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int step_on(const tbsma_params *prm, const tbsma_system *sys,
            const tbsma_cells *cells, const tbsma_nlist *nl,
            const tbsma_forces_out *out, const tbsma_md *md, void *work,
            int64_t n_steps, hipStream_t s) {
  Dev d = make_dev(prm, sys, work);
  attach_lists(d, cells, nl);
  DevMD M = make_devmd(prm, md);
  PotF PF = make_potf(prm);
  PotD PD = make_potd(prm);
  const bool mixed = prm->precision == TBSMA_MIXED;
  launch_call_bounds(d, M, n_steps, s);
  if (M.nh_tau > 0 || M.baro_mass > 0)
    launch_step_begin(d, M, mixed, out->fz, s);
  for (int64_t k = 0; k < n_steps; ++k) enqueue_step(prm, d, M, out, PF, PD, s);
  if (M.nh_tau > 0) launch_nh_finish(d, M, s);
  return finish_run(d, md, s);
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_ptr(void **out) {
  static std::mutex mu;
  static void *ptrs[64] = {nullptr};
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(TBSMA_EDEVICE, "device %d", dev);
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TBSMA_EHIP, "hipGetSymbolAddress(scratch): %s",
                  hipGetErrorString(e));
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return TBSMA_OK;
}

// Instantiated step graphs, keyed by every argument they were captured with
// (pointers, sizes, constants, stream, device); the least recently used one
// is dropped beyond kGraphs entries.
constexpr size_t kGraphs = 16;
struct GraphEntry {
  std::vector<char> key;
  hipGraphExec_t exec = nullptr;
  uint64_t used = 0;
};
struct GraphCache {
  std::mutex mu;
  std::vector<GraphEntry> entries;
  uint64_t clock = 0;
};
GraphCache g_graph;

void append(std::vector<char> &k, const void *p, size_t n) {
  const char *c = static_cast<const char *>(p);
  k.insert(k.end(), c, c + n);
}

}  // namespace

extern "C" {

const char *tbsma_last_error(void) { return g_err.c_str(); }

int tbsma_workspace_query(const tbsma_params *prm, const tbsma_system *sys,
                          size_t *bytes) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!bytes) return fail(TBSMA_EINVAL, "bytes is NULL");
  *bytes = sys->R > 0 ? layout(prm, sys).total : 256;
  return TBSMA_OK;
}

int tbsma_workspace_init(const tbsma_params *prm, const tbsma_system *sys,
                         void *work, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (sys->R == 0) return TBSMA_OK;
  if (!work) return fail(TBSMA_EINVAL, "work is NULL");
  TRY(check_device());
  return workspace_init_on(prm, sys, work, static_cast<hipStream_t>(stream));
}

int tbsma_build_wire(double a, double D, double L, int32_t n_grip,
                     int32_t notch_layers, double notch_depth, double *x,
                     double *y, double *z, uint8_t *flag, int64_t cap,
                     int64_t *n_out) {
  if (!(a > 0) || !(D >= 0) || !(L >= 0) || n_grip < 0 || !n_out)
    return fail(TBSMA_EINVAL, "bad wire arguments");
  if (notch_layers < 0 || !(notch_depth >= 0))
    return fail(TBSMA_EINVAL, "need notch_layers >= 0 and notch_depth >= 0");
  double h = 0.5 * a;
  double rad2 = (D / a) * (D / a);
  int64_t layers = 0;
  while ((double)layers * h < L) ++layers;
  int64_t m = (int64_t)floor(D / a) + 1;
  // ring notch: planes [k0, k0 + notch_layers) around the middle plane lose
  // the sites farther than D/2 - notch_depth from the axis
  const int64_t k0 = layers / 2 - notch_layers / 2;
  const double r_in = 0.5 * D - notch_depth;
  int64_t n = 0;
  for (int64_t k = 0; k < layers; ++k) {
    uint8_t fl = k < n_grip ? TBSMA_GRIP_FIXED
                 : k >= layers - n_grip ? TBSMA_GRIP_PULL
                                        : TBSMA_DYN;
    const bool notch = k >= k0 && k < k0 + notch_layers;
    for (int64_t j = -m; j <= m; ++j)
      for (int64_t i = -m; i <= m; ++i) {
        if ((i + j + k) & 1) continue;
        if ((double)(i * i + j * j) > rad2) continue;
        if (notch) {
          const double px = (double)i * h, py = (double)j * h;
          if (std::sqrt(px * px + py * py) > r_in) continue;
        }
        if (n < cap) {
          x[n] = (double)i * h;
          y[n] = (double)j * h;
          z[n] = (double)k * h;
          flag[n] = fl;
        }
        ++n;
      }
  }
  *n_out = n;
  if (n > cap) return fail(TBSMA_ECAPACITY, "wire has %lld atoms", (long long)n);
  return TBSMA_OK;
}

int tbsma_init_state(const tbsma_params *prm, tbsma_system *sys,
                     const tbsma_md *md, void *work, double jitter,
                     void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  TRY(check_md(md, sys->R));
  if (sys->R == 0) return TBSMA_OK;
  TRY(check_device());
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(prm, sys, work);
  DevMD M = make_devmd(prm, md);
  launch_init(d, M, prm->precision == TBSMA_MIXED, jitter, s);
  launch_set_step(md->step, 0, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return TBSMA_OK;
}

int tbsma_replica_constants(const tbsma_params *prm, const tbsma_system *sys,
                            int32_t *dof, double *vol, double *z_lo,
                            double *z_hi, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (sys->R == 0) return TBSMA_OK;
  if (!dof || !vol || !z_lo || !z_hi)
    return fail(TBSMA_EINVAL, "dof, vol, z_lo and z_hi are required");
  TRY(check_device());
  // the kernel reads only the system's arrays, no workspace
  Dev d;
  memset(&d, 0, sizeof(d));
  d.R = sys->R;
  d.N = sys->N;
  d.rep_off = sys->rep_off;
  d.flag = sys->flag;
  d.z = sys->z;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_replica_constants(d, prm->r0, dof, vol, z_lo, z_hi, s);
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int tbsma_rebase(const tbsma_params *prm, tbsma_system *sys, double *L0,
                 double *baro_s, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (sys->R == 0) return TBSMA_OK;
  if (!L0) return fail(TBSMA_EINVAL, "L0 is required");
  TRY(check_device());
  Dev d;
  memset(&d, 0, sizeof(d));
  d.R = sys->R;
  d.N = sys->N;
  d.z = sys->z;
  d.z0 = sys->z0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_rebase(d, L0, baro_s, s);
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int tbsma_build_cells(const tbsma_params *prm, const tbsma_system *sys,
                      tbsma_cells *cells, void *work, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  TRY(check_lists(prm, cells, nullptr));
  if (!cells) return fail(TBSMA_EINVAL, "cells is NULL");
  if (sys->R == 0) return TBSMA_OK;
  TRY(check_device());
  return build_cells_on(prm, sys, cells, work,
                        static_cast<hipStream_t>(stream));
}

int tbsma_neighbors(const tbsma_params *prm, const tbsma_system *sys,
                    const tbsma_cells *cells, tbsma_nlist *nl, void *work,
                    int32_t *need_cap, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!cells || !nl) return fail(TBSMA_EINVAL, "cells or nlist is NULL");
  TRY(check_lists(prm, cells, nl));
  if (sys->R == 0) return TBSMA_OK;
  TRY(check_device());
  return neighbors_on(prm, sys, cells, nl, work, need_cap,
                      static_cast<hipStream_t>(stream));
}

int tbsma_forces(const tbsma_params *prm, const tbsma_system *sys,
                 const tbsma_nlist *nl, tbsma_forces_out *out, void *work,
                 void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!nl) return fail(TBSMA_EINVAL, "nlist is NULL");
  TRY(check_lists(prm, nullptr, nl));
  TRY(check_out(prm, out));
  if (sys->R == 0) return TBSMA_OK;
  if (!out->rep_energy || !out->rep_wzz)
    return fail(TBSMA_EINVAL, "rep_energy / rep_wzz missing");
  TRY(check_device());
  return forces_on(prm, sys, nl, out, work, static_cast<hipStream_t>(stream));
}

int tbsma_forces_pass(const tbsma_params *prm, const tbsma_system *sys,
                      const tbsma_nlist *nl, tbsma_forces_out *out, void *work,
                      int32_t pass, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!nl) return fail(TBSMA_EINVAL, "nlist is NULL");
  TRY(check_lists(prm, nullptr, nl));
  TRY(check_out(prm, out));
  if (pass < 1 || pass > 3) return fail(TBSMA_EINVAL, "pass must be 1, 2 or 3");
  if (sys->R == 0) return TBSMA_OK;
  TRY(check_device());
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(prm, sys, work);
  attach_lists(d, nullptr, nl);
  if (pass == 3) d.energies = 0;
  launch_force_pass(d, prm->precision == TBSMA_MIXED, pass, make_potf(prm),
                    make_potd(prm), out->fx, out->fy, out->fz, out->e_atom,
                    out->g, s);
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int tbsma_step(const tbsma_params *prm, tbsma_system *sys, tbsma_cells *cells,
               tbsma_nlist *nl, tbsma_forces_out *out, const tbsma_md *md,
               void *work, int64_t n_steps, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!cells || !nl) return fail(TBSMA_EINVAL, "cells or nlist is NULL");
  TRY(check_lists(prm, cells, nl));
  TRY(check_out(prm, out));
  TRY(check_md(md, sys->R));
  if (n_steps < 0) return fail(TBSMA_EINVAL, "n_steps < 0");
  if (sys->R == 0 || n_steps == 0) return TBSMA_OK;
  TRY(check_device());
  return step_on(prm, sys, cells, nl, out, md, work, n_steps,
                 static_cast<hipStream_t>(stream));
}

int tbsma_step_noalloc(const tbsma_params *prm, tbsma_system *sys,
                       tbsma_cells *cells, tbsma_nlist *nl,
                       tbsma_forces_out *out, const tbsma_md *md,
                       int64_t n_steps, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!cells || !nl) return fail(TBSMA_EINVAL, "cells or nlist is NULL");
  TRY(check_lists(prm, cells, nl));
  TRY(check_out(prm, out));
  if (!out->rep_energy || !out->rep_wzz)
    return fail(TBSMA_EINVAL, "rep_energy / rep_wzz missing");
  TRY(check_md(md, sys->R));
  if (n_steps < 0) return fail(TBSMA_EINVAL, "n_steps < 0");
  if (sys->R == 0 || n_steps == 0) return TBSMA_OK;
  const size_t need = layout(prm, sys).total;
  if (need > kScratchBytes)
    return fail(TBSMA_ECAPACITY,
                "system needs %zu bytes of workspace; the static scratch of "
                "tbsma_step_noalloc holds %zu (use tbsma_step with a "
                "workspace)", need, kScratchBytes);
  TRY(check_device());
  void *work = nullptr;
  TRY(scratch_ptr(&work));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the scratch keeps the previous call's contents: put it into the initial
  // state, then lists and forces of the current positions, then the steps
  TRY(workspace_init_on(prm, sys, work, s));
  TRY(build_cells_on(prm, sys, cells, work, s));
  TRY(neighbors_on(prm, sys, cells, nl, work, nullptr, s));
  TRY(forces_on(prm, sys, nl, out, work, s));
  return step_on(prm, sys, cells, nl, out, md, work, n_steps, s);
}

int tbsma_run_batch(const tbsma_params *prm, tbsma_system *sys,
                    tbsma_cells *cells, tbsma_nlist *nl,
                    tbsma_forces_out *out, const tbsma_md *md, void *work,
                    int64_t n_steps, int32_t steps_per_graph, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!cells || !nl) return fail(TBSMA_EINVAL, "cells or nlist is NULL");
  TRY(check_lists(prm, cells, nl));
  TRY(check_out(prm, out));
  TRY(check_md(md, sys->R));
  if (n_steps < 0 || steps_per_graph < 1)
    return fail(TBSMA_EINVAL, "need n_steps >= 0 and steps_per_graph >= 1");
  if (sys->R == 0 || n_steps == 0) return TBSMA_OK;
  TRY(check_device());
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(prm, sys, work);
  attach_lists(d, cells, nl);
  DevMD M = make_devmd(prm, md);
  PotF PF = make_potf(prm);
  PotD PD = make_potd(prm);
  int64_t chunks = n_steps / steps_per_graph;
  int64_t rest = n_steps % steps_per_graph;
  launch_call_bounds(d, M, n_steps, s);
  if (M.nh_tau > 0 || M.baro_mass > 0)
    launch_step_begin(d, M, prm->precision == TBSMA_MIXED, out->fz, s);
  if (chunks > 0) {
    std::lock_guard<std::mutex> lk(g_graph.mu);
    std::vector<char> key;
    append(key, prm, sizeof(*prm));
    append(key, &d, sizeof(d));
    append(key, &M, sizeof(M));
    append(key, out, sizeof(*out));
    append(key, &steps_per_graph, sizeof(steps_per_graph));
    append(key, &s, sizeof(s));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    append(key, &dev, sizeof(dev));
    GraphEntry *hit = nullptr;
    for (GraphEntry &e : g_graph.entries)
      if (e.key == key) hit = &e;
    if (!hit) {
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int32_t k = 0; k < steps_per_graph; ++k)
        enqueue_step(prm, d, M, out, PF, PD, s);
      hipError_t ce = hipStreamEndCapture(s, &graph);
      if (ce != hipSuccess)
        return fail(TBSMA_EHIP, "graph capture: %s", hipGetErrorString(ce));
      hipGraphExec_t exec = nullptr;
      hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess)
        return fail(TBSMA_EHIP, "graph instantiate: %s",
                    hipGetErrorString(ie));
      if (g_graph.entries.size() >= kGraphs) {
        auto lru = std::min_element(
            g_graph.entries.begin(), g_graph.entries.end(),
            [](const GraphEntry &a, const GraphEntry &b) {
              return a.used < b.used;
            });
        (void)hipGraphExecDestroy(lru->exec);
        g_graph.entries.erase(lru);
      }
      g_graph.entries.push_back(GraphEntry{key, exec, 0});
      hit = &g_graph.entries.back();
    }
    hit->used = ++g_graph.clock;
    for (int64_t c = 0; c < chunks; ++c)
      HIPCHK(hipGraphLaunch(hit->exec, s));
  }
  for (int64_t k = 0; k < rest; ++k) enqueue_step(prm, d, M, out, PF, PD, s);
  if (M.nh_tau > 0) launch_nh_finish(d, M, s);
  return finish_run(d, md, s);
}

int tbsma_list_stats(const tbsma_params *prm, const tbsma_system *sys,
                     const tbsma_nlist *nl, void *work, int64_t *out_host,
                     void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!nl || !out_host || !work)
    return fail(TBSMA_EINVAL, "nlist, work or out_host is NULL");
  TRY(check_lists(prm, nullptr, nl));
  for (int k = 0; k < 6; ++k) out_host[k] = 0;
  if (sys->R == 0) return TBSMA_OK;
  TRY(check_device());
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(prm, sys, work);
  attach_lists(d, nullptr, nl);
  launch_list_stats(d, prm->precision == TBSMA_MIXED, s);
  HIPCHK(hipGetLastError());
  unsigned long long h[6];
  HIPCHK(hipMemcpyAsync(h, d.stats, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < 6; ++k)
    out_host[k] = prm->precision == TBSMA_MIXED || k < 2 ? (int64_t)h[k] : 0;
  return TBSMA_OK;
}

int tbsma_rng_fill(uint64_t seed, uint32_t rep_id, uint64_t step,
                   uint32_t stream_id, int64_t n, uint32_t *out_u32,
                   double *out_gauss, void *stream) {
  if (n < 0) return fail(TBSMA_EINVAL, "n < 0");
  if (n == 0) return TBSMA_OK;
  TRY(check_device());
  launch_rng_fill(seed, rep_id, step, stream_id, n, out_u32, out_gauss,
                  nullptr, static_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int tbsma_rng_normals_f32(uint64_t seed, uint32_t rep_id, uint64_t step,
                          uint32_t stream_id, int64_t n, float *out_gauss,
                          void *stream) {
  if (n < 0) return fail(TBSMA_EINVAL, "n < 0");
  if (n > 0 && !out_gauss) return fail(TBSMA_EINVAL, "out_gauss is NULL");
  if (n == 0) return TBSMA_OK;
  TRY(check_device());
  launch_rng_fill(seed, rep_id, step, stream_id, n, nullptr, nullptr,
                  out_gauss, static_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return TBSMA_OK;
}

int tbsma_event_counts(const tbsma_params *prm, const tbsma_system *sys,
                   void *work, int64_t *out_host, void *stream) {
  TRY(check_params(prm));
  TRY(check_system(prm, sys));
  if (!out_host) return fail(TBSMA_EINVAL, "out_host is NULL");
  out_host[0] = out_host[1] = 0;
  if (sys->R == 0) return TBSMA_OK;
  if (!work) return fail(TBSMA_EINVAL, "work is NULL");
  TRY(check_device());
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d = make_dev(prm, sys, work);
  int64_t h[2];
  HIPCHK(hipMemcpyAsync(h, d.callb + kCallRebuilds, sizeof(h),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out_host[0] = h[0];
  out_host[1] = h[1];
  return TBSMA_OK;
}

}  // extern "C"
