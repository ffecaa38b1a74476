/*
 * FP64 CPU oracle for TB-SMA (second-moment tight-binding, Cleri-Rosato)
 * molecular dynamics of gold nanowires under elongation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Every function states the passage of the paper (French, Pervaje, Santos,
 * Iacovella, Cummings, "Probing the Statistical Validity of the
 * Ductile-to-Brittle Transition in Metallic Nanowires using GPU Computing")
 * that it follows.  Where the paper is silent or garbled, the reading taken
 * is stated at the function.
 *
 * Units: Angstrom, eV, amu, ps, K.
 * Axis: the wire axis [100] is z here (the paper's x in eq 5).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Physical constants (CODATA 2018 exact / recommended values).              */
/* ------------------------------------------------------------------------ */
#define ORC_KB 8.617333262e-5                 /* eV / K */
#define ORC_EV_J 1.602176634e-19              /* J per eV */
#define ORC_AMU_KG 1.66053906660e-27          /* kg per amu */
/* 1 eV/(Angstrom amu) expressed in Angstrom/ps^2 */
#define ORC_ACC (ORC_EV_J / ORC_AMU_KG * 1.0e-4)
#define ORC_EVA3_GPA (ORC_EV_J * 1.0e21)       /* 1 eV/A^3 in GPa */

double orc_const_kb(void) { return ORC_KB; }
double orc_const_acc(void) { return ORC_ACC; }
double orc_const_eva3_gpa(void) { return ORC_EVA3_GPA; }

/* ------------------------------------------------------------------------ */
/* Potential parameters.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  double A;      /* eV, repulsive prefactor (Table 1) */
  double xi;     /* eV, band-term hopping integral (Table 1) */
  double p;      /* repulsive decay (Table 1) */
  double q;      /* band decay (Table 1) */
  double r0;     /* Angstrom, reference distance: read as the nearest-neighbour
                    distance a/sqrt(2), see the header of orc_radial */
  double r_tail; /* start of the cubic tail */
  double r_cut;  /* end of the cubic tail; zero beyond */
} orc_pot;

/*
 * Radial functions of eqs 1 and 2 (Methods, "TB-SMA potential"):
 *   phi(r) = xi^2 exp(-2q (r/r0 - 1))    (the summand of eq 1, the density)
 *   V(r)   = A    exp(-p  (r/r0 - 1))    (the summand of eq 2)
 * Reading of the cutoff: the paper applies a hard cut at 5.8 A.  Here each
 * function is kept unchanged up to r_tail and replaced on (r_tail, r_cut] by
 * the cubic Hermite polynomial matching its value and slope at r_tail and
 * reaching value 0, slope 0 at r_cut.  r_tail == r_cut gives the hard cut.
 * Reading of r0: Table 1 prints 4.079 A, which is the lattice constant of Au;
 * with it the FCC crystal is unbound.  The fit the paper describes (cohesive
 * energy and lattice parameter) holds for r0 = a/sqrt(2) = 2.884 A.
 *
 * kind 0 = phi, kind 1 = V.  Returns f(r); *df = f'(r).
 */
static double orc_radial(const orc_pot *P, int kind, double r, double *df) {
  double pre = kind == 0 ? P->xi * P->xi : P->A;
  double k = kind == 0 ? 2.0 * P->q : P->p;
  if (r > P->r_cut) {
    *df = 0.0;
    return 0.0;
  }
  if (r <= P->r_tail) {
    double f = pre * exp(-k * (r / P->r0 - 1.0));
    *df = -(k / P->r0) * f;
    return f;
  }
  /* cubic Hermite on (r_tail, r_cut] */
  double w = P->r_cut - P->r_tail;
  double fs = pre * exp(-k * (P->r_tail / P->r0 - 1.0));
  double ms = -(k / P->r0) * fs * w; /* slope at r_tail times the interval */
  double t = (r - P->r_tail) / w;
  double h00 = 2.0 * t * t * t - 3.0 * t * t + 1.0;
  double h10 = t * t * t - 2.0 * t * t + t;
  double dh00 = 6.0 * t * t - 6.0 * t;
  double dh10 = 3.0 * t * t - 4.0 * t + 1.0;
  *df = (fs * dh00 + ms * dh10) / w;
  return fs * h00 + ms * h10;
}

/* Exposed for the tail pins: f(r) and f'(r) of phi (kind 0) and V (kind 1). */
double orc_radial_eval(const orc_pot *P, int kind, double r, double *df) {
  return orc_radial(P, kind, r, df);
}

/* ------------------------------------------------------------------------ */
/* Nanowire geometry.                                                        */
/* ------------------------------------------------------------------------ */
/*
 * [100]-oriented cylindrical FCC wire (Simulation details; Figure 1):
 * lattice sites (i, j, k) * a/2 with i + j + k even; the cylinder axis runs
 * along z through the atom column at x = y = 0.  A site is kept when
 * (i^2 + j^2) <= (D/a)^2 (that is, x^2 + y^2 <= (D/2)^2) and 0 <= k a/2 < L.
 * Generation order, which is also the tag order: k (z) outermost, then j (y),
 * then i (x), ascending.  The lowest n_grip and highest n_grip (002) planes
 * are the rigid grips: flag 1 at the bottom (fixed), flag 2 at the top (the
 * end that is pulled); every other atom has flag 0 (dynamic).
 * Ring notch (Simulation details; Figure 1 caption: three atoms wide, two
 * deep), reading: with nk planes, the notch covers the notch_layers planes
 * k = nk/2 - notch_layers/2, ..., nk/2 - notch_layers/2 + notch_layers - 1
 * (integer division) and removes there every site whose distance from the
 * axis exceeds D/2 - notch_depth.  notch_layers = 0: no notch.
 * Returns the number of atoms (also when cap is too small: then only the
 * count is computed and nothing is written past cap).
 */
int64_t orc_build_wire(double a, double D, double L, int n_grip,
                       int notch_layers, double notch_depth,
                       double *x, double *y, double *z, uint8_t *flag,
                       int64_t cap) {
  double half = 0.5 * a;
  double lim = (D / a) * (D / a);
  int64_t nk = 0;
  while ((double)nk * half < L) nk++;
  int64_t m = (int64_t)floor(D / a) + 1;
  int64_t k_n0 = nk / 2 - notch_layers / 2;
  int64_t k_n1 = k_n0 + notch_layers; /* exclusive */
  double rin = 0.5 * D - notch_depth;
  int64_t n = 0;
  for (int64_t k = 0; k < nk; k++) {
    int fl = 0;
    if (k < n_grip) fl = 1;
    else if (k >= nk - n_grip) fl = 2;
    int notched = notch_layers > 0 && k >= k_n0 && k < k_n1;
    for (int64_t j = -m; j <= m; j++) {
      for (int64_t i = -m; i <= m; i++) {
        if (((i + j + k) % 2 + 2) % 2 != 0) continue;
        if ((double)(i * i + j * j) > lim) continue;
        double xx = (double)i * half, yy = (double)j * half;
        if (notched && sqrt(xx * xx + yy * yy) > rin) continue;
        if (n < cap) {
          x[n] = xx;
          y[n] = yy;
          z[n] = (double)k * half;
          flag[n] = (uint8_t)fl;
        }
        n++;
      }
    }
  }
  return n;
}

/* ------------------------------------------------------------------------ */
/* Energy and forces.                                                        */
/* ------------------------------------------------------------------------ */
/*
 * Energy of eqs 1-3: E = sum_i E_i with
 *   E_i = -sqrt(rho_i) + sum_{j != i} V(r_ij),   rho_i = sum_{j != i} phi(r_ij)
 * (no factor 1/2 on the repulsive sum: eq 2 sums over all j and eq 3 sums
 * E_R^i over all i).  No periodic images.
 * Forces, from differentiating eqs 1-3 (the dependence on rho of both i and
 * j that the paper notes after Table 1's paragraph):
 *   F_i = sum_j E'_ij (r_j - r_i) / r_ij,
 *   E'_ij = 2 V'(r_ij) - (g_i + g_j) phi'(r_ij) / 2,   g_i = 1/sqrt(rho_i)
 * (g_i = 0 when rho_i = 0).
 * Virial W_ab = -sum_{i<j} E'_ij d_a d_b / r, d = r_j - r_i, stored as
 * xx, yy, zz, xy, xz, yz; the stress of eq 5 uses -W_zz.
 *
 * pairs_of(i) enumeration: brute force over all j (mode 0) or over the 27
 * neighbouring cells of a cell list (mode 1); both visit exactly the j with
 * r_ij <= r_cut.
 */
typedef struct {
  int64_t n;
  const double *x, *y, *z;
  /* cell list (mode 1) */
  int use_cells;
  double lo[3], h;
  int64_t dim[3];
  int64_t *cstart; /* [ncell + 1] */
  int64_t *catom;  /* [n] */
} orc_nbr;

static int64_t orc_cell_coord(double v, double lo, double h, int64_t dim) {
  int64_t c = (int64_t)floor((v - lo) / h);
  if (c < 0) c = 0;
  if (c >= dim) c = dim - 1;
  return c;
}

static void orc_nbr_init(orc_nbr *nb, int64_t n, const double *x,
                         const double *y, const double *z, int use_cells,
                         double h) {
  memset(nb, 0, sizeof(*nb));
  nb->n = n;
  nb->x = x;
  nb->y = y;
  nb->z = z;
  nb->use_cells = use_cells && n > 0;
  if (!nb->use_cells) return;
  const double *c3[3] = {x, y, z};
  int64_t ncell = 1;
  for (int d = 0; d < 3; d++) {
    double mn = c3[d][0], mx = c3[d][0];
    for (int64_t i = 1; i < n; i++) {
      if (c3[d][i] < mn) mn = c3[d][i];
      if (c3[d][i] > mx) mx = c3[d][i];
    }
    nb->lo[d] = mn;
    nb->dim[d] = (int64_t)floor((mx - mn) / h) + 1;
    ncell *= nb->dim[d];
  }
  nb->h = h;
  nb->cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  nb->catom = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t *cid = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) {
    int64_t cx = orc_cell_coord(x[i], nb->lo[0], h, nb->dim[0]);
    int64_t cy = orc_cell_coord(y[i], nb->lo[1], h, nb->dim[1]);
    int64_t cz = orc_cell_coord(z[i], nb->lo[2], h, nb->dim[2]);
    cid[i] = (cz * nb->dim[1] + cy) * nb->dim[0] + cx;
    nb->cstart[cid[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; c++) nb->cstart[c + 1] += nb->cstart[c];
  int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
  memcpy(fill, nb->cstart, (size_t)ncell * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) nb->catom[fill[cid[i]]++] = i;
  free(fill);
  free(cid);
}

static void orc_nbr_free(orc_nbr *nb) {
  free(nb->cstart);
  free(nb->catom);
}

/*
 * Indices j != i with |r_j - r_i| <= rc, written to out (capacity cap);
 * returns the number found (which may exceed cap: then only cap are
 * written).  Brute force or cell list, as set up in nb.
 */
static int64_t orc_neighbors_of(const orc_nbr *nb, int64_t i, double rc,
                                int64_t *out, int64_t cap) {
  int64_t cnt = 0;
  double xi = nb->x[i], yi = nb->y[i], zi = nb->z[i];
  if (!nb->use_cells) {
    for (int64_t j = 0; j < nb->n; j++) {
      if (j == i) continue;
      double dx = nb->x[j] - xi, dy = nb->y[j] - yi, dz = nb->z[j] - zi;
      if (sqrt(dx * dx + dy * dy + dz * dz) > rc) continue;
      if (cnt < cap) out[cnt] = j;
      cnt++;
    }
    return cnt;
  }
  int64_t cx = orc_cell_coord(xi, nb->lo[0], nb->h, nb->dim[0]);
  int64_t cy = orc_cell_coord(yi, nb->lo[1], nb->h, nb->dim[1]);
  int64_t cz = orc_cell_coord(zi, nb->lo[2], nb->h, nb->dim[2]);
  for (int64_t kz = cz - 1; kz <= cz + 1; kz++) {
    if (kz < 0 || kz >= nb->dim[2]) continue;
    for (int64_t ky = cy - 1; ky <= cy + 1; ky++) {
      if (ky < 0 || ky >= nb->dim[1]) continue;
      for (int64_t kx = cx - 1; kx <= cx + 1; kx++) {
        if (kx < 0 || kx >= nb->dim[0]) continue;
        int64_t c = (kz * nb->dim[1] + ky) * nb->dim[0] + kx;
        for (int64_t s = nb->cstart[c]; s < nb->cstart[c + 1]; s++) {
          int64_t j = nb->catom[s];
          if (j == i) continue;
          double dx = nb->x[j] - xi, dy = nb->y[j] - yi, dz = nb->z[j] - zi;
          if (sqrt(dx * dx + dy * dy + dz * dz) > rc) continue;
          if (cnt < cap) out[cnt] = j;
          cnt++;
        }
      }
    }
  }
  return cnt;
}

/* Neighbour indices of i in a growable per-caller buffer. */
static int64_t orc_neighbors(const orc_nbr *nb, int64_t i, double rc,
                             int64_t **buf, int64_t *cap) {
  int64_t c = orc_neighbors_of(nb, i, rc, *buf, *cap);
  if (c > *cap) {
    *cap = 2 * c;
    *buf = (int64_t *)realloc(*buf, (size_t)(*cap) * sizeof(int64_t));
    c = orc_neighbors_of(nb, i, rc, *buf, *cap);
  }
  return c;
}

/*
 * Energies, forces and virial of eqs 1-3 (see the block comment above).
 * Outputs (any may be NULL): rho[n], e_atom[n], fx/fy/fz[n], w6[6].
 * mode 0: brute force over all ordered pairs; mode 1: cell list with cells of
 * edge r_cut (the same pair set).  Returns the total energy E_C of eq 3.
 */
double orc_forces(const orc_pot *P, int64_t n, const double *x,
                  const double *y, const double *z, int mode, double *rho_out,
                  double *e_atom, double *fx, double *fy, double *fz,
                  double *w6) {
  orc_nbr nb;
  orc_nbr_init(&nb, n, x, y, z, mode == 1, P->r_cut);
  double *rho = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double *g = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double *erep = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  const double rc = P->r_cut;

  /* first loop over neighbours: rho_i and the repulsive sum of eq 2 */
#pragma omp parallel
  {
    int64_t cap = 256;
    int64_t *nbr = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
      int64_t c = orc_neighbors(&nb, i, rc, &nbr, &cap);
      double s = 0.0, er = 0.0, d;
      for (int64_t k = 0; k < c; k++) {
        int64_t j = nbr[k];
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        s += orc_radial(P, 0, r, &d);
        er += orc_radial(P, 1, r, &d);
      }
      rho[i] = s;
      erep[i] = er;
      g[i] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    }
    free(nbr);
  }

  /* second loop over neighbours: forces and virial */
  double etot = 0.0;
  double W[6] = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
  {
    double Wl[6] = {0, 0, 0, 0, 0, 0};
    int64_t cap = 256;
    int64_t *nbr = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
#pragma omp for schedule(dynamic, 64) reduction(+ : etot)
    for (int64_t i = 0; i < n; i++) {
      int64_t c = orc_neighbors(&nb, i, rc, &nbr, &cap);
      double Fx = 0.0, Fy = 0.0, Fz = 0.0;
      for (int64_t k = 0; k < c; k++) {
        int64_t j = nbr[k];
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double dphi, dV;
        (void)orc_radial(P, 0, r, &dphi);
        (void)orc_radial(P, 1, r, &dV);
        double ep = 2.0 * dV - 0.5 * (g[i] + g[j]) * dphi;
        double sc = ep / r;
        Fx += sc * dx;
        Fy += sc * dy;
        Fz += sc * dz;
        /* each unordered pair is met twice: half of -E' d d / r each time */
        Wl[0] -= 0.5 * sc * dx * dx;
        Wl[1] -= 0.5 * sc * dy * dy;
        Wl[2] -= 0.5 * sc * dz * dz;
        Wl[3] -= 0.5 * sc * dx * dy;
        Wl[4] -= 0.5 * sc * dx * dz;
        Wl[5] -= 0.5 * sc * dy * dz;
      }
      double ei = -sqrt(rho[i]) + erep[i];
      if (e_atom) e_atom[i] = ei;
      if (fx) fx[i] = Fx;
      if (fy) fy[i] = Fy;
      if (fz) fz[i] = Fz;
      etot += ei;
    }
    free(nbr);
#pragma omp critical
    for (int k = 0; k < 6; k++) W[k] += Wl[k];
  }
  if (w6)
    for (int k = 0; k < 6; k++) w6[k] = W[k];
  if (rho_out) memcpy(rho_out, rho, (size_t)n * sizeof(double));
  free(rho);
  free(g);
  free(erep);
  orc_nbr_free(&nb);
  return etot;
}

/*
 * Force on a chosen set of atoms only (for sampled comparisons on systems
 * too large for the full evaluation): for each listed atom i, rho_i, the rho
 * of each neighbour j and F_i, E_i follow the same definitions as
 * orc_forces, over a cell list.  out: fx, fy, fz, e_atom, rho indexed like
 * idx.
 */
void orc_forces_sampled(const orc_pot *P, int64_t n, const double *x,
                        const double *y, const double *z, int64_t m,
                        const int64_t *idx, double *fx, double *fy, double *fz,
                        double *e_atom, double *rho_out) {
  orc_nbr nb;
  orc_nbr_init(&nb, n, x, y, z, 1, P->r_cut);
  const double rc = P->r_cut;
#pragma omp parallel
  {
    int64_t cap = 256, cap2 = 256;
    int64_t *nbr = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int64_t *nbr2 = (int64_t *)malloc((size_t)cap2 * sizeof(int64_t));
#pragma omp for schedule(dynamic, 1)
    for (int64_t s = 0; s < m; s++) {
      int64_t i = idx[s];
      int64_t c = orc_neighbors(&nb, i, rc, &nbr, &cap);
      double rho_i = 0.0, er = 0.0, d;
      for (int64_t k = 0; k < c; k++) {
        int64_t j = nbr[k];
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        rho_i += orc_radial(P, 0, r, &d);
        er += orc_radial(P, 1, r, &d);
      }
      double gi = rho_i > 0.0 ? 1.0 / sqrt(rho_i) : 0.0;
      double Fx = 0.0, Fy = 0.0, Fz = 0.0;
      for (int64_t k = 0; k < c; k++) {
        int64_t j = nbr[k];
        /* rho_j from j's own neighbours */
        int64_t c2 = orc_neighbors(&nb, j, rc, &nbr2, &cap2);
        double rho_j = 0.0;
        for (int64_t k2 = 0; k2 < c2; k2++) {
          int64_t l = nbr2[k2];
          double ex = x[l] - x[j], ey = y[l] - y[j], ez = z[l] - z[j];
          rho_j += orc_radial(P, 0, sqrt(ex * ex + ey * ey + ez * ez), &d);
        }
        double gj = rho_j > 0.0 ? 1.0 / sqrt(rho_j) : 0.0;
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double dphi, dV;
        (void)orc_radial(P, 0, r, &dphi);
        (void)orc_radial(P, 1, r, &dV);
        double sc = (2.0 * dV - 0.5 * (gi + gj) * dphi) / r;
        Fx += sc * dx;
        Fy += sc * dy;
        Fz += sc * dz;
      }
      fx[s] = Fx;
      fy[s] = Fy;
      fz[s] = Fz;
      if (e_atom) e_atom[s] = -sqrt(rho_i) + er;
      if (rho_out) rho_out[s] = rho_i;
    }
    free(nbr);
    free(nbr2);
  }
  orc_nbr_free(&nb);
}

/*
 * Neighbour pairs within rc (ordered, j != i) by brute force: writes the
 * count of each row into cnt[n] and returns the total.  Used to check
 * neighbour lists as sets.
 */
int64_t orc_count_pairs(int64_t n, const double *x, const double *y,
                        const double *z, double rc, int32_t *cnt) {
  int64_t tot = 0;
#pragma omp parallel for reduction(+ : tot) schedule(dynamic, 64)
  for (int64_t i = 0; i < n; i++) {
    int32_t c = 0;
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
      if (dx * dx + dy * dy + dz * dz < rc * rc) c++;
    }
    cnt[i] = c;
    tot += c;
  }
  return tot;
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers.                                             */
/* ------------------------------------------------------------------------ */
/*
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): a 128-bit counter and a 64-bit key; ten rounds of
 * two 32x32->64 multiplications with an S-box-free Feistel-like permutation;
 * the key is advanced by the Weyl constants between rounds.
 */
static void orc_mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, lo0, hi1, lo1;
    orc_mulhilo(M0, c0, &hi0, &lo0);
    orc_mulhilo(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/*
 * The four uniforms of one counter (tag, lo32(step), rep_id, stream) under
 * key (lo32(seed), hi32(seed)); u = (o + 1/2) 2^-32 lies strictly in (0, 1).
 * Streams: 0 thermostat noise, 1 initial velocities, 2 position jitter.
 */
void orc_uniform4(uint64_t seed, uint32_t rep_id, uint32_t tag, uint64_t step,
                  uint32_t stream, double u[4]) {
  uint32_t ctr[4] = {tag, (uint32_t)step, rep_id, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  for (int k = 0; k < 4; k++) u[k] = ((double)o[k] + 0.5) * 0x1p-32;
}

/*
 * Three standard normals from one counter by the Box-Muller transform:
 * (u0, u1) -> sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1), (u2, u3) -> the
 * cosine branch.
 */
void orc_gauss3(uint64_t seed, uint32_t rep_id, uint32_t tag, uint64_t step,
                uint32_t stream, double nrm[3]) {
  double u[4];
  orc_uniform4(seed, rep_id, tag, step, stream, u);
  const double twopi = 6.283185307179586476925286766559;
  double r0 = sqrt(-2.0 * log(u[0]));
  double r1 = sqrt(-2.0 * log(u[2]));
  nrm[0] = r0 * cos(twopi * u[1]);
  nrm[1] = r0 * sin(twopi * u[1]);
  nrm[2] = r1 * cos(twopi * u[3]);
}

/* ------------------------------------------------------------------------ */
/* Molecular dynamics.                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  double dt;      /* ps; 0.002 (Simulation details) */
  double gamma;   /* Langevin friction, 1/ps; 0 gives velocity Verlet (NVE) */
  double T;       /* K */
  double v_pull;  /* Angstrom/ps of the top grip along +z */
  double z_lo;    /* inner face of the fixed grip at t = 0 */
  double z_hi;    /* inner face of the moving grip at t = 0 */
  double mass;    /* amu */
  uint64_t seed;
  uint32_t rep_id;
  int32_t lab_frame; /* 1: thermostat acts on the lab-frame velocity */
  double nh_tau;     /* ps; > 0: Nose-Hoover thermostat (gamma must be 0) */
  double grip_step;  /* stepwise grips: displacement of each grip per hold, A */
  int64_t grip_hold; /* steps per hold; > 0 selects stepwise symmetric grips */
  double T_start;    /* temperature ramp: target T_start at ramp_begin ... */
  int64_t ramp_begin; /* ... rising linearly to T over ramp_steps steps; */
  int64_t ramp_steps; /* ramp_steps = 0: the target is T throughout */
  double baro_mass;  /* amu; > 0: axial barostat on the grip separation */
  double baro_load;  /* eV/A: outward pull on each grip (0: zero stress) */
  double baro_damp;  /* 1/ps: friction on the barostat coordinate */
} orc_md;

/*
 * Target temperature at time t (in steps) (Simulation details: the
 * equilibration ramps the temperature from 0.01 K to the target value),
 * reading: linear in time from T_start at step ramp_begin to T at step
 * ramp_begin + ramp_steps, constant outside.  The thermostats take it at the
 * time of each operation: the Langevin O step at mid-step, the Nose-Hoover
 * half steps at the start and the end of the step, the initial velocities at
 * step 0.
 */
static double orc_target_T(const orc_md *M, double t) {
  if (M->ramp_steps <= 0) return M->T;
  double f = (t - (double)M->ramp_begin) / (double)M->ramp_steps;
  if (f < 0.0) f = 0.0;
  if (f > 1.0) f = 1.0;
  return M->T_start + (M->T - M->T_start) * f;
}

/*
 * Grips.  Continuous pulling (grip_hold = 0): the bottom grip stays, the top
 * one moves at v_pull, so after s steps the top has moved v_pull s dt.
 * Stepwise symmetric grips (Simulation details: both grips displaced by
 * 0.05 A in opposite directions between 20 ps of MD), reading: each hold of
 * grip_hold steps begins with both grips moving grip_step outwards, so after
 * s steps each has moved grip_step * ceil(s / grip_hold).
 * orc_grip_top / orc_grip_bottom: displacement of the top grip along +z and
 * of the bottom grip along -z; their sum is the elongation D of eq 4.
 */
static double orc_grip_top(const orc_md *M, int64_t s) {
  if (M->grip_hold > 0)
    return M->grip_step * (double)((s + M->grip_hold - 1) / M->grip_hold);
  return M->v_pull * (double)s * M->dt;
}

static double orc_grip_bottom(const orc_md *M, int64_t s) {
  if (M->grip_hold > 0)
    return M->grip_step * (double)((s + M->grip_hold - 1) / M->grip_hold);
  return 0.0;
}

static double orc_elongation(const orc_md *M, int64_t s) {
  return orc_grip_top(M, s) + orc_grip_bottom(M, s);
}

double orc_target_temperature(const orc_md *M, double t) {
  return orc_target_T(M, t);
}

/* Streaming velocity of the affine stretch at axial position zz when the top
 * grip has moved by Dg: v_pull (zz - z_lo) / (z_hi - z_lo + Dg); zero in the
 * lab frame, when the grip does not move, or with stepwise grips (which rest
 * between their displacements). */
static double orc_stream_u(const orc_md *M, double zz, double Dg) {
  if (M->lab_frame || M->v_pull == 0.0 || M->grip_hold > 0 ||
      M->baro_mass > 0.0)
    return 0.0;
  return M->v_pull * (zz - M->z_lo) / (M->z_hi - M->z_lo + Dg);
}

/*
 * Initial state (Simulation details: random Gaussian velocities).  Reading:
 * positions of every atom first receive a uniform jitter amp (2u - 1) per
 * component (stream 2, step 0); dynamic atoms get Gaussian velocities of
 * standard deviation sqrt(kB T / m) (stream 1, step 0); their centre-of-mass
 * velocity is removed and they are rescaled to exactly T with 3 N_dyn - 3
 * degrees of freedom; finally the streaming profile of the stretch at t = 0
 * is added.  Grip atoms: fixed ones at rest, moving ones at v_pull along z
 * (at rest with stepwise grips).
 */
void orc_init_state(const orc_md *M, int64_t n, double *x, double *y,
                    double *z, double *vx, double *vy, double *vz,
                    const uint8_t *flag, double jitter) {
  double u[4];
  for (int64_t i = 0; i < n; i++) {
    if (jitter != 0.0) {
      orc_uniform4(M->seed, M->rep_id, (uint32_t)i, 0, 2, u);
      x[i] += jitter * (2.0 * u[0] - 1.0);
      y[i] += jitter * (2.0 * u[1] - 1.0);
      z[i] += jitter * (2.0 * u[2] - 1.0);
    }
  }
  const double T0 = orc_target_T(M, 0.0);
  double sig = sqrt(ORC_KB * T0 / M->mass * ORC_ACC);
  double px = 0, py = 0, pz = 0;
  int64_t ndyn = 0;
  for (int64_t i = 0; i < n; i++) {
    vx[i] = vy[i] = vz[i] = 0.0;
    if (flag[i] == 2 && M->grip_hold == 0 && M->baro_mass == 0.0)
      vz[i] = M->v_pull;
    if (flag[i] != 0) continue;
    double g3[3];
    orc_gauss3(M->seed, M->rep_id, (uint32_t)i, 0, 1, g3);
    vx[i] = sig * g3[0];
    vy[i] = sig * g3[1];
    vz[i] = sig * g3[2];
    px += vx[i];
    py += vy[i];
    pz += vz[i];
    ndyn++;
  }
  if (ndyn == 0) return;
  px /= (double)ndyn;
  py /= (double)ndyn;
  pz /= (double)ndyn;
  double s2 = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (flag[i] != 0) continue;
    vx[i] -= px;
    vy[i] -= py;
    vz[i] -= pz;
    s2 += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
  }
  int64_t dof = 3 * ndyn - 3;
  double scale = 0.0;
  if (s2 > 0.0 && dof > 0)
    scale = sqrt((double)dof * ORC_KB * T0 / (M->mass * s2 / ORC_ACC));
  for (int64_t i = 0; i < n; i++) {
    if (flag[i] != 0) continue;
    vx[i] *= scale;
    vy[i] *= scale;
    vz[i] *= scale;
    vz[i] += orc_stream_u(M, z[i], 0.0);
  }
}

/*
 * Nose-Hoover thermostat (Simulation details), reading: one friction
 * variable zeta per replica acts on the peculiar velocities w = v - u of the
 * dynamic atoms (u the streaming velocity, see orc_stream_u):
 *   dw/dt = F/m - zeta w,   dzeta/dt = (2K - g kB T) / Q,   Q = g kB T tau^2,
 * with K = sum m |w|^2 / 2 and g = 3 N_dyn - 3.  With deta/dt = zeta,
 * E_pot + K + Q zeta^2 / 2 + g kB T eta is a constant of motion while the
 * grips rest.  The paper does not give its discretisation; this follows the
 * symmetric Trotter splitting of the Liouville operator: a thermostat half
 * step before the velocity Verlet step and one after it, each
 *   zeta += dt/4 G(K);  eta += dt/2 zeta;  w *= exp(-zeta dt/2);
 *   zeta += dt/4 G(K'),   G(K) = (2K / (g kB T) - 1) / tau^2,
 * K' the kinetic energy after the scaling.  A replica with T <= 0 or g <= 0
 * is left unthermostatted.  Dg: top-grip displacement (for u); Tt: the
 * target temperature at the time of the half step.
 */
static void orc_nh_half(const orc_md *M, int64_t n, double *vx, double *vy,
                        double *vz, const double *z, const uint8_t *flag,
                        double Dg, double Tt, double *zeta, double *eta) {
  int64_t ndyn = 0;
  double w2 = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (flag[i] != 0) continue;
    double wz = vz[i] - orc_stream_u(M, z[i], Dg);
    w2 += vx[i] * vx[i] + vy[i] * vy[i] + wz * wz;
    ndyn++;
  }
  double g = (double)(3 * ndyn - 3);
  if (!(g > 0.0) || !(Tt > 0.0)) return;
  double gkT = g * ORC_KB * Tt;
  double tau2 = M->nh_tau * M->nh_tau;
  double K = 0.5 * M->mass * w2 / ORC_ACC;
  *zeta += 0.25 * M->dt * (2.0 * K / gkT - 1.0) / tau2;
  *eta += 0.5 * M->dt * *zeta;
  double sc = exp(-0.5 * M->dt * *zeta);
  w2 = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (flag[i] != 0) continue;
    double u = orc_stream_u(M, z[i], Dg);
    vx[i] *= sc;
    vy[i] *= sc;
    vz[i] = u + sc * (vz[i] - u);
    double wz = vz[i] - u;
    w2 += vx[i] * vx[i] + vy[i] * vy[i] + wz * wz;
  }
  K = 0.5 * M->mass * w2 / ORC_ACC;
  *zeta += 0.25 * M->dt * (2.0 * K / gkT - 1.0) / tau2;
}

/*
 * Axial barostat (Simulation details: the equilibration holds zero pressure
 * along [100] with a Nose-Hoover barostat).  Reading: the wire is finite and
 * held by rigid grips, so the length the barostat controls is the grip
 * separation.  Both grips move by s, outwards, from their reference
 * positions; s is an extended coordinate of mass W (baro_mass) whose
 * equation of motion is
 *   W d2s/dt2 = Q + 2 F_load,   Q = -dE/ds = sum_top F_z - sum_bottom F_z,
 * F_load (baro_load) the outward pull on each grip: zero for zero axial
 * stress.  E_pot + K + W (ds/dt)^2 / 2 - 2 F_load s is then a constant of
 * motion without thermostat.  Atoms are not rescaled: the grips pass the
 * load to the wire.  Integrated with the particles by velocity Verlet.  The
 * barostat coordinate exchanges energy with the wire only through the grips,
 * so an optional friction gamma_b (baro_damp) relaxes it: ds/dt is
 * multiplied by exp(-gamma_b dt/2) before its first and after its second
 * half kick of each step.  The piston then settles where Q = -2 F_load.
 */
static double orc_grip_force(int64_t n, const uint8_t *flag,
                             const double *fz) {
  double q = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (flag[i] == 2) q += fz[i];
    else if (flag[i] == 1) q -= fz[i];
  }
  return q;
}

/*
 * n_steps of velocity Verlet (Simulation details: dt = 2 fs) with the rigid
 * grips of Figure 1 (Simulation details: two rigid layers at each end) and
 * one of three thermostats: none (gamma = 0, nh_tau = 0), the Langevin
 * thermostat of the configurations in BAOAB order (gamma > 0), or the
 * Nose-Hoover thermostat of the paper (nh_tau > 0, orc_nh_half), each at
 * the target temperature of orc_target_T.
 * Step s -> s+1, on dynamic atoms (flag 0):
 *   [Nose-Hoover half step at the positions of step s]
 *   [barostat: ds/dt *= exp(-gamma_b dt/2); ds/dt += dt/2 (Q + 2 F_load)/W
 *    with the forces of step s; s += dt ds/dt]
 *   B: v += dt/2 F/m;  A: x += dt/2 v;
 *   O (Langevin only): v = u + c1 (v - u) + c2 sqrt(kB T/m) n,
 *      c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2), u the streaming velocity at
 *      mid-step (zero in the lab frame), n from the counter (tag, s, rep_id,
 *      stream 0);
 *   A: x += dt/2 v;
 * grips: bottom ones at z0 minus the bottom grip's travel, top ones at z0
 * plus the top grip's travel (x, y unchanged): orc_grip_top/orc_grip_bottom
 * after s+1 steps, or the barostat's s; v = 0 except v_z = v_pull on top
 * when pulling continuously; then forces at the new positions,
 * B: v += dt/2 F/m, [barostat: ds/dt += dt/2 (Q + 2 F_load)/W with the new
 * forces; ds/dt *= exp(-gamma_b dt/2)] and [Nose-Hoover half step at the
 * positions of step s+1].
 * On entry fx, fy, fz hold F at step0; on return F at step0 + n_steps and
 * e_atom (may be NULL) the per-atom energies there.  zeta, eta: the
 * Nose-Hoover variables (used when nh_tau > 0); piston: s and ds/dt of the
 * barostat (used when baro_mass > 0); all read and updated.
 * mode: 0 brute force, 1 cell list (orc_forces).
 */
void orc_run(const orc_pot *P, const orc_md *M, int64_t n, double *x,
             double *y, double *z, double *vx, double *vy, double *vz,
             const double *z0, const uint8_t *flag, double *fx, double *fy,
             double *fz, double *e_atom, int64_t step0, int64_t n_steps,
             int mode, double *zeta, double *eta, double *piston) {
  const double dt = M->dt;
  const double ac = ORC_ACC / M->mass; /* eV/A per amu -> A/ps^2 */
  const double c1 = exp(-M->gamma * dt);
  const double c2 = sqrt(1.0 - c1 * c1);
  const int nh = M->nh_tau > 0.0;
  const int baro = M->baro_mass > 0.0;
  const double acb = baro ? ORC_ACC / M->baro_mass : 0.0;
  const double damp = exp(-0.5 * M->baro_damp * dt);
  for (int64_t s = step0; s < step0 + n_steps; s++) {
    double Dmid = M->v_pull * ((double)s + 0.5) * dt;
    const double sig =
        sqrt(ORC_KB * orc_target_T(M, (double)s + 0.5) / M->mass * ORC_ACC);
    if (nh)
      orc_nh_half(M, n, vx, vy, vz, z, flag, orc_grip_top(M, s),
                  orc_target_T(M, (double)s), zeta, eta);
    if (baro) {
      const double q = orc_grip_force(n, flag, fz) + 2.0 * M->baro_load;
      piston[1] *= damp;
      piston[1] += 0.5 * dt * acb * q;
      piston[0] += dt * piston[1];
    }
    double top = baro ? piston[0] : orc_grip_top(M, s + 1);
    double bottom = baro ? piston[0] : orc_grip_bottom(M, s + 1);
    for (int64_t i = 0; i < n; i++) {
      if (flag[i] == 0) {
        vx[i] += 0.5 * dt * ac * fx[i];
        vy[i] += 0.5 * dt * ac * fy[i];
        vz[i] += 0.5 * dt * ac * fz[i];
        x[i] += 0.5 * dt * vx[i];
        y[i] += 0.5 * dt * vy[i];
        z[i] += 0.5 * dt * vz[i];
        if (M->gamma > 0.0) {
          double g3[3];
          orc_gauss3(M->seed, M->rep_id, (uint32_t)i, (uint64_t)s, 0, g3);
          double uz = orc_stream_u(M, z[i], Dmid);
          vx[i] = c1 * vx[i] + c2 * sig * g3[0];
          vy[i] = c1 * vy[i] + c2 * sig * g3[1];
          vz[i] = uz + c1 * (vz[i] - uz) + c2 * sig * g3[2];
        }
        x[i] += 0.5 * dt * vx[i];
        y[i] += 0.5 * dt * vy[i];
        z[i] += 0.5 * dt * vz[i];
      } else if (flag[i] == 1) {
        z[i] = z0[i] - bottom;
        vx[i] = vy[i] = vz[i] = 0.0;
      } else if (flag[i] == 2) {
        z[i] = z0[i] + top;
        vx[i] = vy[i] = 0.0;
        vz[i] = (M->grip_hold > 0 || baro) ? 0.0 : M->v_pull;
      }
    }
    orc_forces(P, n, x, y, z, mode, NULL, e_atom, fx, fy, fz, NULL);
    for (int64_t i = 0; i < n; i++) {
      if (flag[i] != 0) continue;
      vx[i] += 0.5 * dt * ac * fx[i];
      vy[i] += 0.5 * dt * ac * fy[i];
      vz[i] += 0.5 * dt * ac * fz[i];
    }
    if (baro) {
      const double q = orc_grip_force(n, flag, fz) + 2.0 * M->baro_load;
      piston[1] += 0.5 * dt * acb * q;
      piston[1] *= damp;
    }
    if (nh)
      orc_nh_half(M, n, vx, vy, vz, z, flag, top,
                  orc_target_T(M, (double)(s + 1)), zeta, eta);
  }
}

static int orc_cmp_double(const void *a, const void *b) {
  double da = *(const double *)a, db = *(const double *)b;
  return (da > db) - (da < db);
}

/*
 * Per-replica observables at step s (Results: eqs 4 and 5; failure, the end
 * of the stress-strain runs).  out[0..7]:
 *  0 E_pot (eV, eq 3)             1 KE of dynamic atoms, peculiar (eV)
 *  2 T (K), dof = 3 N_dyn - 3     3 -W_zz = 1/2 sum_i sum_j E'_ij dz^2 / r (eV)
 *  4 sigma_zz (GPa)               5 strain D/L0 (eq 4)
 *  6 largest empty axial gap between consecutive atoms (A)
 *  7 D, the elongation: the sum of both grips' displacements (A)
 * Readings: eq 5's kinetic term is read as m v_z,i^2 (the printed v_x,i v_x,j
 * is a typo), with peculiar velocities v - u (u the streaming profile, zero in
 * the lab frame) over dynamic atoms; V is the constant hard-sphere volume
 * passed in; eq 4's L - L0 is the elongation D (v_pull s dt when pulling
 * continuously, orc_elongation; twice the piston's s with the barostat,
 * piston may be NULL otherwise).
 */
void orc_observe(const orc_pot *P, const orc_md *M, int64_t n,
                 const double *x, const double *y, const double *z,
                 const double *vx, const double *vy, const double *vz,
                 const uint8_t *flag, int64_t step, double vol, double L0,
                 const double *piston, double out[8]) {
  double w6[6];
  double ep = orc_forces(P, n, x, y, z, 1, NULL, NULL, NULL, NULL, NULL, w6);
  double Dg = orc_grip_top(M, step);
  double ke = 0.0, kz = 0.0;
  int64_t ndyn = 0;
  for (int64_t i = 0; i < n; i++) {
    if (flag[i] != 0) continue;
    double uz = orc_stream_u(M, z[i], Dg);
    double wz = vz[i] - uz;
    ke += vx[i] * vx[i] + vy[i] * vy[i] + wz * wz;
    kz += wz * wz;
    ndyn++;
  }
  ke *= 0.5 * M->mass / ORC_ACC;
  kz *= M->mass / ORC_ACC;
  int64_t dof = 3 * ndyn - 3;
  /* largest gap between consecutive z values */
  double *zs = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  memcpy(zs, z, (size_t)n * sizeof(double));
  qsort(zs, (size_t)n, sizeof(double), orc_cmp_double);
  double gap = 0.0;
  for (int64_t i = 1; i < n; i++)
    if (zs[i] - zs[i - 1] > gap) gap = zs[i] - zs[i - 1];
  free(zs);
  out[0] = ep;
  out[1] = ke;
  out[2] = dof > 0 ? 2.0 * ke / ((double)dof * ORC_KB) : 0.0;
  out[3] = -w6[2];
  out[4] = (-w6[2] - kz) / vol * ORC_EVA3_GPA;
  const double D = M->baro_mass > 0.0 ? 2.0 * piston[0]
                                      : orc_elongation(M, step);
  out[5] = D / L0;
  out[6] = gap;
  out[7] = D;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
