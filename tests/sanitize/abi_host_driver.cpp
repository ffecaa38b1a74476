// Runs the host-side code of libtbsma (the wire builder, the argument checks,
// the workspace layout, the size check of the allocation-free entry point and
// the error messages) for a build whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Every call here
// returns before a device is touched, so no GPU is needed.  Test
// infrastructure; exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tbsma.h"

static int failures = 0;

static void check(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "abi host driver: check failed: %s (%s)\n", what,
                 tbsma_last_error());
    failures++;
  }
}

static bool msg_has(const char *s) {
  return std::strstr(tbsma_last_error(), s) != nullptr;
}

static tbsma_params params() {
  tbsma_params p;
  std::memset(&p, 0, sizeof(p));
  p.A = 0.2061;
  p.xi = 1.790;
  p.p = 10.229;
  p.q = 4.036;
  p.r0 = 2.884;
  p.r_tail = 6.5;
  p.r_cut = 7.0;
  p.skin = 1.0;
  p.cell = 8.0;
  p.mass = 196.96657;
  p.precision = TBSMA_MIXED;
  p.qbits = 21;
  p.prune = 0.15;
  return p;
}

int main() {
  // --- wire builder: count, fill, notch, short capacity, bad arguments ------
  int64_t n = 0;
  check(tbsma_build_wire(4.08, 30.0, 40.8, 2, 0, 0.0, nullptr, nullptr,
                         nullptr, nullptr, 0, &n) == TBSMA_ECAPACITY &&
            n > 0,
        "count only");
  std::vector<double> x(n), y(n), z(n);
  std::vector<uint8_t> f(n);
  int64_t m = 0;
  check(tbsma_build_wire(4.08, 30.0, 40.8, 2, 0, 0.0, x.data(), y.data(),
                         z.data(), f.data(), n, &m) == TBSMA_OK &&
            m == n,
        "fill");
  check(tbsma_build_wire(4.08, 30.0, 40.8, 2, 0, 0.0, x.data(), y.data(),
                         z.data(), f.data(), n - 1, &m) == TBSMA_ECAPACITY &&
            m == n,
        "capacity short by one");
  check(tbsma_build_wire(4.08, 30.0, 40.8, 2, 3, 4.08, x.data(), y.data(),
                         z.data(), f.data(), n, &m) == TBSMA_OK &&
            m < n,
        "notch");
  check(tbsma_build_wire(-1.0, 30.0, 40.8, 2, 0, 0.0, nullptr, nullptr,
                         nullptr, nullptr, 0, &m) == TBSMA_EINVAL,
        "negative lattice constant");
  check(tbsma_build_wire(4.08, 30.0, 40.8, 2, -1, 0.0, nullptr, nullptr,
                         nullptr, nullptr, 0, &m) == TBSMA_EINVAL &&
            msg_has("notch"),
        "negative notch");
  check(tbsma_build_wire(4.08, 0.0, 0.0, 0, 0, 0.0, nullptr, nullptr, nullptr,
                         nullptr, 0, &m) == TBSMA_OK &&
            m == 0,
        "empty wire");

  // --- workspace layout of valid systems ------------------------------------
  void *ph = reinterpret_cast<void *>(0x1000);
  auto system = [&](int R, const std::vector<int64_t> &rep,
                    const std::vector<int64_t> &cel) {
    tbsma_system s;
    std::memset(&s, 0, sizeof(s));
    s.R = R;
    s.max_zbins = 64;
    s.N = rep.back();
    s.C = cel.back();
    s.rep_off_h = rep.data();
    s.cell_off_h = cel.data();
    s.rep_off = s.cell_off = static_cast<const int64_t *>(ph);
    s.tile_rep = s.grid_dim = s.rep_id = static_cast<const int32_t *>(ph);
    s.grid_lo = static_cast<const double *>(ph);
    s.x = s.y = s.z = s.vx = s.vy = s.vz = s.z0 = static_cast<double *>(ph);
    s.flag = static_cast<uint8_t *>(ph);
    s.qpos = static_cast<int32_t *>(ph);
    return s;
  };
  tbsma_params p = params();
  std::vector<int64_t> rep3 = {0, 640, 704, 2048}, cel3 = {0, 100, 150, 400};
  tbsma_system s3 = system(3, rep3, cel3);
  size_t b3 = 0, b1 = 0;
  check(tbsma_workspace_query(&p, &s3, &b3) == TBSMA_OK && b3 > 0, "R = 3");
  std::vector<int64_t> rep1 = {0, 64}, cel1 = {0, 8};
  tbsma_system s1 = system(1, rep1, cel1);
  check(tbsma_workspace_query(&p, &s1, &b1) == TBSMA_OK && b1 < b3, "R = 1");
  tbsma_params pd = params();
  pd.precision = TBSMA_FP64;
  check(tbsma_workspace_query(&pd, &s3, &b3) == TBSMA_OK, "FP64");

  // --- refused parameters and layouts --------------------------------------
  struct Bad {
    void (*set)(tbsma_params &);
    const char *msg;
  } bad[] = {
      {[](tbsma_params &q) { q.r_tail = 8.0; }, "r_tail"},
      {[](tbsma_params &q) { q.cell = 7.5; }, "cell"},
      {[](tbsma_params &q) { q.cell = 16.0; }, "cell/2"},
      {[](tbsma_params &q) { q.precision = 7; }, "precision"},
      {[](tbsma_params &q) { q.qbits = 30; }, "qbits"},
      {[](tbsma_params &q) { q.prune = 0.9; }, "prune"},
      {[](tbsma_params &q) { q.mass = 0.0; }, "mass"},
      {[](tbsma_params &q) { q.r0 = std::nan(""); }, "positive"},
  };
  for (const Bad &b : bad) {
    tbsma_params q = params();
    b.set(q);
    size_t bytes = 0;
    check(tbsma_workspace_query(&q, &s1, &bytes) == TBSMA_EINVAL &&
              msg_has(b.msg),
          b.msg);
  }
  std::vector<int64_t> rep_odd = {0, 100}, cel_odd = {0, 8};
  tbsma_system so = system(1, rep_odd, cel_odd);
  size_t bytes = 0;
  check(tbsma_workspace_query(&p, &so, &bytes) == TBSMA_EINVAL, "odd N");
  tbsma_system sn = s1;
  sn.x = nullptr;
  check(tbsma_workspace_query(&p, &sn, &bytes) == TBSMA_EINVAL &&
            msg_has("NULL"),
        "NULL array");
  check(tbsma_workspace_query(nullptr, &s1, &bytes) == TBSMA_EINVAL,
        "NULL params");
  check(tbsma_workspace_query(&p, nullptr, &bytes) == TBSMA_EINVAL,
        "NULL system");

  // --- calls refused before any device work ---------------------------------
  tbsma_cells cells = {static_cast<int32_t *>(ph), static_cast<int32_t *>(ph)};
  tbsma_nlist nl;
  std::memset(&nl, 0, sizeof(nl));
  nl.nl = nl.nn = nl.nl_lane = static_cast<int32_t *>(ph);
  nl.k_cap = 8;
  nl.x_ref = nl.y_ref = nl.z_ref = static_cast<double *>(ph);
  tbsma_forces_out out;
  std::memset(&out, 0, sizeof(out));
  out.fx = out.fy = out.fz = out.e_atom = ph;
  out.rep_energy = out.rep_wzz = static_cast<double *>(ph);
  tbsma_md md;
  std::memset(&md, 0, sizeof(md));
  md.dt = 0.002;
  md.n_log = 10;
  md.n_slots = 4;
  md.T = md.v_pull = md.z_lo = md.z_hi = md.vol = md.L0 =
      static_cast<const double *>(ph);
  md.seed = static_cast<const uint64_t *>(ph);
  md.dof = static_cast<const int32_t *>(ph);
  md.step = static_cast<int64_t *>(ph);
  md.obs = static_cast<double *>(ph);
  md.status = static_cast<uint32_t *>(ph);
  md.gamma = 1.0;
  md.nh_tau = 0.1;  // Langevin and Nose-Hoover exclude each other
  check(tbsma_step(&p, &s1, &cells, &nl, &out, &md, nullptr, 1, nullptr) ==
                TBSMA_EINVAL &&
            msg_has("exclude"),
        "step: thermostats");
  check(tbsma_run_batch(&p, &s1, &cells, &nl, &out, &md, nullptr, 10, 0,
                        nullptr) == TBSMA_EINVAL,
        "run_batch: settings");
  check(tbsma_forces(&p, &s1, nullptr, &out, nullptr, nullptr) ==
            TBSMA_EINVAL,
        "forces: NULL lists");
  nl.k_cap = 12;
  check(tbsma_neighbors(&p, &s1, &cells, &nl, nullptr, nullptr, nullptr) ==
                TBSMA_EINVAL &&
            msg_has("k_cap"),
        "neighbors: k_cap");
  nl.k_cap = 8;
  check(tbsma_forces_pass(&p, &s1, &nl, &out, nullptr, 4, nullptr) ==
            TBSMA_EINVAL,
        "forces_pass: pass number");
  check(tbsma_rng_fill(1, 2, 3, 0, -1, nullptr, nullptr, nullptr) ==
            TBSMA_EINVAL,
        "rng_fill: n < 0");
  check(tbsma_rng_fill(1, 2, 3, 0, 0, nullptr, nullptr, nullptr) == TBSMA_OK,
        "rng_fill: n = 0");
  check(tbsma_event_counts(&p, &s1, nullptr, nullptr, nullptr) ==
            TBSMA_EINVAL,
        "event_counts: NULL");
  int64_t st2[2];
  check(tbsma_list_stats(&p, &s1, &nl, nullptr, st2, nullptr) == TBSMA_EINVAL,
        "list_stats: NULL work");
  std::vector<int64_t> rep0 = {0}, cel0 = {0};
  tbsma_system s0 = system(0, rep0, cel0);
  check(tbsma_step(&p, &s0, &cells, &nl, &out, &md, nullptr, 0, nullptr) ==
            TBSMA_EINVAL,
        "step: settings checked for R = 0");
  md.nh_tau = 0.0;
  check(tbsma_step(&p, &s0, &cells, &nl, &out, &md, nullptr, 5, nullptr) ==
            TBSMA_OK,
        "step: nothing to do for R = 0");

  // --- the other entry points: refusals and no-ops, all before device work
  check(tbsma_workspace_init(&p, &s0, nullptr, nullptr) == TBSMA_OK,
        "workspace_init: nothing to do for R = 0");
  check(tbsma_workspace_init(&p, &s1, nullptr, nullptr) == TBSMA_EINVAL &&
            msg_has("work"),
        "workspace_init: NULL work");
  check(tbsma_init_state(&p, &s0, &md, nullptr, 0.0, nullptr) == TBSMA_OK,
        "init_state: nothing to do for R = 0");
  check(tbsma_init_state(&p, &s1, nullptr, nullptr, 0.0, nullptr) ==
            TBSMA_EINVAL,
        "init_state: NULL md");
  int32_t dof1[1];
  double v1[1], lo1[1], hi1[1];
  check(tbsma_replica_constants(&p, &s1, nullptr, v1, lo1, hi1, nullptr) ==
                TBSMA_EINVAL &&
            msg_has("dof"),
        "replica_constants: NULL dof");
  check(tbsma_replica_constants(&p, &s0, dof1, v1, lo1, hi1, nullptr) ==
            TBSMA_OK,
        "replica_constants: nothing to do for R = 0");
  check(tbsma_rebase(&p, &s1, nullptr, nullptr, nullptr) == TBSMA_EINVAL &&
            msg_has("L0"),
        "rebase: NULL L0");
  check(tbsma_rebase(&p, &s0, v1, nullptr, nullptr) == TBSMA_OK,
        "rebase: nothing to do for R = 0");
  check(tbsma_build_cells(&p, &s1, nullptr, nullptr, nullptr) ==
                TBSMA_EINVAL &&
            msg_has("cells"),
        "build_cells: NULL cells");
  tbsma_cells no_cells = {nullptr, static_cast<int32_t *>(ph)};
  check(tbsma_build_cells(&p, &s1, &no_cells, nullptr, nullptr) ==
                TBSMA_EINVAL &&
            msg_has("cell arrays"),
        "build_cells: cell arrays missing");
  check(tbsma_build_cells(&p, &s0, &cells, nullptr, nullptr) == TBSMA_OK,
        "build_cells: nothing to do for R = 0");
  check(tbsma_rng_normals_f32(1, 2, 3, 0, -1, nullptr, nullptr) ==
            TBSMA_EINVAL,
        "rng_normals_f32: n < 0");
  check(tbsma_rng_normals_f32(1, 2, 3, 0, 4, nullptr, nullptr) ==
            TBSMA_EINVAL,
        "rng_normals_f32: NULL output");
  check(tbsma_rng_normals_f32(1, 2, 3, 0, 0, nullptr, nullptr) == TBSMA_OK,
        "rng_normals_f32: n = 0");
  // launch shapes: both arrays or neither, and only the listed shapes
  int32_t shape_bad[1] = {3}, shape_ok[1] = {TBSMA_SHAPE(2, 0)};
  tbsma_system sh = s1;
  sh.shape_h = shape_ok;
  check(tbsma_workspace_query(&p, &sh, &bytes) == TBSMA_EINVAL &&
            msg_has("both"),
        "shape_h without shape");
  sh.shape = static_cast<const int32_t *>(ph);
  check(tbsma_workspace_query(&p, &sh, &bytes) == TBSMA_OK,
        "a valid launch shape");
  sh.shape_h = shape_bad;
  check(tbsma_workspace_query(&p, &sh, &bytes) == TBSMA_EINVAL &&
            msg_has("launch shape"),
        "3 tiles per block");
  shape_bad[0] = TBSMA_SHAPE(4, 2);
  check(tbsma_workspace_query(&p, &sh, &bytes) == TBSMA_EINVAL,
        "stage class 2");
  // the allocation-free step: settings, then the size of its static scratch
  md.nh_tau = 0.0;
  check(tbsma_step_noalloc(&p, &s1, &cells, &nl, &out, &md, -1, nullptr) ==
            TBSMA_EINVAL,
        "step_noalloc: n_steps < 0");
  check(tbsma_step_noalloc(&p, &s1, &cells, &nl, &out, &md, 0, nullptr) ==
            TBSMA_OK,
        "step_noalloc: zero steps");
  check(tbsma_step_noalloc(&p, &s1, nullptr, &nl, &out, &md, 1, nullptr) ==
            TBSMA_EINVAL,
        "step_noalloc: NULL cells");
  tbsma_forces_out out_nr = out;
  out_nr.rep_energy = nullptr;
  check(tbsma_step_noalloc(&p, &s1, &cells, &nl, &out_nr, &md, 1, nullptr) ==
            TBSMA_EINVAL,
        "step_noalloc: no per-replica outputs");
  std::vector<int64_t> rep_big = {0, (int64_t)64 * 40000}, cel_big = {0, 8};
  tbsma_system sb = system(1, rep_big, cel_big);
  check(tbsma_step_noalloc(&p, &sb, &cells, &nl, &out, &md, 1, nullptr) ==
                TBSMA_ECAPACITY &&
            msg_has("static scratch"),
        "step_noalloc: system beyond its scratch");

  if (failures) return 1;
  std::printf("abi host driver: all checks passed (%lld-atom wire)\n",
              (long long)n);
  return 0;
}
