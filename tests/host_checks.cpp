// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py: the descriptor
// validation, workspace sizing and statistics-to-status functions, which run
// on the host only and must never read the device pointers they are handed
// (here addresses no process can read, so a read would fault under ASan).
// Every call's status is checked; exit code 0 means every check held.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "radiotrace.h"
#include "radiotrace_mlp.h"
#include "radiotrace_solve.h"

namespace {
int failures = 0;
void expect(const char* what, rt_status got, rt_status want) {
  if (got != want) {
    std::printf("FAIL %s: status %d, expected %d (%s)\n", what, (int)got, (int)want,
                rt_last_error());
    ++failures;
  }
}
const void* fake(uintptr_t a) { return reinterpret_cast<const void*>(a); }
const double kNaN = std::numeric_limits<double>::quiet_NaN();
const double kInf = std::numeric_limits<double>::infinity();
}  // namespace

int main() {
  // a two-layer firn scene: air, firn, deep firn; surface and layer planes
  rt_region reg[RT_MAX_REGIONS];
  std::memset(reg, 0, sizeof reg);
  reg[0] = {1.0, 0.0, 0.0, 0.0, -1e9, 0.0, 0, {0, 0, 0}};
  reg[1] = {1.78, 0.0, 0.43, 75.0, 0.0, 150.0, 0, {0, 0, 0}};
  reg[2] = {1.79, 0.0, 0.43, 75.0, 150.0, 1e9, 0, {0, 0, 0}};
  rt_field field;
  std::memset(&field, 0, sizeof field);
  field.n_regions = 3;
  field.regions = reg;
  rt_plane pl[RT_MAX_PLANES];
  std::memset(pl, 0, sizeof pl);
  pl[0] = {{0, 0, 0}, {0, 0, 1}, 1, 0, RT_PLANE_FRESNEL, RT_SHAPE_PLANE, 0.0};
  pl[1] = {{0, 0, 150}, {0, 0, 1}, 2, 1, RT_PLANE_FRESNEL, RT_SHAPE_PLANE, 0.0};
  rt_boundaries bnd;
  std::memset(&bnd, 0, sizeof bnd);
  bnd.n_planes = 2;
  bnd.planes = pl;
  rt_sources src = {static_cast<const double*>(fake(0x10)), 64};
  rt_directions dirs = {static_cast<const double*>(fake(0x20)),
                        static_cast<const int32_t*>(fake(0x30)), 1 << 20};
  rt_step_limits lim;
  std::memset(&lim, 0, sizeof lim);
  lim.h_min = 1e-3;
  lim.h_max = 10.0;
  lim.s_max = 5000.0;
  lim.max_generations = 4;
  lim.model = RT_MODEL_PAPER;
  lim.max_steps_per_ray = 1 << 20;

  expect("valid", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &lim), RT_OK);
  expect("null field", rt_validate(nullptr, &bnd, &src, &dirs, 1e-6, &lim), RT_ERR_INVALID_ARG);
  expect("tol 0", rt_validate(&field, &bnd, &src, &dirs, 0.0, &lim), RT_ERR_INVALID_ARG);
  expect("tol NaN", rt_validate(&field, &bnd, &src, &dirs, kNaN, &lim), RT_ERR_INVALID_ARG);
  {
    rt_step_limits l = lim;
    l.max_generations = 5;
    expect("5 generations", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &l),
           RT_ERR_UNSUPPORTED);
    l = lim;
    l.h_min = 20.0;
    expect("h_min > h_max", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &l),
           RT_ERR_INVALID_ARG);
    l = lim;
    l.s_max = kInf;
    expect("s_max inf", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &l), RT_ERR_INVALID_ARG);
    l = lim;
    l.resume = 2;
    expect("resume 2", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &l), RT_ERR_INVALID_ARG);
  }
  {
    rt_field f = field;
    f.n_regions = RT_MAX_REGIONS + 1;
    expect("too many regions", rt_validate(&f, &bnd, &src, &dirs, 1e-6, &lim),
           RT_ERR_INVALID_ARG);
    reg[1].z0 = 0.0;
    expect("z0 = 0", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &lim), RT_ERR_INVALID_ARG);
    reg[1].z0 = 75.0;
    reg[2].a = kNaN;
    expect("NaN index", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &lim), RT_ERR_INVALID_ARG);
    reg[2].a = 1.79;
  }
  {
    rt_boundaries b = bnd;
    b.n_planes = RT_MAX_PLANES + 1;
    expect("too many planes", rt_validate(&field, &b, &src, &dirs, 1e-6, &lim),
           RT_ERR_INVALID_ARG);
    pl[1].region_neg = 3;
    expect("plane region", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &lim),
           RT_ERR_INVALID_ARG);
    pl[1].region_neg = 1;
    pl[1].shape = RT_SHAPE_SPHERE;
    pl[1].param = -1.0;
    expect("sphere radius", rt_validate(&field, &bnd, &src, &dirs, 1e-6, &lim),
           RT_ERR_INVALID_ARG);
    pl[1].shape = RT_SHAPE_PLANE;
    pl[1].param = 0.0;
    b = bnd;
    b.has_box = 1;
    b.box_lo[0] = b.box_lo[1] = b.box_lo[2] = -1.0;
    b.box_hi[0] = b.box_hi[1] = 1.0;
    b.box_hi[2] = -2.0;
    expect("box lo >= hi", rt_validate(&field, &b, &src, &dirs, 1e-6, &lim), RT_ERR_INVALID_ARG);
  }
  {
    // every table full: 8 media, 16 surfaces of all shapes, a box, 8 anomalies
    rt_region r8[RT_MAX_REGIONS];
    for (int i = 0; i < RT_MAX_REGIONS; ++i)
      r8[i] = {1.3 + 0.01 * i, 1e-4, 0.1, 50.0, 100.0 * i, 100.0 * (i + 1), 0, {0, 0, 0}};
    rt_anomaly an[RT_MAX_ANOMALIES];
    for (int j = 0; j < RT_MAX_ANOMALIES; ++j)
      an[j] = {{10.0 * j, 0, 50}, 0.01, 5.0, j % RT_MAX_REGIONS};
    rt_field f8 = {RT_MAX_REGIONS, r8, {}, RT_MAX_ANOMALIES, an};
    rt_plane p16[RT_MAX_PLANES];
    for (int k = 0; k < RT_MAX_PLANES; ++k)
      p16[k] = {{0, 0, 50.0 * k}, {0, 0, 1}, (k + 1) % RT_MAX_REGIONS, k % RT_MAX_REGIONS,
                k % 2 ? RT_PLANE_ABSORB : RT_PLANE_FRESNEL, k % 3, k % 3 ? 25.0 : 0.0};
    rt_boundaries b16 = {RT_MAX_PLANES, p16, 1, {-1e4, -1e4, -1e4}, {1e4, 1e4, 1e4}};
    expect("full tables", rt_validate(&f8, &b16, &src, &dirs, 1e-6, &lim), RT_OK);
    size_t ws = 0;
    expect("workspace, full tables", rt_workspace_bytes(&f8, 1 << 22, &ws), RT_OK);
    if (ws == 0) {
      std::printf("FAIL workspace bytes 0\n");
      ++failures;
    }
    an[3].sigma = 1e-200;
    expect("tiny sigma", rt_validate(&f8, &b16, &src, &dirs, 1e-6, &lim), RT_ERR_INVALID_ARG);
  }
  {
    // a grid region: sizes and spacing are checked, the data pointer is not read
    rt_region rg[2] = {{1.0, 0, 0, 0, -1e9, 0.0, 0, {0, 0, 0}},
                       {0.0, 0, 0, 0, 0.0, 1e9, 1, {0, 0, 0}}};
    rt_field fg = {2, rg, {}, 0, nullptr};
    fg.grid.n = static_cast<const float*>(fake(0x40));
    fg.grid.nx = 256;
    fg.grid.ny = 256;
    fg.grid.nz = 128;
    for (int a = 0; a < 3; ++a) fg.grid.spacing[a] = 10.0;
    rt_plane p1 = {{0, 0, 0}, {0, 0, 1}, 1, 0, RT_PLANE_FRESNEL, RT_SHAPE_PLANE, 0.0};
    rt_boundaries b1 = {1, &p1, 0, {}, {}};
    expect("grid", rt_validate(&fg, &b1, &src, &dirs, 1e-7, &lim), RT_OK);
    size_t ws = 0;
    expect("grid workspace", rt_workspace_bytes(&fg, 1 << 22, &ws), RT_OK);
    fg.grid.nz = 1;
    expect("grid nz 1", rt_validate(&fg, &b1, &src, &dirs, 1e-7, &lim), RT_ERR_INVALID_ARG);
    fg.grid.nz = 128;
    fg.grid.spacing[1] = 0.0;
    expect("grid spacing 0", rt_validate(&fg, &b1, &src, &dirs, 1e-7, &lim), RT_ERR_INVALID_ARG);
  }
  {
    rt_stats st;
    std::memset(&st, 0, sizeof st);
    st.records = 10;
    st.needed = 10;
    expect("collect ok", rt_collect(&st, 10), RT_OK);
    st.needed = 11;
    expect("collect capacity", rt_collect(&st, 10), RT_ERR_CAPACITY);
    st.needed = 10;
    st.interrupted = 1;
    expect("collect interrupted", rt_collect(&st, 10), RT_INTERRUPTED);
    st.interrupted = 0;
    st.sched_errors = 1;
    expect("collect scheduler", rt_collect(&st, 10), RT_ERR_DEVICE);
    expect("collect null", rt_collect(nullptr, 10), RT_ERR_INVALID_ARG);
  }
  {
    // solves: the surface first, no box, no time limit
    rt_solve_params sp = {64, 60, 4, 1e-4, 1e-3, 1e7};
    expect("solve valid", rt_solve_validate(&field, &bnd, 1e-6, &lim, &sp), RT_OK);
    size_t ws = 0;
    expect("solve workspace", rt_solve_workspace_bytes(&field, 1 << 20, &sp, &ws), RT_OK);
    rt_solve_params bad = sp;
    bad.n_scan = 1;
    expect("n_scan 1", rt_solve_validate(&field, &bnd, 1e-6, &lim, &bad), RT_ERR_INVALID_ARG);
    bad = sp;
    bad.accept_tol = 1e-5;
    expect("accept < miss tol", rt_solve_validate(&field, &bnd, 1e-6, &lim, &bad),
           RT_ERR_INVALID_ARG);
    rt_step_limits l = lim;
    l.t_max = 1e-6;
    expect("solve with t_max", rt_solve_validate(&field, &bnd, 1e-6, &l, &sp),
           RT_ERR_INVALID_ARG);
  }
  if (rt_abi_version() != RT_ABI_VERSION) {
    std::printf("FAIL abi version %d\n", rt_abi_version());
    ++failures;
  }
  if (failures) return 1;
  std::printf("host checks ok\n");
  return 0;
}
