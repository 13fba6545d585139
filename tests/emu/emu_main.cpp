// Driver of the host-emulated library (test infrastructure only): creates a plan
// through the C ABI and runs every entry point once on emulated device memory.
//
//   emu_sgspm nx ny nz precision scheme terms steps A Ms Ku h dt alpha he0 he1 he2 in.bin out.bin
//
// SI units; cubic cells of edge h (m); A (J/m), Ms (A/m), Ku (J/m^3), dt (s), h_e (T).
//
// in.bin: 3N doubles of m0 then 3N doubles of a cotangent (SoA [3][nz][ny][nx]).
// out.bin: m after `steps` steps (3N), its energies (5) and unit error (1); the
// spectral radii of a step from m0 (2); at m0: h_eff (3N), h_s (3N), the heat
// solve of m1 with s = 1 (N); lambda after one adjoint step from m0 (3N) and
// its gradient (4); the same from the no-allocation adjoint (zeros where an
// entry point does not apply).  The taped step and adjoint are checked against
// sgspm_step and sgspm_adjoint_step bit for bit here in runs of every workgroup
// (exit status 5 otherwise).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sgspm.h"

extern "C" long emu_launch_count();
extern "C" long emu_group_count();

static void die(const char* what, int rc) {
  fprintf(stderr, "%s failed: %d %s\n", what, rc, sgspm_last_error());
  exit(3);
}

static sgspm_plan_t plan_for_check = nullptr;

// EMU_BATCH=B: a batched plan of B runs (run b with alpha (1 + b / 2) and h_e (1 + b)
// times the given ones, all from m0) against B single-run plans.  out.bin: the
// batched m (3 B N), energies after the steps (5 B) and before them (5 B), then
// for each single run its energies before the steps (5), m (3 N) and energies
// after them (5).
static int batch_main(sgspm_params p, int B, int steps, double alpha0, const double he0[3], const std::vector<double>& m0,
                      const char* fout) {
  const long N = (long)p.nx * p.ny * p.nz;
  const bool f64 = p.precision == SGSPM_FP64;
  const size_t es = f64 ? 8 : 4;
  std::vector<double> alpha(B), he(3 * B), out;
  for (int b = 0; b < B; ++b) {
    alpha[b] = alpha0 * (1.0 + 0.5 * b);
    for (int c = 0; c < 3; ++c) he[3 * b + c] = he0[c] * (1.0 + b);
  }
  auto put = [&](void* d, long i, double v) {
    if (f64) static_cast<double*>(d)[i] = v;
    else static_cast<float*>(d)[i] = (float)v;
  };
  auto get = [&](const void* d, long i) { return f64 ? static_cast<const double*>(d)[i] : static_cast<const float*>(d)[i]; };
  sgspm_params pb = p;
  pb.batch = B;
  sgspm_plan_t plan;
  int rc = sgspm_plan(&pb, nullptr, &plan);
  if (rc) die("sgspm_plan (batched)", rc);
  void* m;
  hipMalloc(&m, 3 * B * N * es);
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < B; ++b)
      for (long i = 0; i < N; ++i) put(m, (c * B + b) * N + i, m0[c * N + i]);
  // energies before any batched step too (the per-run values are not set yet)
  std::vector<double> e0(5 * B);
  if ((rc = sgspm_energy_batch(plan, m, he.data(), e0.data()))) die("sgspm_energy_batch", rc);
  for (int s = 0; s < steps; ++s)
    if ((rc = sgspm_step_batch(plan, m, alpha.data(), he.data()))) die("sgspm_step_batch", rc);
  if ((rc = sgspm_check(plan))) die("sgspm_check (batched)", rc);
  for (long i = 0; i < 3 * B * N; ++i) out.push_back(get(m, i));
  std::vector<double> e(5 * B);
  if ((rc = sgspm_energy_batch(plan, m, he.data(), e.data()))) die("sgspm_energy_batch", rc);
  out.insert(out.end(), e.begin(), e.end());
  out.insert(out.end(), e0.begin(), e0.end());
  sgspm_destroy(plan);
  hipFree(m);
  for (int b = 0; b < B; ++b) {
    sgspm_plan_t q;
    if ((rc = sgspm_plan(&p, nullptr, &q))) die("sgspm_plan", rc);
    void* mb;
    hipMalloc(&mb, 3 * N * es);
    for (long i = 0; i < 3 * N; ++i) put(mb, i, m0[i]);
    double eb0[5];
    if ((rc = sgspm_energy(q, mb, he.data() + 3 * b, eb0))) die("sgspm_energy", rc);
    out.insert(out.end(), eb0, eb0 + 5);
    for (int s = 0; s < steps; ++s)
      if ((rc = sgspm_step(q, mb, alpha[b], he.data() + 3 * b, nullptr))) die("sgspm_step", rc);
    for (long i = 0; i < 3 * N; ++i) out.push_back(get(mb, i));
    double eb[5];
    if ((rc = sgspm_energy(q, mb, he.data() + 3 * b, eb))) die("sgspm_energy", rc);
    out.insert(out.end(), eb, eb + 5);
    sgspm_destroy(q);
    hipFree(mb);
  }
  FILE* fo = fopen(fout, "wb");
  fwrite(out.data(), 8, out.size(), fo);
  fclose(fo);
  printf("launches %ld workgroups %ld\n", emu_launch_count(), emu_group_count());
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 19) {
    fprintf(stderr, "usage: emu_sgspm nx ny nz precision scheme terms steps A Ms Ku h dt alpha he0 he1 he2 in.bin out.bin\n");
    return 2;
  }
  sgspm_params p{};
  p.nx = atoi(argv[1]);
  p.ny = atoi(argv[2]);
  p.nz = atoi(argv[3]);
  p.precision = atoi(argv[4]);
  p.scheme = atoi(argv[5]);
  p.terms = (uint32_t)atoi(argv[6]);
  const int steps = atoi(argv[7]);
  p.units = SGSPM_UNITS_SI;
  p.A = atof(argv[8]);
  p.Ms = atof(argv[9]);
  p.Ku = atof(argv[10]);
  p.dx = p.dy = p.dz = atof(argv[11]);
  p.dt = atof(argv[12]);
  const double alpha = atof(argv[13]);
  const double he[3] = {atof(argv[14]), atof(argv[15]), atof(argv[16])};

  const long N = (long)p.nx * p.ny * p.nz;
  // with a sample of workgroups per launch the values are not the method's: the
  // projection's numeric flag is then expected
  const bool sampled = getenv("EMU_MAX_GROUPS") && atol(getenv("EMU_MAX_GROUPS")) > 0;
  auto check = [&](const char* where) {
    const int r = sgspm_check(plan_for_check);
    if (r && !(sampled && r == SGSPM_ENUMERIC)) die(where, r);
  };
  const bool f64 = p.precision == SGSPM_FP64;
  const size_t es = f64 ? 8 : 4;

  std::vector<double> in(6 * N);
  FILE* fi = fopen(argv[17], "rb");
  if (!fi || fread(in.data(), 8, in.size(), fi) != in.size()) {
    fprintf(stderr, "cannot read %s\n", argv[17]);
    return 2;
  }
  fclose(fi);
  if (getenv("EMU_BATCH")) {
    std::vector<double> m0(in.begin(), in.begin() + 3 * N);
    return batch_main(p, atoi(getenv("EMU_BATCH")), steps, alpha, he, m0, argv[18]);
  }
  auto upload = [&](const double* src, long n) {
    void* d;
    hipMalloc(&d, n * es);
    for (long i = 0; i < n; ++i) {
      if (f64) static_cast<double*>(d)[i] = src[i];
      else static_cast<float*>(d)[i] = (float)src[i];
    }
    return d;
  };
  auto fetch = [&](const void* d, long n, std::vector<double>& out) {
    for (long i = 0; i < n; ++i) out.push_back(f64 ? static_cast<const double*>(d)[i] : static_cast<const float*>(d)[i]);
  };
  std::vector<double> out;

  int rc = sgspm_plan(&p, nullptr, &plan_for_check);
  sgspm_plan_t plan = plan_for_check;
  if (rc) die("sgspm_plan", rc);
  void* m = upload(in.data(), 3 * N);
  for (int s = 0; s < steps; ++s)
    if ((rc = sgspm_step(plan, m, alpha, he, nullptr))) die("sgspm_step", rc);
  check("sgspm_check after the steps");
  fetch(m, 3 * N, out);

  double e[5] = {0, 0, 0, 0, 0}, ue = 0.0, rho[2] = {0, 0};
  if ((rc = sgspm_energy(plan, m, he, e))) die("sgspm_energy", rc);
  if ((rc = sgspm_unit_error(plan, m, &ue))) die("sgspm_unit_error", rc);
  out.insert(out.end(), e, e + 5);
  out.push_back(ue);
  void* m2 = upload(in.data(), 3 * N);
  if ((rc = sgspm_step_spectral_radius(plan, m2, alpha, he, nullptr, rho))) die("sgspm_step_spectral_radius", rc);
  out.insert(out.end(), rho, rho + 2);

  hipFree(m2);
  m2 = upload(in.data(), 3 * N);  // m0 again
  void* h = upload(in.data(), 3 * N);
  if ((rc = sgspm_field(plan, m2, he, h))) die("sgspm_field", rc);
  fetch(h, 3 * N, out);
  if (p.terms & SGSPM_TERM_STRAY) {
    if ((rc = sgspm_stray(plan, m2, h))) die("sgspm_stray", rc);
    fetch(h, 3 * N, out);
    void* nt = nullptr;
    long P = 1;
    for (int n : {p.nx, p.ny, p.nz}) P *= n > 1 ? 2 * n : 1;
    hipMalloc(&nt, P * 8);
    for (int c = 0; c < 6; ++c)
      if ((rc = sgspm_demag_tensor(plan, c, nt))) die("sgspm_demag_tensor", rc);
    hipFree(nt);
  } else {
    out.insert(out.end(), 3 * N, 0.0);
  }
  if ((rc = sgspm_heat_solve(plan, m2, 1.0, h))) die("sgspm_heat_solve", rc);
  fetch(h, N, out);

  if (p.scheme == SGSPM_SCHEME_SGS) {
    void* m0 = upload(in.data(), 3 * N);
    for (int pass = 0; pass < 2; ++pass) {
      void* lam = upload(in.data() + 3 * N, 3 * N);
      double* g;
      hipMalloc(&g, 32);
      for (int i = 0; i < 4; ++i) g[i] = 0.0;
      rc = pass == 0 ? sgspm_adjoint_step(plan, m0, alpha, he, lam, g) : sgspm_adjoint_step_noalloc(plan, m0, alpha, he, lam, g);
      if (rc == SGSPM_EUNSUPPORTED && pass == 1) {
        out.insert(out.end(), 3 * N + 4, 0.0);
      } else {
        if (rc) die(pass == 0 ? "sgspm_adjoint_step" : "sgspm_adjoint_step_noalloc", rc);
        fetch(lam, 3 * N, out);
        out.insert(out.end(), g, g + 4);
      }
      hipFree(lam);
      hipFree(g);
    }
    // the taped pair: the step equals sgspm_step, the adjoint from its tape equals
    // sgspm_adjoint_step, bit for bit (abort otherwise)
    {
      size_t tb = 0;
      if ((rc = sgspm_tape_bytes(plan, &tb))) die("sgspm_tape_bytes", rc);
      void* tape = nullptr;
      hipMalloc(&tape, tb);
      void* ms = upload(in.data(), 3 * N);
      void* mt = upload(in.data(), 3 * N);
      if ((rc = sgspm_step(plan, ms, alpha, he, nullptr))) die("sgspm_step", rc);
      if ((rc = sgspm_step_taped(plan, mt, alpha, he, tape))) die("sgspm_step_taped", rc);
      void* la = upload(in.data() + 3 * N, 3 * N);
      void* lb = upload(in.data() + 3 * N, 3 * N);
      double *ga, *gb;
      hipMalloc(&ga, 32);
      hipMalloc(&gb, 32);
      for (int i = 0; i < 4; ++i) ga[i] = gb[i] = 0.0;
      if ((rc = sgspm_adjoint_step(plan, m0, alpha, he, la, ga))) die("sgspm_adjoint_step", rc);
      if ((rc = sgspm_adjoint_step_taped(plan, m0, alpha, he, tape, lb, gb))) die("sgspm_adjoint_step_taped", rc);
      std::vector<double> xa, xb;
      fetch(ms, 3 * N, xa);
      fetch(mt, 3 * N, xb);
      fetch(la, 3 * N, xa);
      fetch(lb, 3 * N, xb);
      xa.insert(xa.end(), ga, ga + 4);
      xb.insert(xb.end(), gb, gb + 4);
      // a sampled run leaves the workgroups it skips unwritten: compare full runs only
      const char* sampled = getenv("EMU_MAX_GROUPS");
      const bool full = !sampled || atol(sampled) == 0;
      for (size_t i = 0; full && i < xa.size(); ++i)
        if (xa[i] != xb[i]) {
          fprintf(stderr, "taped step or adjoint differs at %zu: %.17g vs %.17g\n", i, xa[i], xb[i]);
          exit(5);
        }
      for (void* q : {tape, ms, mt, la, lb}) hipFree(q);
      hipFree(ga);
      hipFree(gb);
    }
    hipFree(m0);
  } else {
    out.insert(out.end(), 2 * (3 * N + 4), 0.0);
  }
  check("sgspm_check at the end");
  if ((rc = sgspm_destroy(plan))) die("sgspm_destroy", rc);
  hipFree(m);
  hipFree(m2);
  hipFree(h);
  FILE* fo = fopen(argv[18], "wb");
  fwrite(out.data(), 8, out.size(), fo);
  fclose(fo);
  printf("launches %ld workgroups %ld\n", emu_launch_count(), emu_group_count());
  return 0;
}
