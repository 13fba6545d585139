// Host side of the SGSPM library: validation, unit reduction, plan
// construction (tables, workspace, FP64 demagnetising-tensor spectrum) and the
// stage-by-stage schedule of one SGSPM / GSPM step on the caller's stream.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sgspm.h"
#include "kernels.h"

using namespace sgspm;

// Workspace of sgspm_adjoint_step_noalloc: the adjoint's 16 fields of N cells in
// one file-scope device array (each GPU holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: it is a host-side
// stand-in there.  The device address comes from hipGetSymbolAddress, once per
// device with that device current (at plan creation), and is kept per device.
static constexpr size_t SCRATCH_BYTES = size_t(8) << 20;
static constexpr int ADJ_FIELDS = 16;
// field of the adjoint workspace that holds the recomputed new state
static constexpr int ADJ_MT = 13;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

const double MU0 = 4.0e-7 * M_PI;
const double GAMMA = 1.7609e11;  // rad / (s T)
const int R_FAR = 20;            // cells: Newell sum within, point dipole beyond

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
// n = 2^a 3^b 5^c: the lengths the FFT passes support
bool smooth235(int n) {
  if (n <= 0) return false;
  for (int f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}
long gcdl(long a, long b) {
  while (b) {
    const long t = a % b;
    a = b;
    b = t;
  }
  return a;
}
// length of the table of W_L for every non-power-of-two transform length L of a plan
// (the DCT lengths n_a, and the padded lengths 2 n_a with the stray field), 1 if none
long mixed_table_len(const int n[3], bool stray) {
  long L = 1;
  for (int a = 0; a < 3; ++a) {
    if (n[a] <= 1 || pow2(n[a])) continue;
    const long l = stray ? 2L * n[a] : n[a];
    L = L / gcdl(L, l) * l;
  }
  return L;
}
constexpr long MIXED_TABLE_MAX = 1L << 20;
int ilog2(long n) {
  int l = 0;
  while ((1L << l) < n) ++l;
  return l;
}

int validate(const sgspm_params* p) {
  if (!p) return fail(SGSPM_EINVAL, "params is NULL");
  const int n[3] = {p->nx, p->ny, p->nz};
  const char* nm[3] = {"nx", "ny", "nz"};
  for (int a = 0; a < 3; ++a) {
    if (n[a] <= 0) return fail(SGSPM_EINVAL, std::string(nm[a]) + " must be positive");
    if (n[a] > (a == 0 ? 2048 : 1024))
      return fail(SGSPM_EUNSUPPORTED, std::string(nm[a]) + (a == 0 ? " above 2048" : " above 1024") + " is not supported");
    if (!smooth235(n[a])) return fail(SGSPM_EUNSUPPORTED, std::string(nm[a]) + " must be a product of 2, 3 and 5");
  }
  const double h[3] = {p->dx, p->dy, p->dz};
  for (int a = 0; a < 3; ++a)
    if (!(h[a] > 0.0) || !std::isfinite(h[a])) return fail(SGSPM_EINVAL, "cell sizes must be positive and finite");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(SGSPM_EINVAL, "dt must be positive and finite");
  if (p->units != SGSPM_UNITS_SI && p->units != SGSPM_UNITS_REDUCED) return fail(SGSPM_EINVAL, "unknown units");
  if (p->units == SGSPM_UNITS_SI) {
    if (!(p->Ms > 0.0) || !std::isfinite(p->Ms)) return fail(SGSPM_EINVAL, "Ms must be positive");
    if (!(p->A >= 0.0) || !std::isfinite(p->A)) return fail(SGSPM_EINVAL, "A must be non-negative");
    if (!std::isfinite(p->Ku)) return fail(SGSPM_EINVAL, "Ku must be finite");
  } else {
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return fail(SGSPM_EINVAL, "eps must be non-negative");
    if (!std::isfinite(p->Q)) return fail(SGSPM_EINVAL, "Q must be finite");
  }
  if (p->terms & ~15u) return fail(SGSPM_EINVAL, "unknown term bits");
  if (p->precision != SGSPM_FP32 && p->precision != SGSPM_FP64) return fail(SGSPM_EINVAL, "unknown precision");
  if (p->scheme != SGSPM_SCHEME_SGS && p->scheme != SGSPM_SCHEME_GS && p->scheme != SGSPM_SCHEME_SGS_FF)
    return fail(SGSPM_EINVAL, "unknown scheme");
  if (p->batch < 0 || p->batch > 256) return fail(SGSPM_EINVAL, "batch must be in [0, 256]");
  const long B = std::max(1, (int)p->batch);
  const long N = (long)p->nx * p->ny * p->nz;
  if (N * B > (1L << 28)) return fail(SGSPM_EUNSUPPORTED, "grid too large");
  if (B > 1) {
    if (p->scheme == SGSPM_SCHEME_SGS_FF)
      return fail(SGSPM_EUNSUPPORTED, "batched plans take the SGS or GS scheme");
    if (((long)p->ny * p->nz) % 2)
      return fail(SGSPM_EUNSUPPORTED, "batched plans need ny * nz even (row pairs of one run)");
    const bool fused = yz_reg_plane(p->ny, p->nz) ||
                       (p->precision == SGSPM_FP64 ? yz_fits<double>(p->ny, p->nz, 0) : yz_fits<float>(p->ny, p->nz, 0));
    if (!fused) return fail(SGSPM_EUNSUPPORTED, "batched plans need y-z planes that one workgroup solves");
  }
  const bool fp64 = p->precision == SGSPM_FP64;
  const bool stray = p->terms & SGSPM_TERM_STRAY;
  // the row kernels hold two rows and their (padded) transforms in one tile
  const long rowlen = (stray && p->nx > 1) ? 2L * p->nx : p->nx;
  if (rowlen > (fp64 ? tile_elems<double>() : tile_elems<float>()))
    return fail(SGSPM_EUNSUPPORTED, std::string("nx = ") + std::to_string(p->nx) +
                                        " rows do not fit a row tile at this precision" + (stray ? " with the stray field" : ""));
  // the demagnetising tensor is transformed in FP64 whatever the plan's precision
  if (stray && rowlen > tile_elems<double>())
    return fail(SGSPM_EUNSUPPORTED, std::string("nx = ") + std::to_string(p->nx) +
                                        " rows of the FP64 demagnetising tensor do not fit a row tile");
  if (mixed_table_len(n, stray) > MIXED_TABLE_MAX)
    return fail(SGSPM_EUNSUPPORTED, "the non-power-of-two lengths need too long a twiddle table");
  if (stray) {
    // the last-axis convolution holds three padded pencils of its axis in one tile
    const int nc = p->nz > 1 ? p->nz : p->ny;
    const int L = nc > 1 ? 2 * nc : 1;
    const int lgP = fp64 ? conv_lgP<double>(L, 1, 6) : conv_lgP<float>(L, 1, 6);
    if (lgP < 0 && !(L == 64))
      return fail(SGSPM_EUNSUPPORTED, std::string(p->nz > 1 ? "nz" : "ny") + " = " + std::to_string(nc) +
                                          " is not supported with the stray field at this precision");
  }
  return SGSPM_OK;
}

// eps, Q, dt (reduced), field scale (per tesla), energy scale
void reduce(const sgspm_params* p, double out[5]) {
  const bool ex = p->terms & SGSPM_TERM_EXCHANGE, an = p->terms & SGSPM_TERM_ANISO;
  if (p->units == SGSPM_UNITS_SI) {
    const double sc = MU0 * p->Ms * p->Ms;
    out[0] = ex ? 2.0 * p->A / sc : 0.0;
    out[1] = an ? 2.0 * p->Ku / sc : 0.0;
    out[2] = p->dt * GAMMA * MU0 * p->Ms;
    out[3] = 1.0 / (MU0 * p->Ms);
    out[4] = sc;
  } else {
    out[0] = ex ? p->eps : 0.0;
    out[1] = an ? p->Q : 0.0;
    out[2] = p->dt;
    out[3] = 1.0;
    out[4] = 1.0;
  }
}

}  // namespace

struct sgspm_plan_s {
  sgspm_params prm;
  hipStream_t s = nullptr;
  // one step captured as a HIP graph (sgspm_steps): the private capture stream,
  // the executable graph and the arguments it was captured with
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  void* g_m = nullptr;
  double g_alpha = 0.0, g_he[3] = {0.0, 0.0, 0.0};
  int dev = 0;  // device current at plan creation (owner of the plan's memory)
  bool fp64 = false;
  int nx = 1, ny = 1, nz = 1;
  // cells of one component array: nx ny nz per run, times B runs in a batched plan
  long N = 0;
  int B = 1;            // runs (batched plan: fields [3][B][nz][ny][nx])
  long Nrun = 0;        // nx ny nz
  void* runp = nullptr; // batched plan: per-run values [B][RUNP] of the precision
  int Px = 1, Py = 1, Pz = 1, Kx = 1, Kxp = 1, Hy = 1, Hz = 1;
  bool stray = false, zeeman = false, has_mid = false;
  // the x-level spectra carry their (real) Nyquist bin in bin 0, and the y
  // level holds the DC column and the Nyquist column (blocked layout) apart
  bool dcnq = false;
  bool yz = false;  // heat arrays x-major and solved across y, z by one fused kernel
  double eps = 0, Q = 0, dt = 0, fscale = 1, escale = 1;
  double cxx = 0, cyy = 0, czz = 0;  // eps / h^2 per axis (reduced)
  int lgTw = 0;
  // typed (T) device tables
  void* tw = nullptr;
  // W_Lm^i for the non-power-of-two lengths (Lm = 1: none), typed and FP64
  void* twm = nullptr;
  void* twm64 = nullptr;
  long Lm = 1;
  void* dtw[3] = {nullptr, nullptr, nullptr};
  void* lam[3] = {nullptr, nullptr, nullptr};
  // FP64 twiddles for the tensor precompute
  void* tw64 = nullptr;
  // workspace
  void* fld = nullptr;     // NF fields of N values
  void* heat = nullptr;    // 3 x N
  void* xlev = nullptr;    // 3 x nz*ny*Kxp complex
  void* ylev = nullptr;    // 3 x nz*Py*Kxp complex (3-D) or null
  void* yout = nullptr;    // 3 x conv outputs
  void* tens = nullptr;    // 6 x Hz*Hy*Kt
  int Kt = 1;              // tensor kx pitch: Kx rounded up to 32 (128-byte rows in FP32)
  double* partials = nullptr;
  double* eout = nullptr;
  int* flag = nullptr;
  void* adj = nullptr;     // adjoint workspace (16 fields), allocated on first use
  int nred = 0;
  std::vector<void*> allocs;
  // optional per-kernel-class timing (HIP events around every launch)
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  bool timing = false;
  // first launch-geometry error of the current call (0: none)
  int geom_err = 0;
  std::string geom_msg;
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  std::vector<Rec> recs;
};

namespace {

// F_R0..F_R2: the right-hand sides of the heat solves in flight (one per channel),
// which the inverse passes read to form g = r - correction
enum { F_G2N, F_G3N, F_A1, F_G1S, F_A2, F_G2S, F_A3, F_G3SS, F_B2, F_G2SS, F_B1, F_NRM, F_HS0, F_HS1, F_HS2,
       F_R0, F_R1, F_R2, NF };
// a step's tape: the fields before F_R0 (what the reverse reads) and the new state
constexpr int TAPE_FIELDS = F_R0 + 3;

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SGSPM_OK;
  return fail(SGSPM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int dalloc(sgspm_plan_s* P, void** out, size_t bytes) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SGSPM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  P->allocs.push_back(p);
  *out = p;
  return SGSPM_OK;
}

template <typename T> int upload(sgspm_plan_s* P, void** out, const std::vector<T>& h) {
  int rc = dalloc(P, out, h.size() * sizeof(T));
  if (rc) return rc;
  return hip_check(hipMemcpyAsync(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, P->s), "upload");
}

// Tiles: log2 of the most pencils of length L one tile of the precision holds.
template <typename T> int lg_tile_for(int L) {
  int l = 0;
  while (((long)L << (l + 1)) <= tile_elems<T>()) ++l;
  return l;
}

// twiddle table and stride giving W_L^i = t[i * stride] for a transform length L of
// the plan: the power-of-two table (2^lgTw entries) or the mixed one (Lm entries)
template <typename V> void table_for(const sgspm_plan_s& P, const void* pow2tab, const void* mixtab, int L,
                                     const cx<V>*& t, int& stride) {
  if (lg_or_neg(L) >= 0) {
    t = (const cx<V>*)pow2tab;
    stride = (1 << P.lgTw) / L;
  } else {
    t = (const cx<V>*)mixtab;
    stride = (int)(P.Lm / L);
  }
}

// largest lgP with (2 << lgP) rows not beyond what the rows need
int cap_lgP(int lgP, long count_pencils) {
  int need = ilog2(std::max<long>(1, count_pencils));
  return std::max(0, std::min(lgP, need));
}

// the same for the row kernels, whose grid is the row pairs alone: fewer pencils per
// workgroup until the launch has about 256 workgroups (small grids are latency-bound;
// a full tile per workgroup would leave most of the chip idle)
int row_lgP(int lgP, long count_pencils) {
  const int need = ilog2(std::max<long>(1, count_pencils));
  return std::max(0, std::min(cap_lgP(lgP, count_pencils), need - 8));
}

// ---------------------------------------------------------------------------
template <typename T> struct Eng {
  sgspm_plan_s& P;
  hipStream_t s;
  const cx<T>* tw;
  const cx<T>* dtw[3];
  const T* lam[3];
  T* f[NF];
  T* heat[3];
  void tab(int L, const cx<T>*& t, int& stride) const { table_for<T>(P, P.tw, P.twm, L, t, stride); }
  cx<T>* xlev[3];
  cx<T>* ylev[3];
  cx<T>* yout[3];
  const T* tens;

  explicit Eng(sgspm_plan_s& p) : P(p), s(p.s) {
    tw = (const cx<T>*)P.tw;
    for (int a = 0; a < 3; ++a) {
      dtw[a] = (const cx<T>*)P.dtw[a];
      lam[a] = (const T*)P.lam[a];
    }
    for (int i = 0; i < NF; ++i) f[i] = (T*)P.fld + (long)i * P.N;
    for (int c = 0; c < 3; ++c) heat[c] = (T*)P.heat + (long)c * P.N;
    const long xl = (long)P.B * P.nz * P.ny * P.Kxp;
    const long yl = (long)P.B * P.nz * P.Py * P.Kxp;
    for (int c = 0; c < 3; ++c) {
      xlev[c] = P.xlev ? (cx<T>*)P.xlev + c * xl : nullptr;
      ylev[c] = P.ylev ? (cx<T>*)P.ylev + c * yl : nullptr;
      yout[c] = P.yout ? (cx<T>*)P.yout + c * (P.has_mid ? yl : xl) : nullptr;
    }
    tens = (const T*)P.tens;
  }

  // ---- timing: events around a launch, with the launch's launch-level bytes
  hipEvent_t ev() {
    if (P.evnext == P.evpool.size()) {
      hipEvent_t e;
      (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
      P.evpool.push_back(e);
    }
    return P.evpool[P.evnext++];
  }
  // fn launches one kernel and returns its class (SGSPM_KC_*)
  template <class F> void timed(double bytes, F&& fn) {
    if (!P.timing) {
      (void)note(fn());
      return;
    }
    hipEvent_t a = ev(), b = ev();
    (void)hipEventRecord(a, s);
    const int cls = fn();
    (void)hipEventRecord(b, s);
    if (note(cls)) P.recs.push_back({cls, a, b, bytes});
  }
  // keeps the first launch-geometry error of the call; true for a launch that ran
  bool note(int cls) {
    if (cls >= 0) return true;
    if (!P.geom_err) {
      P.geom_err = cls;
      P.geom_msg = launch_geom_error();
    }
    return false;
  }
  static constexpr double TS = sizeof(T);

  // component spectra at the level the last-axis convolution reads
  cx<T>* comp_spec(int c) { return P.has_mid ? ylev[c] : xlev[c]; }
  // real-to-complex output slot of component c (x level)
  cx<T>* r2c_slot(int c) { return xlev[c]; }
  // complex-to-real source of stray-field component a (x level)
  const cx<T>* c2r_src(int a) { return P.has_mid ? xlev[a] : yout[a]; }

  // ---- row kernels
  struct RowIO {
    const T* u[3] = {nullptr, nullptr, nullptr};
    T a[3] = {1, 1, 1};
    T alo[3] = {0, 0, 0};  // coefficients of u and w near one: a + alo, wc + wclo
    T b = 0;
    T he[3] = {0, 0, 0};
    bool with_hs = false;
    const T* w[3] = {nullptr, nullptr, nullptr};
    T wc[3] = {0, 0, 0};
    T wclo[3] = {0, 0, 0};
    T* val_out[3] = {nullptr, nullptr, nullptr};
    T* hs_out[3] = {nullptr, nullptr, nullptr};
    T* dct_out[3] = {nullptr, nullptr, nullptr};
    cx<T>* xout[3] = {nullptr, nullptr, nullptr};
    // batched plan: the component of each channel (run values by component) and
    // whether this is the damping step's right-hand side
    int rcomp[3] = {0, 1, 2};
    bool per_run = false;  // the heat right-hand sides of a batched plan
    bool stageF = false;
  };
  void row_fwd(int nch, const RowIO& io) {
    RowFwd<T> A{};
    A.nrows = P.ny * P.nz * P.B;
    A.n = P.nx;
    A.lgN = lg_or_neg(P.nx);
    A.Lc = A.Lr = P.Px;
    A.lgLc = A.lgLr = lg_or_neg(P.Px);
    bool any_x = io.with_hs;
    for (int c = 0; c < nch; ++c)
      if (io.xout[c]) any_x = true;
    // the tile holds 2P rows of nx values whether or not a transform runs (a pass
    // with no transform, such as the accumulation of a plan without the stray
    // field, still carries its rows); the padded transforms (Px = 2 nx) set it
    // when they run, and the DCT length nx divides them
    A.Lmax = any_x ? P.Px : P.nx;
    A.lgLmax = lg_or_neg(A.Lmax);
    A.lgP = row_lgP(lg_tile_for<T>(A.Lmax), (A.nrows + 1) / 2);
    if (P.B > 1 && io.per_run) {
      // a tile holds rows of one run
      A.runp = (const T*)P.runp;
      A.rpr = P.ny * P.nz;
      A.rstageF = io.stageF ? 1 : 0;
      for (int c = 0; c < 3; ++c) A.rcomp[c] = io.rcomp[c];
      while (A.lgP > 0 && A.rpr % (2 << A.lgP)) --A.lgP;
    }
    A.lgTw = P.lgTw;
    tab(A.Lmax, A.tw, A.twg);
    A.dtw = dtw[0];
    A.b = io.b;
    A.xin_pitch = P.Kxp;
    A.xout_pitch = P.Kxp;
    A.xpk = P.dcnq ? 1 : 0;
    A.dct_xmajor = P.yz ? 1 : 0;
    for (int c = 0; c < nch; ++c) {
      A.u[c] = io.u[c];
      A.a[c] = io.a[c];
      A.alo[c] = io.alo[c];
      A.he[c] = io.he[c];
      A.w[c] = io.w[c];
      A.wc[c] = io.wc[c];
      A.wclo[c] = io.wclo[c];
      A.val_out[c] = io.val_out[c];
      A.xin[c] = io.with_hs ? c2r_src_for_[c] : nullptr;
      A.hs_out[c] = io.hs_out[c];
      A.dct_out[c] = io.dct_out[c];
      A.xout[c] = io.xout[c];
    }
    double by = 0;
    const double cpx = (double)A.nrows * P.Kx * 2 * TS;
    for (int c = 0; c < nch; ++c)
      by += (A.u[c] ? P.N * TS : 0) + (A.w[c] ? P.N * TS : 0) + (A.xin[c] ? cpx : 0) +
            (A.hs_out[c] ? P.N * TS : 0) + (A.val_out[c] ? P.N * TS : 0) + (A.dct_out[c] ? P.N * TS : 0) +
            (A.xout[c] ? cpx : 0);
    timed(by, [&] { return launch_row_fwd<T>(A, nch, s); });
  }
  const cx<T>* c2r_src_for_[3] = {nullptr, nullptr, nullptr};
  bool tape = false;

  void row_inv(RowInv<T>& A, bool r2c) {
    A.nrows = P.ny * P.nz * P.B;
    A.n = P.nx;
    A.lgN = lg_or_neg(P.nx);
    A.Lr = P.Px;
    A.lgLr = lg_or_neg(P.Px);
    A.Lmax = r2c ? std::max(P.nx, P.Px) : P.nx;
    A.lgLmax = lg_or_neg(A.Lmax);
    A.lgP = row_lgP(lg_tile_for<T>(A.Lmax), (A.nrows + 1) / 2);
    A.lgTw = P.lgTw;
    tab(A.Lmax, A.tw, A.twg);
    A.dtw = dtw[0];
    A.xout_pitch = P.Kxp;
    A.xpk = P.dcnq ? 1 : 0;
    A.heat_xmajor = P.yz ? 1 : 0;
    if (!r2c) A.xout = nullptr;
    // the right-hand sides the forward passes stored, unless the caller names its own
    for (int c = 0; c < A.nch; ++c)
      if (!A.rin[c]) A.rin[c] = f[F_R0 + c];
    double by = 2.0 * A.nch * P.N * TS;
    for (int c = 0; c < A.nch; ++c) by += A.gout[c] ? P.N * TS : 0;
    if (A.op == ROW_OP_GS) by += (4 + (A.src ? 1 : 0) + 1) * P.N * TS;
    if (A.op == ROW_OP_PROJECT) by += (3 + (A.nrm ? 1 : 0)) * P.N * TS;
    if (A.xout) by += (double)A.nrows * P.Kx * 2 * TS;
    timed(by, [&] { return launch_row_inv<T>(A, s); });
  }

  // ---- heat solves: after row_fwd wrote DCT_x(rhs) into heat[0..nch)
  void heat_rest(int nch, T scale, bool stageF = false) {
    T* d[3] = {heat[0], heat[1], heat[2]};
    const T sdt = (T)(scale * P.dt);
    if (P.yz) {
      YZSolve<T> A{};
      for (int c = 0; c < 3; ++c) A.data[c] = d[c];
      // a batched plan: the planes are (x, run) pairs, [nx][B] (the kernels group
      // planes per workgroup by run, as a single-run plan does)
      A.nx = P.nx;
      A.runs = P.B;
      A.runp = (const T*)P.runp;
      A.rstageF = (stageF && P.B > 1) ? 1 : 0;
      A.ny = P.ny;
      A.nz = P.nz;
      A.lgNy = lg_or_neg(P.ny);
      A.lgNz = lg_or_neg(P.nz);
      // planes per workgroup: fill the tile, but keep at least ~256 workgroups,
      // and at least four values per thread (small planes leave most of a
      // workgroup idle otherwise; a batched plan then has B times the workgroups)
      int lgPP = 0;
      while (yz_fits<T>(P.ny, P.nz, lgPP + 1)) ++lgPP;
      const int lgmax = lgPP;
      while (lgPP > 0 && (P.nx >> lgPP) < 256) --lgPP;
      while (lgPP < lgmax && ((long)P.ny * P.nz << lgPP) < 4L * YZ_NT) ++lgPP;
      A.lgPP = lgPP;
      A.dtwy = dtw[1];
      A.dtwz = dtw[2];
      A.tw = tw;
      A.lgTw = P.lgTw;
      tab(P.ny, A.twy, A.twy_s);
      tab(P.nz, A.twz, A.twz_s);
      A.lamX = lam[0];
      A.lamY = lam[1];
      A.lamZ = lam[2];
      A.s = sdt;
      timed(2.0 * nch * P.N * TS, [&] { return launch_yz_solve<T>(A, nch, s); });
      return;
    }
    if (P.has_mid) {
      ColDct<T> A{};
      A.mode = COL_DCT_FWD;
      A.n = P.ny;
      A.lgN = lg_or_neg(P.ny);
      A.lgP = cap_lgP(lg_tile_for<T>(A.n), (P.nx + 1) / 2);
      A.ni = P.nx;
      A.sa = P.nx;
      A.sb = (long)P.ny * P.nx;
      for (int c = 0; c < 3; ++c) A.data[c] = d[c];
      A.dtw = dtw[1];
      tab(A.n, A.tw, A.twg);
      timed(2.0 * nch * P.N * TS, [&] { return launch_col_dct<T>(A, P.nz, nch, s); });
    }
    {
      ColDct<T> A{};
      A.mode = COL_DCT_SOLVE;
      const bool z = P.nz > 1;
      A.n = z ? P.nz : P.ny;
      A.lgN = lg_or_neg(A.n);
      A.lgP = cap_lgP(lg_tile_for<T>(A.n), (P.nx + 1) / 2);
      A.ni = P.nx;
      A.sa = z ? (long)P.ny * P.nx : P.nx;
      A.sb = z ? P.nx : 0;
      for (int c = 0; c < 3; ++c) A.data[c] = d[c];
      A.dtw = dtw[z ? 2 : 1];
      tab(A.n, A.tw, A.twg);
      A.lamX = lam[0];
      A.lamB = z ? lam[1] : lam[2];
      A.lamA = z ? lam[2] : lam[1];
      A.s = sdt;
      timed(2.0 * nch * P.N * TS, [&] { return launch_col_dct<T>(A, z ? P.ny : 1, nch, s); });
    }
    if (P.has_mid) {
      ColDct<T> A{};
      A.mode = COL_DCT_INV;
      A.n = P.ny;
      A.lgN = lg_or_neg(P.ny);
      A.lgP = cap_lgP(lg_tile_for<T>(A.n), (P.nx + 1) / 2);
      A.ni = P.nx;
      A.sa = P.nx;
      A.sb = (long)P.ny * P.nx;
      for (int c = 0; c < 3; ++c) A.data[c] = d[c];
      A.dtw = dtw[1];
      tab(A.n, A.tw, A.twg);
      timed(2.0 * nch * P.N * TS, [&] { return launch_col_dct<T>(A, P.nz, nch, s); });
    }
  }

  // ---- stray field
  // y-pass forward of x-level spectra of the listed components (3-D only)
  void mid_fwd(int mask) {
    if (!P.has_mid) return;
    ColFft<T> A{};
    A.L = P.Py;
    A.lgL = lg_or_neg(P.Py);
    A.n_in = P.ny;
    A.n_out = P.Py;
    A.lgP = cap_lgP(lg_tile_for<T>(A.L), P.Kx);
    A.ni = P.Kx;
    A.sa_in = P.Kxp;
    A.sb_in = (long)P.ny * P.Kxp;
    A.sa_out = P.Kxp;
    A.sb_out = (long)P.Py * P.Kxp;
    int k = 0;
    for (int c = 0; c < 3; ++c)
      if (mask >> c & 1) {
        A.in[k] = xlev[c];
        A.out[k] = ylev[c];
        ++k;
      }
    A.inv = 0;
    A.lgTw = P.lgTw;
    tab(A.L, A.tw, A.twg);
    A.pack = P.dcnq ? 1 : 0;
    const double cb = (double)P.Kx * P.nz * 2 * TS;
    timed(P.B * k * cb * (P.ny + P.Py), [&] { return launch_col_fft<T>(A, P.nz * P.B, k, s); });
  }
  void mid_inv(int mask) {
    if (!P.has_mid) return;
    ColFft<T> A{};
    A.L = P.Py;
    A.lgL = lg_or_neg(P.Py);
    A.n_in = P.Py;
    A.n_out = P.ny;
    A.lgP = cap_lgP(lg_tile_for<T>(A.L), P.Kx);
    A.ni = P.Kx;
    A.sa_in = P.Kxp;
    A.sb_in = (long)P.Py * P.Kxp;
    A.sa_out = P.Kxp;
    A.sb_out = (long)P.ny * P.Kxp;
    int k = 0;
    for (int c = 0; c < 3; ++c)
      if (mask >> c & 1) {
        A.in[k] = yout[c];
        A.out[k] = xlev[c];
        ++k;
      }
    A.inv = 1;
    A.lgTw = P.lgTw;
    tab(A.L, A.tw, A.twg);
    A.pack = P.dcnq ? 1 : 0;
    const double cb = (double)P.Kx * P.nz * 2 * TS;
    timed(P.B * k * cb * (P.ny + P.Py), [&] { return launch_col_fft<T>(A, P.nz * P.B, k, s); });
  }
  void conv(int mask, int smask = 7) {
    Conv<T> A{};
    const bool z = P.nz > 1;
    const int L = z ? P.Pz : P.Py;
    A.L = L;
    A.lgL = lg_or_neg(L);
    A.n = z ? P.nz : P.ny;
    A.ni = P.Kx;
    if (z) {
      A.sa = (P.has_mid ? (long)P.Py : 1L) * P.Kxp;
      A.sb = P.has_mid ? P.Kxp : 0;
      A.Hb = P.has_mid ? P.Hy : 1;
      A.Pb = P.has_mid ? P.Py : 1;
      A.oddc = (1 << 4) | (1 << 5);  // xz, yz odd in z
      A.oddb = (1 << 3) | (1 << 5);  // xy, yz odd in y
    } else {
      A.sa = P.Kxp;
      A.sb = 0;
      A.Hb = 1;
      A.Pb = 1;
      A.oddc = (1 << 3) | (1 << 5);
      A.oddb = 0;
    }
    unsigned used = 0;
    int nout = 0;
    for (int c = 0; c < 3; ++c) {
      A.S[c] = (smask >> c & 1) ? comp_spec(c) : nullptr;
      A.O[c] = (mask >> c & 1) ? yout[c] : nullptr;
      if (mask >> c & 1) {
        ++nout;
        // the tensor components of the inputs present
        for (int b = 0; b < 3; ++b)
          if (smask >> b & 1) used |= 1u << (c == b ? c : 2 + c + b);
      }
    }
    A.nt = 0;
    for (int c = 0; c < 6; ++c) {
      A.cpos[c] = 0;
      if (used >> c & 1) {
        A.cpos[c] = A.nt;
        A.clist[A.nt++] = c;
      }
    }
    A.lgP = conv_lgP<T>(A.L, P.Kx, A.nt);
    {
      // small grids: fewer kx per workgroup until the launch has ~256 workgroups
      const long nbw = ((z && P.has_mid) ? P.Hy : 1) * (long)P.B;
      while (A.lgP > 0 && ((P.Kx + (1L << A.lgP) - 1) >> A.lgP) * nbw < 256) --A.lgP;
    }
    // a batched plan: one grid layer per run
    A.runs = P.B;
    A.rs_in = (long)P.nz * (P.has_mid ? P.Py : P.ny) * P.Kxp;
    A.rs_out = A.rs_in;
    A.tens = tens;
    A.nyqb = P.dcnq ? 1 : 0;
    A.tcs = (long)P.Hz * P.Hy * P.Kt;
    A.tkx = P.Kt;
    A.lgTw = P.lgTw;
    tab(A.L, A.tw, A.twg);
    const int nb = (z && P.has_mid) ? P.Hy : 1;
    const int nrows = (z && P.has_mid) ? P.Py : 1;
    const double slab = (double)A.n * A.ni * nrows * 2 * TS * P.B;
    const double tb = A.nt * (double)(z ? P.Hz : P.Hy) * A.Hb * A.ni * TS;
    const int nin = (smask & 1) + (smask >> 1 & 1) + (smask >> 2 & 1);
    timed(nin * slab + nout * slab + tb, [&] { return launch_conv<T>(A, nb, s); });
  }

  // forward transforms of real fields into the component spectra
  void stray_from_fields(const T* const fields[3], int mask) {
    RowIO io;
    int k = 0;
    for (int c = 0; c < 3; ++c)
      if (mask >> c & 1) {
        io.u[k] = fields[c];
        io.xout[k] = r2c_slot(c);
        ++k;
      }
    row_fwd(k, io);
    mid_fwd(mask);
  }

  // the stray-field components of `mask` as x-level spectra ready for c2r
  void stray_eval(int mask) {
    conv(mask);
    mid_inv(mask);
  }

  void set_c2r(const int comps[3], int nch) {
    for (int c = 0; c < 3; ++c) c2r_src_for_[c] = nullptr;
    for (int c = 0; c < nch; ++c) c2r_src_for_[c] = c2r_src(comps[c]);
  }

  // RHS + forward x DCT for heat solves of components comps[0..nch)
  void heat_rhs(int nch, const int comps[3], const T* const u[3], T beta, const T he[3], T* const hs_store[3] = nullptr,
                bool stageF = false) {
    RowIO io;
    io.per_run = true;
    io.stageF = stageF;
    for (int c = 0; c < nch; ++c) {
      io.rcomp[c] = comps[c];
      io.u[c] = u[c];
      // 1 - beta Q as 1 + (-beta Q)
      io.a[c] = (T)1;
      io.alo[c] = (T)(-(double)beta * (comps[c] > 0 ? P.Q : 0.0));
      io.he[c] = he[comps[c]];
      io.dct_out[c] = heat[c];
      io.val_out[c] = f[F_R0 + c];
      if (hs_store) io.hs_out[c] = hs_store[c];
    }
    io.b = beta;
    io.with_hs = P.stray;
    set_c2r(comps, nch);
    row_fwd(nch, io);
  }

  // One SGSPM / GSPM step (paper §3.2 / §3.1), latest-state reading.
  void step(T* m, double alpha, const double he_in[3], const T* src) {
    if (P.prm.scheme == SGSPM_SCHEME_SGS_FF) {
      step_ff(m, alpha, he_in, src);
      return;
    }
    const long N = P.N;
    T* m1 = m;
    T* m2 = m + N;
    T* m3 = m + 2 * N;
    const T dt = (T)P.dt;
    T he[3];
    for (int c = 0; c < 3; ++c) he[c] = P.zeeman ? (T)(he_in[c] * P.fscale) : (T)0;
    const T* s1 = src ? src : nullptr;
    const T* s2 = src ? src + N : nullptr;
    const T* s3 = src ? src + 2 * N : nullptr;
    const bool st = P.stray;
    const bool sgs = P.prm.scheme == SGSPM_SCHEME_SGS;

    // Stage A: g2^n, g3^n from m^n
    if (st) {
      const T* fl[3] = {m1, m2, m3};
      stray_from_fields(fl, 7);
      stray_eval(6);
    }
    {
      const int comps[3] = {1, 2, 0};
      const T* u[3] = {m2, m3, nullptr};
      heat_rhs(2, comps, u, dt, he);
      heat_rest(2, (T)1);
    }
    // Stage B: m1* = m1 + g2^n m3 - g3^n m2 (+ dt s1); g1* from (m1*, m2, m3)
    {
      RowInv<T> A{};
      A.nch = 2;
      A.heat[0] = heat[0];
      A.heat[1] = heat[1];
      A.gout[0] = f[F_G2N];
      A.gout[1] = f[F_G3N];
      A.op = ROW_OP_GS;
      A.base = m1;
      A.Pch = 0;
      A.Qf = m3;
      A.Rch = 1;
      A.Sf = m2;
      A.src = s1;
      A.ds = dt;
      A.out = f[F_A1];
      A.xout = st ? r2c_slot(0) : nullptr;
      row_inv(A, st);
    }
    single_stage(0, f[F_A1], dt, he, (T)1);
    // Stage C: m2* = m2 + g3^n m1* - g1* m3 (+ dt s2); g2* from (m1*, m2*, m3)
    gs_update(f[F_G1S], m2, f[F_G3N], -1, f[F_A1], 0, m3, s2, dt, f[F_A2], 1);
    single_stage(1, f[F_A2], dt, he, (T)1);
    // Stage D: m3* = m3 + g1* m2* - g2* m1* (+ dt s3)
    gs_update(f[F_G2S], m3, f[F_G1S], -1, f[F_A2], 0, f[F_A1], s3, dt, f[F_A3], 2);
    const T* uF[3];
    if (sgs) {
      // g3** from (m1*, m2*, m3** = m3*)
      single_stage(2, f[F_A3], dt, he, (T)1);
      // Stage E: m2** = m2 + g3** m1* - g1* m3** (+ dt s2); g2** from (m1*, m2**, m3**)
      gs_update(f[F_G3SS], m2, nullptr, 0, f[F_A1], -1, f[F_A3], s2, dt, f[F_B2], 1, f[F_G1S]);
      single_stage(1, f[F_B2], dt, he, (T)1);
      // Stage F: m1** = m1 + g2** m3** - g3** m2** (+ dt s1)
      gs_update(f[F_G2SS], m1, nullptr, 0, f[F_A3], -1, f[F_B2], s1, dt, f[F_B1], 0, f[F_G3SS]);
      if (st) {
        mid_fwd(1);
        stray_eval(7);
      }
      uF[0] = f[F_B1];
      uF[1] = f[F_B2];
      uF[2] = f[F_A3];
    } else {
      if (st) {
        mid_fwd(4);
        stray_eval(7);
      }
      uF[0] = f[F_A1];
      uF[1] = f[F_A2];
      uF[2] = f[F_A3];
    }
    // Step 2: (I - alpha eps dt Lap_h) m*** = m** + alpha dt f**
    {
      const int comps[3] = {0, 1, 2};
      T* hsF[3] = {f[F_HS0], f[F_HS1], f[F_HS2]};
      heat_rhs(3, comps, uF, (T)(alpha * P.dt), he, (tape && P.stray) ? hsF : nullptr, true);
      heat_rest(3, (T)alpha, true);
    }
    // Step 3: projection
    {
      RowInv<T> A{};
      A.nch = 3;
      for (int c = 0; c < 3; ++c) A.heat[c] = heat[c];
      A.op = ROW_OP_PROJECT;
      A.mout[0] = m1;
      A.mout[1] = m2;
      A.mout[2] = m3;
      A.nrm = f[F_NRM];
      A.flag = P.flag;
      row_inv(A, false);
    }
  }

  // One SGSPM step (§3.2) under the frozen-field reading: every f of both sweeps
  // is f(m^n), formed once (its stray and anisotropy parts as three real fields),
  // and Step 2 evaluates f(m**) once: two stray-field evaluations per step instead
  // of six.  Only the updates that produce components of m** (m3*, m2**, m1**)
  // transform their output for the second evaluation.
  void step_ff(T* m, double alpha, const double he_in[3], const T* src) {
    const long N = P.N;
    T* mc[3] = {m, m + N, m + 2 * N};
    const T dt = (T)P.dt;
    T he[3];
    for (int c = 0; c < 3; ++c) he[c] = P.zeeman ? (T)(he_in[c] * P.fscale) : (T)0;
    const T* s1 = src ? src : nullptr;
    const T* s2 = src ? src + N : nullptr;
    const T* s3 = src ? src + 2 * N : nullptr;
    const bool st = P.stray;
    // the frozen part of f at m^n: fz_c = -Q [c > 0] m_c + h_s(m^n)_c; without the
    // stray field the RHS reads m_c^n itself with weight -dt Q
    const T* w[3];
    T wc[3];
    if (st) {
      T* fz[3] = {f[F_HS0], f[F_HS1], f[F_HS2]};
      const T* fl[3] = {mc[0], mc[1], mc[2]};
      stray_from_fields(fl, 7);
      stray_eval(7);
      const int comps[3] = {0, 1, 2};
      set_c2r(comps, 3);
      RowIO io;
      for (int c = 0; c < 3; ++c) {
        io.u[c] = mc[c];
        io.a[c] = (T)(c > 0 ? -P.Q : 0.0);
        io.val_out[c] = fz[c];
        w[c] = fz[c];
        wc[c] = dt;
      }
      io.b = (T)1;
      io.with_hs = true;
      row_fwd(3, io);
    } else {
      for (int c = 0; c < 3; ++c) {
        wc[c] = (T)(c > 0 ? -P.dt * P.Q : 0.0);
        w[c] = wc[c] != (T)0 ? mc[c] : nullptr;
      }
    }
    // RHS u_c + dt (f_c(m^n)) and the transforms of the precession solves
    auto solve_rhs = [&](int nch, const int comps[], const T* const u[]) {
      RowIO io;
      for (int k = 0; k < nch; ++k) {
        io.u[k] = u[k];
        io.a[k] = (T)1;
        io.he[k] = he[comps[k]];
        io.w[k] = w[comps[k]];
        io.wc[k] = wc[comps[k]];
        io.dct_out[k] = heat[k];
        io.val_out[k] = f[F_R0 + k];
      }
      io.b = dt;
      io.with_hs = false;
      row_fwd(nch, io);
      heat_rest(nch, (T)1);
    };
    {
      const int comps[2] = {1, 2};
      const T* u[2] = {mc[1], mc[2]};
      solve_rhs(2, comps, u);
    }
    // forward sweep: m1*, m2*, m3* (only m3* = m3** is transformed for Step 2)
    {
      RowInv<T> A{};
      A.nch = 2;
      A.heat[0] = heat[0];
      A.heat[1] = heat[1];
      A.gout[0] = f[F_G2N];
      A.gout[1] = f[F_G3N];
      A.op = ROW_OP_GS;
      A.base = mc[0];
      A.Pch = 0;
      A.Qf = mc[2];
      A.Rch = 1;
      A.Sf = mc[1];
      A.src = s1;
      A.ds = dt;
      A.out = f[F_A1];
      A.xout = nullptr;
      row_inv(A, false);
    }
    {
      const int comps[1] = {0};
      const T* u[1] = {f[F_A1]};
      solve_rhs(1, comps, u);
    }
    gs_update(f[F_G1S], mc[1], f[F_G3N], -1, f[F_A1], 0, mc[2], s2, dt, f[F_A2], 1, nullptr, false);
    {
      const int comps[1] = {1};
      const T* u[1] = {f[F_A2]};
      solve_rhs(1, comps, u);
    }
    gs_update(f[F_G2S], mc[2], f[F_G1S], -1, f[F_A2], 0, f[F_A1], s3, dt, f[F_A3], 2, nullptr, true);
    {
      const int comps[1] = {2};
      const T* u[1] = {f[F_A3]};
      solve_rhs(1, comps, u);
    }
    // backward sweep: m2**, m1** (rebased on m^n)
    gs_update(f[F_G3SS], mc[1], nullptr, 0, f[F_A1], -1, f[F_A3], s2, dt, f[F_B2], 1, f[F_G1S], true);
    {
      const int comps[1] = {1};
      const T* u[1] = {f[F_B2]};
      solve_rhs(1, comps, u);
    }
    gs_update(f[F_G2SS], mc[0], nullptr, 0, f[F_A3], -1, f[F_B2], s1, dt, f[F_B1], 0, f[F_G3SS], true);
    // Step 2 with f(m**): the second stray-field evaluation
    if (st) {
      mid_fwd(7);
      stray_eval(7);
    }
    {
      const int comps[3] = {0, 1, 2};
      const T* uF[3] = {f[F_B1], f[F_B2], f[F_A3]};
      heat_rhs(3, comps, uF, (T)(alpha * P.dt), he);
      heat_rest(3, (T)alpha);
    }
    {
      RowInv<T> A{};
      A.nch = 3;
      for (int c = 0; c < 3; ++c) A.heat[c] = heat[c];
      A.op = ROW_OP_PROJECT;
      for (int c = 0; c < 3; ++c) A.mout[c] = mc[c];
      A.nrm = f[F_NRM];
      A.flag = P.flag;
      row_inv(A, false);
    }
  }

  // stray evaluation for component c of the state (if on) followed by the RHS
  // and the transforms of its precession solve (leaves DCT-level data in heat[0])
  void single_stage(int c, const T* u_c, T beta, const T he[3], T scale) {
    if (P.stray) {
      mid_fwd(1 << c);
      stray_eval(1 << c);
    }
    const int comps[3] = {c, 0, 0};
    const T* u[3] = {u_c, nullptr, nullptr};
    heat_rhs(1, comps, u, beta, he);
    heat_rest(1, scale);
  }

  // Inverse x DCT of heat[0] into gstore, then out = base + Pv Q - Rv S (+ ds src)
  // where a null Pv / Rv pointer (with Pch / Rch = 0) means the inverted array.
  // If `other` is given it replaces the non-inverted operand among P/R.
  void gs_update(T* gstore, const T* base, const T* Pv, int Pch_unused, const T* Q, int Rch_unused, const T* S,
                 const T* src, T ds, T* out, int comp_out, const T* other = nullptr, bool r2c = true) {
    (void)Pch_unused;
    (void)Rch_unused;
    RowInv<T> A{};
    A.nch = 1;
    A.heat[0] = heat[0];
    A.gout[0] = gstore;
    A.op = ROW_OP_GS;
    A.base = base;
    A.Qf = Q;
    A.Sf = S;
    if (Pv) {  // the inverted array is R
      A.Pch = -1;
      A.Pf = Pv;
      A.Rch = 0;
    } else {   // the inverted array is P, R is `other`
      A.Pch = 0;
      A.Rch = -1;
      A.Rf = other;
    }
    A.src = src;
    A.ds = ds;
    A.out = out;
    const bool x = P.stray && r2c;
    A.xout = x ? r2c_slot(comp_out) : nullptr;
    row_inv(A, x);
  }

  // h_s of m into hs (3 fields)
  void stray_to(const T* m, T* hs) {
    const T* fl[3] = {m, m + P.N, m + 2 * P.N};
    stray_from_fields(fl, 7);
    stray_eval(7);
    const int comps[3] = {0, 1, 2};
    set_c2r(comps, 3);
    RowIO io;
    io.with_hs = true;
    for (int c = 0; c < 3; ++c) io.hs_out[c] = hs + c * P.N;
    row_fwd(3, io);
  }

  void heat_solve(const T* r, T scale, T* g) {
    const T* in[3] = {r, nullptr, nullptr};
    T* out[3] = {g, nullptr, nullptr};
    heat_solve_n(1, in, scale, out);
  }

  // g_c = (I - scale eps dt Lap_h)^{-1} r_c for nch channels (in place allowed); with one
  // channel, xout0 (optional) receives the zero-padded r2c of g (the x-level spectrum)
  void heat_solve_n(int nch, const T* const r[3], T scale, T* const g[3], cx<T>* xout0 = nullptr) {
    RowIO io;
    for (int c = 0; c < nch; ++c) {
      io.u[c] = r[c];
      io.dct_out[c] = heat[c];
    }
    row_fwd(nch, io);
    heat_rest(nch, scale);
    RowInv<T> A{};
    A.nch = nch;
    for (int c = 0; c < nch; ++c) {
      A.heat[c] = heat[c];
      A.rin[c] = r[c];
      A.gout[c] = g[c];
    }
    A.op = ROW_OP_NONE;
    A.xout = nch == 1 ? xout0 : nullptr;
    row_inv(A, A.xout != nullptr);
  }

  // acc_a = acc_in_a + kscale K(v)_a + wc_a w_a for a = 0, 1, 2 (null v_c: zero component,
  // null acc_in / w: zero); the stray operator is skipped when the plan has no stray field
  // spectra: the x-level spectra of v are already in place (r2c_slot), as the heat
  // solve that produced v can leave them
  void stray_accumulate(const T* const v[3], T kscale, T* const acc[3], const T* const acc_in[3],
                        const T* const w[3], const T wc[3], const T* wclo = nullptr, bool spectra = false) {
    int mask = 0;
    for (int c = 0; c < 3; ++c)
      if (v[c]) mask |= 1 << c;
    if (P.stray && mask) {
      if (spectra) mid_fwd(mask);
      else stray_from_fields(v, mask);
      conv(7, mask);
      mid_inv(7);
      const int comps[3] = {0, 1, 2};
      set_c2r(comps, 3);
    }
    RowIO io;
    for (int c = 0; c < 3; ++c) {
      io.u[c] = acc_in[c];
      io.a[c] = 1;
      io.w[c] = w[c];
      io.wc[c] = wc[c];
      io.wclo[c] = wclo ? wclo[c] : (T)0;
      io.val_out[c] = acc[c];
    }
    io.b = kscale;
    io.with_hs = P.stray && mask;
    row_fwd(3, io);
  }

  void pw(std::initializer_list<PwTerm<T>> terms) {
    std::vector<PwTerm<T>> t(terms);
    double by = 0;
    for (auto& x : t) by += TS * P.N * (1 + x.acc + (x.x0 ? 1 : 0) + (x.y0 ? 1 : 0) + (x.x1 ? 1 : 0) + (x.y1 ? 1 : 0));
    timed(by, [&] { launch_pw<T>(t.data(), (int)t.size(), P.N, s); return (int)SGSPM_KC_OTHER; });
  }
  static PwTerm<T> set1(T* out, double c0, const T* x0, const T* y0 = nullptr) {
    return PwTerm<T>{out, 0, c0, 0.0, x0, y0, nullptr, nullptr};
  }
  static PwTerm<T> add1(T* out, double c0, const T* x0, const T* y0 = nullptr) {
    return PwTerm<T>{out, 1, c0, 0.0, x0, y0, nullptr, nullptr};
  }
  void sums(std::initializer_list<const T*> xs, std::initializer_list<double> ws, std::initializer_list<int> slots,
            double* grad) {
    const T* x[4] = {nullptr, nullptr, nullptr, nullptr};
    double w[4] = {0, 0, 0, 0};
    int sl[4] = {0, 0, 0, 0};
    int k = 0;
    for (auto v : xs) x[k++] = v;
    k = 0;
    for (auto v : ws) w[k++] = v;
    int n = 0;
    for (auto v : slots) sl[n++] = v;
    timed(n * P.N * TS, [&] { launch_wsum<T>(x, w, sl, n, P.N, P.partials, P.nred, grad, s); return (int)SGSPM_KC_OTHER; });
  }

  // Adjoint of one SGSPM step (latest-state reading): the step recomputed from m_n,
  // its tape left in the workspace fields, then the reverse.
  void adjoint(const T* m_n, double alpha, const double he_in[3], T* lam, double* grad, void* work) {
    T* mt = (T*)work + (long)ADJ_MT * P.N;
    (void)hipMemcpyAsync(mt, m_n, 3 * P.N * sizeof(T), hipMemcpyDeviceToDevice, s);
    tape = true;
    step(mt, alpha, he_in, nullptr);
    tape = false;
    reverse(m_n, mt, alpha, he_in, lam, grad, work);
  }

  // the step's intermediate fields (the tape) live in tp: fields 0 .. F_R0 - 1 of f,
  // then the new state (3 fields); the right-hand-side fields stay in the workspace
  void use_tape(T* tp) {
    for (int i = 0; i < F_R0; ++i) f[i] = tp + (long)i * P.N;
  }

  // The reverse of one step from its tape (f) and its new state u; J = work.
  void reverse(const T* m_n, const T* u, double alpha, const double he_in[3], T* lam, double* grad, void* work) {
    const long N = P.N;
    T* J = (T*)work;
    enum { LA1, LA2, LA3, LB1, LB2, LG1, LG3, LG3N, TMP, MU, LW, MT = LW + 3, NJ = MT + 3 };
    static_assert(MT == ADJ_MT, "adjoint workspace layout");
    T* LW_[3] = {J + (long)LW * N, J + (long)(LW + 1) * N, J + (long)(LW + 2) * N};
    auto Jf = [&](int k) { return J + (long)k * N; };
    const T* m2 = m_n + N;
    const T* m3 = m_n + 2 * N;
    T* lam0 = lam;
    T* lam1 = lam + N;
    T* lam2 = lam + 2 * N;
    const double dt = P.dt;
    const double Q = P.Q;
    const double dh = P.zeeman ? dt * P.fscale : 0.0;  // d(reduced h_e)/d(argument) * dt
    double he[3];
    for (int c = 0; c < 3; ++c) he[c] = P.zeeman ? he_in[c] * P.fscale : 0.0;
    const T* nrm = f[F_NRM];
    // projection and heat flow
    // reads lam, u (3 N each) and |c| (N), writes 3 N
    timed(10.0 * N * TS, [&] { launch_adj_project<T>(lam, u, nrm, LW_[0], N, s); return (int)SGSPM_KC_OTHER; });
    {
      const T* in[3] = {LW_[0], LW_[1], LW_[2]};
      heat_solve_n(3, in, (T)alpha, LW_);
    }
    {
      const T* uF[3] = {f[F_B1], f[F_B2], f[F_A3]};
      const double ex = P.eps;
      // reads w, u, the damping operands and h_s (3 N each) and |c| (N)
      const double by = (P.stray ? 13.0 : 10.0) * N * TS;
      timed(by, [&] {
        launch_adj_damp<T>(LW_[0], u, nrm, uF, P.stray ? f[F_HS0] : nullptr, P.nx, P.ny, P.nz,
                           P.nx > 1 ? ex / (P.prm.dx * P.prm.dx) : 0.0, P.ny > 1 ? ex / (P.prm.dy * P.prm.dy) : 0.0,
                           P.nz > 1 ? ex / (P.prm.dz * P.prm.dz) : 0.0, Q, he, dt, alpha * dh, P.partials, P.nred,
                           grad, s);
        return (int)SGSPM_KC_OTHER;
      });
    }
    {
      const T* v[3] = {LW_[0], LW_[1], LW_[2]};
      T* acc[3] = {Jf(LB1), Jf(LB2), Jf(LA3)};
      const T wc[3] = {0, (T)(-alpha * dt * Q), (T)(-alpha * dt * Q)};
      stray_accumulate(v, (T)(alpha * dt), acc, v, v, wc);
    }
    // the coefficient 1 - dt Q of the precession right-hand sides, as 1 + (-dt Q)
    const T cql = (T)(-dt * Q);
    const T dtt = (T)dt;
    // m1** = m1 + g2** m3** - g3** m2**
    pw({set1(lam0, 1, Jf(LB1)), set1(Jf(TMP), 1, Jf(LB1), f[F_A3]), add1(Jf(LA3), 1, Jf(LB1), f[F_G2SS]),
        set1(Jf(LG3), -1, Jf(LB1), f[F_B2]), add1(Jf(LB2), -1, Jf(LB1), f[F_G3SS])});
    // g2** = H(m2** + dt f2(m1*, m2**, m3**))
    {
      const T* in[3] = {Jf(TMP)};
      T* out[3] = {Jf(MU)};
      heat_solve_n(1, in, (T)1, out, P.stray ? r2c_slot(1) : nullptr);
      sums({Jf(MU)}, {dh}, {1}, grad);
      const T* v[3] = {nullptr, Jf(MU), nullptr};
      T* acc[3] = {Jf(LA1), Jf(LB2), Jf(LA3)};
      const T* ai[3] = {nullptr, Jf(LB2), Jf(LA3)};
      const T* w[3] = {nullptr, Jf(MU), nullptr};
      const T wc[3] = {0, 1, 0}, wl[3] = {0, cql, 0};
      stray_accumulate(v, dtt, acc, ai, w, wc, wl, P.stray);
    }
    // m2** = m2 + g3** m1* - g1* m3**
    pw({set1(lam1, 1, Jf(LB2)), add1(Jf(LG3), 1, Jf(LB2), f[F_A1]), add1(Jf(LA1), 1, Jf(LB2), f[F_G3SS]),
        set1(Jf(LG1), -1, Jf(LB2), f[F_A3]), add1(Jf(LA3), -1, Jf(LB2), f[F_G1S])});
    // g3** = H(m3** + dt f3(m1*, m2*, m3**))
    {
      const T* in[3] = {Jf(LG3)};
      T* out[3] = {Jf(MU)};
      heat_solve_n(1, in, (T)1, out, P.stray ? r2c_slot(2) : nullptr);
      sums({Jf(MU)}, {dh}, {2}, grad);
      const T* v[3] = {nullptr, nullptr, Jf(MU)};
      T* acc[3] = {Jf(LA1), Jf(LA2), Jf(LA3)};
      const T* ai[3] = {Jf(LA1), nullptr, Jf(LA3)};
      const T* w[3] = {nullptr, nullptr, Jf(MU)};
      const T wc[3] = {0, 0, 1}, wl[3] = {0, 0, cql};
      stray_accumulate(v, dtt, acc, ai, w, wc, wl, P.stray);
    }
    // m3* = m3 + g1* m2* - g2* m1*
    pw({set1(lam2, 1, Jf(LA3)), add1(Jf(LG1), 1, Jf(LA3), f[F_A2]), add1(Jf(LA2), 1, Jf(LA3), f[F_G1S]),
        set1(Jf(TMP), -1, Jf(LA3), f[F_A1]), add1(Jf(LA1), -1, Jf(LA3), f[F_G2S])});
    // g2* = H(m2* + dt f2(m1*, m2*, m3))
    {
      const T* in[3] = {Jf(TMP)};
      T* out[3] = {Jf(MU)};
      heat_solve_n(1, in, (T)1, out, P.stray ? r2c_slot(1) : nullptr);
      sums({Jf(MU)}, {dh}, {1}, grad);
      const T* v[3] = {nullptr, Jf(MU), nullptr};
      T* acc[3] = {Jf(LA1), Jf(LA2), lam2};
      const T* ai[3] = {Jf(LA1), Jf(LA2), lam2};
      const T* w[3] = {nullptr, Jf(MU), nullptr};
      const T wc[3] = {0, 1, 0}, wl[3] = {0, cql, 0};
      stray_accumulate(v, dtt, acc, ai, w, wc, wl, P.stray);
    }
    // m2* = m2 + g3^n m1* - g1* m3
    pw({add1(lam1, 1, Jf(LA2)), set1(Jf(LG3N), 1, Jf(LA2), f[F_A1]), add1(Jf(LA1), 1, Jf(LA2), f[F_G3N]),
        add1(Jf(LG1), -1, Jf(LA2), m3), add1(lam2, -1, Jf(LA2), f[F_G1S])});
    // g1* = H(m1* + dt f1(m1*, m2, m3))
    {
      const T* in[3] = {Jf(LG1)};
      T* out[3] = {Jf(MU)};
      heat_solve_n(1, in, (T)1, out, P.stray ? r2c_slot(0) : nullptr);
      sums({Jf(MU)}, {dh}, {0}, grad);
      const T* v[3] = {Jf(MU), nullptr, nullptr};
      T* acc[3] = {Jf(LA1), lam1, lam2};
      const T* ai[3] = {Jf(LA1), lam1, lam2};
      const T* w[3] = {Jf(MU), nullptr, nullptr};
      const T wc[3] = {1, 0, 0};
      stray_accumulate(v, dtt, acc, ai, w, wc, nullptr, P.stray);
    }
    // m1* = m1 + g2^n m3 - g3^n m2
    pw({add1(lam0, 1, Jf(LA1)), set1(Jf(TMP), 1, Jf(LA1), m3), add1(lam2, 1, Jf(LA1), f[F_G2N]),
        add1(Jf(LG3N), -1, Jf(LA1), m2), add1(lam1, -1, Jf(LA1), f[F_G3N])});
    // g2^n = H(m2 + dt f2(m)), g3^n = H(m3 + dt f3(m))
    {
      const T* in[3] = {Jf(TMP), Jf(LG3N)};
      T* out[3] = {Jf(MU), Jf(LG3)};
      heat_solve_n(2, in, (T)1, out);
      sums({Jf(MU), Jf(LG3)}, {dh, dh}, {1, 2}, grad);
      const T* v[3] = {nullptr, Jf(MU), Jf(LG3)};
      T* acc[3] = {lam0, lam1, lam2};
      const T* ai[3] = {lam0, lam1, lam2};
      const T* w[3] = {nullptr, Jf(MU), Jf(LG3)};
      const T wc[3] = {0, 1, 1}, wl[3] = {0, cql, cql};
      stray_accumulate(v, dtt, acc, ai, w, wc, wl);
    }
    static_assert(NJ == ADJ_FIELDS, "adjoint workspace fields");
  }
};

// ---------------------------------------------------------------------------
// cell edges in units of the largest (the tensor is scale free)
void cell_ratios(const sgspm_plan_s* P, double& hx, double& hy, double& hz) {
  const double hs = std::max(P->prm.dx, std::max(P->prm.dy, P->prm.dz));
  hx = P->prm.dx / hs;
  hy = P->prm.dy / hs;
  hz = P->prm.dz / hs;
}

// Plan-time FP64 demagnetising tensor spectrum.
int build_tensor(sgspm_plan_s* P) {
  const long padded = (long)P->Px * P->Py * P->Pz;
  const long speclen = (long)P->Pz * P->Py * P->Kxp;
  void* real = nullptr;
  void* spec = nullptr;
  int rc;
  if ((rc = dalloc(P, &real, padded * sizeof(double)))) return rc;
  if ((rc = dalloc(P, &spec, speclen * sizeof(cx<double>)))) return rc;
  double hx, hy, hz;
  cell_ratios(P, hx, hy, hz);
  const long tcs = (long)P->Hz * P->Hy * P->Kt;
  const double scale = -1.0 / (double)padded;
  for (int comp = 0; comp < 6; ++comp) {
    launch_newell_fill((double*)real, comp, P->nx, P->ny, P->nz, P->Px, P->Py, P->Pz, hx, hy, hz, R_FAR, P->s);
    // x: real-to-complex, full length
    {
      RowFwd<double> A{};
      A.nrows = P->Py * P->Pz;
      A.n = A.Lr = A.Lc = A.Lmax = P->Px;
      A.lgN = A.lgLr = A.lgLc = A.lgLmax = lg_or_neg(P->Px);
      A.lgP = cap_lgP(lg_tile_for<double>(A.Lmax), (A.nrows + 1) / 2);
      A.lgTw = P->lgTw;
      table_for<double>(*P, P->tw64, P->twm64, A.Lmax, A.tw, A.twg);
      A.u[0] = (const double*)real;
      A.a[0] = 1.0;
      A.b = 0.0;
      A.xout[0] = (cx<double>*)spec;
      A.xout_pitch = P->Kxp;
      if (launch_row_fwd<double>(A, 1, P->s) < 0) return fail(SGSPM_EUNSUPPORTED, launch_geom_error());
    }
    // y and z: complex, full length, in place
    for (int ax = 1; ax <= 2; ++ax) {
      const int L = ax == 1 ? P->Py : P->Pz;
      if (L == 1) continue;
      ColFft<double> A{};
      A.L = L;
      A.lgL = lg_or_neg(L);
      A.n_in = L;
      A.n_out = L;
      A.lgP = cap_lgP(lg_tile_for<double>(L), P->Kx);
      A.ni = P->Kx;
      if (ax == 1) {
        A.sa_in = A.sa_out = P->Kxp;
        A.sb_in = A.sb_out = (long)P->Py * P->Kxp;
      } else {
        A.sa_in = A.sa_out = (long)P->Py * P->Kxp;
        A.sb_in = A.sb_out = P->Kxp;
      }
      A.in[0] = (const cx<double>*)spec;
      A.out[0] = (cx<double>*)spec;
      A.inv = 0;
      A.lgTw = P->lgTw;
      table_for<double>(*P, P->tw64, P->twm64, L, A.tw, A.twg);
      if (launch_col_fft<double>(A, ax == 1 ? P->Pz : P->Py, 1, P->s) < 0)
        return fail(SGSPM_EUNSUPPORTED, launch_geom_error());
    }
    if (P->fp64)
      launch_tensor_pack<double>((const cx<double>*)spec, (double*)P->tens + comp * tcs, P->Hz, P->Hy, P->Kx, P->Kxp, P->Kt,
                                 P->Py, scale, P->s);
    else
      launch_tensor_pack<float>((const cx<double>*)spec, (float*)P->tens + comp * tcs, P->Hz, P->Hy, P->Kx, P->Kxp, P->Kt,
                                P->Py, scale, P->s);
  }
  rc = hip_check(hipGetLastError(), "tensor kernels");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(P->s), "tensor sync");
  // release the FP64 scratch
  for (void* p : {real, spec}) {
    (void)hipFree(p);
    P->allocs.erase(std::find(P->allocs.begin(), P->allocs.end(), p));
  }
  return rc;
}

template <typename T> int make_tables(sgspm_plan_s* P) {
  int rc;
  const int Lmax = 1 << P->lgTw;
  std::vector<cx<T>> tw(Lmax);
  std::vector<cx<double>> tw64(Lmax);
  for (int i = 0; i < Lmax; ++i) {
    const double a = -2.0 * M_PI * (double)i / (double)Lmax;
    tw64[i].x = std::cos(a);
    tw64[i].y = std::sin(a);
    tw[i].x = (T)tw64[i].x;
    tw[i].y = (T)tw64[i].y;
  }
  if ((rc = upload(P, &P->tw, tw))) return rc;
  if ((rc = upload(P, &P->tw64, tw64))) return rc;
  const int n[3] = {P->nx, P->ny, P->nz};
  // W_Lm for the non-power-of-two transform lengths
  P->Lm = mixed_table_len(n, P->stray);
  if (P->Lm > 1) {
    std::vector<cx<T>> m(P->Lm);
    std::vector<cx<double>> m64(P->Lm);
    for (long i = 0; i < P->Lm; ++i) {
      const double a = -2.0 * M_PI * (double)i / (double)P->Lm;
      m64[i].x = std::cos(a);
      m64[i].y = std::sin(a);
      m[i].x = (T)m64[i].x;
      m[i].y = (T)m64[i].y;
    }
    if ((rc = upload(P, &P->twm, m))) return rc;
    if ((rc = upload(P, &P->twm64, m64))) return rc;
  }
  const double c[3] = {P->cxx, P->cyy, P->czz};
  for (int a = 0; a < 3; ++a) {
    std::vector<cx<T>> d(n[a]);
    std::vector<T> l(n[a]);
    for (int k = 0; k < n[a]; ++k) {
      const double ang = -M_PI * k / (2.0 * n[a]);
      d[k].x = (T)std::cos(ang);
      d[k].y = (T)std::sin(ang);
      const double sn = std::sin(M_PI * k / (2.0 * n[a]));
      l[k] = (T)(4.0 * c[a] * sn * sn);
    }
    if ((rc = upload(P, &P->dtw[a], d))) return rc;
    if ((rc = upload(P, &P->lam[a], l))) return rc;
  }
  return SGSPM_OK;
}

// device address of this device's copy of `scratch` (once per device)
int scratch_setup(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= MAX_DEVICES) return fail(SGSPM_EUNSUPPORTED, "device ordinal beyond the supported range");
  if (g_scratch_ptr[dev]) return SGSPM_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(SGSPM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = ptr;
  return SGSPM_OK;
}

template <typename T> int alloc_workspace(sgspm_plan_s* P) {
  int rc;
  if ((rc = dalloc(P, &P->fld, (size_t)NF * P->N * sizeof(T)))) return rc;
  if ((rc = dalloc(P, &P->heat, (size_t)3 * P->N * sizeof(T)))) return rc;
  if (P->B > 1) {
    // per-run values start at zero (each batched step fills them first)
    if ((rc = dalloc(P, &P->runp, (size_t)P->B * RUNP * sizeof(T)))) return rc;
    if ((rc = hip_check(hipMemsetAsync(P->runp, 0, (size_t)P->B * RUNP * sizeof(T), P->s), "per-run clear"))) return rc;
  }
  if (P->stray) {
    const long xl = (long)P->B * P->nz * P->ny * P->Kxp;
    const long yl = (long)P->B * P->nz * P->Py * P->Kxp;
    if ((rc = dalloc(P, &P->xlev, 3 * xl * sizeof(cx<T>)))) return rc;
    if (P->has_mid) {
      if ((rc = dalloc(P, &P->ylev, 3 * yl * sizeof(cx<T>)))) return rc;
      if ((rc = dalloc(P, &P->yout, 3 * yl * sizeof(cx<T>)))) return rc;
    } else {
      if ((rc = dalloc(P, &P->yout, 3 * xl * sizeof(cx<T>)))) return rc;
    }
    if ((rc = dalloc(P, &P->tens, (size_t)6 * P->Hz * P->Hy * P->Kt * sizeof(T)))) return rc;
  }
  P->nred = (int)std::min<long>(1024, (P->N + NT - 1) / NT);
  if ((rc = dalloc(P, (void**)&P->partials, (size_t)P->nred * 4 * sizeof(double)))) return rc;
  if ((rc = dalloc(P, (void**)&P->eout, (size_t)std::max(8, 4 * P->B) * sizeof(double)))) return rc;
  if ((rc = dalloc(P, (void**)&P->flag, sizeof(int)))) return rc;
  rc = hip_check(hipMemsetAsync(P->flag, 0, sizeof(int), P->s), "flag clear");
  if (rc) return rc;
  return make_tables<T>(P);
}

// status of the launches of one call: a launch-geometry error first (nothing was
// launched for it), then the runtime's launch error; clears the geometry error
int launch_status(sgspm_plan_s* P, const char* what) {
  if (P->geom_err) {
    P->geom_err = 0;
    (void)hipGetLastError();
    return fail(SGSPM_EUNSUPPORTED, std::string(what) + ": " + P->geom_msg);
  }
  return hip_check(hipGetLastError(), what);
}

template <typename T> int dispatch_step(sgspm_plan_s* P, void* m, double alpha, const double he[3], const void* src) {
  Eng<T> e(*P);
  e.step((T*)m, alpha, he, (const T*)src);
  return launch_status(P, "sgspm_step launch");
}

// per-run values of a batched plan into its device buffer (stream-ordered)
template <typename T> int upload_runs(sgspm_plan_s* P, const double* alpha, const double* h_e) {
  std::vector<T> v((size_t)P->B * RUNP, (T)0);
  for (int b = 0; b < P->B; ++b) {
    T* r = v.data() + (size_t)b * RUNP;
    // the values the single-run step forms from (alpha, h_e), by the same expressions
    for (int c = 0; c < 3; ++c) r[c] = P->zeeman ? (T)(h_e[3 * b + c] * P->fscale) : (T)0;
    const T beta = (T)(alpha[b] * P->dt);
    for (int c = 0; c < 3; ++c) {
      r[3 + c] = (T)1;
      r[8 + c] = (T)(-(double)beta * (c > 0 ? P->Q : 0.0));
    }
    r[6] = beta;
    const T scale = (T)alpha[b];
    r[7] = (T)(scale * P->dt);
  }
  launch_fill<T>((T*)P->runp, v.data(), (long)v.size(), P->s);
  return hip_check(hipGetLastError(), "per-run values");
}

int check_batch_args(sgspm_plan_s* P, const void* m, const double* alpha, const double* h_e, const char* what) {
  if (!P || !m || !alpha || !h_e) return fail(SGSPM_EINVAL, std::string(what) + ": NULL argument");
  if (P->B < 2) return fail(SGSPM_EINVAL, std::string(what) + ": the plan is not batched");
  for (int b = 0; b < P->B; ++b) {
    if (!(alpha[b] >= 0.0) || !std::isfinite(alpha[b])) return fail(SGSPM_EINVAL, "alpha must be >= 0 and finite");
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(h_e[3 * b + c])) return fail(SGSPM_EINVAL, "h_e must be finite");
  }
  return SGSPM_OK;
}

// energies of every run of a batched plan: the stray field of all runs at once,
// then run by run its components and their stray field gathered contiguous in
// the workspace and reduced as for one run
template <typename T> int energy_runs(sgspm_plan_s* P, const void* m, const double* h_e) {
  const double cx_ = P->nx > 1 ? 1.0 / (P->prm.dx * P->prm.dx) : 0.0;
  const double cy_ = P->ny > 1 ? 1.0 / (P->prm.dy * P->prm.dy) : 0.0;
  const double cz_ = P->nz > 1 ? 1.0 / (P->prm.dz * P->prm.dz) : 0.0;
  const long n = P->Nrun, NB = P->N;
  Eng<T> e(*P);
  T* hs = P->stray ? e.f[F_HS0] : nullptr;
  if (hs) e.stray_to((const T*)m, hs);
  // 6 n values from the start of the workspace (below the stray field, which
  // starts at F_HS0 NB >= 12 n)
  T* tm = e.f[0];
  T* th = tm + 3 * n;
  int rc = SGSPM_OK;
  for (int b = 0; b < P->B && !rc; ++b) {
    double he[3];
    for (int c = 0; c < 3; ++c) he[c] = P->zeeman ? h_e[3 * b + c] * P->fscale : 0.0;
    for (int c = 0; c < 3 && !rc; ++c) {
      rc = hip_check(hipMemcpyAsync(tm + c * n, (const T*)m + c * NB + b * n, n * sizeof(T), hipMemcpyDeviceToDevice,
                                    P->s), "energy gather");
      if (!rc && hs)
        rc = hip_check(hipMemcpyAsync(th + c * n, hs + c * NB + b * n, n * sizeof(T), hipMemcpyDeviceToDevice, P->s),
                       "energy gather");
    }
    if (!rc)
      launch_energy<T>(tm, hs ? th : nullptr, P->nx, P->ny, P->nz, cx_, cy_, cz_, he, P->partials, P->nred,
                       P->eout + 4 * b, P->s);
  }
  return rc;
}
}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

int sgspm_validate(const sgspm_params* p) { return validate(p); }

int sgspm_reduced_constants(const sgspm_params* p, double out[5]) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return fail(SGSPM_EINVAL, "out is NULL");
  reduce(p, out);
  return SGSPM_OK;
}

const char* sgspm_last_error(void) { return g_err.c_str(); }

int sgspm_plan(const sgspm_params* p, void* hip_stream, sgspm_plan_t* out) {
  if (!out) return fail(SGSPM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  int dev = 0;
  rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  rc = scratch_setup(dev);
  if (rc) return rc;
  sgspm_plan_s* P = new sgspm_plan_s();
  P->prm = *p;
  P->dev = dev;
  P->s = (hipStream_t)hip_stream;
  P->fp64 = p->precision == SGSPM_FP64;
  P->nx = p->nx;
  P->ny = p->ny;
  P->nz = p->nz;
  P->B = std::max(1, (int)p->batch);
  P->Nrun = (long)p->nx * p->ny * p->nz;
  P->N = P->Nrun * P->B;
  P->Px = p->nx > 1 ? 2 * p->nx : 1;
  P->Py = p->ny > 1 ? 2 * p->ny : 1;
  P->Pz = p->nz > 1 ? 2 * p->nz : 1;
  P->Kx = P->Px / 2 + 1;
  P->Kxp = (P->Kx + 15) / 16 * 16;
  P->Kt = (P->Kx + 31) / 32 * 32;
  P->Hy = P->Py / 2 + 1;
  P->Hz = P->Pz / 2 + 1;
  P->stray = p->terms & SGSPM_TERM_STRAY;
  P->zeeman = p->terms & SGSPM_TERM_ZEEMAN;
  P->has_mid = p->nz > 1 && p->ny > 1;
  // only where every pass over the spectra supports it: the 512-point y pass
  // (ny = 256) and the 64-point z convolution (nz = 32), rows of x bins with 16
  // slots of padding (nx a multiple of 16)
  P->dcnq = P->has_mid && p->ny == 256 && p->nz == 32 && p->nx >= 16 && p->nx % 16 == 0 &&
            P->Kxp == P->Kx - 1 + 16;
  P->yz = yz_reg_plane(p->ny, p->nz) || (P->fp64 ? yz_fits<double>(p->ny, p->nz, 0) : yz_fits<float>(p->ny, p->nz, 0));
  double red[5];
  reduce(p, red);
  P->eps = red[0];
  P->Q = red[1];
  P->dt = red[2];
  P->fscale = red[3];
  P->escale = red[4];
  P->cxx = p->nx > 1 ? P->eps / (p->dx * p->dx) : 0.0;
  P->cyy = p->ny > 1 ? P->eps / (p->dy * p->dy) : 0.0;
  P->czz = p->nz > 1 ? P->eps / (p->dz * p->dz) : 0.0;
  P->lgTw = std::max(2, ilog2(std::max(std::max(P->Px, P->Py), P->Pz)));
  rc = P->fp64 ? alloc_workspace<double>(P) : alloc_workspace<float>(P);
  if (!rc && P->stray) rc = build_tensor(P);
  if (!rc) rc = hip_check(hipStreamSynchronize(P->s), "plan sync");
  if (rc) {
    std::string keep = g_err;
    sgspm_destroy(P);
    g_err = keep;
    return rc;
  }
  *out = P;
  return SGSPM_OK;
}

int sgspm_step(sgspm_plan_t P, void* m, double alpha, const double h_e[3], const void* src) {
  if (!P || !m || !h_e) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_step: a batched plan takes the batched entry points");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SGSPM_EINVAL, "alpha must be >= 0 and finite");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(h_e[c])) return fail(SGSPM_EINVAL, "h_e must be finite");
  return P->fp64 ? dispatch_step<double>(P, m, alpha, h_e, src) : dispatch_step<float>(P, m, alpha, h_e, src);
}

// Capture one step of (m, alpha, h_e) on the plan's private stream as a graph.
int capture_step(sgspm_plan_s* P, void* m, double alpha, const double h_e[3]) {
  int rc;
  if (P->gexec) {
    (void)hipGraphExecDestroy(P->gexec);
    P->gexec = nullptr;
  }
  if (!P->cap) {
    rc = hip_check(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking), "capture stream");
    if (rc) return rc;
  }
  const bool timing = P->timing;
  P->timing = false;  // no event records inside the graph
  hipStream_t keep = P->s;
  P->s = P->cap;
  rc = hip_check(hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed), "begin capture");
  if (!rc) {
    const int src = P->fp64 ? dispatch_step<double>(P, m, alpha, h_e, nullptr)
                            : dispatch_step<float>(P, m, alpha, h_e, nullptr);
    const std::string msg = g_err;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(P->cap, &g);
    rc = src ? fail(src, msg) : hip_check(e, "end capture");
    if (!rc) rc = hip_check(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0), "graph instantiate");
    if (g) (void)hipGraphDestroy(g);
  }
  P->s = keep;
  P->timing = timing;
  if (rc) return rc;
  P->g_m = m;
  P->g_alpha = alpha;
  for (int c = 0; c < 3; ++c) P->g_he[c] = h_e[c];
  return SGSPM_OK;
}

int sgspm_step_spectral_radius(sgspm_plan_t P, void* m, double alpha, const double h_e[3], const void* src,
                               double rho_out[2]) {
  if (!rho_out) return fail(SGSPM_EINVAL, "NULL argument");
  int rc = sgspm_step(P, m, alpha, h_e, src);
  if (rc) return rc;
  const int sgs = P->prm.scheme != SGSPM_SCHEME_GS;
  const double k = P->eps * P->dt;
  const double kx = P->nx > 1 ? k / (P->prm.dx * P->prm.dx) : 0.0;
  const double ky = P->ny > 1 ? k / (P->prm.dy * P->prm.dy) : 0.0;
  const double kz = P->nz > 1 ? k / (P->prm.dz * P->prm.dz) : 0.0;
  const int tape[6] = {F_G2N, F_G3N, F_G1S, F_G2S, F_G3SS, F_G2SS};
  if (P->fp64) {
    Eng<double> e(*P);
    const double* g[6];
    for (int i = 0; i < 6; ++i) g[i] = e.f[tape[i]];
    launch_rho<double>(g, P->nx, P->ny, P->nz, kx, ky, kz, sgs, P->partials, P->nred, P->eout, P->s);
  } else {
    Eng<float> e(*P);
    const float* g[6];
    for (int i = 0; i < 6; ++i) g[i] = e.f[tape[i]];
    launch_rho<float>(g, P->nx, P->ny, P->nz, kx, ky, kz, sgs, P->partials, P->nred, P->eout, P->s);
  }
  rc = launch_status(P, "sgspm_step_spectral_radius launch");
  if (rc) return rc;
  double r[2];
  rc = hip_check(hipMemcpyAsync(r, P->eout, sizeof(r), hipMemcpyDeviceToHost, P->s), "spectral radius copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(P->s), "spectral radius sync");
  if (rc) return rc;
  rho_out[0] = r[0];
  rho_out[1] = sgs ? r[1] : std::nan("");
  return SGSPM_OK;
}

int sgspm_steps(sgspm_plan_t P, void* m, int nsteps, double alpha, const double h_e[3]) {
  if (!P || !m || !h_e) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_steps: a batched plan takes the batched entry points");
  if (nsteps < 0) return fail(SGSPM_EINVAL, "nsteps must be >= 0");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SGSPM_EINVAL, "alpha must be >= 0 and finite");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(h_e[c])) return fail(SGSPM_EINVAL, "h_e must be finite");
  if (nsteps == 0) return SGSPM_OK;
  int rc;
  if (!P->gexec || P->g_m != m || P->g_alpha != alpha || P->g_he[0] != h_e[0] || P->g_he[1] != h_e[1] ||
      P->g_he[2] != h_e[2]) {
    rc = capture_step(P, m, alpha, h_e);
    if (rc) return rc;
  }
  for (int k = 0; k < nsteps; ++k) {
    rc = hip_check(hipGraphLaunch(P->gexec, P->s), "graph launch");
    if (rc) return rc;
  }
  return SGSPM_OK;
}

int sgspm_step_batch(sgspm_plan_t P, void* m, const double* alpha, const double* h_e) {
  int rc = check_batch_args(P, m, alpha, h_e, "sgspm_step_batch");
  if (rc) return rc;
  rc = P->fp64 ? upload_runs<double>(P, alpha, h_e) : upload_runs<float>(P, alpha, h_e);
  if (rc) return rc;
  const double zero[3] = {0.0, 0.0, 0.0};
  return P->fp64 ? dispatch_step<double>(P, m, 0.0, zero, nullptr) : dispatch_step<float>(P, m, 0.0, zero, nullptr);
}

int sgspm_steps_batch(sgspm_plan_t P, void* m, int nsteps, const double* alpha, const double* h_e) {
  int rc = check_batch_args(P, m, alpha, h_e, "sgspm_steps_batch");
  if (rc) return rc;
  if (nsteps < 0) return fail(SGSPM_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return SGSPM_OK;
  rc = P->fp64 ? upload_runs<double>(P, alpha, h_e) : upload_runs<float>(P, alpha, h_e);
  if (rc) return rc;
  // the graph reads the per-run values from the plan's buffer at every replay: it
  // is captured again only for another array
  const double zero[3] = {0.0, 0.0, 0.0};
  if (!P->gexec || P->g_m != m) {
    rc = capture_step(P, m, 0.0, zero);
    if (rc) return rc;
  }
  for (int k = 0; k < nsteps; ++k) {
    rc = hip_check(hipGraphLaunch(P->gexec, P->s), "graph launch");
    if (rc) return rc;
  }
  return SGSPM_OK;
}

int sgspm_energy_batch(sgspm_plan_t P, const void* m, const double* h_e, double* e_out) {
  if (!P || !e_out) return fail(SGSPM_EINVAL, "NULL argument");
  const std::vector<double> zero_alpha((size_t)std::max(1, P->B), 0.0);
  int rc = check_batch_args(P, m, zero_alpha.data(), h_e, "sgspm_energy_batch");
  if (rc) return rc;
  rc = P->fp64 ? energy_runs<double>(P, m, h_e) : energy_runs<float>(P, m, h_e);
  if (rc) return rc;
  rc = launch_status(P, "sgspm_energy_batch launch");
  if (rc) return rc;
  std::vector<double> acc((size_t)4 * P->B);
  rc = hip_check(hipMemcpyAsync(acc.data(), P->eout, acc.size() * sizeof(double), hipMemcpyDeviceToHost, P->s),
                 "energy copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(P->s), "energy sync");
  if (rc) return rc;
  const double V = P->prm.dx * P->prm.dy * P->prm.dz;
  const double es = P->escale;
  for (int b = 0; b < P->B; ++b) {
    const double* a = acc.data() + 4 * b;
    const double ex = 0.5 * P->eps * V * a[0];
    const double an = 0.5 * P->Q * V * a[1];
    const double st = -0.5 * V * a[2];
    const double ze = -V * a[3];
    double* o = e_out + 5 * b;
    o[1] = ex * es;
    o[2] = an * es;
    o[3] = st * es;
    o[4] = ze * es;
    o[0] = (ex + an + st + ze) * es;
  }
  return SGSPM_OK;
}

int sgspm_stray(sgspm_plan_t P, const void* m, void* hs_out) {
  if (!P || !m || !hs_out) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_stray: a batched plan takes the batched entry points");
  if (!P->stray) {
    const size_t bytes = 3 * P->N * (P->fp64 ? 8 : 4);
    return hip_check(hipMemsetAsync(hs_out, 0, bytes, P->s), "stray zero");
  }
  if (P->fp64) Eng<double>(*P).stray_to((const double*)m, (double*)hs_out);
  else Eng<float>(*P).stray_to((const float*)m, (float*)hs_out);
  return launch_status(P, "sgspm_stray launch");
}

int sgspm_field(sgspm_plan_t P, const void* m, const double h_e[3], void* h_out) {
  if (!P || !m || !h_e || !h_out) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_field: a batched plan takes the batched entry points");
  double he[3];
  for (int c = 0; c < 3; ++c) he[c] = P->zeeman ? h_e[c] * P->fscale : 0.0;
  const bool ex = P->eps != 0.0;
  if (P->fp64) {
    Eng<double> e(*P);
    double* hs = P->stray ? e.f[F_HS0] : nullptr;
    if (hs) e.stray_to((const double*)m, hs);
    launch_field_assemble<double>((const double*)m, hs, (double*)h_out, P->nx, P->ny, P->nz,
                                  ex ? 1.0 / (P->prm.dx * P->prm.dx) : 0.0, ex ? 1.0 / (P->prm.dy * P->prm.dy) : 0.0,
                                  ex ? 1.0 / (P->prm.dz * P->prm.dz) : 0.0, P->eps, P->Q, he, P->s);
  } else {
    Eng<float> e(*P);
    float* hs = P->stray ? e.f[F_HS0] : nullptr;
    if (hs) e.stray_to((const float*)m, hs);
    launch_field_assemble<float>((const float*)m, hs, (float*)h_out, P->nx, P->ny, P->nz,
                                 ex ? 1.0 / (P->prm.dx * P->prm.dx) : 0.0, ex ? 1.0 / (P->prm.dy * P->prm.dy) : 0.0,
                                 ex ? 1.0 / (P->prm.dz * P->prm.dz) : 0.0, P->eps, P->Q, he, P->s);
  }
  return launch_status(P, "sgspm_field launch");
}

int sgspm_heat_solve(sgspm_plan_t P, const void* r, double s, void* g) {
  if (!P || !r || !g) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_heat_solve: a batched plan takes the batched entry points");
  if (!(s >= 0.0) || !std::isfinite(s)) return fail(SGSPM_EINVAL, "s must be >= 0 and finite");
  if (P->fp64) Eng<double>(*P).heat_solve((const double*)r, s, (double*)g);
  else Eng<float>(*P).heat_solve((const float*)r, (float)s, (float*)g);
  return launch_status(P, "sgspm_heat_solve launch");
}

int sgspm_energy(sgspm_plan_t P, const void* m, const double h_e[3], double e_out[5]) {
  if (!P || !m || !h_e || !e_out) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_energy: a batched plan takes the batched entry points");
  double he[3];
  for (int c = 0; c < 3; ++c) he[c] = P->zeeman ? h_e[c] * P->fscale : 0.0;
  const double cx_ = P->nx > 1 ? 1.0 / (P->prm.dx * P->prm.dx) : 0.0;
  const double cy_ = P->ny > 1 ? 1.0 / (P->prm.dy * P->prm.dy) : 0.0;
  const double cz_ = P->nz > 1 ? 1.0 / (P->prm.dz * P->prm.dz) : 0.0;
  if (P->fp64) {
    Eng<double> e(*P);
    double* hs = P->stray ? e.f[F_HS0] : nullptr;
    if (hs) e.stray_to((const double*)m, hs);
    launch_energy<double>((const double*)m, hs, P->nx, P->ny, P->nz, cx_, cy_, cz_, he, P->partials, P->nred, P->eout,
                          P->s);
  } else {
    Eng<float> e(*P);
    float* hs = P->stray ? e.f[F_HS0] : nullptr;
    if (hs) e.stray_to((const float*)m, hs);
    launch_energy<float>((const float*)m, hs, P->nx, P->ny, P->nz, cx_, cy_, cz_, he, P->partials, P->nred, P->eout,
                         P->s);
  }
  int rc = launch_status(P, "sgspm_energy launch");
  if (rc) return rc;
  double acc[4];
  rc = hip_check(hipMemcpyAsync(acc, P->eout, sizeof(acc), hipMemcpyDeviceToHost, P->s), "energy copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(P->s), "energy sync");
  if (rc) return rc;
  const double V = P->prm.dx * P->prm.dy * P->prm.dz;
  const double es = P->escale;
  const double ex = 0.5 * P->eps * V * acc[0];
  const double an = 0.5 * P->Q * V * acc[1];
  const double st = -0.5 * V * acc[2];
  const double ze = -V * acc[3];
  e_out[1] = ex * es;
  e_out[2] = an * es;
  e_out[3] = st * es;
  e_out[4] = ze * es;
  e_out[0] = (ex + an + st + ze) * es;
  return SGSPM_OK;
}

int sgspm_unit_error(sgspm_plan_t P, const void* m, double* out) {
  if (!P || !m || !out) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->fp64) launch_unit_error<double>((const double*)m, P->N, P->partials, P->nred, P->eout, P->s);
  else launch_unit_error<float>((const float*)m, P->N, P->partials, P->nred, P->eout, P->s);
  int rc = launch_status(P, "sgspm_unit_error launch");
  if (rc) return rc;
  rc = hip_check(hipMemcpyAsync(out, P->eout, sizeof(double), hipMemcpyDeviceToHost, P->s), "unit error copy");
  if (rc) return rc;
  return hip_check(hipStreamSynchronize(P->s), "unit error sync");
}

int sgspm_adjoint_step(sgspm_plan_t P, const void* m_n, double alpha, const double h_e[3], void* lam,
                       double* grad_dev) {
  if (!P || !m_n || !h_e || !lam || !grad_dev) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_adjoint_step: a batched plan takes the batched entry points");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SGSPM_EINVAL, "alpha must be >= 0 and finite");
  if (P->prm.scheme != SGSPM_SCHEME_SGS) return fail(SGSPM_EUNSUPPORTED, "the adjoint covers the SGS scheme only");
  if (!P->adj) {
    int rc = dalloc(P, &P->adj, (size_t)ADJ_FIELDS * P->N * (P->fp64 ? 8 : 4));
    if (rc) return rc;
  }
  if (P->fp64) Eng<double>(*P).adjoint((const double*)m_n, alpha, h_e, (double*)lam, grad_dev, P->adj);
  else Eng<float>(*P).adjoint((const float*)m_n, alpha, h_e, (float*)lam, grad_dev, P->adj);
  return launch_status(P, "sgspm_adjoint_step launch");
}

int sgspm_tape_bytes(sgspm_plan_t P, size_t* bytes) {
  if (!P || !bytes) return fail(SGSPM_EINVAL, "NULL argument");
  *bytes = (size_t)TAPE_FIELDS * P->N * (P->fp64 ? 8 : 4);
  return SGSPM_OK;
}

int sgspm_step_taped(sgspm_plan_t P, void* m, double alpha, const double h_e[3], void* tape) {
  if (!P || !m || !h_e || !tape) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_step_taped: a batched plan takes the batched entry points");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SGSPM_EINVAL, "alpha must be >= 0 and finite");
  if (P->prm.scheme != SGSPM_SCHEME_SGS) return fail(SGSPM_EUNSUPPORTED, "the adjoint covers the SGS scheme only");
  if (P->fp64) {
    Eng<double> e(*P);
    e.use_tape((double*)tape);
    e.tape = true;
    e.step((double*)m, alpha, h_e, nullptr);
    (void)hipMemcpyAsync((double*)tape + (long)F_R0 * P->N, m, 3 * P->N * sizeof(double), hipMemcpyDeviceToDevice, P->s);
  } else {
    Eng<float> e(*P);
    e.use_tape((float*)tape);
    e.tape = true;
    e.step((float*)m, alpha, h_e, nullptr);
    (void)hipMemcpyAsync((float*)tape + (long)F_R0 * P->N, m, 3 * P->N * sizeof(float), hipMemcpyDeviceToDevice, P->s);
  }
  return launch_status(P, "sgspm_step_taped launch");
}

int sgspm_adjoint_step_taped(sgspm_plan_t P, const void* m_n, double alpha, const double h_e[3], const void* tape,
                             void* lam, double* grad_dev) {
  if (!P || !m_n || !h_e || !tape || !lam || !grad_dev) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_adjoint_step_taped: a batched plan takes the batched entry points");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SGSPM_EINVAL, "alpha must be >= 0 and finite");
  if (P->prm.scheme != SGSPM_SCHEME_SGS) return fail(SGSPM_EUNSUPPORTED, "the adjoint covers the SGS scheme only");
  if (!P->adj) {
    int rc = dalloc(P, &P->adj, (size_t)ADJ_FIELDS * P->N * (P->fp64 ? 8 : 4));
    if (rc) return rc;
  }
  // the reverse only reads the tape
  if (P->fp64) {
    Eng<double> e(*P);
    double* tp = const_cast<double*>(static_cast<const double*>(tape));
    e.use_tape(tp);
    e.reverse((const double*)m_n, tp + (long)F_R0 * P->N, alpha, h_e, (double*)lam, grad_dev, P->adj);
  } else {
    Eng<float> e(*P);
    float* tp = const_cast<float*>(static_cast<const float*>(tape));
    e.use_tape(tp);
    e.reverse((const float*)m_n, tp + (long)F_R0 * P->N, alpha, h_e, (float*)lam, grad_dev, P->adj);
  }
  return launch_status(P, "sgspm_adjoint_step_taped launch");
}

int sgspm_adjoint_step_noalloc(sgspm_plan_t P, const void* m_n, double alpha, const double h_e[3], void* lam,
                               double* grad_dev) {
  if (!P || !m_n || !h_e || !lam || !grad_dev) return fail(SGSPM_EINVAL, "NULL argument");
  if (P->B > 1) return fail(SGSPM_EINVAL, "sgspm_adjoint_step_noalloc: a batched plan takes the batched entry points");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SGSPM_EINVAL, "alpha must be >= 0 and finite");
  if (P->prm.scheme != SGSPM_SCHEME_SGS) return fail(SGSPM_EUNSUPPORTED, "the adjoint covers the SGS scheme only");
  const size_t need = (size_t)ADJ_FIELDS * P->N * (P->fp64 ? 8 : 4);
  if (need > SCRATCH_BYTES)
    return fail(SGSPM_EUNSUPPORTED, "sgspm_adjoint_step_noalloc: the grid needs " + std::to_string(need) +
                                        " bytes of workspace; the static workspace holds " +
                                        std::to_string(SCRATCH_BYTES) + " (at most " +
                                        std::to_string(SCRATCH_BYTES / (ADJ_FIELDS * 4)) + " cells in FP32, " +
                                        std::to_string(SCRATCH_BYTES / (ADJ_FIELDS * 8)) + " in FP64)");
  void* work = g_scratch_ptr[P->dev];
  if (!work) return fail(SGSPM_EHIP, "the static workspace of this device has no address");
  if (P->fp64) Eng<double>(*P).adjoint((const double*)m_n, alpha, h_e, (double*)lam, grad_dev, work);
  else Eng<float>(*P).adjoint((const float*)m_n, alpha, h_e, (float*)lam, grad_dev, work);
  return launch_status(P, "sgspm_adjoint_step_noalloc launch");
}

int sgspm_demag_tensor(sgspm_plan_t P, int comp, void* out) {
  if (!P || !out) return fail(SGSPM_EINVAL, "NULL argument");
  if (comp < 0 || comp > 5) return fail(SGSPM_EINVAL, "comp must be 0..5 (xx yy zz xy xz yz)");
  if (!P->stray) return fail(SGSPM_EINVAL, "the plan has no stray field");
  double hx, hy, hz;
  cell_ratios(P, hx, hy, hz);
  launch_newell_fill((double*)out, comp, P->nx, P->ny, P->nz, P->Px, P->Py, P->Pz, hx, hy, hz, R_FAR, P->s);
  return hip_check(hipGetLastError(), "sgspm_demag_tensor launch");
}

int sgspm_timing(sgspm_plan_t P, int enable) {
  if (!P) return fail(SGSPM_EINVAL, "NULL plan");
  P->timing = enable != 0;
  P->recs.clear();
  P->evnext = 0;
  return SGSPM_OK;
}

int sgspm_timing_read(sgspm_plan_t P, double ms[SGSPM_KC_COUNT], double bytes[SGSPM_KC_COUNT],
                      int64_t launches[SGSPM_KC_COUNT]) {
  if (!P || !ms || !bytes || !launches) return fail(SGSPM_EINVAL, "NULL argument");
  int rc = hip_check(hipStreamSynchronize(P->s), "timing sync");
  if (rc) return rc;
  for (int k = 0; k < SGSPM_KC_COUNT; ++k) {
    ms[k] = 0.0;
    bytes[k] = 0.0;
    launches[k] = 0;
  }
  for (const auto& r : P->recs) {
    float t = 0.f;
    rc = hip_check(hipEventElapsedTime(&t, r.a, r.b), "event elapsed");
    if (rc) return rc;
    ms[r.cls] += t;
    bytes[r.cls] += r.bytes;
    launches[r.cls] += 1;
  }
  P->recs.clear();
  P->evnext = 0;
  return SGSPM_OK;
}

int sgspm_check(sgspm_plan_t P) {
  if (!P) return fail(SGSPM_EINVAL, "NULL plan");
  int h = 0;
  int rc = hip_check(hipMemcpyAsync(&h, P->flag, sizeof(int), hipMemcpyDeviceToHost, P->s), "flag copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(P->s), "flag sync");
  if (rc) return rc;
  if (h) {
    rc = hip_check(hipMemsetAsync(P->flag, 0, sizeof(int), P->s), "flag clear");
    if (rc) return rc;
    return fail(SGSPM_ENUMERIC, "a projection met |m***| = 0 or a non-finite value");
  }
  return SGSPM_OK;
}

int sgspm_destroy(sgspm_plan_t P) {
  if (!P) return SGSPM_OK;
  if (P->s || !P->allocs.empty()) (void)hipStreamSynchronize(P->s);
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  for (void* p : P->allocs) (void)hipFree(p);
  for (hipEvent_t e : P->evpool) (void)hipEventDestroy(e);
  delete P;
  return SGSPM_OK;
}

}  // extern "C"
