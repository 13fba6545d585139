// Argument blocks of the gfx950 kernels of the SGSPM step and their launchers.
//
// Array conventions (all device memory):
//   real field       [nz][ny][nx], x fastest (row pitch nx)
//   x-level spectrum [nz][ny][Kxp] complex: the zero-padded real-to-complex
//                    transform along x of a field (Kx = Px/2 + 1 bins, pitch Kxp)
//   y-level spectrum [nz][Py][Kxp] complex: the above, also transformed (padded)
//                    along y
//   heat array       [nz][ny][nx] real: a field after type-II cosine transforms
//                    along some of its axes
// A "channel" is one of up to three independent arrays handled by one launch
// (grid.z); each argument block carries one pointer per channel.
//
// Packed DC and Nyquist bins (x-level spectra of real rows): both bins are real,
// so bin 0 holds X[0] + i X[N] and bin N is not stored; the y pass transforms
// that column like any other.  At the y level the forward pass splits it again:
// the DC column in column 0, the Nyquist column in the blocked layout (spectra
// whose Nyquist bin N = Kx - 1 is a multiple of 16, with Kxp = N + 16, in planes
// whose row count is a multiple of 16): the Nyquist bin of row r is not at
// (r, N) but at (r & ~15, N + (r & 15)), in the row padding, so that the Nyquist
// bins of 16 consecutive rows form one 128-byte line.  The convolution keeps
// that layout, and the inverse y pass packs the two columns again.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "../../include/sgspm.h"

namespace sgspm {

// element offset of the Nyquist bin `nyq` of row `row` (rows of `pitch` complex)
__host__ __device__ inline long nyq_off(long row, long pitch, int nyq, bool blocked) {
  return blocked ? (row & ~15L) * pitch + nyq + (row & 15) : row * pitch + nyq;
}

// Row kernels (pencils along x; two real rows share one complex FFT).
// Lengths: every transform length is 2^a 3^b 5^c; each length field n comes
// with lgN = log2 n when n is a power of two, else -1 (the kernels then divide
// instead of shifting).  The generic kernels take their twiddles W_Lmax^i from
// tw[i * twg]; the register kernels (power-of-two lengths only) from
// tw[i << (lgTw - log2 L)], tw then being the power-of-two table.
template <typename T> struct RowFwd {
  int nrows;       // real rows per channel
  int n, lgN;      // values per real row
  int Lmax, lgLmax;  // the longest FFT in the launch (sets the tile); the others divide it
  int lgP;         // log2 of complex pencils per tile (2P rows)
  int lgTw;        // log2 length of the power-of-two twiddle table
  int twg;         // stride of W_Lmax in tw (generic kernel)
  const cx<T>* tw;
  // row value v = (b (hs + he[ch]) + alo[ch] u + wclo[ch] w) + a[ch] u + wc[ch] w;
  // u and w may be null (0). A coefficient near one (1 - beta Q) comes as a = 1 and
  // alo = -beta Q: rounded to the working precision as one number it would keep
  // few of beta Q's digits, and lose the same ones at every step.
  const T* u[3];
  T a[3];
  T alo[3];
  T b;
  T he[3];
  const T* w[3];
  T wc[3];
  T wclo[3];
  T* val_out[3];    // optional store of v (may alias u)
  // optional hs by complex-to-real transform (crop) of an x-level spectrum
  const cx<T>* xin[3];
  int Lc, lgLc;
  int xin_pitch;
  T* hs_out[3];     // optional store of hs
  T* dct_out[3];    // optional type-II DCT of v along x
  int dct_xmajor;   // store it x-major: [nx][nrows] instead of [nrows][nx]
  const cx<T>* dtw; // exp(-i pi k / (2n)), k < n
  cx<T>* xout[3];   // optional zero-padded real-to-complex transform of v
  int Lr, lgLr;
  int xout_pitch;
  int xpk;          // xin and xout hold the Nyquist bin in the imaginary part of bin 0
  // independent runs of a batched plan (runp null: one run): rows b rpr ...
  // (b + 1) rpr - 1 belong to run b, and a tile never holds rows of two runs.
  // Run b's applied field (he[ch] <- runp[b RUNP + rcomp[ch]]) replaces he; in
  // the damping step (rstageF) its a[ch], alo[ch] and b as well (runp[b RUNP + 3 +
  // rcomp], runp[b RUNP + 8 + rcomp], runp[b RUNP + 6])
  const T* runp;
  int rpr;
  int rstageF;
  int rcomp[3];
};
// per-run values of a batched plan, in the plan's precision: the applied field
// (3, by component), the damping step's a (3, by component) and b, its heat
// scale s = alpha dt, and the damping step's alo (3, by component)
constexpr int RUNP = 12;

enum { ROW_OP_NONE = 0, ROW_OP_GS = 1, ROW_OP_PROJECT = 2 };

template <typename T> struct RowInv {
  int nrows, n, lgN, Lmax, lgLmax, lgP, lgTw, twg;
  const cx<T>* tw;
  const cx<T>* dtw;
  int nch;             // heat arrays to invert along x (1..3)
  const T* heat[3];
  int heat_xmajor;     // heat arrays are [nx][nrows]
  // the right-hand sides r of the heat solves: the heat arrays hold the spectra of
  // the corrections q r (q = x / (1 + x)), and channel c inverts to g = rin[c] - its
  // inverse transform
  const T* rin[3];
  T* gout[3];          // optional stores of the inverted arrays
  int op;
  // ROW_OP_GS: out = base + Pf * Qf - Rf * Sf + ds * src; Pch/Rch >= 0 select an
  // inverted channel in place of Pf / Rf
  const T* base;
  const T* Pf;
  const T* Qf;
  const T* Rf;
  const T* Sf;
  int Pch, Rch;
  const T* src;
  T ds;
  T* out;
  // ROW_OP_PROJECT: mout = c / |c| over the three channels, nrm = |c|
  T* mout[3];
  T* nrm;
  int* flag;
  // optional zero-padded real-to-complex transform of `out`
  cx<T>* xout;
  int Lr, lgLr;
  int xout_pitch;
  int xpk;             // xout holds the Nyquist bin in the imaginary part of bin 0
};

// Column kernels (pencils along a strided axis; tiles of consecutive inner indices).
enum { COL_DCT_FWD = 0, COL_DCT_INV = 1, COL_DCT_SOLVE = 2 };

template <typename T> struct ColDct {
  int mode;
  int n, lgN;        // pencil length
  int lgP;           // complex pencils per tile (2P real pencils)
  int ni;            // inner extent
  long sa, sb;       // element strides along the axis and along the batch (grid.y)
  T* data[3];        // in place
  const cx<T>* dtw;
  const cx<T>* tw;
  int twg;           // W_n^i = tw[i * twg]
  // COL_DCT_SOLVE diagonal q = x / (1 + x), x = s (lamX[i] + lamB[batch] + lamA[k])
  // (the spectrum of the correction r - g of the heat solve g = (1 + x)^-1 r)
  const T* lamX;
  const T* lamB;
  const T* lamA;
  T s;
};

template <typename T> struct ColFft {
  int L, lgL, n_in, n_out, lgP, ni;
  long sa_in, sb_in, sa_out, sb_out;
  const cx<T>* in[3];
  cx<T>* out[3];
  int inv;
  const cx<T>* tw;
  int lgTw;          // the 512-point kernel: power-of-two table
  int twg;           // the generic kernel: W_L^i = tw[i * twg]
  // the x-level side packs the DC and Nyquist columns in column 0 (ni - 1
  // columns are transformed); the y-level side holds them apart, the Nyquist
  // column ni - 1 in the blocked layout (nyq_off)
  int pack;
};

// Heat solve across y and z of x-major planes [nx][nz][ny] (after the x DCT-II):
// y DCT-II, z DCT-II, the diagonal q = x / (1 + x), x = s (lamX + lamY + lamZ)
// (the spectrum of the correction r - g), z and y inverse, in place, 2^lgPP planes
// per workgroup.
template <typename T> struct YZSolve {
  T* data[3];
  int nx, ny, lgNy, nz, lgNz, lgPP;
  const cx<T>* dtwy;
  const cx<T>* dtwz;
  const cx<T>* tw;   // the register kernel: power-of-two table of 2^lgTw entries
  int lgTw;
  const cx<T>* twy;  // the generic kernel: W_ny^i = twy[i * twy_s], W_nz^i = twz[i * twz_s]
  int twy_s;
  const cx<T>* twz;
  int twz_s;
  const T* lamX;
  const T* lamY;
  const T* lamZ;
  T s;
  // a batched plan: nx planes per run, stored [nx][runs] (plane x of run b at
  // x runs + b); in the damping step (rstageF) the planes of run b take
  // s = runp[b RUNP + 7] (runs 0: one run)
  int runs;
  const T* runp;
  int rstageF;
};
template <typename T> int launch_yz_solve(const YZSolve<T>& a, int nch, hipStream_t s);
// largest plane (ny * nz reals) the fused yz solve holds in one workgroup
template <typename T> constexpr int yz_max_plane() { return sizeof(T) == 4 ? 8192 : 4096; }
// ny * nz * planes <= this many reals per workgroup (16 per thread of 512)
constexpr int YZ_MAX_VALUES = 8192;
// threads of the generic y-z solve's workgroup
constexpr int YZ_NT = 512;
// the generic y-z solve holds 2^lgPP planes of ny x nz in one workgroup
template <typename T> bool yz_fits(int ny, int nz, int lgPP);
// planes that the register y-z kernel handles in either precision
inline bool yz_reg_plane(int ny, int nz) { return ny == 256 && nz == 32; }

// Last-axis convolution: FFT of the three component spectra, multiply by the
// six-component symmetric tensor spectrum, inverse FFT of the requested outputs.
template <typename T> struct Conv {
  int L, lgL, n, lgP, ni;
  long sa, sb;
  const cx<T>* S[3]; // null = component identically zero
  cx<T>* O[3];       // null = output not requested
  const T* tens;     // [6][Hc][Hb][tkx]
  long tcs;
  int tkx;           // kx pitch of the tensor rows (a multiple of 32)
  int nt;            // tensor components used (listed in clist; cpos maps component -> slot)
  int clist[6];
  int cpos[6];
  int Hb, Pb;        // folded / full length of the batch axis
  int oddc, oddb;    // bitmask of components odd along the pencil / batch axis
  const cx<T>* tw;
  int lgTw;          // the 64-point kernel: power-of-two table
  int twg;           // the generic kernel: W_L^i = tw[i * twg]
  int nyqb;          // S and O hold the Nyquist column ni - 1 in the blocked layout over the batch rows
  // a batched plan: runs of the plan (grid z; 0 or 1: one run), run b's S and O
  // at S[c] + b rs_in and O[a] + b rs_out
  int runs;
  long rs_in, rs_out;
};

// Launch-geometry errors.  Every launcher checks, before it launches, the
// invariants its kernel's indexing relies on (tile capacity, LDS bytes, table
// lengths, pencil lengths); when one fails it launches nothing and returns
// LAUNCH_EGEOM, and launch_geom_error() names the kernel and the invariant.
constexpr int LAUNCH_EGEOM = -100;
const char* launch_geom_error();
// LDS of one workgroup on gfx950 (160 KiB per CU)
constexpr size_t LDS_LIMIT = 160 * 1024;

template <typename T> int launch_row_fwd(const RowFwd<T>& a, int nch, hipStream_t s);
template <typename T> int launch_row_inv(const RowInv<T>& a, hipStream_t s);
template <typename T> int launch_col_dct(const ColDct<T>& a, int nbatch, int nch, hipStream_t s);
template <typename T> int launch_col_fft(const ColFft<T>& a, int nbatch, int nch, hipStream_t s);
template <typename T> int launch_conv(const Conv<T>& a, int nbatch, hipStream_t s);
// kx tile (log2) of the convolution for a padded pencil of L and nt tensor components
// (-1: no tile fits)
template <typename T> int conv_lgP(int L, int ni, int nt);

// Demagnetising tensor (FP64): fill the padded real array of one component.
void launch_newell_fill(double* out, int comp, int nx, int ny, int nz, int Px, int Py, int Pz, double hx, double hy,
                        double hz, int rfar, hipStream_t s);
// Real part of the FP64 spectrum on the folded octant, times scale, as T.
template <typename T>
void launch_tensor_pack(const cx<double>* spec, T* out, int Hz, int Hy, int Kx, int Kxp, int Kt, int Py, double scale,
                        hipStream_t s);

// dst[i] = values[i], i < n (host values passed in the launch arguments, 256
// per launch): the per-run values of a batched plan, stream-ordered and
// capturable without a host buffer that must outlive the call
template <typename T> void launch_fill(T* dst, const T* values, long n, hipStream_t s);

// Pointwise product terms: for each term t in order,
//   out_t = (acc_t ? out_t : 0) + c0_t * x0_t * y0_t + c1_t * x1_t * y1_t
// (a null y means 1, a null x drops the product).
template <typename T> struct PwTerm {
  T* out;
  int acc;
  double c0, c1;
  const T *x0, *y0, *x1, *y1;
};
constexpr int PW_MAX = 6;
template <typename T> void launch_pw(const PwTerm<T>* terms, int nterms, long N, hipStream_t s);

// Adjoint of the projection: lc_i = (lam_i - (lam . u) u_i) / nrm.
template <typename T> void launch_adj_project(const T* lam, const T* u, const T* nrm, T* lc, long N, hipStream_t s);

// Deterministic weighted sums: grad[slot_k] += w_k * sum(x_k) (FP64 accumulation).
template <typename T>
void launch_wsum(const T* const x[4], const double w[4], const int slot[4], int nterms, long N, double* partials,
                 int nblocks, double* grad, hipStream_t s);

// Damping-stage sums of the adjoint: grad[3] += dt * sum lw . (eps Lap_h c + F),
// grad[0..2] += wdh * sum lw_i, with c = nrm u, F_i = -Q_i uF_i + hsF_i + he_i.
template <typename T>
void launch_adj_damp(const T* lw, const T* u, const T* nrm, const T* const uF[3], const T* hsF, int nx, int ny,
                     int nz, double ecx, double ecy, double ecz, double Q, const double he[3], double dt, double wdh,
                     double* partials, int nblocks, double* grad, hipStream_t s);

// Spectral radii of the sweep matrices of the last step from its precession
// solves g = {g2^n, g3^n, g1*, g2*, g3**, g2**} (coefficients eps dt Lap_h g,
// k_a = eps dt / h_a^2, 0 for an axis of one cell): out[0] = rho(G_GS),
// out[1] = rho(G_SGS) (only if sgs; else 0).
template <typename T>
void launch_rho(const T* const g[6], int nx, int ny, int nz, double kx, double ky, double kz, int sgs,
                double* partials, int nblocks, double* out, hipStream_t s);

// out[0] = max over cells of | |m| - 1 | in FP64 (out[1] is overwritten).
template <typename T> void launch_unit_error(const T* m, long N, double* partials, int nblocks, double* out, hipStream_t s);

// Pointwise and reduction kernels.
template <typename T>
void launch_field_assemble(const T* m, const T* hs, T* out, int nx, int ny, int nz, double cxx, double cyy, double czz,
                           double eps_on, double Q, const double he[3], hipStream_t s);
template <typename T>
void launch_energy(const T* m, const T* hs, int nx, int ny, int nz, double cxx, double cyy, double czz,
                   const double he[3], double* partials, int nblocks, double* out, hipStream_t s);

}  // namespace sgspm
