// gfx950 kernels of one SGSPM step: x-row transforms with fused pointwise
// prologues/epilogues, strided column transforms, the last-axis fused
// DCT-diagonal-IDCT heat solve, the last-axis fused FFT-tensor-IFFT stray-field
// convolution, the FP64 Newell tensor, and FP64 reductions.
//
// Heat-type solve (paper §3, g = (I - c Lap_h)^{-1} r with Neumann BC): the
// mirror-ghost Lap_h is diagonal in the type-II DCT basis (the solve runs in
// correction form, g = r - DCT^-1 (q DCT r), see heat_q); each 1-D DCT-II of
// length n is computed by Makhoul's method, a length-n complex FFT of the
// even/odd-reordered sequence followed by a twiddle, with two real pencils
// packed into one complex FFT.  Stray field (h_s = -N (*) m): zero-padded
// real-to-complex FFT along x, complex FFTs along y and z, multiplication by the
// precomputed real tensor spectrum, inverse transforms cropped to the grid.
#include <cmath>

#include "kernels.h"

namespace sgspm {

template <typename T> __device__ __forceinline__ cx<T> zero() { return mk<T>((T)0, (T)0); }

// Heat solves g = (1 + x)^-1 r per mode, x = s (lx + ly + lz) >= 0, run in
// correction form: the spectral pass multiplies by q = x / (1 + x) and the last
// inverse pass forms g = r - T^-1 (q T r). The transforms then touch only the
// correction, which is small on the smooth modes: in single precision the pair
// T^-1 T is not the identity (the rounded twiddles shrink their inputs by ~1e-7
// per solve, the same way at every step), and the damping solve's low modes have
// x of order 1e-7, which 1 + x rounded to single precision would keep one or two
// digits of. q keeps x's relative precision.
template <typename T> __device__ __forceinline__ T heat_q(T x) { return x / ((T)1 + x); }

// element at a byte offset from a base pointer
template <typename V> __device__ __forceinline__ V ld_off(const V* base, unsigned byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename V> __device__ __forceinline__ void st_off(V* base, unsigned byte_off, V v) {
  *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Workgroups go to the 8 XCDs round-robin by linear id, and each XCD has its
// own L2.  Renumber them so that consecutive logical workgroups (neighbours
// that read the two halves of the same 128-byte lines) run on one XCD.
struct Blk {
  int x, y, z;
};
__device__ __forceinline__ Blk xcd_block() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int n = gx * gy * (int)gridDim.z;
  const int L = (int)blockIdx.x + gx * ((int)blockIdx.y + gy * (int)blockIdx.z);
  const int q = n >> 3, rem = n & 7, xc = L & 7;
  const int lg = xc * q + min(xc, rem) + (L >> 3);
  Blk b;
  b.x = lg % gx;
  b.y = (lg / gx) % gy;
  b.z = lg / (gx * gy);
  return b;
}

// ---------------------------------------------------------------------------
// Shared row-kernel helpers (tile: P complex pencils = 2P real rows).  Lengths
// are any 2^a 3^b 5^c; qdiv / qmod shift when a length is a power of two.

// Zero-padded real-to-complex transform of the per-thread row values `val`
// (element e = tid + i NT of the tile) and store of bins 0..Lr/2.
template <typename T, int NV, bool MX>
__device__ __forceinline__ void row_r2c_store(cx<T>* buf, const cx<T>* tw, const T (&val)[NV], int tot, int n, int lgN,
                                              int Lr, int lgLr, int Lmax, int lgP, int row0, int nrows, cx<T>* xout,
                                              int pitch, bool xpk) {
  const int P = 1 << lgP;
  T* bufr = reinterpret_cast<T*>(buf);
  const int ps = Lr + 1;
  for (int t = threadIdx.x; t < P * Lr; t += NT) {
    const int x = qmod<MX>(t, Lr, lgLr);
    if (x >= n) buf[qdiv<MX>(t, Lr, lgLr) * ps + x] = zero<T>();
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < tot) {
      const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
      bufr[2 * ((row >> 1) * ps + x) + (row & 1)] = val[i];
    }
  }
  __syncthreads();
  FftGeom g{Lr, lgLr, lgP, 1, false, ps, 1, Lmax / Lr};
  fft_lds<T, Tile<T>::VPT, NT, MX>(buf, tw, g, false);
  const int half = Lr >> 1;
  for (int t = threadIdx.x; t < P * Lr; t += NT) {
    const int k = qmod<MX>(t, Lr, lgLr);
    if (k > half || (xpk && k == half)) continue;
    const int q = qdiv<MX>(t, Lr, lgLr);
    const cx<T> Zk = buf[q * ps + k];
    const cx<T> Zm = buf[q * ps + (k ? Lr - k : 0)];
    // X_a = (Z_k + conj Z_{-k}) / 2 ; X_b = (Z_k - conj Z_{-k}) / (2i)
    cx<T> Xa = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
    cx<T> Xb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
    if (xpk && k == 0) {
      // packed: X_a[half] = Re Z_half and X_b[half] = Im Z_half (both real) in the
      // imaginary part of bin 0
      const cx<T> Zh = buf[q * ps + half];
      Xa.y = Zh.x;
      Xb.y = Zh.y;
    }
    const int ra = row0 + 2 * q;
    if (ra < nrows) xout[(long)ra * pitch + k] = Xa;
    if (ra + 1 < nrows) xout[(long)(ra + 1) * pitch + k] = Xb;
  }
  __syncthreads();
}

// the FFT twiddles W_Lmax^i and the DCT twiddles of length n <= Lmax into LDS, both
// loads of an index issued before either store; the DCT table is optional (a plain
// r2c launch, such as the tensor build's, passes none)
template <typename T>
__device__ __forceinline__ void load_row_tables(cx<T>* tw, cx<T>* dtl, const cx<T>* gtw, int twg, const cx<T>* gdt,
                                                int Lmax, int n) {
  for (int i = threadIdx.x; i < Lmax; i += NT) {
    const cx<T> a = gtw[i * twg];
    const cx<T> d = gdt ? gdt[min(i, n - 1)] : zero<T>();
    tw[i] = a;
    if (i < n) dtl[i] = d;
  }
}

// ---------------------------------------------------------------------------
// Row forward kernel: [c2r of x-level hs] -> v = a u + b (hs + he) ->
// [DCT-II along x] and/or [zero-padded r2c along x].
template <typename T, bool MX>
__global__ __launch_bounds__(NT) void k_row_fwd(const RowFwd<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NV = 2 * Tile<T>::VPT, VPT = Tile<T>::VPT;
  const int ch = blockIdx.z;
  const int Lmax = A.Lmax;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + Lmax;
  const int P = 1 << A.lgP;
  const int row0 = blockIdx.x * 2 * P;
  const int n = A.n, lgN = A.lgN;
  const int tot = 2 * P * n;
  // the DCT twiddles in LDS after the tile (no global load among the stores)
  cx<T>* dtl = buf + P * (Lmax + 1);
  T hs[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) hs[i] = (T)0;

  const cx<T>* xin = A.xin[ch];
  const int Lc = A.Lc, lgLc = A.lgLc;
  const int half = Lc >> 1;
  // the spectra first (at most VPT per thread: P Lc fits the tile), then the tables,
  // then the LDS stores: one round trip to memory
  cx<T> Ra[VPT], Rb[VPT];
  if (xin) {
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int t = threadIdx.x + j * NT;
      Ra[j] = Rb[j] = zero<T>();
      if (t < P * Lc) {
        const int q = qdiv<MX>(t, Lc, lgLc), k = qmod<MX>(t, Lc, lgLc);
        const int ra = row0 + 2 * q;
        const int kk = k > half ? Lc - k : k;
        const int kl = A.xpk && kk == half ? 0 : kk;  // packed: the Nyquist bin is in bin 0
        if (ra < A.nrows) Ra[j] = xin[(long)ra * A.xin_pitch + kl];
        if (ra + 1 < A.nrows) Rb[j] = xin[(long)(ra + 1) * A.xin_pitch + kl];
      }
    }
  }
  load_row_tables<T>(tw, dtl, A.tw, A.twg, A.dtw, Lmax, n);
  __syncthreads();
  if (xin) {
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int t = threadIdx.x + j * NT;
      if (t < P * Lc) {
        const int q = qdiv<MX>(t, Lc, lgLc), k = qmod<MX>(t, Lc, lgLc);
        const bool cj = k > half;
        const int kk = cj ? Lc - k : k;
        cx<T> Xa = Ra[j], Xb = Rb[j];
        if (kk == 0 || kk == half) {
          if (A.xpk && kk == half) {
            Xa.x = Xa.y;
            Xb.x = Xb.y;
          }
          Xa.y = (T)0;
          Xb.y = (T)0;
        }
        if (cj) {
          Xa.y = -Xa.y;
          Xb.y = -Xb.y;
        }
        buf[q * (Lc + 1) + k] = mk<T>(Xa.x - Xb.y, Xa.y + Xb.x);
      }
    }
    __syncthreads();
    FftGeom g{Lc, lgLc, A.lgP, 1, false, Lc + 1, 1, Lmax / Lc};
    fft_lds<T, Tile<T>::VPT, NT, MX>(buf, tw, g, true);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < tot) {
        const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
        const cx<T> z = buf[(row >> 1) * (Lc + 1) + x];
        hs[i] = (row & 1) ? z.y : z.x;
      }
    }
    __syncthreads();
  }

  T val[NV];
  const T* u = A.u[ch];
  const T* w = A.w[ch];
  T* hso = A.hs_out[ch];
  T* vo = A.val_out[ch];
  T ac = A.a[ch], aloc = A.alo[ch], hec = A.he[ch], bc = A.b;
  const T wcc = A.wc[ch], wcloc = A.wclo[ch];
  if (A.runp) {
    // every row of the tile belongs to one run
    const T* r = A.runp + (long)(min(row0, A.nrows - 1) / A.rpr) * RUNP;
    hec = r[A.rcomp[ch]];
    if (A.rstageF) {
      ac = r[3 + A.rcomp[ch]];
      aloc = r[8 + A.rcomp[ch]];
      bc = r[6];
    }
  }
  // loads of every element first (clamped indices, no branch between them), stores
  // after (loads and stores share one in-order counter)
  auto cidx = [&](int i) {
    const int e = min((int)threadIdx.x + i * NT, tot - 1);
    return (long)min(row0 + qdiv<MX>(e, n, lgN), A.nrows - 1) * n + qmod<MX>(e, n, lgN);
  };
#pragma unroll
  for (int i = 0; i < NV; ++i) val[i] = bc * (hs[i] + hec);
  // the small parts first, the leading coefficients last
  T pu[NV], pw[NV];
  if (u) {
#pragma unroll
    for (int i = 0; i < NV; ++i) pu[i] = u[cidx(i)];
#pragma unroll
    for (int i = 0; i < NV; ++i) val[i] += aloc * pu[i];
  }
  if (w) {
#pragma unroll
    for (int i = 0; i < NV; ++i) pw[i] = w[cidx(i)];
#pragma unroll
    for (int i = 0; i < NV; ++i) val[i] += wcloc * pw[i];
  }
  if (u) {
#pragma unroll
    for (int i = 0; i < NV; ++i) val[i] += ac * pu[i];
  }
  if (w) {
#pragma unroll
    for (int i = 0; i < NV; ++i) val[i] += wcc * pw[i];
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < tot) {
      const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
      const int grow = row0 + row;
      if (grow < A.nrows) {
        const long idx = (long)grow * n + x;
        if (hso) hso[idx] = hs[i];
        if (vo) vo[idx] = val[i];
      }
    }
  }

  T* dout = A.dct_out[ch];
  if (dout) {
    T* bufr = reinterpret_cast<T*>(buf);
    const int ps = n + 1;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < tot) {
        const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
        bufr[2 * ((row >> 1) * ps + makhoul_pos(x, n)) + (row & 1)] = val[i];
      }
    }
    __syncthreads();
    FftGeom g{n, lgN, A.lgP, 1, false, ps, 1, Lmax / n};
    fft_lds<T, Tile<T>::VPT, NT, MX>(buf, tw, g, false);
    for (int t = threadIdx.x; t < P * n; t += NT) {
      // x-major stores take consecutive rows per thread group, row-major consecutive k
      const int q = A.dct_xmajor ? (t & (P - 1)) : qdiv<MX>(t, n, lgN);
      const int k = A.dct_xmajor ? (t >> A.lgP) : qmod<MX>(t, n, lgN);
      const cx<T> Zk = buf[q * ps + k];
      const cx<T> Zm = buf[q * ps + (k ? n - k : 0)];
      const cx<T> Va = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
      const cx<T> Vb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
      const cx<T> w = dtl[k];
      const int ra = row0 + 2 * q;
      const T xa = w.x * Va.x - w.y * Va.y, xb = w.x * Vb.x - w.y * Vb.y;
      if (A.dct_xmajor) {
        if (ra < A.nrows) dout[(long)k * A.nrows + ra] = xa;
        if (ra + 1 < A.nrows) dout[(long)k * A.nrows + ra + 1] = xb;
      } else {
        if (ra < A.nrows) dout[(long)ra * n + k] = xa;
        if (ra + 1 < A.nrows) dout[(long)(ra + 1) * n + k] = xb;
      }
    }
    __syncthreads();
  }

  cx<T>* xo = A.xout[ch];
  if (xo)
    row_r2c_store<T, NV, MX>(buf, tw, val, tot, n, lgN, A.Lr, A.lgLr, Lmax, A.lgP, row0, A.nrows, xo, A.xout_pitch,
                         A.xpk != 0);
}

// ---------------------------------------------------------------------------
// Row inverse kernel: inverse DCT-II along x of 1..3 heat arrays, then a
// Gauss-Seidel update or the projection, then optionally the zero-padded r2c
// transform of the updated component.
template <typename T, bool MX>
__global__ __launch_bounds__(NT) void k_row_inv(const RowInv<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NV = 2 * Tile<T>::VPT, VPT = Tile<T>::VPT;
  const int Lmax = A.Lmax;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + Lmax;
  const int P = 1 << A.lgP;
  const int row0 = blockIdx.x * 2 * P;
  const int n = A.n, lgN = A.lgN;
  const int tot = 2 * P * n;
  cx<T>* dtl = buf + P * (Lmax + 1);  // DCT twiddles
  load_row_tables<T>(tw, dtl, A.tw, A.twg, A.dtw, Lmax, n);
  const T invn = (T)1 / (T)n;
  T g[3][NV];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int i = 0; i < NV; ++i) g[c][i] = (T)0;
  }
  // one channel: inverse x DCT of heat array c into gc (one call per channel, so
  // that every register array is indexed by constants)
  auto channel = [&](int c, T(&gc)[NV]) {
    __syncthreads();
    // the right-hand side r into gc first (clamped indices), g = r - the inverse
    // transform of the correction at the end
    {
      const T* R = A.rin[c];
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int e = min((int)threadIdx.x + i * NT, tot - 1);
        gc[i] = R[(long)min(row0 + qdiv<MX>(e, n, lgN), A.nrows - 1) * n + qmod<MX>(e, n, lgN)];
      }
    }
    const T* H = A.heat[c];
    const int ps = n + 1;
    // loads in groups of four rows of the loop (at most VPT per thread), each
    // group issued before its LDS stores
    constexpr int CH = 4;
#pragma unroll
    for (int j0 = 0; j0 < VPT; j0 += CH) {
      T rak[CH], ram[CH], rbk[CH], rbm[CH];
#pragma unroll
      for (int jj = 0; jj < CH; ++jj) {
        const int t = threadIdx.x + (j0 + jj) * NT;
        rak[jj] = ram[jj] = rbk[jj] = rbm[jj] = (T)0;
        if (t < P * n) {
          const int q = A.heat_xmajor ? (t & (P - 1)) : qdiv<MX>(t, n, lgN);
          const int k = A.heat_xmajor ? (t >> A.lgP) : qmod<MX>(t, n, lgN);
          const int ra = row0 + 2 * q;
          if (A.heat_xmajor) {
            const long nr = A.nrows;
            if (ra < A.nrows) {
              rak[jj] = H[(long)k * nr + ra];
              if (k) ram[jj] = H[(long)(n - k) * nr + ra];
            }
            if (ra + 1 < A.nrows) {
              rbk[jj] = H[(long)k * nr + ra + 1];
              if (k) rbm[jj] = H[(long)(n - k) * nr + ra + 1];
            }
          } else {
            if (ra < A.nrows) {
              rak[jj] = H[(long)ra * n + k];
              if (k) ram[jj] = H[(long)ra * n + n - k];
            }
            if (ra + 1 < A.nrows) {
              rbk[jj] = H[(long)(ra + 1) * n + k];
              if (k) rbm[jj] = H[(long)(ra + 1) * n + n - k];
            }
          }
        }
      }
#pragma unroll
      for (int jj = 0; jj < CH; ++jj) {
        const int t = threadIdx.x + (j0 + jj) * NT;
        if (t < P * n) {
          const int q = A.heat_xmajor ? (t & (P - 1)) : qdiv<MX>(t, n, lgN);
          const int k = A.heat_xmajor ? (t >> A.lgP) : qmod<MX>(t, n, lgN);
          const cx<T> w = conjg(dtl[k]);
          const cx<T> Va = cmul(w, mk<T>(rak[jj], -ram[jj]));
          const cx<T> Vb = cmul(w, mk<T>(rbk[jj], -rbm[jj]));
          buf[q * ps + k] = mk<T>(Va.x - Vb.y, Va.y + Vb.x);
        }
      }
    }
    __syncthreads();
    FftGeom gm{n, lgN, A.lgP, 1, false, ps, 1, Lmax / n};
    fft_lds<T, Tile<T>::VPT, NT, MX>(buf, tw, gm, true);
    T* go = A.gout[c];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < tot) {
        const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
        const cx<T> z = buf[(row >> 1) * ps + makhoul_pos(x, n)];
        gc[i] -= ((row & 1) ? z.y : z.x) * invn;
        if (go && row0 + row < A.nrows) go[(long)(row0 + row) * n + x] = gc[i];
      }
    }
  };
  channel(0, g[0]);
  if (A.nch > 1) channel(1, g[1]);
  if (A.nch > 2) channel(2, g[2]);
  __syncthreads();

  if (A.op == ROW_OP_GS) {
    // loads of every element first, stores after
    T val[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = threadIdx.x + i * NT;
      val[i] = (T)0;
      if (e < tot) {
        const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
        if (row0 + row < A.nrows) {
          const long idx = (long)(row0 + row) * n + x;
          const T pv = A.Pch == 0 ? g[0][i] : (A.Pch == 1 ? g[1][i] : A.Pf[idx]);
          const T rv = A.Rch == 0 ? g[0][i] : (A.Rch == 1 ? g[1][i] : A.Rf[idx]);
          T o = A.base[idx] + pv * A.Qf[idx] - rv * A.Sf[idx];
          if (A.src) o += A.ds * A.src[idx];
          val[i] = o;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < tot) {
        const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
        if (row0 + row < A.nrows) A.out[(long)(row0 + row) * n + x] = val[i];
      }
    }
    if (A.xout)
      row_r2c_store<T, NV, MX>(buf, tw, val, tot, n, lgN, A.Lr, A.lgLr, Lmax, A.lgP, row0, A.nrows, A.xout, A.xout_pitch,
                           A.xpk != 0);
  } else if (A.op == ROW_OP_PROJECT) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < tot) {
        const int row = qdiv<MX>(e, n, lgN), x = qmod<MX>(e, n, lgN);
        if (row0 + row < A.nrows) {
          const long idx = (long)(row0 + row) * n + x;
          const T c0 = g[0][i], c1 = g[1][i], c2 = g[2][i];
          const T nr = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
          if (!(nr > (T)0) || !isfinite(nr)) A.flag[0] = 1;
          const T inr = (T)1 / nr;
          A.mout[0][idx] = c0 * inr;
          A.mout[1][idx] = c1 * inr;
          A.mout[2][idx] = c2 * inr;
          if (A.nrm) A.nrm[idx] = nr;
        }
      }
    }
  } else if (A.op == ROW_OP_NONE && A.nch == 1 && A.xout) {
    // a plain inverse of one channel: the r2c of its result
    row_r2c_store<T, NV, MX>(buf, tw, g[0], tot, n, lgN, A.Lr, A.lgLr, Lmax, A.lgP, row0, A.nrows, A.xout,
                             A.xout_pitch, A.xpk != 0);
  }
}

// ---------------------------------------------------------------------------
// Column DCT kernel (in place): forward DCT-II, inverse, or the full heat solve
// along the pencil axis (forward, diagonal, inverse).  Real pencils
// i0 + q and i0 + q + P share complex pencil q; LDS layout buf[j * P + q].
template <typename T, bool MX>
__global__ __launch_bounds__(NT) void k_col_dct(const ColDct<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int VPT = Tile<T>::VPT;
  const int n = A.n, lgN = A.lgN;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + n;
  load_twiddles(tw, A.tw, n, A.twg);
  const int P = 1 << A.lgP;
  const int i0 = blockIdx.x * 2 * P;
  const int b = blockIdx.y;
  T* D = A.data[blockIdx.z] + (long)b * A.sb;
  T* bufr = reinterpret_cast<T*>(buf);
  const T invn = (T)1 / (T)n;
  __syncthreads();

  if (A.mode == COL_DCT_FWD || A.mode == COL_DCT_SOLVE) {
    for (int t = threadIdx.x; t < 2 * P * n; t += NT) {
      const int j = t >> (A.lgP + 1), ii = t & (2 * P - 1);
      const int i = i0 + ii;
      const T v = (i < A.ni) ? D[(long)j * A.sa + i] : (T)0;
      bufr[2 * (makhoul_pos(j, n) * P + (ii & (P - 1))) + (ii >> A.lgP)] = v;
    }
    __syncthreads();
    FftGeom g{n, lgN, A.lgP, 1, true, 1, P, 1};
    fft_lds<T, Tile<T>::VPT, NT, MX>(buf, tw, g, false);
    T xa[VPT], xb[VPT];
#pragma unroll
    for (int s = 0; s < VPT; ++s) {
      const int t = threadIdx.x + s * NT;
      xa[s] = xb[s] = (T)0;
      if (t < P * n) {
        const int k = t >> A.lgP, q = t & (P - 1);
        const cx<T> Zk = buf[k * P + q];
        const cx<T> Zm = buf[(k ? n - k : 0) * P + q];
        const cx<T> Va = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
        const cx<T> Vb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
        const cx<T> w = A.dtw[k];
        xa[s] = w.x * Va.x - w.y * Va.y;
        xb[s] = w.x * Vb.x - w.y * Vb.y;
        const int ia = i0 + q, ib = i0 + q + P;
        if (A.mode == COL_DCT_FWD) {
          if (ia < A.ni) D[(long)k * A.sa + ia] = xa[s];
          if (ib < A.ni) D[(long)k * A.sa + ib] = xb[s];
        } else {
          const T lb = (A.lamB ? A.lamB[b] : (T)0) + A.lamA[k];
          if (ia < A.ni) xa[s] *= heat_q(A.s * (A.lamX[ia] + lb));
          if (ib < A.ni) xb[s] *= heat_q(A.s * (A.lamX[ib] + lb));
        }
      }
    }
    if (A.mode == COL_DCT_FWD) return;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < VPT; ++s) {
      const int t = threadIdx.x + s * NT;
      if (t < P * n) buf[t] = mk<T>(xa[s], xb[s]);
    }
    __syncthreads();
  }

  // inverse: V_k = exp(+i pi k / 2n) (X_k - i X_{n-k}); x = IFFT(V) / n, un-reordered
  {
    cx<T> z[VPT];
#pragma unroll
    for (int s = 0; s < VPT; ++s) {
      const int t = threadIdx.x + s * NT;
      z[s] = zero<T>();
      if (t < P * n) {
        const int k = t >> A.lgP, q = t & (P - 1);
        T xak, xam = 0, xbk, xbm = 0;
        if (A.mode == COL_DCT_INV) {
          const int ia = i0 + q, ib = i0 + q + P;
          xak = (ia < A.ni) ? D[(long)k * A.sa + ia] : (T)0;
          xbk = (ib < A.ni) ? D[(long)k * A.sa + ib] : (T)0;
          if (k) {
            xam = (ia < A.ni) ? D[(long)(n - k) * A.sa + ia] : (T)0;
            xbm = (ib < A.ni) ? D[(long)(n - k) * A.sa + ib] : (T)0;
          }
        } else {
          const cx<T> Xk = buf[k * P + q];
          xak = Xk.x;
          xbk = Xk.y;
          if (k) {
            const cx<T> Xm = buf[(n - k) * P + q];
            xam = Xm.x;
            xbm = Xm.y;
          }
        }
        const cx<T> w = conjg(A.dtw[k]);
        const cx<T> Va = cmul(w, mk<T>(xak, -xam));
        const cx<T> Vb = cmul(w, mk<T>(xbk, -xbm));
        z[s] = mk<T>(Va.x - Vb.y, Va.y + Vb.x);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < VPT; ++s) {
      const int t = threadIdx.x + s * NT;
      if (t < P * n) buf[t] = z[s];
    }
    __syncthreads();
    FftGeom g{n, lgN, A.lgP, 1, true, 1, P, 1};
    fft_lds<T, Tile<T>::VPT, NT, MX>(buf, tw, g, true);
    for (int t = threadIdx.x; t < 2 * P * n; t += NT) {
      const int j = t >> (A.lgP + 1), ii = t & (2 * P - 1);
      const int i = i0 + ii;
      if (i < A.ni) D[(long)j * A.sa + i] = bufr[2 * (makhoul_pos(j, n) * P + (ii & (P - 1))) + (ii >> A.lgP)] * invn;
    }
  }
}


// ---------------------------------------------------------------------------
// Fused yz heat solve on x-major planes.  Values travel between the passes in
// registers; each pass scatters them into an element-major LDS layout with a
// padded pencil stride (es = pencils + 1) and two real pencils per complex one
// (pencil rho in slot rho mod H, real or imaginary part by rho / H, with H the
// number of complex pencils, ceil(real pencils / 2)).
constexpr int YZ_VPT = 8;

template <typename T, bool MX>
__global__ __launch_bounds__(YZ_NT) void k_yz_solve(const YZSolve<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NTH = YZ_NT;
  constexpr int NV = 2 * YZ_VPT;  // reals per thread
  const int ny = A.ny, nz = A.nz, lgNy = A.lgNy, lgNz = A.lgNz;
  const int M = ny * nz, lgM = lg_or_neg(M);
  const int PP = 1 << A.lgPP;
  const int R = M * PP;
  // y pass: real pencils rho = (p, z), NPy of them, paired rho <-> rho + Hy
  const int NPy = PP * nz, Hy = (NPy + 1) >> 1, esy = Hy + 1;
  const int lgHy = lg_or_neg(Hy);
  // z pass: real pencils rho' = (p, ky)
  const int NPz = PP * ny, Hz = (NPz + 1) >> 1, esz = Hz + 1;
  const int lgHz = lg_or_neg(Hz);
  // LDS: the y and z twiddles, the transpose buffer, then the DCT twiddles and eigenvalues
  cx<T>* Wy = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* Wz = Wy + ny;
  cx<T>* buf = Wz + nz;
  T* bufr = reinterpret_cast<T*>(buf);
  cx<T>* Dy = buf + max(ny * esy, nz * esz);
  cx<T>* Dz = Dy + ny;
  T* Ly = reinterpret_cast<T*>(Dz + nz);
  T* Lz = Ly + ny;
  T* Lx = Lz + nz;
  T* Sx = Lx + PP;  // the scale s of each plane
  // a batched plan: workgroup (xg, run b) holds planes x0 ... x0 + PP - 1 of run b,
  // which sit runs planes apart ([nx][runs][nz][ny]); its pairing of rows into
  // complex pencils is the single-run plan's
  const int runs = A.runs > 0 ? A.runs : 1;
  const int rb = blockIdx.x % runs;
  const int p0 = (blockIdx.x / runs) << A.lgPP;
  const int nplanes = min(PP, A.nx - p0);
  const long pstride = (long)runs * M;
  T* D = A.data[blockIdx.z] + ((long)p0 * runs + rb) * M;
  auto doff = [&](int e) { return (long)qdiv<MX>(e, M, lgM) * pstride + qmod<MX>(e, M, lgM); };
  // one round trip to memory: the planes, then the tables (each table loop loads
  // before it stores)
  T v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int e = threadIdx.x + i * NTH;
    v[i] = (e < R && e < nplanes * M) ? D[doff(e)] : (T)0;
  }
  {
    const int nt = max(max(ny, nz), PP);
    for (int i = threadIdx.x; i < nt; i += NTH) {
      const int iy = min(i, ny - 1), iz = min(i, nz - 1);
      const cx<T> wy = A.twy[iy * A.twy_s], wz = A.twz[iz * A.twz_s];
      const cx<T> dy = A.dtwy[iy], dz = A.dtwz[iz];
      const T ly = A.lamY[iy], lz = A.lamZ[iz];
      const T lx = A.lamX[min(p0 + min(i, PP - 1), A.nx - 1)];
      const T sp = (A.runp && A.rstageF) ? A.runp[(long)rb * RUNP + 7] : A.s;
      if (i < ny) {
        Wy[i] = wy;
        Dy[i] = dy;
        Ly[i] = ly;
      }
      if (i < nz) {
        Wz[i] = wz;
        Dz[i] = dz;
        Lz[i] = lz;
      }
      if (i < PP) {
        Lx[i] = p0 + i < A.nx ? lx : (T)0;
        Sx[i] = sp;
      }
    }
  }
  // pencils of a pass as (lgP, ncomp) of the FFT engine: a power-of-two count
  // pencil-fastest, any other as ncomp groups of one
  const int gyP = lgHy >= 0 ? lgHy : 0, gyC = lgHy >= 0 ? 1 : Hy;
  const int gzP = lgHz >= 0 ? lgHz : 0, gzC = lgHz >= 0 ? 1 : Hz;
  // current order of v[]: 0 plane order (e = tid + i NTH), 1 after the y pass, 2 after the z pass
  int order = 0;
  auto decode = [&](int i, int& p, int& z, int& y) -> bool {
    if (order == 1) {
      const int t = threadIdx.x + (i >> 1) * NTH, part = i & 1;
      if (t >= Hy * ny) return false;
      const int rho = qmod<MX>(t, Hy, lgHy) + part * Hy;
      if (rho >= NPy) return false;
      p = qdiv<MX>(rho, nz, lgNz);
      z = qmod<MX>(rho, nz, lgNz);
      y = qdiv<MX>(t, Hy, lgHy);
      return true;
    }
    if (order == 2) {
      const int t = threadIdx.x + i * NTH;
      if (t >= R) return false;
      const int rho = qdiv<MX>(t, nz, lgNz);
      p = qdiv<MX>(rho, ny, lgNy);
      y = qmod<MX>(rho, ny, lgNy);
      z = qmod<MX>(t, nz, lgNz);
      return true;
    }
    const int e = threadIdx.x + i * NTH;
    if (e >= R) return false;
    p = e / M;
    const int r = e - p * M;
    z = qdiv<MX>(r, ny, lgNy);
    y = qmod<MX>(r, ny, lgNy);
    return true;
  };
  __syncthreads();

  if (ny > 1) {
    if (NPy & 1)
      for (int t = threadIdx.x; t < ny * esy; t += NTH) buf[t] = zero<T>();
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int p, z, y;
      if (decode(i, p, z, y)) {
        const int rho = p * nz + z;
        bufr[2 * (makhoul_pos(y, ny) * esy + qmod<MX>(rho, Hy, lgHy)) + qdiv<MX>(rho, Hy, lgHy)] = v[i];
      }
    }
    __syncthreads();
    FftGeom g{ny, lgNy, gyP, gyC, true, 1, esy, 1};
    fft_lds<T, YZ_VPT, NTH, MX>(buf, Wy, g, false);
#pragma unroll
    for (int s2 = 0; s2 < YZ_VPT; ++s2) {
      const int t = threadIdx.x + s2 * NTH;
      v[2 * s2] = v[2 * s2 + 1] = (T)0;
      if (t < Hy * ny) {
        const int k = qdiv<MX>(t, Hy, lgHy), q = qmod<MX>(t, Hy, lgHy);
        const cx<T> Zk = buf[k * esy + q];
        const cx<T> Zm = buf[(k ? ny - k : 0) * esy + q];
        const cx<T> Va = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
        const cx<T> Vb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
        const cx<T> w = Dy[k];
        v[2 * s2] = w.x * Va.x - w.y * Va.y;
        v[2 * s2 + 1] = w.x * Vb.x - w.y * Vb.y;
      }
    }
    order = 1;
    __syncthreads();
  }

  if (nz > 1) {
    if (NPz & 1)
      for (int t = threadIdx.x; t < nz * esz; t += NTH) buf[t] = zero<T>();
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int p, z, y;
      if (decode(i, p, z, y)) {
        const int rho = p * ny + y;
        bufr[2 * (makhoul_pos(z, nz) * esz + qmod<MX>(rho, Hz, lgHz)) + qdiv<MX>(rho, Hz, lgHz)] = v[i];
      }
    }
    __syncthreads();
    FftGeom g{nz, lgNz, gzP, gzC, true, 1, esz, 1};
    fft_lds<T, YZ_VPT, NTH, MX>(buf, Wz, g, false);
    T xa[YZ_VPT], xb[YZ_VPT];
#pragma unroll
    for (int s2 = 0; s2 < YZ_VPT; ++s2) {
      const int t = threadIdx.x + s2 * NTH;
      xa[s2] = xb[s2] = (T)0;
      if (t < Hz * nz) {
        const int k = qdiv<MX>(t, Hz, lgHz), q = qmod<MX>(t, Hz, lgHz);
        const cx<T> Zk = buf[k * esz + q];
        const cx<T> Zm = buf[(k ? nz - k : 0) * esz + q];
        const cx<T> Va = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
        const cx<T> Vb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
        const cx<T> w = Dz[k];
        const int ra = q, rb = q + Hz;
        const int pa = qdiv<MX>(ra, ny, lgNy), pb = min(qdiv<MX>(rb, ny, lgNy), PP - 1);
        const T lx_a = Lx[pa], lx_b = Lx[pb];
        xa[s2] = (w.x * Va.x - w.y * Va.y) * heat_q(Sx[pa] * (lx_a + Ly[qmod<MX>(ra, ny, lgNy)] + Lz[k]));
        xb[s2] = (w.x * Vb.x - w.y * Vb.y) * heat_q(Sx[pb] * (lx_b + Ly[qmod<MX>(rb, ny, lgNy)] + Lz[k]));
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < YZ_VPT; ++s2) {
      const int t = threadIdx.x + s2 * NTH;
      if (t < Hz * nz) buf[qdiv<MX>(t, Hz, lgHz) * esz + qmod<MX>(t, Hz, lgHz)] = mk<T>(xa[s2], xb[s2]);
    }
    __syncthreads();
    cx<T> zz[YZ_VPT];
#pragma unroll
    for (int s2 = 0; s2 < YZ_VPT; ++s2) {
      const int t = threadIdx.x + s2 * NTH;
      zz[s2] = zero<T>();
      if (t < Hz * nz) {
        const int k = qdiv<MX>(t, Hz, lgHz), q = qmod<MX>(t, Hz, lgHz);
        const cx<T> Xk = buf[k * esz + q];
        const cx<T> Xm = k ? buf[(nz - k) * esz + q] : zero<T>();
        const cx<T> w = conjg(Dz[k]);
        const cx<T> Va = cmul(w, mk<T>(Xk.x, -Xm.x));
        const cx<T> Vb = cmul(w, mk<T>(Xk.y, -Xm.y));
        zz[s2] = mk<T>(Va.x - Vb.y, Va.y + Vb.x);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < YZ_VPT; ++s2) {
      const int t = threadIdx.x + s2 * NTH;
      if (t < Hz * nz) buf[qdiv<MX>(t, Hz, lgHz) * esz + qmod<MX>(t, Hz, lgHz)] = zz[s2];
    }
    __syncthreads();
    fft_lds<T, YZ_VPT, NTH, MX>(buf, Wz, g, true);
    const T invn = (T)1 / (T)nz;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int t = threadIdx.x + i * NTH;
      v[i] = (T)0;
      if (t < R) {
        const int rho = qdiv<MX>(t, nz, lgNz), z = qmod<MX>(t, nz, lgNz);
        const cx<T> c = buf[makhoul_pos(z, nz) * esz + qmod<MX>(rho, Hz, lgHz)];
        v[i] = (qdiv<MX>(rho, Hz, lgHz) ? c.y : c.x) * invn;
      }
    }
    order = 2;
    __syncthreads();
  } else {
    // no z axis: the diagonal acts on the y (or plane) coefficients directly
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int p, z, y;
      if (decode(i, p, z, y)) {
        v[i] *= heat_q(Sx[p] * (Lx[p] + Ly[y] + Lz[0]));
      }
    }
  }

  if (ny > 1) {
    if (NPy & 1)
      for (int t = threadIdx.x; t < ny * esy; t += NTH) buf[t] = zero<T>();
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int p, z, y;
      if (decode(i, p, z, y)) {
        const int rho = p * nz + z;
        bufr[2 * (y * esy + qmod<MX>(rho, Hy, lgHy)) + qdiv<MX>(rho, Hy, lgHy)] = v[i];
      }
    }
    __syncthreads();
    cx<T> zz[YZ_VPT];
#pragma unroll
    for (int s2 = 0; s2 < YZ_VPT; ++s2) {
      const int t = threadIdx.x + s2 * NTH;
      zz[s2] = zero<T>();
      if (t < Hy * ny) {
        const int k = qdiv<MX>(t, Hy, lgHy), q = qmod<MX>(t, Hy, lgHy);
        const cx<T> Xk = buf[k * esy + q];
        const cx<T> Xm = k ? buf[(ny - k) * esy + q] : zero<T>();
        const cx<T> w = conjg(Dy[k]);
        const cx<T> Va = cmul(w, mk<T>(Xk.x, -Xm.x));
        const cx<T> Vb = cmul(w, mk<T>(Xk.y, -Xm.y));
        zz[s2] = mk<T>(Va.x - Vb.y, Va.y + Vb.x);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < YZ_VPT; ++s2) {
      const int t = threadIdx.x + s2 * NTH;
      if (t < Hy * ny) buf[qdiv<MX>(t, Hy, lgHy) * esy + qmod<MX>(t, Hy, lgHy)] = zz[s2];
    }
    __syncthreads();
    FftGeom g{ny, lgNy, gyP, gyC, true, 1, esy, 1};
    fft_lds<T, YZ_VPT, NTH, MX>(buf, Wy, g, true);
    const T invn = (T)1 / (T)ny;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = threadIdx.x + i * NTH;
      v[i] = (T)0;
      if (e < R) {
        const int rho = qdiv<MX>(e, ny, lgNy), y = qmod<MX>(e, ny, lgNy);
        const cx<T> c = buf[makhoul_pos(y, ny) * esy + qmod<MX>(rho, Hy, lgHy)];
        v[i] = (qdiv<MX>(rho, Hy, lgHy) ? c.y : c.x) * invn;
      }
    }
    order = 0;
  }
  // plane order here (with ny == 1 the z-pass order coincides with it)
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int e = threadIdx.x + i * NTH;
    if (e < R && e < nplanes * M) D[doff(e)] = v[i];
  }
}

// ---------------------------------------------------------------------------
// Column complex FFT (forward with zero padding n_in -> L, or inverse with
// crop L -> n_out).  In place allowed (in == out, same strides).
template <typename T, bool MX>
__global__ __launch_bounds__(NT) void k_col_fft(const ColFft<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = A.L;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + L;
  const int P = 1 << A.lgP;
  const int i0 = blockIdx.x * P;
  const int b = blockIdx.y;
  const cx<T>* in = A.in[blockIdx.z] + (long)b * A.sb_in;
  cx<T>* out = A.out[blockIdx.z] + (long)b * A.sb_out;
  // the tile's loads first (at most VPT per thread), then the twiddles, then the LDS
  // stores: one round trip to memory
  constexpr int VPT = Tile<T>::VPT;
  cx<T> r[VPT];
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int t = threadIdx.x + u * NT;
    const int j = t >> A.lgP, q = t & (P - 1);
    const int i = i0 + q;
    r[u] = (t < P * L && j < A.n_in && i < A.ni) ? in[(long)j * A.sa_in + i] : zero<T>();
  }
  load_twiddles(tw, A.tw, L, A.twg);
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t < P * L) buf[t] = r[u];
  }
  __syncthreads();
  FftGeom g{L, A.lgL, A.lgP, 1, true, 1, P, 1};
  fft_lds<T, Tile<T>::VPT, NT, MX>(buf, tw, g, A.inv != 0);
  for (int t = threadIdx.x; t < P * A.n_out; t += NT) {
    const int j = t >> A.lgP, q = t & (P - 1);
    const int i = i0 + q;
    if (i < A.ni) out[(long)j * A.sa_out + i] = buf[t];
  }
}


// ---------------------------------------------------------------------------
// 512-point column FFT in registers: 512 = 8 x 8 x 8, 64 threads per pencil,
// 8 values per thread.  Forward: thread t holds n = t + 64 m; DFT-8 over m and
// W_512^{t k2}; transpose; thread (k2, t0) takes t = t0 + 8 t1, DFT-8 over t1
// and W_64^{t0 ka}; transpose; thread (k2, ka) finishes with a DFT-8 over t0
// and owns k = k2 + 8 ka + 64 kb.  The inverse runs the same digits backwards.
// LDS rows are padded (fft512_stride) against bank conflicts: with 64 four-byte
// banks, the 8 rows x P pencils that half a wave touches in a transpose fall in
// distinct banks when the row stride is P mod 32 complex (float) or P mod 16
// (double).
template <typename T, int P> constexpr int fft512_stride() { return 9 * P; }

template <typename T, int P, bool INV>
__global__ __launch_bounds__(64 * P) void k_fft512(const ColFft<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // row stride of the transposes: 8 mod 32 complex (float) or 4 mod 16 (double), so the
  // 8 rows x P columns a half-wave touches fall in distinct banks
  constexpr int S = fft512_stride<T, P>();
  // double precision takes its twiddles as powers of one or two table entries
  // (W^k by repeated products: k - 1 roundings of 2^-53), so that without the
  // 8 KiB table in LDS four workgroups fit a CU
  constexpr bool TWR = sizeof(T) == 8;
  cx<T>* w = reinterpret_cast<cx<T>*>(smem_raw);  // W_512^i (single precision)
  cx<T>* xb = TWR ? w : w + 512;                   // [64][S]
  const int tid = threadIdx.x;
  const int q = tid % P;
  const int t = tid / P;  // 0..63
  const Blk bk = xcd_block();
  const int kx = bk.x * P + q;
  const bool act = kx < A.ni;
  // A.pack: the x-level DC and Nyquist columns (both real) share the pencil of
  // tile 0, lane q = 0, as c0 + i cN, packed so in column 0 of the x-level side;
  // the y-level side holds them apart, C0 in column 0 and CN in column A.ni in
  // the blocked layout.  The forward output splits by Hermitian symmetry; the
  // inverse packs C0 + i CN on input and returns c0 + i cN.  So ni / 8
  // workgroups cover ni + 1 columns: 1024 instead of 1056 for 257 columns, one
  // round at four per CU (two rounds of 1024 instead of three in double
  // precision, with P = 4).
  const bool pk = A.pack && bk.x == 0;
  const bool pkl = pk && q == 0;
  const int b = bk.y;
  // byte offsets from the uniform pencil-set bases (inactive lanes read kx = ni - 1)
  const cx<T>* in = A.in[bk.z];
  cx<T>* out = A.out[bk.z];
  constexpr unsigned CB = sizeof(cx<T>);
  const unsigned ioff = (unsigned)(b * A.sb_in + min(kx, A.ni - 1)) * CB, isa = (unsigned)A.sa_in * CB;
  const unsigned ooff = (unsigned)(b * A.sb_out + kx) * CB, osa = (unsigned)A.sa_out * CB;
  // the y-level Nyquist column (blocked layout: row r at (r & ~15, ni + (r & 15))),
  // staged through LDS for or from the packed lane, 512 / (64 P) entries per
  // thread.  With 8 padding entries per transpose row (single precision), entry
  // i sits in the padding of row i % 64 (columns 8 P + i / 64, which no
  // transpose touches), so no barrier separates it from the transposes;
  // otherwise it sits in the transpose buffer, behind a barrier each way.
  const unsigned nbase_in = (unsigned)(b * A.sb_in + A.ni) * CB, nbase_out = (unsigned)(b * A.sb_out + A.ni) * CB;
  auto noff_in = [&](int r) { return nbase_in + (unsigned)(r & ~15) * isa + (unsigned)(r & 15) * CB; };
  auto noff_out = [&](int r) { return nbase_out + (unsigned)(r & ~15) * osa + (unsigned)(r & 15) * CB; };
  constexpr bool PADST = S - 8 * P >= 8;
  constexpr int NPT = 512 / (64 * P);
  static_assert(NPT == 1 || NPT == 2, "one or two staged entries per thread");
  auto xn = [&](int i) -> cx<T>& { return PADST ? xb[(i & 63) * S + 8 * P + (i >> 6)] : xb[i]; };
  constexpr bool inv = INV;
  auto W = [&](int e) {  // W_512^{e} (conjugated for the inverse), from the LDS table
    cx<T> v = w[e & 511];
    if (inv) v.y = -v.y;
    return v;
  };
  auto G = [&](int e) {  // the same from the global table
    cx<T> v = A.tw[(e & 511) << (A.lgTw - 9)];
    if (inv) v.y = -v.y;
    return v;
  };
  // v[j] *= a b^j for j = j0..7 (b^j by repeated products)
  auto tw_pow = [](cx<T>(&v)[8], cx<T> a, cx<T> b, int j0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= j0) v[j] = cmul(v[j], a);
      a = cmul(a, b);
    }
  };
  // the pencil first, then the W table: one round trip to memory
  cx<T> v[8];
  if (!inv) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int row = t + 64 * m;
      v[m] = row < A.n_in ? ld_off(in, ioff + (unsigned)row * isa) : zero<T>();
    }
  } else {
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      const int k = (t >> 3) + 8 * (t & 7) + 64 * kb;
      v[kb] = k < A.n_in ? ld_off(in, ioff + (unsigned)k * isa) : zero<T>();
    }
  }
  // twiddle bases of this thread (double precision): forward W^t and W^(8 (t & 7)),
  // inverse W^(8 (t & 7)), W^((t & 7) (t >> 3)) and W^(8 (t >> 3))
  cx<T> tb0{}, tb1{}, tb2{};
  if constexpr (TWR) {
    tb0 = inv ? G(8 * (t & 7)) : G(t);
    tb1 = inv ? G((t & 7) * (t >> 3)) : G(8 * (t & 7));
    if (inv) tb2 = G(8 * (t >> 3));
  }
  if constexpr (INV) {
    // the staging loads are unconditional: other workgroups re-read their own
    // first element (a valid address, the value unused), since a branch around
    // a load makes the compiler wait for it there.  Rows past n_in are masked
    // where the packed lane reads them.
    const int r1 = tid + 64 * P;
    const cx<T> nq0 = ld_off(in, pk ? noff_in(min(tid, A.n_in - 1)) : ioff);
    const cx<T> nq1 = NPT == 2 ? ld_off(in, pk ? noff_in(min(r1, A.n_in - 1)) : ioff) : zero<T>();
    cx<T> wv{};
    if constexpr (!TWR) wv = A.tw[tid << (A.lgTw - 9)];
    // every load above is issued before the first LDS store waits for one
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (!TWR) {
      static_assert(TWR || 64 * P == 512, "one table entry per thread");
      w[tid] = wv;
    }
    if (pk) {
      xn(tid) = nq0;
      if (NPT == 2) xn(r1) = nq1;
    }
  } else if constexpr (!TWR) {
    for (int i = tid; i < 512; i += 64 * P) w[i] = A.tw[i << (A.lgTw - 9)];
  }
  __syncthreads();
  if (INV && pkl) {
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      const int k = (t >> 3) + 8 * (t & 7) + 64 * kb;
      const cx<T> cn = k < A.n_in ? xn(k) : zero<T>();
      v[kb] = mk<T>(v[kb].x - cn.y, v[kb].y + cn.x);
    }
  }
  if (INV && !PADST && pk) __syncthreads();  // the first transpose overwrites the staging
  if (!inv) {
    if (A.n_in <= 256) dft8_lo4(v, false);  // zero-padded half: rows t + 64 m, m >= 4
    else dft8(v, false);
    const int t0 = t & 7, t1 = t >> 3;
    if constexpr (TWR) tw_pow(v, mk<T>((T)1, (T)0), tb0, 1);
    else {
#pragma unroll
      for (int k2 = 1; k2 < 8; ++k2) v[k2] = cmul(v[k2], W(t * k2));
    }
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) xb[(k2 * 8 + t0) * S + t1 * P + q] = v[k2];
    __syncthreads();
    {
      const int k2 = t >> 3, u0 = t & 7;
#pragma unroll
      for (int u1 = 0; u1 < 8; ++u1) v[u1] = xb[(k2 * 8 + u0) * S + u1 * P + q];
      dft8(v, false);
      if constexpr (TWR) tw_pow(v, mk<T>((T)1, (T)0), tb1, 1);
      else {
#pragma unroll
        for (int ka = 1; ka < 8; ++ka) v[ka] = cmul(v[ka], W(8 * u0 * ka));
      }
      __syncthreads();
#pragma unroll
      for (int ka = 0; ka < 8; ++ka) xb[(k2 * 8 + ka) * S + u0 * P + q] = v[ka];
    }
    __syncthreads();
    {
      const int k2 = t >> 3, ka = t & 7;
#pragma unroll
      for (int u0 = 0; u0 < 8; ++u0) v[u0] = xb[(k2 * 8 + ka) * S + u0 * P + q];
      dft8(v, false);
      const int s0 = k2 + 8 * ka, s1 = (64 - s0) & 63;
      cx<T> cn[8];  // the packed lane's FFT(cN)
      if (pkl) {
        // Z = FFT(c0 + i cN): FFT(c0)[k] = (Z[k] + conj Z[-k]) / 2 and
        // FFT(cN)[k] = (Z[k] - conj Z[-k]) / 2i.  With s = k2 + 8 ka, Z[-k] is
        // output 7 - kb of the thread with s' = 64 - s (output (8 - kb) % 8 of this
        // thread for s = 0); this lane repeats that thread's last DFT from the
        // same LDS rows instead of waiting for it at a barrier.  FFT(c0) leaves
        // with the other lanes' outputs, FFT(cN) through LDS.
        cx<T> u[8];
#pragma unroll
        for (int u0 = 0; u0 < 8; ++u0) u[u0] = xb[((s1 & 7) * 8 + (s1 >> 3)) * S + u0 * P + q];
        dft8(u, false);
        cx<T> c0[8];
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
          const cx<T> Z = v[kb], Zm = s0 ? u[7 - kb] : v[(8 - kb) & 7];
          cn[kb] = mk<T>((Z.y + Zm.y) * (T)0.5, (Zm.x - Z.x) * (T)0.5);
          c0[kb] = mk<T>((Z.x + Zm.x) * (T)0.5, (Z.y - Zm.y) * (T)0.5);
          if (PADST) xn(s0 + 64 * kb) = cn[kb];
        }
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) v[kb] = c0[kb];
      }
      if (act) {
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
          const int k = k2 + 8 * ka + 64 * kb;
          if (k < A.n_out) st_off(out, ooff + (unsigned)k * osa, v[kb]);
        }
      }
      if (pk) {
        // the Nyquist column, one row per thread: whole lines of the blocked
        // layout instead of scattered 8-byte stores
        if constexpr (!PADST) {
          __syncthreads();  // every thread has read the transpose buffer
          if (pkl) {
#pragma unroll
            for (int kb = 0; kb < 8; ++kb) xn(s0 + 64 * kb) = cn[kb];
          }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NPT; ++j)
          if (tid + j * 64 * P < A.n_out) st_off(out, noff_out(tid + j * 64 * P), xn(tid + j * 64 * P));
      }
    }
  } else {
    const int k2 = t >> 3, ka = t & 7;
    dft8(v, true);  // index t0
    if constexpr (TWR) tw_pow(v, mk<T>((T)1, (T)0), tb0, 1);
    else {
#pragma unroll
      for (int t0 = 1; t0 < 8; ++t0) v[t0] = cmul(v[t0], W(8 * t0 * ka));
    }
#pragma unroll
    for (int t0 = 0; t0 < 8; ++t0) xb[(k2 * 8 + t0) * S + ka * P + q] = v[t0];
    __syncthreads();
    {
      const int kk2 = t >> 3, t0 = t & 7;
#pragma unroll
      for (int a = 0; a < 8; ++a) v[a] = xb[(kk2 * 8 + t0) * S + a * P + q];
      dft8(v, true);  // index t1
      if constexpr (TWR) tw_pow(v, tb1, tb2, 0);
      else {
#pragma unroll
        for (int t1 = 0; t1 < 8; ++t1) v[t1] = cmul(v[t1], W((t0 + 8 * t1) * kk2));
      }
      __syncthreads();
#pragma unroll
      for (int t1 = 0; t1 < 8; ++t1) xb[(t0 + 8 * t1) * S + kk2 * P + q] = v[t1];
    }
    __syncthreads();
#pragma unroll
    for (int kk2 = 0; kk2 < 8; ++kk2) v[kk2] = xb[t * S + kk2 * P + q];
    // index m: x[t + 64 m]; a cropped output keeps m < 4
    if (A.n_out <= 256) dft8_first4(v, true);
    else dft8(v, true);
    if (act) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int row = t + 64 * m;
        if (row < A.n_out) st_off(out, ooff + (unsigned)row * osa, v[m]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Last-axis stray-field convolution.  LDS layout buf[j * 3P + c * P + q].
__device__ __forceinline__ int comp_index(int a, int b) {
  // xx yy zz xy xz yz
  if (a == b) return a;
  const int s = a + b;  // 1: xy, 2: xz, 3: yz
  return 2 + s;
}

// One workgroup: P consecutive kx, the full padded pencil along the last axis,
// and the pair of batch rows b and Pb - b that share one folded tensor row (the
// tensor tile is read once into LDS and used for both).  LDS layout of the
// spectra: buf[j * 3P + c * P + q].
constexpr int CONV_NT = 512;
constexpr int CONV_VPT = 8;

template <typename T, bool MX>
__global__ __launch_bounds__(CONV_NT) void k_conv(const Conv<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = A.L;
  const int LH = (L >> 1) + 1;
  const int P = 1 << A.lgP;
  const int es = 3 * P;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + L;
  T* tt = reinterpret_cast<T*>(buf + 3 * P * L);  // [ncomp][LH][P]
  load_twiddles<T, CONV_NT>(tw, A.tw, L, A.twg);
  const int i0 = blockIdx.x * P;
  const int bf = blockIdx.y;
  // folded tensor tile: per chunk of the [LH][P] tile, every used component's entry
  // loaded before any is stored (one round trip per chunk, component lists read as
  // uniform values)
  for (int t0 = 0; t0 < LH * P; t0 += CONV_NT) {
    const int t = t0 + threadIdx.x;
    const int tc = min(t, LH * P - 1);
    const int q = tc % P, kf = tc / P;
    const int kx = min(i0 + q, A.ni - 1);
    T tv[6];
#pragma unroll
    for (int ci = 0; ci < 6; ++ci)
      tv[ci] = ci < A.nt ? A.tens[(long)A.clist[ci] * A.tcs + ((long)kf * A.Hb + bf) * A.tkx + kx] : (T)0;
    if (t < LH * P) {
#pragma unroll
      for (int ci = 0; ci < 6; ++ci)
        if (ci < A.nt) tt[ci * LH * P + t] = (i0 + q < A.ni) ? tv[ci] : (T)0;
    }
  }
  const bool mirror = A.Pb > 1 && bf != 0 && 2 * bf != A.Pb;
  const int ch = L >> 1;
  for (int pass = 0; pass < (mirror ? 2 : 1); ++pass) {
    const int b = pass ? A.Pb - bf : bf;
    const bool bneg = pass == 1;
    const long boff = (long)b * A.sb;
    __syncthreads();
    // the three components' loads first, then the LDS stores.  The kx tile keeps
    // 3 P L <= CONV_VPT CONV_NT and P L <= 2 CONV_NT: two loads per component and thread
    cx<T> r[3][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<T>* S = A.S[c] ? A.S[c] + (long)blockIdx.z * A.rs_in : nullptr;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = threadIdx.x + u * CONV_NT;
        const int j = t >> A.lgP, q = t & (P - 1);
        const int i = i0 + q;
        r[c][u] = (S && t < P * L && j < A.n && i < A.ni) ? S[boff + (long)j * A.sa + i] : zero<T>();
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = threadIdx.x + u * CONV_NT;
        if (t < P * L) buf[(t >> A.lgP) * es + c * P + (t & (P - 1))] = r[c][u];
      }
    __syncthreads();
    {
      FftGeom g{L, A.lgL, A.lgP, 3, true, 1, es, 1};
      fft_lds<T, CONV_VPT, CONV_NT, MX>(buf, tw, g, false);
    }
    for (int t = threadIdx.x; t < P * L; t += CONV_NT) {
      const int j = t >> A.lgP, q = t & (P - 1);
      if (i0 + q >= A.ni) continue;
      const bool cneg = j > ch;
      const int kf = cneg ? L - j : j;
      const cx<T> s0 = buf[j * es + q], s1 = buf[j * es + P + q], s2 = buf[j * es + 2 * P + q];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (!A.O[a]) continue;
        T tv[3];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          // an absent input component: its tensor components are not loaded
          const int c = comp_index(a, bb);
          T v = A.S[bb] ? tt[(A.cpos[c] * LH + kf) * P + q] : (T)0;
          if (cneg && ((A.oddc >> c) & 1)) v = -v;
          if (bneg && ((A.oddb >> c) & 1)) v = -v;
          tv[bb] = v;
        }
        buf[j * es + a * P + q] =
            mk<T>(tv[0] * s0.x + tv[1] * s1.x + tv[2] * s2.x, tv[0] * s0.y + tv[1] * s1.y + tv[2] * s2.y);
      }
    }
    __syncthreads();
    if (A.O[0] && A.O[1] && A.O[2]) {
      FftGeom g{L, A.lgL, A.lgP, 3, true, 1, es, 1};
      fft_lds<T, CONV_VPT, CONV_NT, MX>(buf, tw, g, true);
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (A.O[a]) {
          FftGeom g{L, A.lgL, A.lgP, 1, true, 1, es, 1};
          fft_lds<T, CONV_VPT, CONV_NT, MX>(buf + a * P, tw, g, true);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<T>* O = A.O[a];
      if (!O) continue;
      O += boff + (long)blockIdx.z * A.rs_out;
      for (int t = threadIdx.x; t < P * A.n; t += CONV_NT) {
        const int j = t >> A.lgP, q = t & (P - 1);
        const int i = i0 + q;
        if (i < A.ni) O[(long)j * A.sa + i] = buf[j * es + a * P + q];
      }
    }
  }
}


// Convolution for a 64-point padded pencil (last axis of extent 32): four-step
// FFT 64 = 8 x 8 in registers.  Eight threads share a pencil, thread t holding
// elements n = t + 8 m; after a register DFT-8 over m and the twiddles
// W_64^{t k2} one LDS transpose lets thread k2 finish with a DFT-8 over t, so
// thread k2 ends with the frequencies k2 + 8 k1.  The tensor multiply needs no
// exchange (all three components of a frequency sit in one thread); the inverse
// mirrors the forward and leaves thread b with z = 8 a + b.  A workgroup covers
// P consecutive kx and the batch rows b and Pb - b that share a tensor row.
constexpr int C64_NT = 256;
// log2 of the kx per workgroup: 16 in single precision, 8 in double (16 KiB of
// transpose buffer either way); a compile-time constant, so that every LDS
// offset of the transposes and the tile is an immediate
template <typename T> constexpr int c64_lgP() { return sizeof(T) == 4 ? 4 : 3; }
// tensor tile entries per thread and component: 33 rows x P kx over 16 P threads
constexpr int C64_TILE_PT = (33 + 15) / 16;

template <typename T>
__device__ __forceinline__ void tw64_apply(cx<T>* v, const cx<T>* w64, int t, bool inv) {
#pragma unroll
  for (int k = 1; k < 8; ++k) {
    cx<T> w = w64[(t * k) & 63];
    if (inv) w.y = -w.y;
    v[k] = cmul(v[k], w);
  }
}

// LDS index of pencil pen in transpose row (a, b) of channel c (rows of NP
// pencils): on odd a + b the two halves of the row swap, so that the two t
// values of a half-wave fall in distinct banks both when t is the column index
// (writes) and when it is the row index (reads)
__device__ __forceinline__ int c64_idx(int c, int a, int b, int NP, int pen) {
  return ((c * 8 + a) * 8 + b) * NP + (pen ^ (((a + b) & 1) * (NP >> 1)));
}

template <typename T>
__global__ __launch_bounds__(C64_NT, sizeof(T) == 4 ? 5 : 1) void k_conv64(const Conv<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int LGP = c64_lgP<T>(), P = 1 << LGP;
  constexpr int NP = 2 * P;  // pencils per workgroup (two batch rows)
  cx<T>* w64 = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* xb = w64 + 64;                          // [8][8][NP]: one transpose at a time
  T* tt = reinterpret_cast<T*>(xb + 64 * NP);    // tensor tile [nt][33 folded kz][P kx]
  const int tid = threadIdx.x;
  const int q = tid & (P - 1);
  const int t = (tid >> LGP) & 7;
  const int r = tid >> (LGP + 3);
  const Blk bk = xcd_block();
  const int bf = bk.y;
  const int kx0 = bk.x * P;
  const bool mirror = A.Pb > 1 && bf != 0 && 2 * bf != A.Pb;
  const int kx = kx0 + q;
  const bool act = kx < A.ni && (r == 0 || mirror);
  // inactive lanes read valid addresses and are never stored
  const int kxc = min(kx, A.ni - 1);
  const int b = (r && mirror) ? A.Pb - bf : bf;
  // byte offsets from uniform base pointers (scalar base + 32-bit vector offset);
  // the Nyquist column may be in the blocked layout over the batch rows
  const unsigned soff =
      (unsigned)(A.nyqb && kxc == A.ni - 1 ? nyq_off(b, A.sb, kxc, true) : (long)b * A.sb + kxc) *
      (unsigned)sizeof(cx<T>);
  const unsigned sa = (unsigned)A.sa * (unsigned)sizeof(cx<T>);
  const int pen = r * P + q;

  // forward: load z = t + 8 m (m < 4; the padded half is zero), DFT-8 over m,
  // twiddle, transpose, DFT-8 over t
  cx<T> v[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T>* S = A.S[c] ? A.S[c] + (long)bk.z * A.rs_in : nullptr;
#pragma unroll
    for (int m = 0; m < 4; ++m) v[c][m] = S ? ld_off(S, soff + (unsigned)(t + 8 * m) * sa) : zero<T>();
  }
  // the tensor tile of this workgroup (the used components, the 33 folded kz rows
  // of batch row bf, its P kx) and the W table into LDS, loaded with the pencils:
  // one round trip to memory, and no tensor load in the output loop
  {
    const int nth = 16 * P, ncp = 33 * P;  // entries per component: 33 rows x P kx
    // 32-bit byte offsets from the uniform tensor base
    const unsigned rowb = (unsigned)(bf * A.tkx) * (unsigned)sizeof(T), kzb = (unsigned)(A.Hb * A.tkx) * (unsigned)sizeof(T);
    T tv[6][C64_TILE_PT];
#pragma unroll
    for (int cp = 0; cp < 6; ++cp) {
      if (cp >= A.nt) break;
      const unsigned cb = (unsigned)A.clist[cp] * (unsigned)A.tcs * (unsigned)sizeof(T) + rowb;
#pragma unroll
      for (int j = 0; j < C64_TILE_PT; ++j) {
        const int i = min(tid + j * nth, ncp - 1);
        const unsigned off = cb + (unsigned)(i >> LGP) * kzb + (unsigned)min(kx0 + (i & (P - 1)), A.ni - 1) * (unsigned)sizeof(T);
        tv[cp][j] = ld_off(A.tens, off);
      }
    }
    const cx<T> wv = A.tw[min(tid, 63) << (A.lgTw - 6)];
    // every load above is issued before the first LDS store waits for one
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int cp = 0; cp < 6; ++cp) {
      if (cp >= A.nt) break;
#pragma unroll
      for (int j = 0; j < C64_TILE_PT; ++j)
        if (tid + j * nth < ncp) tt[cp * ncp + tid + j * nth] = tv[cp][j];
    }
    if (tid < 64) w64[tid] = wv;
  }
  __syncthreads();  // w64 and the tile are in LDS
  // this thread's twiddles W_64^{t k}, k < 8 (conjugated for the inverse), read
  // from LDS at each use: held in registers they would cost a wave per SIMD
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    dft8_lo4(v[c], false);
    tw64_apply(v[c], w64, t, false);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) xb[c64_idx(0, k2, t, NP, pen)] = v[c][k2];
    __syncthreads();
#pragma unroll
    for (int tt2 = 0; tt2 < 8; ++tt2) v[c][tt2] = xb[c64_idx(0, t, tt2, NP, pen)];
    __syncthreads();
    dft8(v[c], false);  // v[c][k1] = X[t + 8 k1]
  }

  // folded tensor rows, shared by every component and output: kz = t + 8 k1 reads
  // row kz up to 32, above that row 64 - kz of a z-odd component negated (with
  // t < 8 that is k1 > 4, and k1 = 4 for t > 0)
  auto kzf = [&](int k1) { return k1 < 4 ? t + 8 * k1 : (k1 > 4 ? 64 - t - 8 * k1 : (t ? 32 - t : 32)); };
  auto zsg = [&](int k1) -> T { return k1 < 4 ? (T)1 : (k1 > 4 ? (T)-1 : (t ? (T)-1 : (T)1)); };
  const bool bneg = r == 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!A.O[a]) continue;
    cx<T> o[8];
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) o[k1] = zero<T>();
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      // an absent input component: its tensor components are not loaded
      if (!A.S[bb]) continue;
      const int c = comp_index(a, bb);
      const T* tc = tt + A.cpos[c] * 33 * P + q;
      const bool zodd = (A.oddc >> c) & 1;
      const T ys = (bneg && ((A.oddb >> c) & 1)) ? (T)-1 : (T)1;
#pragma unroll
      for (int k1 = 0; k1 < 8; ++k1) {
        T w = tc[kzf(k1) * P] * ys;
        if (zodd) w *= zsg(k1);
        o[k1] = mk<T>(o[k1].x + w * v[bb][k1].x, o[k1].y + w * v[bb][k1].y);
      }
    }
    dft8(o, true);
    tw64_apply(o, w64, t, true);
#pragma unroll
    for (int bb = 0; bb < 8; ++bb) xb[c64_idx(0, bb, t, NP, pen)] = o[bb];
    __syncthreads();
    cx<T>* O = A.O[a] + (long)bk.z * A.rs_out;
    cx<T> u[8];
#pragma unroll
    for (int tt2 = 0; tt2 < 8; ++tt2) u[tt2] = xb[c64_idx(0, t, tt2, NP, pen)];
    __syncthreads();
    dft8_first4(u, true);  // u[a'] = x[8 a' + t], a' < 4: z < 32
    if (act) {
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) st_off(O, soff + (unsigned)(8 * aa + t) * sa, u[aa]);
    }
  }
}

// ---------------------------------------------------------------------------
// Newell cell-averaged demagnetising tensor (FP64), point-dipole beyond rfar.
__device__ __forceinline__ double asinh_ratio(double a, double b) { return b != 0.0 ? asinh(a / b) : 0.0; }
__device__ __forceinline__ double atan_ratio(double a, double b) { return b != 0.0 ? atan(a / b) : 0.0; }

__device__ double newell_f(double x, double y, double z) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double t = (2.0 * x2 - y2 - z2) * R / 6.0;
  t += 0.5 * y * (z2 - x2) * asinh_ratio(y, sqrt(x2 + z2));
  t += 0.5 * z * (y2 - x2) * asinh_ratio(z, sqrt(x2 + y2));
  t -= x * y * z * atan_ratio(y * z, x * R);
  return t;
}

__device__ double newell_g(double x, double y, double z) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double t = -x * y * R / 3.0;
  t += x * y * z * asinh_ratio(z, sqrt(x2 + y2));
  t += y / 6.0 * (3.0 * z2 - y2) * asinh_ratio(x, sqrt(y2 + z2));
  t += x / 6.0 * (3.0 * z2 - x2) * asinh_ratio(y, sqrt(x2 + z2));
  t -= z2 * z / 6.0 * atan_ratio(x * y, z * R);
  t -= z * y2 / 2.0 * atan_ratio(x * z, y * R);
  t -= z * x2 / 2.0 * atan_ratio(y * z, x * R);
  return t;
}

template <int G>
__device__ double newell_sum(double X, double Y, double Z, double a, double b, double c) {
  const double w[3] = {-1.0, 2.0, -1.0};
  double acc = 0.0;
  for (int i = -1; i <= 1; ++i)
    for (int j = -1; j <= 1; ++j)
      for (int k = -1; k <= 1; ++k) {
        const double f = G ? newell_g(X + i * a, Y + j * b, Z + k * c) : newell_f(X + i * a, Y + j * b, Z + k * c);
        acc += w[i + 1] * w[j + 1] * w[k + 1] * f;
      }
  return acc / (4.0 * M_PI * a * b * c);
}

__global__ void k_newell_fill(double* out, int comp, int nx, int ny, int nz, int Px, int Py, int Pz, double hx,
                              double hy, double hz, int rfar) {
  const long total = (long)Px * Py * Pz;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int kx = (int)(t % Px);
    const int ky = (int)((t / Px) % Py);
    const int kz = (int)(t / ((long)Px * Py));
    const int ix = kx < nx ? kx : kx - Px;
    const int iy = ky < ny ? ky : ky - Py;
    const int iz = kz < nz ? kz : kz - Pz;
    double v = 0.0;
    if (abs(ix) <= nx - 1 && abs(iy) <= ny - 1 && abs(iz) <= nz - 1) {
      const double X = ix * hx, Y = iy * hy, Z = iz * hz;
      const int mx = max(abs(ix), max(abs(iy), abs(iz)));
      if (mx > rfar) {
        const double r2 = X * X + Y * Y + Z * Z;
        const double s = hx * hy * hz / (4.0 * M_PI) / (r2 * r2 * sqrt(r2));
        switch (comp) {
          case 0: v = s * (r2 - 3.0 * X * X); break;
          case 1: v = s * (r2 - 3.0 * Y * Y); break;
          case 2: v = s * (r2 - 3.0 * Z * Z); break;
          case 3: v = s * (-3.0 * X * Y); break;
          case 4: v = s * (-3.0 * X * Z); break;
          default: v = s * (-3.0 * Y * Z); break;
        }
      } else {
        switch (comp) {
          case 0: v = newell_sum<0>(X, Y, Z, hx, hy, hz); break;
          case 1: v = newell_sum<0>(Y, X, Z, hy, hx, hz); break;
          case 2: v = newell_sum<0>(Z, Y, X, hz, hy, hx); break;
          case 3: v = newell_sum<1>(X, Y, Z, hx, hy, hz); break;
          case 4: v = newell_sum<1>(X, Z, Y, hx, hz, hy); break;
          default: v = newell_sum<1>(Y, Z, X, hy, hz, hx); break;
        }
      }
    }
    out[t] = v;
  }
}

template <typename T>
__global__ void k_tensor_pack(const cx<double>* spec, T* out, int Hz, int Hy, int Kx, int Kxp, int Kt, int Py,
                              double scale) {
  const long total = (long)Hz * Hy * Kt;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int kx = (int)(t % Kt);
    const int ky = (int)((t / Kt) % Hy);
    const int kz = (int)(t / ((long)Kt * Hy));
    out[t] = kx < Kx ? (T)(spec[((long)kz * Py + ky) * Kxp + kx].x * scale) : (T)0;
  }
}

// ---------------------------------------------------------------------------
// Pointwise: effective field h = eps Lap_h m - Q (m2 e2 + m3 e3) + hs + he.
template <typename T>
__global__ void k_field_assemble(const T* m, const T* hs, T* out, int nx, int ny, int nz, double cxx, double cyy,
                                 double czz, double eps_on, double Q, double he0, double he1, double he2) {
  const long N = (long)nx * ny * nz;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < N; idx += (long)gridDim.x * blockDim.x) {
    const int x = (int)(idx % nx);
    const int y = (int)((idx / nx) % ny);
    const int z = (int)(idx / ((long)nx * ny));
    const double he[3] = {he0, he1, he2};
    for (int c = 0; c < 3; ++c) {
      const T* mc = m + c * N;
      const double v = mc[idx];
      double lap = 0.0;
      if (nx > 1) lap += cxx * ((double)mc[x > 0 ? idx - 1 : idx] + (double)mc[x < nx - 1 ? idx + 1 : idx] - 2.0 * v);
      if (ny > 1) lap += cyy * ((double)mc[y > 0 ? idx - nx : idx] + (double)mc[y < ny - 1 ? idx + nx : idx] - 2.0 * v);
      if (nz > 1)
        lap += czz * ((double)mc[z > 0 ? idx - (long)nx * ny : idx] + (double)mc[z < nz - 1 ? idx + (long)nx * ny : idx] -
                      2.0 * v);
      double h = eps_on * lap + he[c];
      if (c > 0) h -= Q * v;
      if (hs) h += (double)hs[c * N + idx];
      out[c * N + idx] = (T)h;
    }
  }
}

// ---------------------------------------------------------------------------
// Energies: per-cell FP64 densities, fixed-order block partials, fixed final sum.
// acc[0] = sum over faces |dm|^2 / h^2 (times per-axis weights cxx, cyy, czz)
// acc[1] = sum m2^2 + m3^2, acc[2] = sum m . hs, acc[3] = sum m . he
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_energy(const T* m, const T* hs, int nx, int ny, int nz, double cxx, double cyy,
                                               double czz, double he0, double he1, double he2, double* partials) {
  const long N = (long)nx * ny * nz;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long idx = blockIdx.x * (long)NT + threadIdx.x; idx < N; idx += (long)gridDim.x * NT) {
    const int x = (int)(idx % nx);
    const int y = (int)((idx / nx) % ny);
    const int z = (int)(idx / ((long)nx * ny));
    const double m0 = m[idx], m1 = m[N + idx], m2 = m[2 * N + idx];
    double ex = 0.0;
    if (x < nx - 1) {
      const double d0 = m[idx + 1] - m0, d1 = m[N + idx + 1] - m1, d2 = m[2 * N + idx + 1] - m2;
      ex += cxx * (d0 * d0 + d1 * d1 + d2 * d2);
    }
    if (y < ny - 1) {
      const long o = idx + nx;
      const double d0 = m[o] - m0, d1 = m[N + o] - m1, d2 = m[2 * N + o] - m2;
      ex += cyy * (d0 * d0 + d1 * d1 + d2 * d2);
    }
    if (z < nz - 1) {
      const long o = idx + (long)nx * ny;
      const double d0 = m[o] - m0, d1 = m[N + o] - m1, d2 = m[2 * N + o] - m2;
      ex += czz * (d0 * d0 + d1 * d1 + d2 * d2);
    }
    acc[0] += ex;
    acc[1] += m1 * m1 + m2 * m2;
    if (hs) acc[2] += m0 * (double)hs[idx] + m1 * (double)hs[N + idx] + m2 * (double)hs[2 * N + idx];
    acc[3] += m0 * he0 + m1 * he1 + m2 * he2;
  }
  static __shared__ double red[4][NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[k][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[threadIdx.x][w];
    partials[(long)blockIdx.x * 4 + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(NT) void k_energy_final(const double* partials, int nblocks, double* out) {
  static __shared__ double red[4][NT];
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) s += partials[(long)b * 4 + k];
    red[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Spectral radius of the sweep matrices (paper §4, eqs. GS-matrix and SGS-matrix):
// per cell the coefficients c = eps dt Lap_h g of the step's six precession
// solves (7-point stencil, mirror ghosts), the 3x3 iteration matrices
// G_GS = (D - L)^{-1} U and G_SGS = (D - U)^{-1} L G_GS, whose first columns
// vanish, so that rho is the larger modulus of the eigenvalues of the trailing
// 2x2 block; block maxima into partials[4 b], partials[4 b + 1].
__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

__device__ __forceinline__ double rho2(double p, double q, double r, double s) {
  const double tr = p + s, det = p * s - q * r, disc = tr * tr - 4.0 * det;
  return disc >= 0.0 ? 0.5 * (fabs(tr) + sqrt(disc)) : sqrt(det);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_rho(const T* g2n, const T* g3n, const T* g1s, const T* g2s, const T* g3ss,
                                            const T* g2ss, int nx, int ny, int nz, double kx, double ky, double kz,
                                            int sgs, double* partials) {
  const int N = nx * ny * nz, nxy = nx * ny;
  double rg = 0.0, rs = 0.0;
  for (int idx = blockIdx.x * NT + threadIdx.x; idx < N; idx += gridDim.x * NT) {
    const int x = idx % nx, y = (idx / nx) % ny, z = idx / nxy;
    const int xm = x > 0 ? idx - 1 : idx, xp = x < nx - 1 ? idx + 1 : idx;
    const int ym = y > 0 ? idx - nx : idx, yp = y < ny - 1 ? idx + nx : idx;
    const int zm = z > 0 ? idx - nxy : idx, zp = z < nz - 1 ? idx + nxy : idx;
    auto lap = [&](const T* g) {
      const double c = g[idx];
      return kx * ((double)g[xm] + (double)g[xp] - 2.0 * c) + ky * ((double)g[ym] + (double)g[yp] - 2.0 * c) +
             kz * ((double)g[zm] + (double)g[zp] - 2.0 * c);
    };
    const double a = lap(g3n), b = lap(g2n), c = lap(g1s), d = lap(g2s);
    // G_GS by forward substitution of (D - L) with D - L = [[1,0,0],[-a,1,0],[d,-c,1]]
    // and U = [[0,-a,b],[0,0,-c],[0,0,0]]: columns 1 and 2
    const double g01 = -a, g02 = b;
    const double g11 = -a * a, g12 = a * b - c;
    const double g21 = a * d - a * a * c, g22 = a * b * c - b * d - c * c;
    rg = fmax(rg, rho2(g11, g12, g21, g22));
    if (sgs) {
      const double e = lap(g3ss), f = lap(g2ss);
      // Y = L G_GS with L = [[0,0,0],[e,0,0],[-d,c,0]], then back substitution of
      // D - U = [[1,e,-f],[0,1,c],[0,0,1]]: rows 1 and 2
      const double y11 = e * g01, y12 = e * g02;
      const double y21 = -d * g01 + c * g11, y22 = -d * g02 + c * g12;
      const double x21 = y21, x22 = y22;
      const double x11 = y11 - c * x21, x12 = y12 - c * x22;
      rs = fmax(rs, rho2(x11, x12, x21, x22));
    }
  }
  static __shared__ double red[2][NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double mg = wave_max(rg), ms = wave_max(rs);
  if (lane == 0) {
    red[0][wv] = mg;
    red[1][wv] = ms;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = 0.0;
    for (int w = 0; w < NT / 64; ++w) v = fmax(v, red[threadIdx.x][w]);
    partials[(long)blockIdx.x * 4 + threadIdx.x] = v;
  }
}

// max over cells of | |m| - 1 | (FP64), block maxima into partials[4 b]
template <typename T>
__global__ __launch_bounds__(NT) void k_unit_error(const T* m, long N, double* partials) {
  double v = 0.0;
  for (long idx = blockIdx.x * (long)NT + threadIdx.x; idx < N; idx += (long)gridDim.x * NT) {
    const double a = m[idx], b = m[N + idx], c = m[2 * N + idx];
    v = fmax(v, fabs(sqrt(a * a + b * b + c * c) - 1.0));
  }
  static __shared__ double red[NT / 64];
  const double w = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < NT / 64; ++k) r = fmax(r, red[k]);
    partials[(long)blockIdx.x * 4] = r;
    partials[(long)blockIdx.x * 4 + 1] = 0.0;
  }
}

__global__ __launch_bounds__(NT) void k_rho_final(const double* partials, int nblocks, double* out) {
  static __shared__ double red[2][NT];
  for (int k = 0; k < 2; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) v = fmax(v, partials[(long)b * 4 + k]);
    red[k][threadIdx.x] = v;
  }
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 2; ++k) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 2) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Adjoint helpers
template <typename T> struct PwPack {
  PwTerm<T> t[PW_MAX];
  int n;
};

// One element per thread.  No term reads an array that an earlier term of the pack
// writes (the launcher splits packs that would), so the kernel issues every load of
// the pack, then computes, then stores: one round trip to memory.
template <typename T> __global__ __launch_bounds__(NT) void k_pw(const PwPack<T> A, int N) {
  const int idx = blockIdx.x * NT + threadIdx.x;
  if (idx >= N) return;
  T ro[PW_MAX], ra0[PW_MAX], rb0[PW_MAX], ra1[PW_MAX], rb1[PW_MAX];
#pragma unroll
  for (int k = 0; k < PW_MAX; ++k) {
    if (k >= A.n) break;
    const PwTerm<T>& t = A.t[k];
    ro[k] = t.acc ? t.out[idx] : (T)0;
    ra0[k] = t.x0 ? t.x0[idx] : (T)0;
    rb0[k] = t.y0 ? t.y0[idx] : (T)1;
    ra1[k] = t.x1 ? t.x1[idx] : (T)0;
    rb1[k] = t.y1 ? t.y1[idx] : (T)1;
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < PW_MAX; ++k) {
    if (k >= A.n) break;
    const PwTerm<T>& t = A.t[k];
    const double v = (double)ro[k] + t.c0 * (double)ra0[k] * (double)rb0[k] + t.c1 * (double)ra1[k] * (double)rb1[k];
    t.out[idx] = (T)v;
  }
}

template <typename T>
__global__ void k_adj_project(const T* lam, const T* u, const T* nrm, T* lc, long N) {
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < N; idx += (long)gridDim.x * blockDim.x) {
    const T l0 = lam[idx], l1 = lam[N + idx], l2 = lam[2 * N + idx];
    const T u0 = u[idx], u1 = u[N + idx], u2 = u[2 * N + idx];
    const T d = l0 * u0 + l1 * u1 + l2 * u2;
    const T r = (T)1 / nrm[idx];
    lc[idx] = (l0 - d * u0) * r;
    lc[N + idx] = (l1 - d * u1) * r;
    lc[2 * N + idx] = (l2 - d * u2) * r;
  }
}

__device__ __forceinline__ void block_partials4(double acc[4], double* partials) {
  static __shared__ double red[4][NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[k][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[threadIdx.x][w];
    partials[(long)blockIdx.x * 4 + threadIdx.x] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_wsum(const T* x0, const T* x1, const T* x2, const T* x3, int nterms, long N,
                                              double* partials) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const T* xs[4] = {x0, x1, x2, x3};
  for (long idx = blockIdx.x * (long)NT + threadIdx.x; idx < N; idx += (long)gridDim.x * NT) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < nterms) acc[k] += (double)xs[k][idx];
  }
  block_partials4(acc, partials);
}

// Adds the weighted totals of the block partials into grad (one thread: fixed order).
__global__ void k_partials_to_grad(const double* partials, int nblocks, int nterms, double w0, double w1, double w2,
                                   double w3, int s0, int s1, int s2, int s3, double* grad) {
  static __shared__ double red[4][NT];
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) s += partials[(long)b * 4 + k];
    red[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ws[4] = {w0, w1, w2, w3};
    const int ss[4] = {s0, s1, s2, s3};
    for (int k = 0; k < nterms; ++k) grad[ss[k]] += ws[k] * red[k][0];
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_adj_damp(const T* lw, const T* u, const T* nrm, const T* uF0, const T* uF1,
                                                  const T* uF2, const T* hsF, int nx, int ny, int nz, double ecx,
                                                  double ecy, double ecz, double Q, double he0, double he1, double he2,
                                                  double* partials) {
  // N <= 2^28: 32-bit indices
  const int N = nx * ny * nz, nxy = nx * ny;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const T* uF[3] = {uF0, uF1, uF2};
  const double he[3] = {he0, he1, he2};
  for (int idx = blockIdx.x * NT + threadIdx.x; idx < N; idx += gridDim.x * NT) {
    const int x = idx % nx, y = (idx / nx) % ny, z = idx / nxy;
    const int xm = x > 0 ? idx - 1 : idx, xp = x < nx - 1 ? idx + 1 : idx;
    const int ym = y > 0 ? idx - nx : idx, yp = y < ny - 1 ? idx + nx : idx;
    const int zm = z > 0 ? idx - nxy : idx, zp = z < nz - 1 ? idx + nxy : idx;
    double t = 0.0;
    for (int c = 0; c < 3; ++c) {
      const T* uc = u + c * N;
      const double cc = (double)nrm[idx] * uc[idx];
      double lap = 0.0;
      if (nx > 1) lap += ecx * ((double)nrm[xm] * uc[xm] + (double)nrm[xp] * uc[xp] - 2.0 * cc);
      if (ny > 1) lap += ecy * ((double)nrm[ym] * uc[ym] + (double)nrm[yp] * uc[yp] - 2.0 * cc);
      if (nz > 1) lap += ecz * ((double)nrm[zm] * uc[zm] + (double)nrm[zp] * uc[zp] - 2.0 * cc);
      double F = he[c] + (hsF ? (double)hsF[c * N + idx] : 0.0);
      if (c > 0) F -= Q * (double)uF[c][idx];
      const double l = lw[c * N + idx];
      t += l * (lap + F);
      acc[c] += l;
    }
    acc[3] += t;
  }
  block_partials4(acc, partials);
}

// ---------------------------------------------------------------------------
// Launchers
static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

namespace {
thread_local const char* g_geom = "";
int geom_fail(const char* what) {
  g_geom = what;
  return LAUNCH_EGEOM;
}
}  // namespace

const char* launch_geom_error() { return g_geom; }

// 1 / x: the hardware reciprocal in single precision (within 1 ulp), a correctly
// rounded division in double
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------
// Register version of the y-z heat solve for one x-major plane [NZ][NY] per
// workgroup (NY = 16 R2, NZ = 32), one thread team of R2 threads per pair of
// z rows (a = r, b = r + NZ/2) packed as one complex pencil.
//  y forward: Makhoul reordering on the load, 16-point DFT in registers over
//    the stride-R2 digit, twiddle, one padded LDS transpose, length-R2 DFTs:
//    the pencil's spectrum lands in row r of the LDS array Zs.
//  z: thread c owns column c.  It separates the two rows of every pencil into
//    the y-DCT coefficients of its column, then does the z DCT-II of that real
//    column as a 16-point complex FFT of its even / odd Makhoul samples, the
//    diagonal q (heat_q) and the z DCT-III the same way,
//    all in registers, and writes the column to LDS (over Zs, as reals).
//  y inverse: each team forms the pre-twiddled inverse input of its two rows
//    from that array, then the forward steps mirrored; stores undo the
//    reordering and scale by 2 / (NY NZ) (the half-length z inverse leaves 2).
template <typename T, int LGY, int LGZ>
__global__ __launch_bounds__((1 << (LGZ - 1)) * (1 << (LGY - 4))) void k_yz_reg(const YZSolve<T> A) {
  constexpr int NY = 1 << LGY, NZ = 1 << LGZ, HZ = NZ / 2;
  constexpr int R2 = NY / 16, G = 16 / R2, NTH = HZ * R2, RS = NY + 16;
  static_assert(LGY >= 5 && LGY <= 8 && LGZ == 5, "unsupported plane");
  static_assert(NTH == NY, "one z thread per column");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* Wy = reinterpret_cast<cx<T>*>(smem_raw);  // W_NY^i
  cx<T>* Dy = Wy + NY;                             // y DCT twiddles
  cx<T>* Dz = Dy + NY;                             // z DCT twiddles
  cx<T>* Zs = Dz + NZ;                             // [HZ][RS] complex, reused as [NZ][RS] reals
  T* Ly = reinterpret_cast<T*>(Zs + HZ * RS);      // y eigenvalues
  T* Lz = Ly + NY;                                 // z eigenvalues
  T* Yr = reinterpret_cast<T*>(Zs);
  const int tid = threadIdx.x;
  const int r = tid / R2, t = tid % R2;
  T* D = A.data[blockIdx.z] + (long)blockIdx.x * (NY * NZ);
  cx<T>* zs = Zs + r * RS;
  auto minv = [](int p) { return p < NY / 2 ? 2 * p : 2 * (NY - 1 - p) + 1; };
  T lx, sp;

  // ---- y forward
  {
    // the plane first, then the tables into LDS: one round trip to memory
    cx<T> v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int y = minv(t + R2 * m);
      v[m] = mk<T>(D[r * NY + y], D[(r + HZ) * NY + y]);
    }
    // one table entry per thread (NTH = NY)
    const cx<T> w_i = A.tw[tid << (A.lgTw - LGY)], dy_i = A.dtwy[tid];
    const T ly_i = A.lamY[tid];
    const int iz = min(tid, NZ - 1);
    const cx<T> dz_i = A.dtwz[iz];
    const T lz_i = A.lamZ[iz];
    // a batched plan: plane blockIdx.x = x runs + b
    const int runs = A.runs > 0 ? A.runs : 1;
    lx = A.lamX[blockIdx.x / runs];
    sp = (A.runp && A.rstageF) ? A.runp[(long)(blockIdx.x % runs) * RUNP + 7] : A.s;
    Wy[tid] = w_i;
    Dy[tid] = dy_i;
    Ly[tid] = ly_i;
    // threads past NZ repeat entry NZ - 1 (same value, same slot): no branch for the
    // compiler to sink these loads into
    Dz[iz] = dz_i;
    Lz[iz] = lz_i;
    __syncthreads();
    dft16(v, false);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], Wy[(t * k1) & (NY - 1)]);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) zs[k1 * (R2 + 1) + t] = v[k1];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int k1 = t * G + g;
#pragma unroll
      for (int q = 0; q < R2; ++q) v[g * R2 + q] = zs[k1 * (R2 + 1) + q];
      dft_reg<T, R2>(v + g * R2, false);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int k1 = t * G + g;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) zs[k1 + 16 * k2] = v[g * R2 + k2];
    }
    __syncthreads();
  }

  // ---- z pass: one real column per thread
  {
    const int c = tid;
    const int cm = (NY - c) & (NY - 1);
    const cx<T> wy = Dy[c];
    cx<T> u[HZ];  // u_n = v_2n + i v_2n+1, v the Makhoul order of the column
#pragma unroll
    for (int q = 0; q < HZ; ++q) {
      const cx<T> Zk = Zs[q * RS + c], Zm = Zs[q * RS + cm];
      const cx<T> Va = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
      const cx<T> Vb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
      // rows q and q + HZ of the column sit at Makhoul positions pa, pb
      const int za = q, zb = q + HZ;
      const int pa = (za & 1) ? NZ - 1 - (za >> 1) : (za >> 1);
      const int pb = (zb & 1) ? NZ - 1 - (zb >> 1) : (zb >> 1);
      const T ya = wy.x * Va.x - wy.y * Va.y, yb = wy.x * Vb.x - wy.y * Vb.y;
      if (pa & 1) u[pa >> 1].y = ya;
      else u[pa >> 1].x = ya;
      if (pb & 1) u[pb >> 1].y = yb;
      else u[pb >> 1].x = yb;
    }
    dft16(u, false);
    const T xc = sp * (lx + Ly[c]);
    T X[NZ];
    // V_k = E_k + W_32^k O_k from U_k and conj U_(16-k); V_(32-k) = conj V_k
#pragma unroll
    for (int k = 0; k <= HZ; ++k) {
      const cx<T> Uk = u[k & (HZ - 1)];
      const cx<T> Um = conjg(u[(HZ - k) & (HZ - 1)]);
      const cx<T> E = mk<T>((Uk.x + Um.x) * (T)0.5, (Uk.y + Um.y) * (T)0.5);
      const cx<T> O = mk<T>((Uk.y - Um.y) * (T)0.5, (Um.x - Uk.x) * (T)0.5);
      const cx<T> V = E + tw32v(O, k, false);
      const cx<T> wk = Dz[k];
      const T xk = xc + sp * Lz[k];
      X[k] = (wk.x * V.x - wk.y * V.y) * (xk * recip((T)1 + xk));
      if (k > 0 && k < HZ) {
        const cx<T> wm = Dz[NZ - k];
        const T xm = xc + sp * Lz[NZ - k];
        X[NZ - k] = (wm.x * V.x + wm.y * V.y) * (xm * recip((T)1 + xm));
      }
    }
    // DCT-III input V_j = conj(dtwz_j) (X_j - i X_(32-j)), folded to 16 points:
    // E = (V_k + V_(k+16)) / 2, O = (V_k - V_(k+16)) conj(W_32^k) / 2, u_k = E + i O
#pragma unroll
    for (int k = 0; k < HZ; ++k) {
      const cx<T> Vk = cmul(conjg(Dz[k]), mk<T>(X[k], k ? -X[NZ - k] : (T)0));
      const cx<T> Vj = cmul(conjg(Dz[k + HZ]), mk<T>(X[k + HZ], -X[HZ - k]));
      const cx<T> E = mk<T>((Vk.x + Vj.x) * (T)0.5, (Vk.y + Vj.y) * (T)0.5);
      const cx<T> O = tw32v(mk<T>((Vk.x - Vj.x) * (T)0.5, (Vk.y - Vj.y) * (T)0.5), k, true);
      u[k] = mk<T>(E.x - O.y, E.y + O.x);
    }
    dft16(u, true);
    __syncthreads();  // every thread has read Zs
#pragma unroll
    for (int z = 0; z < NZ; ++z) {
      const int p = (z & 1) ? NZ - 1 - (z >> 1) : (z >> 1);
      Yr[z * RS + c] = (p & 1) ? u[p >> 1].y : u[p >> 1].x;
    }
  }
  __syncthreads();

  // ---- y inverse
  {
    cx<T> v[16];
    const T* ya = Yr + r * RS;
    const T* yb = Yr + (r + HZ) * RS;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int k1 = t * G + g;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int k = k1 + 16 * k2;
        const cx<T> w = conjg(Dy[k]);
        const cx<T> Va = cmul(w, mk<T>(ya[k], k ? -ya[NY - k] : (T)0));
        const cx<T> Vb = cmul(w, mk<T>(yb[k], k ? -yb[NY - k] : (T)0));
        v[g * R2 + k2] = mk<T>(Va.x - Vb.y, Va.y + Vb.x);
      }
      dft_reg<T, R2>(v + g * R2, true);
#pragma unroll
      for (int q = 1; q < R2; ++q) v[g * R2 + q] = cmul(v[g * R2 + q], conjg(Wy[(q * k1) & (NY - 1)]));
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int k1 = t * G + g;
#pragma unroll
      for (int q = 0; q < R2; ++q) zs[k1 * (R2 + 1) + q] = v[g * R2 + q];
    }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) v[k1] = zs[k1 * (R2 + 1) + t];
    dft16(v, true);
    const T sc = (T)2 / (T)(NY * NZ);
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int y = minv(t + R2 * m);
      D[r * NY + y] = v[m].x * sc;
      D[(r + HZ) * NY + y] = v[m].y * sc;
    }
  }
}

// ---------------------------------------------------------------------------
// Row kernels for rows of N = 256 with 64 threads per pair of rows.  A DCT-II of
// length N is the real part of the twiddled, zero-padded 2N-point DFT, and the
// inverse DCT a cropped 2N-point inverse DFT of the Hermitian extension of the
// pre-twiddled coefficients, so all four row transforms (cropped c2r, DCT-II,
// inverse DCT, zero-padded r2c) are 512-point FFTs with the same 8 x 8 x 8
// four-step structure, and between them every thread t holds x = t + 64 m, m < 4.
// Two real rows share one complex pencil (a in .x, b in .y); P pencils per
// workgroup, thread (q = tid % P, t = tid / P).

// The 512-point row kernels keep W_512^e in LDS at slot e + e / 8: the twiddles
// that a wave reads at once are spaced by multiples of 8 entries, which one pad
// entry per 8 spreads over the banks.
constexpr int W512_SLOTS = 512 + 64;
__host__ __device__ __forceinline__ int w512_slot(int e) { return e + (e >> 3); }

// natural order in: v[m] = x[t + 64 m]; digit order out: v[kb] = X[(t >> 3) + 8 (t & 7) + 64 kb],
// the forward DFT, or with INV the unnormalised inverse (conjugate twiddles);
// xb the LDS transpose buffer [64][S], W the table W_512^i in LDS;
// lo4: x[t + 64 m] = 0 for m >= 4; first4: only kb < 4 is needed
template <typename T, int P, int S, bool INV>
__device__ __forceinline__ void f512_dif(cx<T> (&v)[8], int t, int q, cx<T>* xb, const cx<T>* W, bool lo4,
                                         bool first4) {
  auto tw = [&](int e) {
    cx<T> w = W[w512_slot(e & 511)];
    if (INV) w.y = -w.y;
    return w;
  };
  if (lo4) dft8_lo4(v, INV);
  else dft8(v, INV);
  {
    const int t0 = t & 7, t1 = t >> 3;
#pragma unroll
    for (int k2 = 1; k2 < 8; ++k2) v[k2] = cmul(v[k2], tw(t * k2));
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) xb[(k2 * 8 + t0) * S + t1 * P + q] = v[k2];
  }
  __syncthreads();
  {
    const int k2 = t >> 3, u0 = t & 7;
#pragma unroll
    for (int u1 = 0; u1 < 8; ++u1) v[u1] = xb[(k2 * 8 + u0) * S + u1 * P + q];
    dft8(v, INV);
#pragma unroll
    for (int ka = 1; ka < 8; ++ka) v[ka] = cmul(v[ka], tw(8 * u0 * ka));
    __syncthreads();
#pragma unroll
    for (int ka = 0; ka < 8; ++ka) xb[(k2 * 8 + ka) * S + u0 * P + q] = v[ka];
  }
  __syncthreads();
  {
    const int k2 = t >> 3, ka = t & 7;
#pragma unroll
    for (int u0 = 0; u0 < 8; ++u0) v[u0] = xb[(k2 * 8 + ka) * S + u0 * P + q];
  }
  __syncthreads();
  if (first4) dft8_first4(v, INV);
  else dft8(v, INV);
}
template <typename T, int P, int S>
__device__ __forceinline__ void f512_fwd(cx<T> (&v)[8], int t, int q, cx<T>* xb, const cx<T>* W, bool lo4) {
  f512_dif<T, P, S, false>(v, t, q, xb, W, lo4, false);
}

// inverse (unnormalised): v[kb] = X[(t >> 3) + 8 (t & 7) + 64 kb] in, v[m] = x[t + 64 m]
// out; first4: only m < 4 is needed
template <typename T, int P, int S>
__device__ __forceinline__ void f512_inv(cx<T> (&v)[8], int t, int q, cx<T>* xb, const cx<T>* W, bool first4) {
  {
    const int k2 = t >> 3, ka = t & 7;
    dft8(v, true);
#pragma unroll
    for (int t0 = 1; t0 < 8; ++t0) v[t0] = cmul(v[t0], conjg(W[w512_slot((8 * t0 * ka) & 511)]));
#pragma unroll
    for (int t0 = 0; t0 < 8; ++t0) xb[(k2 * 8 + t0) * S + ka * P + q] = v[t0];
  }
  __syncthreads();
  {
    const int kk2 = t >> 3, t0 = t & 7;
#pragma unroll
    for (int a = 0; a < 8; ++a) v[a] = xb[(kk2 * 8 + t0) * S + a * P + q];
    dft8(v, true);
#pragma unroll
    for (int t1 = 0; t1 < 8; ++t1) v[t1] = cmul(v[t1], conjg(W[w512_slot(((t0 + 8 * t1) * kk2) & 511)]));
    __syncthreads();
#pragma unroll
    for (int t1 = 0; t1 < 8; ++t1) xb[(t0 + 8 * t1) * S + kk2 * P + q] = v[t1];
  }
  __syncthreads();
#pragma unroll
  for (int kk2 = 0; kk2 < 8; ++kk2) v[kk2] = xb[t * S + kk2 * P + q];
  __syncthreads();
  if (first4) dft8_first4(v, true);
  else dft8(v, true);
}

// X[k] of pencil q in natural order: row k & 63, column (k >> 6) P + q of xb, the
// column XORed with P ((k >> 3) & 7).  The spill writes rows 8 apart at once; the
// swizzle puts them in distinct banks (the columns of a row stay within 8 P).
template <typename T, int P, int S> __device__ __forceinline__ int f512_slot(int k, int q) {
  const int r = k & 63;
  return r * S + ((((k >> 6) * P) ^ (P * ((r >> 3) & 7))) + q);
}
// the spectrum of this thread's pencil, after f512_fwd (digit order), to its natural
// slots; NKB: the first NKB digits only
template <typename T, int P, int S, int NKB = 8>
__device__ __forceinline__ void f512_spill(const cx<T> (&v)[8], int t, int q, cx<T>* xb) {
  const int kl = (t >> 3) + 8 * (t & 7);
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) xb[f512_slot<T, P, S>(kl + 64 * kb, q)] = v[kb];
}
template <typename T, int P, int S> __device__ __forceinline__ cx<T> f512_at(const cx<T>* xb, int k, int q) {
  return xb[f512_slot<T, P, S>(k, q)];
}

// Memory order in both kernels: every global load (operands, spectra, DCT
// twiddles, then the W table) is issued before the first wait, and no load
// follows a store.  The hardware counts loads and stores in one in-order
// counter, so a load issued after a store would make its wait cover the store.
template <typename T, int P>
__global__ __launch_bounds__(64 * P) void k_row_fwd512(const RowFwd<T> A) {
  constexpr int N = 256, S = fft512_stride<T, P>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* W = reinterpret_cast<cx<T>*>(smem_raw);  // W_512^i at w512_slot(i)
  cx<T>* xb = W + W512_SLOTS;
  const Blk bk = xcd_block();
  const int tid = threadIdx.x, q = tid % P, t = tid / P, ch = bk.z;
  const int ra = bk.x * 2 * P + 2 * q;
  const bool oka = ra < A.nrows, okb = ra + 1 < A.nrows;
  constexpr unsigned TB = sizeof(T), CB = sizeof(cx<T>);
  // loads read rows clamped into range (finite data for rows that are never stored)
  const unsigned ra1c = (unsigned)min(ra, A.nrows - 1), rb1c = (unsigned)min(ra + 1, A.nrows - 1);
  const unsigned la = ra1c * (N * TB), lb = rb1c * (N * TB);
  const T* u = A.u[ch];
  const T* w = A.w[ch];
  const cx<T>* xin = A.xin[ch];
  T* dout = A.dct_out[ch];
  cx<T>* xo = A.xout[ch];
  cx<T> Xa[8], Xb[8];
  if (xin) {
    // x-level half spectra (k <= 256) of both rows at k = t + 64 m (consecutive
    // lanes read consecutive k; above 256 the mirrored 512 - k)
    const unsigned pa = ra1c * (unsigned)A.xin_pitch * CB, pb = rb1c * (unsigned)A.xin_pitch * CB;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int k = t + 64 * m;
      const unsigned kk = (unsigned)(k <= 256 ? k : 512 - k);
      // packed: the Nyquist bin (thread 0, m = 4) is the imaginary part of bin 0
      const unsigned kl = m == 4 && A.xpk && kk == 256u ? 0u : kk;
      Xa[m] = ld_off(xin, pa + kl * CB);
      Xb[m] = ld_off(xin, pb + kl * CB);
    }
  }
  cx<T> pu[4], pw[4], wk[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const unsigned xo4 = (unsigned)(t + 64 * m) * TB;
    pu[m] = u ? mk<T>(ld_off(u, la + xo4), ld_off(u, lb + xo4)) : zero<T>();
    pw[m] = w ? mk<T>(ld_off(w, la + xo4), ld_off(w, lb + xo4)) : zero<T>();
    wk[m] = dout ? A.dtw[t + 64 * m] : zero<T>();
  }
  for (int i = tid; i < 512; i += 64 * P) W[w512_slot(i)] = A.tw[i << (A.lgTw - 9)];
  __syncthreads();
  cx<T> v[8];
  if (xin) {
    // cropped c2r: Hermitian completion above k = 256, both rows packed as a + i b
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int k = t + 64 * m;
      const int kk = k <= 256 ? k : 512 - k;
      cx<T> xa = Xa[m], xbb = Xb[m];
      if (kk == 0 || kk == 256) {
        if (A.xpk && kk == 256) {
          xa.x = xa.y;
          xbb.x = xbb.y;
        }
        xa.y = (T)0;
        xbb.y = (T)0;
      }
      if (k > 256) {
        xa.y = -xa.y;
        xbb.y = -xbb.y;
      }
      v[m] = mk<T>(xa.x - xbb.y, xa.y + xbb.x);
    }
    // x in digit order, only x < 256 (kb < 4); back to x = t + 64 m through LDS
    f512_dif<T, P, S, true>(v, t, q, xb, W, false, true);
    f512_spill<T, P, S, 4>(v, t, q, xb);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = f512_at<T, P, S>(xb, t + 64 * m, q);
    __syncthreads();  // xb is reused by the forward transform
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = zero<T>();
  }
  // v = b (hs + he) + (alo + a) u + (wclo + wc) w at x = t + 64 m
  {
    T* hso = A.hs_out[ch];
    T* vo = A.val_out[ch];
    T ac = A.a[ch], aloc = A.alo[ch], hec = A.he[ch], bc = A.b;
    const T wcc = A.wc[ch], wcloc = A.wclo[ch];
    if (A.runp) {
      // every row of the tile belongs to one run
      const T* rp = A.runp + (long)(min(bk.x * 2 * P, A.nrows - 1) / A.rpr) * RUNP;
      hec = rp[A.rcomp[ch]];
      if (A.rstageF) {
        ac = rp[3 + A.rcomp[ch]];
        aloc = rp[8 + A.rcomp[ch]];
        bc = rp[6];
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const unsigned xo4 = (unsigned)(t + 64 * m) * TB;
      const T hsa = v[m].x, hsb = v[m].y;
      T va = bc * (hsa + hec), vb = bc * (hsb + hec);
      // the small parts first, the leading coefficients last
      if (u) {
        va += aloc * pu[m].x;
        vb += aloc * pu[m].y;
      }
      if (w) {
        va += wcloc * pw[m].x;
        vb += wcloc * pw[m].y;
      }
      if (u) {
        va += ac * pu[m].x;
        vb += ac * pu[m].y;
      }
      if (w) {
        va += wcc * pw[m].x;
        vb += wcc * pw[m].y;
      }
      if (hso) {
        if (oka) st_off(hso, la + xo4, hsa);
        if (okb) st_off(hso, lb + xo4, hsb);
      }
      if (vo) {
        if (oka) st_off(vo, la + xo4, va);
        if (okb) st_off(vo, lb + xo4, vb);
      }
      v[m] = mk<T>(va, vb);
    }
  }
  if (dout || xo) {
    // one zero-padded forward transform serves the DCT-II and the r2c
#pragma unroll
    for (int m = 4; m < 8; ++m) v[m] = zero<T>();
    f512_fwd<T, P, S>(v, t, q, xb, W, true);
    f512_spill<T, P, S>(v, t, q, xb);
    __syncthreads();
    if (dout) {
      const unsigned nr = (unsigned)A.nrows;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = t + 64 * j;
        const cx<T> Zk = f512_at<T, P, S>(xb, k, q), Zm = f512_at<T, P, S>(xb, (512 - k) & 511, q);
        const cx<T> Fa = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
        const cx<T> Fb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
        const T xa = wk[j].x * Fa.x - wk[j].y * Fa.y, xbv = wk[j].x * Fb.x - wk[j].y * Fb.y;
        if (A.dct_xmajor) {
          // [N][nrows] with nrows even: the pair (ra, ra + 1) is one aligned vector
          if (oka) st_off(reinterpret_cast<cx<T>*>(dout), ((unsigned)k * nr + (unsigned)ra) * TB, mk<T>(xa, xbv));
        } else {
          if (oka) st_off(dout, la + (unsigned)k * TB, xa);
          if (okb) st_off(dout, lb + (unsigned)k * TB, xbv);
        }
      }
    }
    if (xo) {
      const unsigned pitch = (unsigned)A.xout_pitch;
#pragma unroll
      for (int j = 0; j <= 4; ++j) {
        const int k = t + 64 * j;
        if (j == 4 && (t || A.xpk)) break;  // packed: the Nyquist bin goes with bin 0
        const cx<T> Zk = f512_at<T, P, S>(xb, k, q), Zm = f512_at<T, P, S>(xb, (512 - k) & 511, q);
        cx<T> Xa2 = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
        cx<T> Xb2 = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
        if (j == 0 && A.xpk && t == 0) {
          // X[256] of both rows (real: Re Z_256, Im Z_256) as bin 0's imaginary part
          const cx<T> Zn = f512_at<T, P, S>(xb, 256, q);
          Xa2.y = Zn.x;
          Xb2.y = Zn.y;
        }
        if (oka) st_off(xo, ((unsigned)ra * pitch + (unsigned)k) * CB, Xa2);
        if (okb) st_off(xo, ((unsigned)(ra + 1) * pitch + (unsigned)k) * CB, Xb2);
      }
    }
  }
}

template <typename T, int P, int NCH, bool XM, int OP>
__global__ __launch_bounds__(64 * P) void k_row_inv512(const RowInv<T> A) {
  constexpr int N = 256, S = fft512_stride<T, P>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* W = reinterpret_cast<cx<T>*>(smem_raw);  // W_512^i at w512_slot(i)
  cx<T>* xb = W + W512_SLOTS;
  const Blk bk = xcd_block();
  const int tid = threadIdx.x, q = tid % P, t = tid / P;
  const int ra = bk.x * 2 * P + 2 * q;
  const bool oka = ra < A.nrows, okb = ra + 1 < A.nrows;
  constexpr unsigned TB = sizeof(T);
  const unsigned ra1c = (unsigned)min(ra, A.nrows - 1), rb1c = (unsigned)min(ra + 1, A.nrows - 1);
  const unsigned la = ra1c * (N * TB), lb = rb1c * (N * TB);
  constexpr bool gs = OP == ROW_OP_GS;
  const int kl = (t >> 3) + 8 * (t & 7);
  // heat coefficients of every channel at this thread's slots k = kl + 64 kb
  // (their Hermitian-extension index kk), and the DCT twiddles of those slots
  T ha[NCH][8], hb[NCH][8];
  cx<T> wq[8];
  {
    // x-major arrays [N][nrows] (nrows even): rows ra, ra + 1 are one aligned vector
    const unsigned rp = XM ? (unsigned)min(ra, A.nrows - 2) : 0u, nr = (unsigned)A.nrows;
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      const int k = kl + 64 * kb;
      const unsigned kk = (unsigned)(k < 256 ? k : (k == 256 ? 0 : 512 - k));
      wq[kb] = A.dtw[kk];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        if (XM) {
          const cx<T> h2 = ld_off(reinterpret_cast<const cx<T>*>(A.heat[c]), (kk * nr + rp) * TB);
          ha[c][kb] = h2.x;
          hb[c][kb] = h2.y;
        } else {
          ha[c][kb] = ld_off(A.heat[c], la + kk * TB);
          hb[c][kb] = ld_off(A.heat[c], lb + kk * TB);
        }
      }
    }
  }
  // Gauss-Seidel operands: at most one of P, R is an array (the other an inverted
  // channel), the caller guarantees it
  const T* PR = A.Pch < 0 ? A.Pf : (A.Rch < 0 ? A.Rf : nullptr);
  cx<T> pre_b[4], pre_q[4], pre_s[4], pre_pr[4], pre_src[4];
  if (gs) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const unsigned xo = (unsigned)(t + 64 * m) * TB;
      pre_b[m] = mk<T>(ld_off(A.base, la + xo), ld_off(A.base, lb + xo));
      pre_q[m] = mk<T>(ld_off(A.Qf, la + xo), ld_off(A.Qf, lb + xo));
      pre_s[m] = mk<T>(ld_off(A.Sf, la + xo), ld_off(A.Sf, lb + xo));
      pre_pr[m] = PR ? mk<T>(ld_off(PR, la + xo), ld_off(PR, lb + xo)) : zero<T>();
      pre_src[m] = A.src ? mk<T>(ld_off(A.src, la + xo), ld_off(A.src, lb + xo)) : zero<T>();
    }
  }
  // the right-hand sides r: g = r - the inverse transform of the correction
  cx<T> g[NCH][4];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const unsigned xo = (unsigned)(t + 64 * m) * TB;
      g[c][m] = mk<T>(ld_off(A.rin[c], la + xo), ld_off(A.rin[c], lb + xo));
    }
  }
  for (int i = tid; i < 512; i += 64 * P) W[w512_slot(i)] = A.tw[i << (A.lgTw - 9)];
  __syncthreads();
  const T invn = (T)1 / (T)N;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    cx<T> v[8];
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      // Hermitian extension of G_k = conj(dtw_k) X_k (k < 256), G_256 = 0
      const int k = kl + 64 * kb;
      cx<T> wk = wq[kb];
      if (k < 256) wk.y = -wk.y;  // conj(dtw_k) below 256, dtw_(512-k) above
      cx<T> ga = mk<T>(wk.x * ha[c][kb], wk.y * ha[c][kb]), gb = mk<T>(wk.x * hb[c][kb], wk.y * hb[c][kb]);
      if (k == 256) ga = gb = zero<T>();
      v[kb] = mk<T>(ga.x - gb.y, ga.y + gb.x);
    }
    f512_inv<T, P, S>(v, t, q, xb, W, true);
    T* go = A.gout[c];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      g[c][m] = mk<T>(g[c][m].x - v[m].x * invn, g[c][m].y - v[m].y * invn);
      if (go) {
        const unsigned xo = (unsigned)(t + 64 * m) * TB;
        if (oka) st_off(go, la + xo, g[c][m].x);
        if (okb) st_off(go, lb + xo, g[c][m].y);
      }
    }
  }
  // the zero-padded r2c of this thread's two rows (v[m] at x = t + 64 m, m < 4) into A.xout
  auto r2c_store = [&](cx<T>(&v)[8]) {
#pragma unroll
    for (int m = 4; m < 8; ++m) v[m] = zero<T>();
    f512_fwd<T, P, S>(v, t, q, xb, W, true);
    f512_spill<T, P, S>(v, t, q, xb);
    __syncthreads();
    constexpr unsigned CB = sizeof(cx<T>);
    const unsigned pitch = (unsigned)A.xout_pitch;
#pragma unroll
    for (int j = 0; j <= 4; ++j) {
      const int k = t + 64 * j;
      if (j == 4 && (t || A.xpk)) break;  // packed: the Nyquist bin goes with bin 0
      const cx<T> Zk = f512_at<T, P, S>(xb, k, q), Zm = f512_at<T, P, S>(xb, (512 - k) & 511, q);
      cx<T> Xa = mk<T>((Zk.x + Zm.x) * (T)0.5, (Zk.y - Zm.y) * (T)0.5);
      cx<T> Xb = mk<T>((Zk.y + Zm.y) * (T)0.5, (Zm.x - Zk.x) * (T)0.5);
      if (j == 0 && A.xpk && t == 0) {
        // X[256] of both rows (real: Re Z_256, Im Z_256) as bin 0's imaginary part
        const cx<T> Zn = f512_at<T, P, S>(xb, 256, q);
        Xa.y = Zn.x;
        Xb.y = Zn.y;
      }
      if (oka) st_off(A.xout, ((unsigned)ra * pitch + (unsigned)k) * CB, Xa);
      if (okb) st_off(A.xout, ((unsigned)(ra + 1) * pitch + (unsigned)k) * CB, Xb);
    }
  };
  if constexpr (gs) {
    constexpr int C1 = NCH > 1 ? 1 : 0;
    const T ds = A.ds;
    cx<T> v[8];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const unsigned xo = (unsigned)(t + 64 * m) * TB;
      T o[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const T g0 = h ? g[0][m].y : g[0][m].x;
        const T g1 = NCH > 1 ? (h ? g[C1][m].y : g[C1][m].x) : (T)0;
        const T prv = h ? pre_pr[m].y : pre_pr[m].x;
        const T pv = A.Pch == 0 ? g0 : (A.Pch == 1 ? g1 : prv);
        const T rv = A.Rch == 0 ? g0 : (A.Rch == 1 ? g1 : prv);
        o[h] = (h ? pre_b[m].y : pre_b[m].x) + pv * (h ? pre_q[m].y : pre_q[m].x) -
               rv * (h ? pre_s[m].y : pre_s[m].x) + ds * (h ? pre_src[m].y : pre_src[m].x);
      }
      if (oka) st_off(A.out, la + xo, o[0]);
      if (okb) st_off(A.out, lb + xo, o[1]);
      v[m] = mk<T>(o[0], o[1]);
    }
    if (A.xout) r2c_store(v);
  } else if constexpr (NCH == 1 && OP == ROW_OP_NONE) {
    // a plain inverse of one channel: optionally the r2c of its result
    if (A.xout) {
      cx<T> v[8];
#pragma unroll
      for (int m = 0; m < 4; ++m) v[m] = g[0][m];
      r2c_store(v);
    }
  } else if constexpr (NCH == 3 && OP == ROW_OP_PROJECT) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const unsigned xo = (unsigned)(t + 64 * m) * TB;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (!(h ? okb : oka)) continue;
        const unsigned bo = (h ? lb : la) + xo;
        const T c0 = h ? g[0][m].y : g[0][m].x, c1 = h ? g[NCH > 1 ? 1 : 0][m].y : g[NCH > 1 ? 1 : 0][m].x,
                c2 = h ? g[NCH > 2 ? 2 : 0][m].y : g[NCH > 2 ? 2 : 0][m].x;
        const T nr = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        if (!(nr > (T)0) || !isfinite(nr)) A.flag[0] = 1;
        const T inr = (T)1 / nr;
        st_off(A.mout[0], bo, c0 * inr);
        st_off(A.mout[1], bo, c1 * inr);
        st_off(A.mout[2], bo, c2 * inr);
        if (A.nrm) st_off(A.nrm, bo, nr);
      }
    }
  }
}

// pencils (pairs of rows) per workgroup of the 512-point row kernels.  The lanes
// of a wave cover P pencils x 64/P positions, so a row-major access touches 2P
// rows per instruction and an x-major one 2P consecutive values.  Single
// precision: 2 for the forward kernel, whose loads are row-major (10% faster than
// 4 or 8; 16 was slower still), 4 for the inverse kernel, which reads its heat
// arrays x-major (2 measured 7% slower, 8 measured 8% slower for one channel and
// 25% for two)
template <typename T> constexpr int row_fwd512_pencils() { return sizeof(T) == 4 ? 2 : 4; }
template <typename T> constexpr int row_inv512_pencils() { return 4; }

template <typename T> bool row256(int lgN, int lgLc, int lgLr, bool c2r, bool r2c) {
  return lgN == 8 && (!c2r || lgLc == 9) && (!r2c || lgLr == 9);
}

template <typename T> int launch_row_fwd(const RowFwd<T>& a, int nch, hipStream_t s) {
  bool c2r = false, r2c = false;
  for (int c = 0; c < nch; ++c) {
    c2r = c2r || a.xin[c];
    r2c = r2c || a.xout[c];
  }
  // x-major DCT output is stored as row pairs (2r, 2r + 1) of 8 bytes: an even row
  // count (or one row, where the layouts coincide); the generic kernel takes the rest
  const bool xm_ok = !a.dct_xmajor || a.nrows == 1 || a.nrows % 2 == 0;
  if (xm_ok && row256<T>(a.lgN, a.lgLc, a.lgLr, c2r, r2c) && (!a.runp || a.rpr % (2 * row_fwd512_pencils<T>()) == 0)) {
    constexpr int P = row_fwd512_pencils<T>();
    const size_t lds = (W512_SLOTS + (size_t)64 * fft512_stride<T, P>()) * sizeof(cx<T>);
    const dim3 grid(ceil_div(a.nrows, 2 * P), 1, nch);
    RowFwd<T> b = a;
    b.dct_xmajor = a.dct_xmajor && a.nrows > 1;  // one row: both layouts coincide
    hipLaunchKernelGGL((k_row_fwd512<T, P>), grid, dim3(64 * P), lds, s, b);
    return SGSPM_KC_ROW_FWD512;
  }
  const int rows = 2 << a.lgP;
  dim3 grid(ceil_div(a.nrows, rows), 1, nch);
  // twiddles, the tile, the DCT twiddles
  const size_t lds = ((size_t)a.Lmax + ((size_t)1 << a.lgP) * (a.Lmax + 1) + (size_t)a.n) * sizeof(cx<T>);
  // every transform length and the row length divide Lmax (the LDS pitch and the
  // twiddle table), and P Lmax complex values fit the tile: each thread then holds
  // its 2 VPT row values and VPT spectrum values, and every FFT stage its butterflies
  if (nch < 1 || nch > 3) return geom_fail("k_row_fwd: 1 to 3 channels");
  if (a.n < 1 || a.Lmax % a.n || (c2r && a.Lmax % a.Lc) || (r2c && a.Lmax % a.Lr))
    return geom_fail("k_row_fwd: a row or transform length does not divide Lmax");
  if (a.lgP < 0 || ((long)a.Lmax << a.lgP) > tile_elems<T>()) return geom_fail("k_row_fwd: P Lmax beyond the tile");
  if (a.twg < 1) return geom_fail("k_row_fwd: no twiddle stride");
  if (lds > LDS_LIMIT) return geom_fail("k_row_fwd: LDS beyond the limit");
  if (a.runp && (a.rpr < 1 || a.rpr % rows)) return geom_fail("k_row_fwd: a tile holds rows of two runs");
  if (a.lgN < 0 || a.lgLmax < 0 || (c2r && a.lgLc < 0) || (r2c && a.lgLr < 0))
    hipLaunchKernelGGL((k_row_fwd<T, true>), grid, dim3(NT), lds, s, a);
  else
    hipLaunchKernelGGL((k_row_fwd<T, false>), grid, dim3(NT), lds, s, a);
  return SGSPM_KC_ROW_FWD;
}

template <typename T, int NCH, bool XM>
void launch_row_inv512_op(const RowInv<T>& a, dim3 grid, size_t lds, hipStream_t s) {
  constexpr int P = row_inv512_pencils<T>();
  const dim3 blk(64 * P);
  if constexpr (NCH < 3) {
    if (a.op == ROW_OP_GS) {
      hipLaunchKernelGGL((k_row_inv512<T, P, NCH, XM, ROW_OP_GS>), grid, blk, lds, s, a);
      return;
    }
  } else {
    if (a.op == ROW_OP_PROJECT) {
      hipLaunchKernelGGL((k_row_inv512<T, P, NCH, XM, ROW_OP_PROJECT>), grid, blk, lds, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_row_inv512<T, P, NCH, XM, ROW_OP_NONE>), grid, blk, lds, s, a);
}
template <typename T> void launch_row_inv512_mode(const RowInv<T>& a, dim3 grid, size_t lds, hipStream_t s) {
  const bool xm = a.heat_xmajor != 0 && a.nrows > 1;  // one row: both layouts coincide
  if (a.nch == 1) xm ? launch_row_inv512_op<T, 1, true>(a, grid, lds, s) : launch_row_inv512_op<T, 1, false>(a, grid, lds, s);
  else if (a.nch == 2) xm ? launch_row_inv512_op<T, 2, true>(a, grid, lds, s) : launch_row_inv512_op<T, 2, false>(a, grid, lds, s);
  else xm ? launch_row_inv512_op<T, 3, true>(a, grid, lds, s) : launch_row_inv512_op<T, 3, false>(a, grid, lds, s);
}

template <typename T> int launch_row_inv(const RowInv<T>& a, hipStream_t s) {
  for (int c = 0; c < a.nch && c < 3; ++c)
    if (!a.rin[c]) return geom_fail("k_row_inv: a channel without its right-hand side");
  // the r2c output follows a Gauss-Seidel update or a plain inverse of one channel
  if (a.xout && !(a.op == ROW_OP_GS || (a.op == ROW_OP_NONE && a.nch == 1)))
    return geom_fail("k_row_inv: an r2c output needs a Gauss-Seidel update or one plain channel");
  // the register kernel covers the sweeps (update with one or two channels), the
  // projection (three) and plain inverse transforms (one to three)
  const bool mode_ok = (a.op == ROW_OP_GS && a.nch < 3 && !(a.Pch < 0 && a.Rch < 0)) ||
                       (a.op == ROW_OP_PROJECT && a.nch == 3) || a.op == ROW_OP_NONE;
  // x-major heat arrays are read as row pairs (2r, 2r + 1) of 8 bytes: an even row
  // count (or one row, where the layouts coincide); the generic kernel takes the rest
  const bool xm_ok = !a.heat_xmajor || a.nrows == 1 || a.nrows % 2 == 0;
  if (mode_ok && xm_ok && row256<T>(a.lgN, a.lgLr, a.lgLr, false, a.xout != nullptr)) {
    constexpr int P = row_inv512_pencils<T>();
    const size_t lds = (W512_SLOTS + (size_t)64 * fft512_stride<T, P>()) * sizeof(cx<T>);
    const dim3 grid(ceil_div(a.nrows, 2 * P));
    launch_row_inv512_mode<T>(a, grid, lds, s);
    return SGSPM_KC_ROW_INV512;
  }
  const int rows = 2 << a.lgP;
  dim3 grid(ceil_div(a.nrows, rows), 1, 1);
  // twiddles, the tile, the DCT twiddles
  const size_t lds = ((size_t)a.Lmax + ((size_t)1 << a.lgP) * (a.Lmax + 1) + (size_t)a.n) * sizeof(cx<T>);
  if (a.nch < 1 || a.nch > 3) return geom_fail("k_row_inv: 1 to 3 channels");
  if (a.n < 1 || a.Lmax % a.n || (a.xout && a.Lmax % a.Lr))
    return geom_fail("k_row_inv: a row or transform length does not divide Lmax");
  if (a.lgP < 0 || ((long)a.Lmax << a.lgP) > tile_elems<T>()) return geom_fail("k_row_inv: P Lmax beyond the tile");
  if (a.twg < 1) return geom_fail("k_row_inv: no twiddle stride");
  if (lds > LDS_LIMIT) return geom_fail("k_row_inv: LDS beyond the limit");
  if (a.lgN < 0 || a.lgLmax < 0 || (a.xout && a.lgLr < 0))
    hipLaunchKernelGGL((k_row_inv<T, true>), grid, dim3(NT), lds, s, a);
  else
    hipLaunchKernelGGL((k_row_inv<T, false>), grid, dim3(NT), lds, s, a);
  return SGSPM_KC_ROW_INV;
}

template <typename T> int launch_col_dct(const ColDct<T>& a, int nbatch, int nch, hipStream_t s) {
  dim3 grid(ceil_div(a.ni, 2 << a.lgP), nbatch, nch);
  const size_t lds = ((size_t)a.n + ((size_t)a.n << a.lgP)) * sizeof(cx<T>);
  if (nch < 1 || nch > 3) return geom_fail("k_col_dct: 1 to 3 channels");
  if (a.n < 1 || a.lgP < 0 || ((long)a.n << a.lgP) > tile_elems<T>()) return geom_fail("k_col_dct: P n beyond the tile");
  if (a.twg < 1) return geom_fail("k_col_dct: no twiddle stride");
  if (lds > LDS_LIMIT) return geom_fail("k_col_dct: LDS beyond the limit");
  if (a.lgN < 0)
    hipLaunchKernelGGL((k_col_dct<T, true>), grid, dim3(NT), lds, s, a);
  else
    hipLaunchKernelGGL((k_col_dct<T, false>), grid, dim3(NT), lds, s, a);
  return SGSPM_KC_COL_DCT;
}

template <typename T> int launch_col_fft(const ColFft<T>& a, int nbatch, int nch, hipStream_t s) {
  if (nch < 1 || nch > 3) return geom_fail("k_col_fft: 1 to 3 channels");
  if (a.n_in < 1 || a.n_out < 1 || a.n_in > a.L || a.n_out > a.L)
    return geom_fail("k_col_fft: input or output longer than the transform");
  if (a.lgL == 9) {
    if (a.lgTw < 9) return geom_fail("k_fft512: twiddle table shorter than the transform");
    constexpr int P = sizeof(T) == 4 ? 8 : 4;
    // packed DC and Nyquist columns: the kernel's ni counts the columns before
    // the Nyquist column, which is column ni
    ColFft<T> b = a;
    b.pack = a.pack && a.ni > 1;
    if (b.pack) b.ni = a.ni - 1;
    dim3 grid(ceil_div(b.ni, P), nbatch, nch);
    // the twiddle table (single precision) and the transpose buffer
    const size_t lds = ((sizeof(T) == 4 ? 512 : 0) + (size_t)64 * fft512_stride<T, P>()) * sizeof(cx<T>);
    if (a.inv) hipLaunchKernelGGL((k_fft512<T, P, true>), grid, dim3(64 * P), lds, s, b);
    else hipLaunchKernelGGL((k_fft512<T, P, false>), grid, dim3(64 * P), lds, s, b);
    return SGSPM_KC_FFT512;
  }
  dim3 grid(ceil_div(a.ni, 1 << a.lgP), nbatch, nch);
  const size_t lds = ((size_t)a.L + ((size_t)a.L << a.lgP)) * sizeof(cx<T>);
  if (a.lgP < 0 || ((long)a.L << a.lgP) > tile_elems<T>()) return geom_fail("k_col_fft: P L beyond the tile");
  if (a.twg < 1) return geom_fail("k_col_fft: no twiddle stride");
  if (lds > LDS_LIMIT) return geom_fail("k_col_fft: LDS beyond the limit");
  if (a.lgL < 0)
    hipLaunchKernelGGL((k_col_fft<T, true>), grid, dim3(NT), lds, s, a);
  else
    hipLaunchKernelGGL((k_col_fft<T, false>), grid, dim3(NT), lds, s, a);
  return SGSPM_KC_COL_FFT;
}

// LDS of the generic y-z solve and its complex pencils per pass
template <typename T> size_t yz_lds(int ny, int nz, int lgPP) {
  const size_t PP = (size_t)1 << lgPP;
  const size_t Hy = (PP * nz + 1) / 2, Hz = (PP * ny + 1) / 2;
  const size_t nbuf = std::max((size_t)ny * (Hy + 1), (size_t)nz * (Hz + 1));
  // y and z twiddles, buffer, y and z DCT twiddles; eigenvalues of y, z and the
  // planes, and the planes' scales
  return (2 * ((size_t)ny + nz) + nbuf) * sizeof(cx<T>) + ((size_t)ny + nz + 2 * PP) * sizeof(T);
}
// the generic y-z solve holds 2^lgPP planes of ny x nz in one workgroup
template <typename T> bool yz_fits(int ny, int nz, int lgPP) {
  const long PP = 1L << lgPP;
  const long R = PP * ny * nz;
  const long Hy = (PP * nz + 1) / 2, Hz = (PP * ny + 1) / 2;
  return R <= YZ_MAX_VALUES && R <= yz_max_plane<T>() * 1L && Hy * ny <= (long)YZ_VPT * YZ_NT &&
         Hz * nz <= (long)YZ_VPT * YZ_NT && yz_lds<T>(ny, nz, lgPP) <= LDS_LIMIT;
}

template <typename T> int launch_yz_solve(const YZSolve<T>& a, int nch, hipStream_t s) {
  if (nch < 1 || nch > 3) return geom_fail("k_yz_solve: 1 to 3 channels");
  if (yz_reg_plane(a.ny, a.nz)) {
    if (a.lgTw < 8) return geom_fail("k_yz_reg: twiddle table shorter than the y axis");
    constexpr int NY = 256, NZ = 32;
    // W, y and z DCT twiddles, the [NZ/2][NY + 16] buffer, y and z eigenvalues
    const size_t lr = (2 * NY + NZ + (size_t)(NZ / 2) * (NY + 16)) * sizeof(cx<T>) + (NY + NZ) * sizeof(T);
    hipLaunchKernelGGL((k_yz_reg<T, 8, 5>), dim3(a.nx * std::max(1, a.runs), 1, nch), dim3((NZ / 2) * (NY / 16)), lr, s,
                       a);
    return SGSPM_KC_YZ_REG;
  }
  // the planes of a workgroup within the 2 YZ_VPT reals each thread holds, and each
  // pass's complex pencils within the YZ_VPT values per thread of the FFT stages
  if (a.lgPP < 0 || !yz_fits<T>(a.ny, a.nz, a.lgPP)) return geom_fail("k_yz_solve: planes beyond the tile");
  if (a.twy_s < 1 || a.twz_s < 1) return geom_fail("k_yz_solve: no twiddle stride");
  dim3 grid(ceil_div(a.nx, 1 << a.lgPP) * std::max(1, a.runs), 1, nch);
  if (a.lgNy < 0 || a.lgNz < 0)
    hipLaunchKernelGGL((k_yz_solve<T, true>), grid, dim3(YZ_NT), yz_lds<T>(a.ny, a.nz, a.lgPP), s, a);
  else
    hipLaunchKernelGGL((k_yz_solve<T, false>), grid, dim3(YZ_NT), yz_lds<T>(a.ny, a.nz, a.lgPP), s, a);
  return SGSPM_KC_YZ_SOLVE;
}

template <typename T> size_t conv_lds(int L, int lgP, int nt) {
  const size_t P = (size_t)1 << lgP;
  return ((size_t)L + 3 * P * L) * sizeof(cx<T>) + (size_t)nt * (L / 2 + 1) * P * sizeof(T);
}

template <typename T> int conv_lgP(int L, int ni, int nt) {
  // widest power-of-two kx tile whose three padded pencils fit the FFT capacity,
  // with at most two loads per component and thread, and whose LDS (spectra +
  // folded tensor tile) stays within 48 KiB; -1 when a single kx does not fit
  int lgP = -1;
  for (int nl = 0;; ++nl) {
    const long pl = (long)L << nl;
    if (3 * pl > (long)CONV_VPT * CONV_NT || pl > 2L * CONV_NT) break;
    if (conv_lds<T>(L, nl, nt) > 48 * 1024) break;
    if (nl > 0 && (1 << nl) > 2 * ni) break;
    lgP = nl;
  }
  return lgP;
}

template <typename T> int launch_conv(const Conv<T>& a, int nbatch, hipStream_t s) {
  if (a.n < 1 || a.n > a.L) return geom_fail("k_conv: pencil longer than the padded transform");
  if (a.nt < 0 || a.nt > 6) return geom_fail("k_conv: at most six tensor components");
  if (a.lgL == 6 && a.n == 32) {
    if (a.lgTw < 6) return geom_fail("k_conv64: twiddle table shorter than the transform");
    // register four-step kernel: P kx x 2 batch rows x 8 threads per pencil
    // 16 kx per workgroup in single precision, 8 in double (LDS 16 / 16 KiB)
    Conv<T> b = a;
    b.lgP = c64_lgP<T>();
    const int P = 1 << b.lgP;
    dim3 grid(ceil_div(a.ni, P), nbatch, std::max(1, a.runs));
    // W_64, the transpose buffer, the tensor tile
    const size_t lds = (64 + (size_t)64 * 2 * P) * sizeof(cx<T>) + (size_t)a.nt * 33 * P * sizeof(T);
    hipLaunchKernelGGL(k_conv64<T>, grid, dim3(16 * P), lds, s, b);
    return SGSPM_KC_CONV64;
  }
  // three components' P L values within the FFT capacity, and at most two loads
  // per component and thread
  const long pl = (long)a.L << a.lgP;
  if (a.lgP < 0 || 3 * pl > (long)CONV_VPT * CONV_NT || pl > 2L * CONV_NT) return geom_fail("k_conv: P L beyond the tile");
  if (a.twg < 1) return geom_fail("k_conv: no twiddle stride");
  if (conv_lds<T>(a.L, a.lgP, a.nt) > LDS_LIMIT) return geom_fail("k_conv: LDS beyond the limit");
  dim3 grid(ceil_div(a.ni, 1 << a.lgP), nbatch, std::max(1, a.runs));
  if (a.lgL < 0)
    hipLaunchKernelGGL((k_conv<T, true>), grid, dim3(CONV_NT), conv_lds<T>(a.L, a.lgP, a.nt), s, a);
  else
    hipLaunchKernelGGL((k_conv<T, false>), grid, dim3(CONV_NT), conv_lds<T>(a.L, a.lgP, a.nt), s, a);
  return SGSPM_KC_CONV;
}

void launch_newell_fill(double* out, int comp, int nx, int ny, int nz, int Px, int Py, int Pz, double hx, double hy,
                        double hz, int rfar, hipStream_t s) {
  const long total = (long)Px * Py * Pz;
  const int blocks = (int)std::min<long>((total + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_newell_fill, dim3(blocks), dim3(NT), 0, s, out, comp, nx, ny, nz, Px, Py, Pz, hx, hy, hz, rfar);
}

template <typename T>
void launch_tensor_pack(const cx<double>* spec, T* out, int Hz, int Hy, int Kx, int Kxp, int Kt, int Py, double scale,
                        hipStream_t s) {
  const long total = (long)Hz * Hy * Kt;
  const int blocks = (int)std::min<long>((total + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_tensor_pack<T>, dim3(blocks), dim3(NT), 0, s, spec, out, Hz, Hy, Kx, Kxp, Kt, Py, scale);
}

template <typename T>
void launch_field_assemble(const T* m, const T* hs, T* out, int nx, int ny, int nz, double cxx, double cyy, double czz,
                           double eps_on, double Q, const double he[3], hipStream_t s) {
  const long N = (long)nx * ny * nz;
  const int blocks = (int)std::min<long>((N + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_field_assemble<T>, dim3(blocks), dim3(NT), 0, s, m, hs, out, nx, ny, nz, cxx, cyy, czz, eps_on, Q,
                     he[0], he[1], he[2]);
}

template <typename T>
void launch_energy(const T* m, const T* hs, int nx, int ny, int nz, double cxx, double cyy, double czz,
                   const double he[3], double* partials, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy<T>, dim3(nblocks), dim3(NT), 0, s, m, hs, nx, ny, nz, cxx, cyy, czz, he[0], he[1], he[2],
                     partials);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(NT), 0, s, partials, nblocks, out);
}

template <typename T> void launch_pw(const PwTerm<T>* terms, int nterms, long N, hipStream_t s) {
  // a term that reads what an earlier term of the pack writes starts a new pack
  int k0 = 0;
  while (k0 < nterms) {
    int k1 = k0 + 1;
    for (; k1 < nterms; ++k1) {
      const PwTerm<T>& t = terms[k1];
      bool dep = false;
      for (int j = k0; j < k1; ++j) {
        const T* w = terms[j].out;
        dep = dep || w == t.x0 || w == t.y0 || w == t.x1 || w == t.y1 || w == t.out;
      }
      if (dep) break;
    }
    PwPack<T> A{};
    for (int k = k0; k < k1; ++k) A.t[k - k0] = terms[k];
    A.n = k1 - k0;
    hipLaunchKernelGGL(k_pw<T>, dim3(ceil_div(N, NT)), dim3(NT), 0, s, A, (int)N);
    k0 = k1;
  }
}

template <typename T> void launch_adj_project(const T* lam, const T* u, const T* nrm, T* lc, long N, hipStream_t s) {
  const int blocks = (int)std::min<long>((N + NT - 1) / NT, 8192);
  hipLaunchKernelGGL(k_adj_project<T>, dim3(blocks), dim3(NT), 0, s, lam, u, nrm, lc, N);
}

template <typename T>
void launch_wsum(const T* const x[4], const double w[4], const int slot[4], int nterms, long N, double* partials,
                 int nblocks, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_wsum<T>, dim3(nblocks), dim3(NT), 0, s, x[0], nterms > 1 ? x[1] : nullptr,
                     nterms > 2 ? x[2] : nullptr, nterms > 3 ? x[3] : nullptr, nterms, N, partials);
  hipLaunchKernelGGL(k_partials_to_grad, dim3(1), dim3(NT), 0, s, partials, nblocks, nterms, w[0], w[1], w[2], w[3],
                     slot[0], slot[1], slot[2], slot[3], grad);
}

template <typename T>
void launch_adj_damp(const T* lw, const T* u, const T* nrm, const T* const uF[3], const T* hsF, int nx, int ny,
                     int nz, double ecx, double ecy, double ecz, double Q, const double he[3], double dt, double wdh,
                     double* partials, int nblocks, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_damp<T>, dim3(nblocks), dim3(NT), 0, s, lw, u, nrm, uF[0], uF[1], uF[2], hsF, nx, ny, nz,
                     ecx, ecy, ecz, Q, he[0], he[1], he[2], partials);
  hipLaunchKernelGGL(k_partials_to_grad, dim3(1), dim3(NT), 0, s, partials, nblocks, 4, wdh, wdh, wdh, dt, 0, 1, 2, 3,
                     grad);
}

template <typename T>
void launch_rho(const T* const g[6], int nx, int ny, int nz, double kx, double ky, double kz, int sgs,
                double* partials, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rho<T>, dim3(nblocks), dim3(NT), 0, s, g[0], g[1], g[2], g[3], g[4], g[5], nx, ny, nz, kx, ky,
                     kz, sgs, partials);
  hipLaunchKernelGGL(k_rho_final, dim3(1), dim3(NT), 0, s, partials, nblocks, out);
}

template <typename T> struct FillArgs {
  T* dst;
  int n;
  T v[256];
};
template <typename T> __global__ __launch_bounds__(256) void k_fill(const FillArgs<T> a) {
  if ((int)threadIdx.x < a.n) a.dst[threadIdx.x] = a.v[threadIdx.x];
}
template <typename T> void launch_fill(T* dst, const T* values, long n, hipStream_t s) {
  for (long i0 = 0; i0 < n; i0 += 256) {
    FillArgs<T> a;
    a.dst = dst + i0;
    a.n = (int)std::min<long>(256, n - i0);
    for (int i = 0; i < a.n; ++i) a.v[i] = values[i0 + i];
    hipLaunchKernelGGL(k_fill<T>, dim3(1), dim3(256), 0, s, a);
  }
}

template <typename T> void launch_unit_error(const T* m, long N, double* partials, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_unit_error<T>, dim3(nblocks), dim3(NT), 0, s, m, N, partials);
  hipLaunchKernelGGL(k_rho_final, dim3(1), dim3(NT), 0, s, partials, nblocks, out);
}

#define SGSPM_INSTANTIATE(T)                                                                                          \
  template int launch_row_fwd<T>(const RowFwd<T>&, int, hipStream_t);                                              \
  template int launch_row_inv<T>(const RowInv<T>&, hipStream_t);                                                   \
  template int launch_col_dct<T>(const ColDct<T>&, int, int, hipStream_t);                                         \
  template int launch_col_fft<T>(const ColFft<T>&, int, int, hipStream_t);                                         \
  template int launch_conv<T>(const Conv<T>&, int, hipStream_t);                                                   \
  template int conv_lgP<T>(int, int, int);                                                                          \
  template bool yz_fits<T>(int, int, int);                                                                          \
  template int launch_yz_solve<T>(const YZSolve<T>&, int, hipStream_t);                                            \
  template void launch_tensor_pack<T>(const cx<double>*, T*, int, int, int, int, int, int, double, hipStream_t);    \
  template void launch_field_assemble<T>(const T*, const T*, T*, int, int, int, double, double, double, double,    \
                                         double, const double*, hipStream_t);                                       \
  template void launch_energy<T>(const T*, const T*, int, int, int, double, double, double, const double*, double*, \
                                 int, double*, hipStream_t);                                                       \
  template void launch_pw<T>(const PwTerm<T>*, int, long, hipStream_t);                                             \
  template void launch_adj_project<T>(const T*, const T*, const T*, T*, long, hipStream_t);                         \
  template void launch_wsum<T>(const T* const*, const double*, const int*, int, long, double*, int, double*,        \
                               hipStream_t);                                                                        \
  template void launch_adj_damp<T>(const T*, const T*, const T*, const T* const*, const T*, int, int, int, double,  \
                                   double, double, double, const double*, double, double, double*, int, double*,   \
                                   hipStream_t);                                                                    \
  template void launch_rho<T>(const T* const*, int, int, int, double, double, double, int, double*, int, double*,   \
                              hipStream_t);                                                                         \
  template void launch_unit_error<T>(const T*, long, double*, int, double*, hipStream_t);                          \
  template void launch_fill<T>(T*, const T*, long, hipStream_t);

SGSPM_INSTANTIATE(float)
SGSPM_INSTANTIATE(double)

}  // namespace sgspm
