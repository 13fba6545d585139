// In-LDS complex FFT engine for gfx950 (wave64, 256-thread workgroups).
//
// A workgroup holds a tile of pencils in LDS and transforms all of them along
// their length L = 2^lgL with self-sorting Stockham stages (radix 8, plus one
// radix-4 or radix-2 stage when lgL is not a multiple of 3).  Every stage is
// done in place: each thread loads its butterflies into registers, the group
// synchronises, then every thread stores its results.  Each thread owns at
// most VPT complex values per stage, so a tile holds at most VPT * NT values.
//
// Layout of element j of pencil p in the LDS buffer: buf[p * ps + j * es].
// Pencils are numbered p = c * P + q with q < P = 2^lgP and c < ncomp, which
// lets one call transform several equally sized groups (e.g. the three
// magnetisation components) that share a buffer.  With pf (pencil-fastest)
// consecutive threads take consecutive pencils (for element-major layouts,
// ps = 1), otherwise consecutive elements of one pencil (pencil-major, es = 1).
//
// Twiddles: tw[i] = exp(-2 pi i i / Ltw) in LDS with Ltw = L << twshift; an
// inverse transform conjugates them (unnormalised in both directions).
#pragma once
#include <hip/hip_runtime.h>

namespace sgspm {

constexpr int NT = 256;

template <typename T> struct cx { T x, y; };

template <typename T> struct Tile;
template <> struct Tile<float> { static constexpr int VPT = 16; };
template <> struct Tile<double> { static constexpr int VPT = 8; };
template <typename T> constexpr int tile_elems() { return Tile<T>::VPT * NT; }

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by -i (forward sign) or +i (inverse sign)
template <typename T> __device__ __forceinline__ cx<T> rot(cx<T> a, bool inv) {
  return inv ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

template <typename T> __device__ __forceinline__ void dft2(cx<T>* v, bool) {
  cx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T> __device__ __forceinline__ void dft4v(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3, bool inv) {
  cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = rot(a1 - a3, inv);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <typename T> __device__ __forceinline__ void dft4(cx<T>* v, bool inv) { dft4v(v[0], v[1], v[2], v[3], inv); }

template <typename T> __device__ __forceinline__ void dft8(cx<T>* v, bool inv) {
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4v(e0, e1, e2, e3, inv);
  dft4v(o0, o1, o2, o3, inv);
  const T s = (T)0.70710678118654752440084436210485;
  // o_k times W_8^{+-k}
  cx<T> w1 = inv ? mk(s * (o1.x - o1.y), s * (o1.x + o1.y)) : mk(s * (o1.x + o1.y), s * (o1.y - o1.x));
  cx<T> w2 = rot(o2, inv);
  cx<T> w3 = inv ? mk(-s * (o3.x + o3.y), s * (o3.x - o3.y)) : mk(s * (o3.y - o3.x), -s * (o3.x + o3.y));
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + w1;
  v[5] = e1 - w1;
  v[2] = e2 + w2;
  v[6] = e2 - w2;
  v[3] = e3 + w3;
  v[7] = e3 - w3;
}

// v * W_32^e (conjugated for the inverse) for a compile-time exponent e
template <typename T, int E> __device__ __forceinline__ cx<T> tw32(cx<T> a, bool inv) {
  constexpr int e = E & 31;
  if constexpr (e == 0) return a;
  else if constexpr (e == 8) return rot(a, inv);
  else if constexpr (e == 16) return mk(-a.x, -a.y);
  else if constexpr (e == 24) return rot(a, !inv);
  else {
    // cos and sin of pi e / 16, built from cos and sin of pi/16, 2 pi/16, 3 pi/16, 4 pi/16
    constexpr double C1 = 0.98078528040323044912618223613424163, S1 = 0.19509032201612826784828486847702224;
    constexpr double C2 = 0.92387953251128675612818318939678829, S2 = 0.38268343236508977172845998403039887;
    constexpr double C3 = 0.83146961230254523707878837761790760, S3 = 0.55557023301960222474283081394853288;
    constexpr double R2 = 0.70710678118654752440084436210484904;
    constexpr double cq[9] = {1, C1, C2, C3, R2, S3, S2, S1, 0};  // cos(pi q / 16), q = 0..8
    constexpr int q = e & 15;
    constexpr double c0 = q <= 8 ? cq[q] : -cq[16 - q];
    constexpr double s0 = q <= 8 ? cq[8 - q] : cq[q - 8];
    constexpr double c = e < 16 ? c0 : -c0;
    constexpr double sn = e < 16 ? s0 : -s0;
    const T cr = (T)c;
    const T sg = inv ? (T)sn : (T)-sn;
    return mk(a.x * cr - a.y * sg, a.x * sg + a.y * cr);
  }
}
template <typename T, int E> __device__ __forceinline__ cx<T> tw16(cx<T> a, bool inv) { return tw32<T, 2 * E>(a, inv); }
// v * W_32^e for an exponent that is a compile-time constant once the caller's
// loop is unrolled (table lookups then fold into literals)
template <typename T> __device__ __forceinline__ cx<T> tw32v(cx<T> a, int e, bool inv) {
  constexpr double C1 = 0.98078528040323044912618223613424163, S1 = 0.19509032201612826784828486847702224;
  constexpr double C2 = 0.92387953251128675612818318939678829, S2 = 0.38268343236508977172845998403039887;
  constexpr double C3 = 0.83146961230254523707878837761790760, S3 = 0.55557023301960222474283081394853288;
  constexpr double R2 = 0.70710678118654752440084436210484904;
  constexpr double cq[9] = {1, C1, C2, C3, R2, S3, S2, S1, 0};
  e &= 31;
  if (e == 0) return a;
  if (e == 8) return rot(a, inv);
  if (e == 16) return mk(-a.x, -a.y);
  if (e == 24) return rot(a, !inv);
  const int q = e & 15;
  const double c0 = q <= 8 ? cq[q] : -cq[16 - q];
  const double s0 = q <= 8 ? cq[8 - q] : cq[q - 8];
  const T cr = (T)(e < 16 ? c0 : -c0);
  const T sn = (T)(e < 16 ? s0 : -s0);
  const T sg = inv ? sn : -sn;
  return mk(a.x * cr - a.y * sg, a.x * sg + a.y * cr);
}


// 16-point DFT in registers (4 x 4): natural order in and out
template <typename T> __device__ __forceinline__ void dft16(cx<T>* v, bool inv) {
  cx<T> u[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    cx<T> a0 = v[n1], a1 = v[n1 + 4], a2 = v[n1 + 8], a3 = v[n1 + 12];
    dft4v(a0, a1, a2, a3, inv);
    u[4 * n1] = a0;
    u[4 * n1 + 1] = a1;
    u[4 * n1 + 2] = a2;
    u[4 * n1 + 3] = a3;
  }
  u[5] = tw16<T, 1>(u[5], inv);
  u[6] = tw16<T, 2>(u[6], inv);
  u[7] = tw16<T, 3>(u[7], inv);
  u[9] = tw16<T, 2>(u[9], inv);
  u[10] = tw16<T, 4>(u[10], inv);
  u[11] = tw16<T, 6>(u[11], inv);
  u[13] = tw16<T, 3>(u[13], inv);
  u[14] = tw16<T, 6>(u[14], inv);
  u[15] = tw16<T, 9>(u[15], inv);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a0 = u[k1], a1 = u[4 + k1], a2 = u[8 + k1], a3 = u[12 + k1];
    dft4v(a0, a1, a2, a3, inv);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

// 16-point DFT of a sequence whose entries 8..15 are zero (natural order out)
template <typename T> __device__ __forceinline__ void dft16_lo8(cx<T>* v, bool inv) {
  cx<T> u[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    const cx<T> a0 = v[n1], r1 = rot(v[n1 + 4], inv);
    u[4 * n1] = a0 + v[n1 + 4];
    u[4 * n1 + 1] = a0 + r1;
    u[4 * n1 + 2] = a0 - v[n1 + 4];
    u[4 * n1 + 3] = a0 - r1;
  }
  u[5] = tw16<T, 1>(u[5], inv);
  u[6] = tw16<T, 2>(u[6], inv);
  u[7] = tw16<T, 3>(u[7], inv);
  u[9] = tw16<T, 2>(u[9], inv);
  u[10] = tw16<T, 4>(u[10], inv);
  u[11] = tw16<T, 6>(u[11], inv);
  u[13] = tw16<T, 3>(u[13], inv);
  u[14] = tw16<T, 6>(u[14], inv);
  u[15] = tw16<T, 9>(u[15], inv);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a0 = u[k1], a1 = u[4 + k1], a2 = u[8 + k1], a3 = u[12 + k1];
    dft4v(a0, a1, a2, a3, inv);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

// 32-point DFT in registers (even / odd halves), natural order
template <typename T, int K = 0> __device__ __forceinline__ void dft32_merge(cx<T>* v, const cx<T>* e, const cx<T>* o,
                                                                             bool inv) {
  if constexpr (K < 16) {
    const cx<T> t = tw32<T, K>(o[K], inv);
    v[K] = e[K] + t;
    v[K + 16] = e[K] - t;
    dft32_merge<T, K + 1>(v, e, o, inv);
  }
}
template <typename T> __device__ __forceinline__ void dft32(cx<T>* v, bool inv) {
  cx<T> e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft16(e, inv);
  dft16(o, inv);
  dft32_merge<T>(v, e, o, inv);
}

// N-point DFT in registers, natural order, N <= 32 a power of two
template <typename T, int N> __device__ __forceinline__ void dft_reg(cx<T>* v, bool inv) {
  if constexpr (N == 2) dft2(v, inv);
  else if constexpr (N == 4) dft4(v, inv);
  else if constexpr (N == 8) dft8(v, inv);
  else if constexpr (N == 16) dft16(v, inv);
  else if constexpr (N == 32) dft32(v, inv);
}

// 8-point DFT of a sequence whose entries 4..7 are zero (natural order out)
template <typename T> __device__ __forceinline__ void dft8_lo4(cx<T>* v, bool inv) {
  const cx<T> r2 = rot(v[2], inv), r3 = rot(v[3], inv);
  const cx<T> e0 = v[0] + v[2], e1 = v[0] + r2, e2 = v[0] - v[2], e3 = v[0] - r2;
  cx<T> o0 = v[1] + v[3], o1 = v[1] + r3, o2 = v[1] - v[3], o3 = v[1] - r3;
  const T s = (T)0.70710678118654752440084436210485;
  const cx<T> w1 = inv ? mk(s * (o1.x - o1.y), s * (o1.x + o1.y)) : mk(s * (o1.x + o1.y), s * (o1.y - o1.x));
  const cx<T> w2 = rot(o2, inv);
  const cx<T> w3 = inv ? mk(-s * (o3.x + o3.y), s * (o3.x - o3.y)) : mk(s * (o3.y - o3.x), -s * (o3.x + o3.y));
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + w1;
  v[5] = e1 - w1;
  v[2] = e2 + w2;
  v[6] = e2 - w2;
  v[3] = e3 + w3;
  v[7] = e3 - w3;
}

// outputs 0..3 of an 8-point DFT (entries 4..7 of v are left undefined)
template <typename T> __device__ __forceinline__ void dft8_first4(cx<T>* v, bool inv) {
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4v(e0, e1, e2, e3, inv);
  dft4v(o0, o1, o2, o3, inv);
  const T s = (T)0.70710678118654752440084436210485;
  const cx<T> w1 = inv ? mk(s * (o1.x - o1.y), s * (o1.x + o1.y)) : mk(s * (o1.x + o1.y), s * (o1.y - o1.x));
  const cx<T> w2 = rot(o2, inv);
  const cx<T> w3 = inv ? mk(-s * (o3.x + o3.y), s * (o3.x - o3.y)) : mk(s * (o3.y - o3.x), -s * (o3.x + o3.y));
  v[0] = e0 + o0;
  v[1] = e1 + w1;
  v[2] = e2 + w2;
  v[3] = e3 + w3;
}

template <typename T, int R> __device__ __forceinline__ void dftR(cx<T>* v, bool inv) {
  if constexpr (R == 2) dft2(v, inv);
  else if constexpr (R == 4) dft4(v, inv);
  else dft8(v, inv);
}

template <int R> struct Lg;
template <> struct Lg<2> { static constexpr int v = 1; };
template <> struct Lg<4> { static constexpr int v = 2; };
template <> struct Lg<8> { static constexpr int v = 3; };

// Geometry of one FFT call.
struct FftGeom {
  int lgL;    // transform length 2^lgL
  int lgP;    // pencils per group 2^lgP
  int ncomp;  // number of groups
  bool pf;    // pencil-fastest thread mapping
  int ps, es; // LDS strides of pencil and element
  int twshift;
};

template <typename T, int R, int VPT, int NTH>
__device__ __forceinline__ void fft_stage(cx<T>* __restrict__ buf, const cx<T>* __restrict__ tw, const FftGeom& g,
                                          int Ns, bool inv) {
  constexpr int NB = VPT / R;
  constexpr int lgR = Lg<R>::v;
  const int lgLR = g.lgL - lgR;
  const int LR = 1 << lgLR;
  const int total = (g.ncomp << g.lgP) << lgLR;
  cx<T> v[NB][R];
  int dst[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * NTH;
    dst[i] = -1;
    if (b < total) {
      int p, j;
      if (g.pf) {
        const int q = b & ((1 << g.lgP) - 1);
        const int rest = b >> g.lgP;
        j = rest & (LR - 1);
        p = ((rest >> lgLR) << g.lgP) + q;
      } else {
        j = b & (LR - 1);
        p = b >> lgLR;
      }
      const int k = j & (Ns - 1);
      const int base = p * g.ps;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[base + (j + r * LR) * g.es];
      if (Ns > 1) {
        // W_{Ns R}^{r k} = W_L^{r k L / (Ns R)}
        const int stp = (LR / Ns) << g.twshift;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * stp];
          if (inv) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      dftR<T, R>(v[i], inv);
      dst[i] = base + ((j - k) * R + k) * g.es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (dst[i] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[i] + r * Ns * g.es] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform; the caller has synchronised after filling buf.  A workgroup
// of NTH threads holds at most VPT * NTH values per stage.
template <typename T, int VPT = Tile<T>::VPT, int NTH = NT>
__device__ __forceinline__ void fft_lds(cx<T>* __restrict__ buf, const cx<T>* __restrict__ tw, const FftGeom& g,
                                        bool inv) {
  int Ns = 1;
  int rem = g.lgL;
  if (rem % 3 == 1) {
    fft_stage<T, 2, VPT, NTH>(buf, tw, g, Ns, inv);
    Ns <<= 1;
    rem -= 1;
  } else if (rem % 3 == 2) {
    fft_stage<T, 4, VPT, NTH>(buf, tw, g, Ns, inv);
    Ns <<= 2;
    rem -= 2;
  }
  while (rem > 0) {
    fft_stage<T, 8, VPT, NTH>(buf, tw, g, Ns, inv);
    Ns <<= 3;
    rem -= 3;
  }
}

// Copy the length-2^lgL twiddle table (from a global table of length 2^lgTw) into LDS.
template <typename T, int NTH = NT>
__device__ __forceinline__ void load_twiddles(cx<T>* __restrict__ lds, const cx<T>* __restrict__ gtw, int lgL, int lgTw) {
  const int L = 1 << lgL;
  const int sh = lgTw - lgL;
  for (int i = threadIdx.x; i < L; i += NTH) lds[i] = gtw[i << sh];
}

// Makhoul's reordering for the DCT-II through a length-n FFT:
// element x goes to v[x/2] if x is even, to v[n - 1 - (x-1)/2] if odd.
__device__ __forceinline__ int makhoul_pos(int x, int n) { return (x & 1) ? (n - 1 - (x >> 1)) : (x >> 1); }

}  // namespace sgspm
