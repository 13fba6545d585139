// In-LDS complex FFT engine for gfx950 (wave64, 256-thread workgroups).
//
// A workgroup holds a tile of pencils in LDS and transforms all of them along
// their length L = 2^a 3^b 5^c with self-sorting Stockham stages (radix 8, one
// radix-4 or radix-2 stage when a is not a multiple of 3, then radix 5 and
// radix 3).  Every stage is done in place: each thread loads its butterflies
// into registers, the group synchronises, then every thread stores its
// results.  Each thread owns ceil(VPT / R) butterflies of a radix-R stage
// (VPT complex values for the power-of-two radices, a few more for 3 and 5),
// so a tile holds at most VPT * NT values.
//
// Layout of element j of pencil p in the LDS buffer: buf[p * ps + j * es].
// Pencils are numbered p = c * P + q with q < P = 2^lgP and c < ncomp, which
// lets one call transform several equally sized groups (e.g. the three
// magnetisation components) that share a buffer.  With pf (pencil-fastest)
// consecutive threads take consecutive pencils (for element-major layouts,
// ps = 1), otherwise consecutive elements of one pencil (pencil-major, es = 1).
//
// Twiddles: tw[i] = exp(-2 pi i i / Ltw) in LDS with Ltw = L * tws; an
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

// 3- and 5-point DFTs (forward sign e^{-2 pi i / R}; the inverse conjugates)
template <typename T> __device__ __forceinline__ void dft3(cx<T>* v, bool inv) {
  const T h = (T)0.86602540378443864676372317075294;  // sin(2 pi / 3)
  const cx<T> a = v[0], t1 = v[1] + v[2];
  const cx<T> t2 = mk<T>(a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y);
  const cx<T> d = rot(v[1] - v[2], inv);
  const cx<T> t3 = mk<T>(h * d.x, h * d.y);
  v[0] = a + t1;
  v[1] = t2 + t3;
  v[2] = t2 - t3;
}

template <typename T> __device__ __forceinline__ void dft5(cx<T>* v, bool inv) {
  // cos and sin of 2 pi / 5 and 4 pi / 5
  const T c1 = (T)0.30901699437494742410229341718282, c2 = (T)-0.80901699437494742410229341718282;
  const T s1 = (T)0.95105651629515357211643933337938, s2 = (T)0.58778525229247312916870595463907;
  const cx<T> x0 = v[0];
  const cx<T> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
  const cx<T> a1 = mk<T>(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
  const cx<T> a2 = mk<T>(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
  const cx<T> b1 = rot(mk<T>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y), inv);
  const cx<T> b2 = rot(mk<T>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y), inv);
  v[0] = x0 + t1 + t2;
  v[1] = a1 + b1;
  v[4] = a1 - b1;
  v[2] = a2 + b2;
  v[3] = a2 - b2;
}

template <typename T, int R> __device__ __forceinline__ void dftR(cx<T>* v, bool inv) {
  if constexpr (R == 2) dft2(v, inv);
  else if constexpr (R == 3) dft3(v, inv);
  else if constexpr (R == 4) dft4(v, inv);
  else if constexpr (R == 5) dft5(v, inv);
  else dft8(v, inv);
}

// Quotient and remainder by a runtime divisor d = 2^lgd (MX false: every length
// of the launch is a power of two) or any d, by shifts when lgd >= 0 (MX true).
template <bool MX> __host__ __device__ __forceinline__ int qdiv(int a, int d, int lgd) {
  if constexpr (!MX) return a >> lgd;
  else return lgd >= 0 ? a >> lgd : a / d;
}
template <bool MX> __host__ __device__ __forceinline__ int qmod(int a, int d, int lgd) {
  if constexpr (!MX) return a & (d - 1);
  else return lgd >= 0 ? (a & (d - 1)) : a % d;
}

// log2 of n if n is a power of two, else -1
__host__ __device__ __forceinline__ int lg_or_neg(int n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Geometry of one FFT call.
struct FftGeom {
  int L;      // transform length, a product of 2, 3 and 5
  int lgL;    // log2 L when L is a power of two, else -1
  int lgP;    // pencils per group 2^lgP
  int ncomp;  // number of groups
  bool pf;    // pencil-fastest thread mapping
  int ps, es; // LDS strides of pencil and element
  int tws;    // twiddle stride: the LDS table holds W_{L tws}^i
};

// Each thread takes ceil(VPT / R) butterflies of a radix-R stage, so a tile of
// VPT * NTH complex values fits every stage whatever the radices.
template <typename T, int R, int VPT, int NTH, bool MX>
__device__ __forceinline__ void fft_stage(cx<T>* __restrict__ buf, const cx<T>* __restrict__ tw, const FftGeom& g,
                                          int Ns, int lgNs, bool inv) {
  constexpr int NB = (VPT + R - 1) / R;
  const int LR = g.L / R;
  const int lgLR = g.lgL >= 0 ? g.lgL - (R == 2 ? 1 : R == 4 ? 2 : 3) : -1;
  const int total = (g.ncomp << g.lgP) * LR;
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
        j = qmod<MX>(rest, LR, lgLR);
        p = (qdiv<MX>(rest, LR, lgLR) << g.lgP) + q;
      } else {
        j = qmod<MX>(b, LR, lgLR);
        p = qdiv<MX>(b, LR, lgLR);
      }
      const int k = qmod<MX>(j, Ns, lgNs);
      const int base = p * g.ps;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[base + (j + r * LR) * g.es];
      if (Ns > 1) {
        // W_{Ns R}^{r k} = W_L^{r k L / (Ns R)}
        const int stp = qdiv<MX>(LR, Ns, lgNs) * g.tws;
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
// of NTH threads holds at most VPT * NTH values.  Stages: the
// power-of-two part (one radix-2 or radix-4 stage, then radix 8), then radix 5,
// then radix 3 (self-sorting Stockham, any order of radices).  MX false compiles
// the power-of-two stages only (L must then be a power of two).
template <typename T, int VPT = Tile<T>::VPT, int NTH = NT, bool MX = false>
__device__ __forceinline__ void fft_lds(cx<T>* __restrict__ buf, const cx<T>* __restrict__ tw, const FftGeom& g,
                                        bool inv) {
  int Ns = 1, lgNs = 0;
  int m = g.L, e2 = 0;
  if constexpr (MX) {
    while (!(m & 1)) {
      m >>= 1;
      ++e2;
    }
  } else {
    e2 = g.lgL;
  }
  if (e2 % 3 == 1) {
    fft_stage<T, 2, VPT, NTH, MX>(buf, tw, g, Ns, lgNs, inv);
    Ns <<= 1;
    ++lgNs;
    e2 -= 1;
  } else if (e2 % 3 == 2) {
    fft_stage<T, 4, VPT, NTH, MX>(buf, tw, g, Ns, lgNs, inv);
    Ns <<= 2;
    lgNs += 2;
    e2 -= 2;
  }
  while (e2 > 0) {
    fft_stage<T, 8, VPT, NTH, MX>(buf, tw, g, Ns, lgNs, inv);
    Ns <<= 3;
    lgNs += 3;
    e2 -= 3;
  }
  if constexpr (MX) {
    while (m % 5 == 0) {
      fft_stage<T, 5, VPT, NTH, MX>(buf, tw, g, Ns, -1, inv);
      Ns *= 5;
      m /= 5;
    }
    while (m % 3 == 0) {
      fft_stage<T, 3, VPT, NTH, MX>(buf, tw, g, Ns, -1, inv);
      Ns *= 3;
      m /= 3;
    }
  }
}

// Copy the twiddles W_L^i, i < L, into LDS from a global table whose entry
// i * stride is W_L^i.
template <typename T, int NTH = NT>
__device__ __forceinline__ void load_twiddles(cx<T>* __restrict__ lds, const cx<T>* __restrict__ gtw, int L, int stride) {
  for (int i = threadIdx.x; i < L; i += NTH) lds[i] = gtw[i * stride];
}

// Makhoul's reordering for the DCT-II through a length-n FFT:
// element x goes to v[x/2] if x is even, to v[n - 1 - (x-1)/2] if odd.
__device__ __forceinline__ int makhoul_pos(int x, int n) { return (x & 1) ? (n - 1 - (x >> 1)) : (x >> 1); }

}  // namespace sgspm
