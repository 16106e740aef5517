// Device-side building blocks of the even-odd Wilson-Dirac library for gfx950:
// packed layouts, link decompression, the spin-projected 8-neighbour hop and
// deterministic wave/grid reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace qiral {

constexpr int WAVE = 64;   // CDNA wavefront; also the site-block of the packed layouts
constexpr int WG = 256;    // work-group: 4 waves
// Minimum waves per SIMD asked of the compiler for a hop kernel (storage S, T
// waves per site block, NR right-hand sides per lane): caps the VGPR budget at
// 512 / waves so enough waves stay resident to cover memory latency, while
// leaving the larger NR / smaller T variants room to avoid spilling (the FP64
// 1-RHS hops spill at 128).
#define HOP_MIN_WAVES(S, T, NR) ((S) == 0 ? ((NR) == 1 ? 3 : 2) : (NR) == 1 ? ((T) == 4 ? 4 : 3) : (NR) == 2 ? ((T) == 4 ? 3 : 2) : 2)

// ---------------------------------------------------------------------------
// Lattice geometry of one parity-checkerboarded lattice.
// Sites of one parity are numbered by the checkerboard index
// s = lex(x,y,z,t) >> 1 with lex = ((t*Lz + z)*Ly + y)*Lx + x (x fastest).
struct Geo {
  int lx, ly, lz, lt;
  int lxh;     // Lx / 2
  int vh;      // sites per parity
  int nb;      // 64-site blocks per parity (vh rounded up)
  int sy, sz, st;  // checkerboard-index strides of y, z, t
  double rlxh, rly, rlz;   // 1 / (Lx/2), 1 / Ly, 1 / Lz for the coordinate divisions
};

inline Geo make_geo(const int32_t d[4]) {
  Geo g;
  g.lx = d[0]; g.ly = d[1]; g.lz = d[2]; g.lt = d[3];
  g.lxh = d[0] / 2;
  g.vh = (int)((int64_t)d[0] * d[1] * d[2] * d[3] / 2);
  g.nb = (g.vh + WAVE - 1) / WAVE;
  g.sy = g.lxh; g.sz = g.lxh * g.ly; g.st = g.sz * g.lz;
  g.rlxh = 1.0 / g.lxh; g.rly = 1.0 / g.ly; g.rlz = 1.0 / g.lz;
  return g;
}

// ---------------------------------------------------------------------------
// Complex arithmetic
template <class R> struct cpx { R re, im; };

template <class R> __device__ __forceinline__ cpx<R> cmake(R a, R b) { cpx<R> c; c.re = a; c.im = b; return c; }
template <class R> __device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return cmake(a.re + b.re, a.im + b.im); }
template <class R> __device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return cmake(a.re - b.re, a.im - b.im); }
template <class R> __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return cmake(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// conj(a) * b
template <class R> __device__ __forceinline__ cpx<R> cjmul(cpx<R> a, cpx<R> b) {
  return cmake(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class R> __device__ __forceinline__ cpx<R> cscale(R s, cpx<R> a) { return cmake(s * a.re, s * a.im); }
// s * a + b (FP32), one rounding per part
__device__ __forceinline__ cpx<float> cfma(float s, cpx<float> a, cpx<float> b) {
  return cmake(__builtin_fmaf(s, a.re, b.re), __builtin_fmaf(s, a.im, b.im));
}
__device__ __forceinline__ float rfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double rfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a * b + c and conj(a) * b + c as chains of fused multiply-adds (4 per
// complex product; the compiler does not fuse an add into a product's result)
template <class R> __device__ __forceinline__ cpx<R> cmac(cpx<R> a, cpx<R> b, cpx<R> c) {
  return cmake(rfma(a.re, b.re, rfma(-a.im, b.im, c.re)), rfma(a.re, b.im, rfma(a.im, b.re, c.im)));
}
template <class R> __device__ __forceinline__ cpx<R> cjmac(cpx<R> a, cpx<R> b, cpx<R> c) {
  return cmake(rfma(a.re, b.re, rfma(a.im, b.im, c.re)), rfma(a.re, b.im, rfma(-a.im, b.re, c.im)));
}
template <class R> __device__ __forceinline__ cpx<R> cneg(cpx<R> a) { return cmake(-a.re, -a.im); }
// multiply by +i and -i
template <class R> __device__ __forceinline__ cpx<R> ci(cpx<R> a) { return cmake(-a.im, a.re); }
template <class R> __device__ __forceinline__ cpx<R> cmi(cpx<R> a) { return cmake(a.im, -a.re); }

// ---------------------------------------------------------------------------
// Packed spinor half-fields.  Blocks of 64 sites; inside a block, "unit" j of
// lane l sits at ((block * UNITS + j) * 64 + l), so a wavefront reads each unit
// of 64 consecutive sites as one contiguous, fully coalesced segment.
//   F64 : unit = 16 B = one complex128,         12 units per site
//   F32 : unit = 16 B = two complex64,            6 units
//   F16S: unit = 16 B = four complex FP16,        3 units, then one FP32 scale
//         per site stored after all units of the half-field.
// Component order inside a site is k = 4 * colour + spin.
enum { S_F64 = 0, S_F32 = 1, S_F16S = 2 };

// Non-temporal (streaming) 16- and 8-byte accesses: data read or written once
// per launch (links, hop outputs) is marked so that it does not displace the
// neighbour spinors that other sites re-read from L2.  Used only when a hop's
// working set exceeds the last-level cache (otherwise the streaming hint keeps
// links and outputs from staying cached between launches, which costs more).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 ld_nt(const float4 *p) {
  const f32x4 v = __builtin_nontemporal_load((const f32x4 *)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
  const f64x2 v = __builtin_nontemporal_load((const f64x2 *)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ uint2 ld_nt(const uint2 *p) {
  const u32x2 v = __builtin_nontemporal_load((const u32x2 *)p);
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(float4 *p, float4 v) {
  f32x4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, (f32x4 *)p);
}
__device__ __forceinline__ void st_nt(double2 *p, double2 v) {
  f64x2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, (f64x2 *)p);
}
__device__ __forceinline__ void st_nt(uint4 *p, uint4 v) {
  u32x4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, (u32x4 *)p);
}
__device__ __forceinline__ void st_nt(float *p, float v) { __builtin_nontemporal_store(v, p); }

template <int S> struct SpinorIO;

template <> struct SpinorIO<S_F64> {
  using R = double;
  static constexpr int UNITS = 12;
  static constexpr size_t SITE_BYTES = 192;
  struct Raw { double2 q[12]; };
  __device__ static void fetch(const void *base, int s, size_t npad, Raw &r) {
    (void)npad;
    const double2 *p = (const double2 *)base + (size_t)(s >> 6) * (12 * WAVE) + (s & 63);
#pragma unroll
    for (int k = 0; k < 12; ++k) r.q[k] = p[k * WAVE];
  }
  __device__ static void decode(const Raw &r, cpx<double> v[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = cmake(r.q[k].x, r.q[k].y);
  }
  __device__ static void load(const void *base, int s, size_t npad, cpx<double> v[12]) {
    Raw r;
    fetch(base, s, npad, r);
    decode(r, v);
  }
  __device__ static void store(void *base, int s, size_t npad, const cpx<double> v[12]) {
    (void)npad;
    double2 *p = (double2 *)base + (size_t)(s >> 6) * (12 * WAVE) + (s & 63);
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k * WAVE] = make_double2(v[k].re, v[k].im);
  }
  template <bool NT = false>
  __device__ static void store_fast(void *base, int s, size_t npad, const cpx<double> v[12]) {
    if (!NT) return store(base, s, npad, v);
    double2 *p = (double2 *)base + (size_t)(s >> 6) * (12 * WAVE) + (s & 63);
#pragma unroll
    for (int k = 0; k < 12; ++k) st_nt(p + k * WAVE, make_double2(v[k].re, v[k].im));
  }
};

template <> struct SpinorIO<S_F32> {
  using R = float;
  static constexpr int UNITS = 6;
  static constexpr size_t SITE_BYTES = 96;
  struct Raw { float4 q[6]; };
  __device__ static void fetch(const void *base, int s, size_t npad, Raw &r) {
    (void)npad;
    const float4 *p = (const float4 *)base + (size_t)(s >> 6) * (6 * WAVE) + (s & 63);
#pragma unroll
    for (int j = 0; j < 6; ++j) r.q[j] = p[j * WAVE];
  }
  __device__ static void decode(const Raw &r, cpx<float> v[12]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      v[2 * j] = cmake(r.q[j].x, r.q[j].y);
      v[2 * j + 1] = cmake(r.q[j].z, r.q[j].w);
    }
  }
  __device__ static void load(const void *base, int s, size_t npad, cpx<float> v[12]) {
    Raw r;
    fetch(base, s, npad, r);
    decode(r, v);
  }
  __device__ static void store(void *base, int s, size_t npad, const cpx<float> v[12]) {
    (void)npad;
    float4 *p = (float4 *)base + (size_t)(s >> 6) * (6 * WAVE) + (s & 63);
#pragma unroll
    for (int j = 0; j < 6; ++j) p[j * WAVE] = make_float4(v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im);
  }
  template <bool NT = false>
  __device__ static void store_fast(void *base, int s, size_t npad, const cpx<float> v[12]) {
    if (!NT) return store(base, s, npad, v);
    float4 *p = (float4 *)base + (size_t)(s >> 6) * (6 * WAVE) + (s & 63);
#pragma unroll
    for (int j = 0; j < 6; ++j) st_nt(p + j * WAVE, make_float4(v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im));
  }
};

__device__ __forceinline__ float h2f(unsigned short h) { return __half2float(__ushort_as_half(h)); }
__device__ __forceinline__ unsigned short f2h(float f) { return __half_as_ushort(__float2half_rn(f)); }

// FP64 -> FP16 with one rounding to nearest even.  Going through FP32 with
// ordinary rounding would round twice (1 + 2^-11 + 2^-30 would become 1 instead
// of 1 + 2^-10).  Rounding to FP32 "to odd" first -- toward zero, then setting
// the last bit if the conversion was inexact -- and then to FP16 to nearest
// gives the directly rounded result, because FP32 keeps at least two more bits
// than FP16 (Boldo and Melquiond, IEEE Trans. Computers 57 (2008) 462).
__device__ __forceinline__ unsigned short d2h(double d) {
  float f = __double2float_rz(d);
  if ((double)f != d) f = __uint_as_float(__float_as_uint(f) | 1u);
  return f2h(f);
}


template <> struct SpinorIO<S_F16S> {
  using R = float;
  static constexpr int UNITS = 3;
  static constexpr size_t SITE_BYTES = 52;
  __device__ static float *scale_ptr(const void *base, size_t npad) {
    return (float *)((char *)base + npad * 48);
  }
  __device__ static void load(const void *base, int s, size_t npad, cpx<float> v[12]) {
    const uint4 *p = (const uint4 *)base + (size_t)(s >> 6) * (3 * WAVE) + (s & 63);
    const float sc = scale_ptr(base, npad)[s];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      uint4 q = p[j * WAVE];
      unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int c = 0; c < 4; ++c)
        v[4 * j + c] = cmake(h2f((unsigned short)(w[c] & 0xffffu)) * sc, h2f((unsigned short)(w[c] >> 16)) * sc);
    }
  }
  // The stored FP16 values, unscaled, and the site's scale: the value is sc * v.
  struct Raw { uint4 q[3]; float sc; };
  __device__ static void fetch(const void *base, int s, size_t npad, Raw &r) {
    const uint4 *p = (const uint4 *)base + (size_t)(s >> 6) * (3 * WAVE) + (s & 63);
#pragma unroll
    for (int j = 0; j < 3; ++j) r.q[j] = p[j * WAVE];
    r.sc = scale_ptr(base, npad)[s];
  }
  __device__ static void decode_raw(const Raw &r, cpx<float> v[12], float &sc) {
    sc = r.sc;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      unsigned w[4] = {r.q[j].x, r.q[j].y, r.q[j].z, r.q[j].w};
#pragma unroll
      for (int c = 0; c < 4; ++c)
        v[4 * j + c] = cmake(h2f((unsigned short)(w[c] & 0xffffu)), h2f((unsigned short)(w[c] >> 16)));
    }
  }
  __device__ static void load_raw(const void *base, int s, size_t npad, cpx<float> v[12], float &sc) {
    Raw r;
    fetch(base, s, npad, r);
    decode_raw(r, v, sc);
  }
  // Quantise: scale = max |real| over the site's 24 reals, half = RNE(real / scale).
  __device__ static void store(void *base, int s, size_t npad, const cpx<float> v[12]) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
    uint4 *p = (uint4 *)base + (size_t)(s >> 6) * (3 * WAVE) + (s & 63);
    const bool zero = !(m > 0.f);
    const float d = zero ? 1.f : m;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      unsigned w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        unsigned lo = zero ? 0u : f2h(v[4 * j + c].re / d);
        unsigned hi = zero ? 0u : f2h(v[4 * j + c].im / d);
        w[c] = lo | (hi << 16);
      }
      p[j * WAVE] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    scale_ptr(base, npad)[s] = zero ? 0.f : m;
  }
  // Same format, quantised with one reciprocal per site (values may differ from
  // store() in the last FP16 bit); used for the outputs of the hot kernels.
  template <bool NT = false>
  __device__ static void store_fast(void *base, int s, size_t npad, const cpx<float> v[12]) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
    uint4 *p = (uint4 *)base + (size_t)(s >> 6) * (3 * WAVE) + (s & 63);
    const bool zero = !(m > 0.f);
    // 1/m overflows for m below ~3e-39 (FP32 denormals, e.g. far from a point
    // source); such sites are pre-scaled by 2^64 so the reciprocal stays finite.
    const float pre = m < 0x1p-64f ? 0x1p64f : 1.f;
    const float r = zero ? 0.f : 1.f / (m * pre);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      unsigned w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        w[c] = (unsigned)f2h((v[4 * j + c].re * pre) * r) | ((unsigned)f2h((v[4 * j + c].im * pre) * r) << 16);
      if (NT) st_nt(p + j * WAVE, make_uint4(w[0], w[1], w[2], w[3]));
      else p[j * WAVE] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (NT) st_nt(scale_ptr(base, npad) + s, m);
    else scale_ptr(base, npad)[s] = m;
  }
};

// ---------------------------------------------------------------------------
// Packed links.  Forward links U_mu(x) of the sites of parity p, in the same
// 64-site blocking; block index ((p * 4 + mu) * nb + (s >> 6)).
//   L_F64R18: 9 units of 16 B (complex128), row-major; the hops read the 6
//             units of rows 0-1 (96 B) and rebuild row 2, like the others
//   L_F32R12: 3 units of 16 B (rows 0-1, six complex64)
//   L_F16R12: 3 units of 8 B  (rows 0-1, six complex FP16)
// Row 2 of an SU(3) link is conj(row0 x row1) (unitarity and det = 1).
enum { L_F64R18 = 0, L_F32R12 = 1, L_F16R12 = 2 };

template <class R> __device__ __forceinline__ void recon_row2(cpx<R> u[9]) {
  // u[6 + c] = conj( (row0 x row1)_c )
  cpx<R> a0 = u[0], a1 = u[1], a2 = u[2], b0 = u[3], b1 = u[4], b2 = u[5];
  cpx<R> c0 = cmac(a1, b2, cneg(cmul(a2, b1)));
  cpx<R> c1 = cmac(a2, b0, cneg(cmul(a0, b2)));
  cpx<R> c2 = cmac(a0, b1, cneg(cmul(a1, b0)));
  u[6] = cmake(c0.re, -c0.im);
  u[7] = cmake(c1.re, -c1.im);
  u[8] = cmake(c2.re, -c2.im);
}

template <int L> struct LinkIO;

// Each link store has fetch (the loads only, into Raw), decode (conversion
// and row-2 rebuild) and load (both).
template <> struct LinkIO<L_F64R18> {
  using R = double;
  static constexpr size_t LINK_BYTES = 144;   // stored; a hop reads 96
  struct Raw { double2 q[6]; };
  template <bool NT = false>
  __device__ static void fetch(const void *g, int par, int mu, int s, int nb, Raw &r) {
    const double2 *p = (const double2 *)g + ((size_t)((par * 4 + mu) * nb + (s >> 6)) * 9) * WAVE + (s & 63);
    // each unit is one contiguous 1 KB wave access: skipping row 2's three
    // units skips their bytes entirely
#pragma unroll
    for (int j = 0; j < 6; ++j) r.q[j] = NT ? ld_nt(p + j * WAVE) : p[j * WAVE];
  }
  __device__ static void decode(const Raw &r, cpx<double> u[9]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) u[j] = cmake(r.q[j].x, r.q[j].y);
    recon_row2(u);
  }
  template <bool NT = false>
  __device__ static void load(const void *g, int par, int mu, int s, int nb, cpx<double> u[9]) {
    Raw r;
    fetch<NT>(g, par, mu, s, nb, r);
    decode(r, u);
  }
};

template <> struct LinkIO<L_F32R12> {
  using R = float;
  static constexpr size_t LINK_BYTES = 48;
  struct Raw { float4 q[3]; };
  template <bool NT = false>
  __device__ static void fetch(const void *g, int par, int mu, int s, int nb, Raw &r) {
    const float4 *p = (const float4 *)g + ((size_t)((par * 4 + mu) * nb + (s >> 6)) * 3) * WAVE + (s & 63);
#pragma unroll
    for (int j = 0; j < 3; ++j) r.q[j] = NT ? ld_nt(p + j * WAVE) : p[j * WAVE];
  }
  __device__ static void decode(const Raw &r, cpx<float> u[9]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      u[2 * j] = cmake(r.q[j].x, r.q[j].y);
      u[2 * j + 1] = cmake(r.q[j].z, r.q[j].w);
    }
    recon_row2(u);
  }
  template <bool NT = false>
  __device__ static void load(const void *g, int par, int mu, int s, int nb, cpx<float> u[9]) {
    Raw r;
    fetch<NT>(g, par, mu, s, nb, r);
    decode(r, u);
  }
};

template <> struct LinkIO<L_F16R12> {
  using R = float;
  static constexpr size_t LINK_BYTES = 24;
  struct Raw { uint2 q[3]; };
  template <bool NT = false>
  __device__ static void fetch(const void *g, int par, int mu, int s, int nb, Raw &r) {
    const uint2 *p = (const uint2 *)g + ((size_t)((par * 4 + mu) * nb + (s >> 6)) * 3) * WAVE + (s & 63);
#pragma unroll
    for (int j = 0; j < 3; ++j) r.q[j] = NT ? ld_nt(p + j * WAVE) : p[j * WAVE];
  }
  __device__ static void decode(const Raw &r, cpx<float> u[9]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const uint2 q = r.q[j];
      u[2 * j] = cmake(h2f((unsigned short)(q.x & 0xffffu)), h2f((unsigned short)(q.x >> 16)));
      u[2 * j + 1] = cmake(h2f((unsigned short)(q.y & 0xffffu)), h2f((unsigned short)(q.y >> 16)));
    }
    recon_row2(u);
  }
  template <bool NT = false>
  __device__ static void load(const void *g, int par, int mu, int s, int nb, cpx<float> u[9]) {
    Raw r;
    fetch<NT>(g, par, mu, s, nb, r);
    decode(r, u);
  }
};

// ---------------------------------------------------------------------------
// The hop.  Chiral basis gamma_mu = [[0, B_mu], [B_mu^+, 0]] with
// B_x = -i sigma_x, B_y = -i sigma_y, B_z = -i sigma_z, B_t = 1:
// (1 + S gamma_mu) psi has upper half h = psi_up + S B psi_lo and lower half
// S B^+ h, so each of the 8 terms is one spin projection to a half spinor (6
// complex), two SU(3) x colour-vector products, and a reconstruction.
//
// A site's directions are shared by the T waves of its work item (T = 1, 2 or
// 4): wave group g takes directions g, g + T, ...  The direction is uniform
// over a wave, so each is compiled on its own with the spin matrices as
// constants (the projections are additions with swapped or negated parts), and
// the groups' partial sums are added in LDS in a fixed order.

// w = U h (ADJ = false) or U^+ h (ADJ = true) for both spin components of h.
template <bool ADJ, class R>
__device__ __forceinline__ void su3_mul(const cpx<R> u[9], const cpx<R> h[6], cpx<R> w[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      cpx<R> r;
      if (!ADJ) {
        r = cmul(u[3 * a + 0], h[0 + sp]);
        r = cmac(u[3 * a + 1], h[2 + sp], r);
        r = cmac(u[3 * a + 2], h[4 + sp], r);
      } else {
        r = cjmul(u[0 + a], h[0 + sp]);
        r = cjmac(u[3 + a], h[2 + sp], r);
        r = cjmac(u[6 + a], h[4 + sp], r);
      }
      w[2 * a + sp] = r;
    }
  }
}

template <class Rd, class Rs> __device__ __forceinline__ void cvt12(const cpx<Rs> a[12], cpx<Rd> b[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = cmake((Rd)a[k].re, (Rd)a[k].im);
}

// Coordinates of checkerboard site s of parity p.  The divisions by Lx/2, Ly
// and Lz use (n + 1/2) * (1/d) in FP64, exact for n < 2^30 and d < 2^16.
struct SiteC { int s, xh, y, z, t, x; };

__device__ __forceinline__ int qdiv(int n, double r) { return (int)(((double)n + 0.5) * r); }

__device__ __forceinline__ SiteC site_c(const Geo &g, int s, int p) {
  SiteC c;
  c.s = s;
  const int q1 = qdiv(s, g.rlxh);
  c.xh = s - q1 * g.lxh;
  const int q2 = qdiv(q1, g.rly);
  c.y = q1 - q2 * g.ly;
  c.t = qdiv(q2, g.rlz);
  c.z = q2 - c.t * g.lz;
  c.x = 2 * c.xh + ((p + c.y + c.z + c.t) & 1);
  return c;
}

// Checkerboard index of the neighbour in direction mu, forward or backward.
__device__ __forceinline__ int nbr(const Geo &g, const SiteC &c, int mu, bool fwd) {
  if (mu == 0) {
    const int xn = fwd ? (c.x + 1 == g.lx ? 0 : c.x + 1) : (c.x == 0 ? g.lx - 1 : c.x - 1);
    return c.s - c.xh + (xn >> 1);
  }
  // Selected arithmetically: a conditional over the struct members lets the
  // compiler index the coordinate struct at run time (per lane), which moves it
  // out of registers into LDS or scratch.
  const int m1 = mu == 1, m2 = mu == 2, m3 = mu == 3;
  const int co = m1 * c.y + m2 * c.z + m3 * c.t;
  const int L = m1 * g.ly + m2 * g.lz + m3 * g.lt;
  const int st = m1 * g.sy + m2 * g.sz + m3 * g.st;
  if (fwd) return (co + 1 == L) ? c.s - (L - 1) * st : c.s + st;
  return (co == 0) ? c.s + (L - 1) * st : c.s - st;
}

// Field loaders: NF packed fields (right-hand sides) read at one site and
// converted to the compute type R.
template <int S, int N> struct FieldLd {
  using R = typename SpinorIO<S>::R;
  static constexpr int NF = N;
  const void *base[N];
  size_t npad;
  __device__ __forceinline__ void operator()(int r, int s, cpx<R> v[12]) const { SpinorIO<S>::load(base[r], s, npad, v); }
  // F16S: the hop reads the unscaled FP16 values and applies the site scale
  // once, in its accumulation (see hop_term)
  static constexpr bool RAW = S == S_F16S;
  __device__ __forceinline__ void raw(int r, int s, cpx<R> v[12], R &sc) const {
    if constexpr (RAW) SpinorIO<S>::load_raw(base[r], s, npad, v, sc);
  }
  // One FP32 field: the hop issues the loads of both directions of a dimension
  // before it uses either (hop_mu), one memory round trip instead of two.
  // Measured: 6% off the latency-bound 16^3x32 hop; the F16S hop, bound by its
  // vector work, lost occupancy and ran up to 11% slower, and the FP64 hop has
  // no registers to spare.
  static constexpr bool PAIR = N == 1 && S == S_F32;
  using Raw = typename SpinorIO<S>::Raw;
  __device__ __forceinline__ void fetch(int r, int s, Raw &w) const { SpinorIO<S>::fetch(base[r], s, npad, w); }
  __device__ __forceinline__ void decode(const Raw &w, cpx<R> v[12], R &sc) const {
    if constexpr (RAW) SpinorIO<S>::decode_raw(w, v, sc);
    else { SpinorIO<S>::decode(w, v); sc = (R)1; }
  }
};

// Sum of an FP64 field and an FP32 field (the solution of a mixed-precision
// solve: FP64 accumulated part plus the FP32 part not yet folded in).
struct SumLd {
  using R = double;
  static constexpr int NF = 1;
  static constexpr bool RAW = false;
  static constexpr bool PAIR = false;
  __device__ __forceinline__ void raw(int, int, cpx<double> *, double &) const {}
  const void *a;   // F64
  const void *b;   // F32, or null
  size_t npad;
  __device__ __forceinline__ void operator()(int, int s, cpx<double> v[12]) const {
    SpinorIO<S_F64>::load(a, s, npad, v);
    if (b) {
      cpx<float> w[12];
      SpinorIO<S_F32>::load(b, s, npad, w);
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = cadd(v[k], cmake((double)w[k].re, (double)w[k].im));
    }
  }
};

// B_mu and B_mu^+ as (source component, phase) per row: row i of B psi_lo is
// phase f_i times component j_i of psi_lo; row i of B^+ h is phase e_i times
// component j_i of h.  Phase codes: 0 -> 1, 1 -> i, 2 -> -1, 3 -> -i.
template <int MU> struct SpinB {
  static constexpr int j0 = (MU == 0 || MU == 1) ? 1 : 0, j1 = 1 - j0;
  static constexpr int f0 = MU == 0 ? 3 : MU == 1 ? 2 : MU == 2 ? 3 : 0;
  static constexpr int f1 = MU == 0 ? 3 : MU == 1 ? 0 : MU == 2 ? 1 : 0;
  static constexpr int e0 = MU == 0 ? 1 : MU == 1 ? 0 : MU == 2 ? 1 : 0;
  static constexpr int e1 = MU == 0 ? 1 : MU == 1 ? 2 : MU == 2 ? 3 : 0;
};

template <int F, class R> __device__ __forceinline__ cpx<R> cph(cpx<R> z) {
  constexpr int f = F & 3;
  if constexpr (f == 0) return z;
  else if constexpr (f == 1) return cmake(-z.im, z.re);
  else if constexpr (f == 2) return cmake(-z.re, -z.im);
  else return cmake(z.im, -z.re);
}

// One term of the hop for every field of the loader: DIR 0 is the forward
// neighbour with U_mu(x) and (1 - gamma_mu) (DAG: 1 + gamma_mu), DIR 1 the
// backward neighbour with U_mu(x - mu)^+ and (1 + gamma_mu) (DAG: 1 - gamma_mu).
// Each link is loaded and rebuilt once for all fields.  FIRST: the term
// initialises the accumulators.
// The arithmetic of one term for one field: project psi (RAW: the unscaled
// FP16 values of an F16S site with scale sc), multiply by the link, rebuild
// the lower half and accumulate.
template <int MU, int DIR, bool DAG, bool FIRST, bool RAW, class R>
__device__ __forceinline__ void term_acc(const cpx<R> u[9], const cpx<R> psi[12], R sc, cpx<R> acc[12]) {
  using B = SpinB<MU>;
  constexpr int ph = ((DIR == 0) == DAG) ? 0 : 2;   // the projection sign as a phase
  cpx<R> h[6], w[6];
  if constexpr (RAW) {
    // F16S: each real of h is one mixed-precision fma (FP16 sources converted
    // in the instruction), with a multiplier of 1 the compiler cannot fold
    // away; the site scale sc enters below, as the multiplier of the
    // accumulation (or of h for the term that initialises the accumulators).
    R one = (R)1;
    asm volatile("" : "+s"(one));
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const cpx<R> l0 = cph<B::f0 + ph>(psi[4 * cc + 2 + B::j0]), l1 = cph<B::f1 + ph>(psi[4 * cc + 2 + B::j1]);
      h[2 * cc] = cmake(__builtin_fmaf(l0.re, one, psi[4 * cc].re), __builtin_fmaf(l0.im, one, psi[4 * cc].im));
      h[2 * cc + 1] =
          cmake(__builtin_fmaf(l1.re, one, psi[4 * cc + 1].re), __builtin_fmaf(l1.im, one, psi[4 * cc + 1].im));
    }
    if (FIRST && DIR == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = cscale(sc, h[k]);
    }
  } else {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      h[2 * cc] = cadd(psi[4 * cc], cph<B::f0 + ph>(psi[4 * cc + 2 + B::j0]));
      h[2 * cc + 1] = cadd(psi[4 * cc + 1], cph<B::f1 + ph>(psi[4 * cc + 2 + B::j1]));
    }
  }
  su3_mul<DIR == 1>(u, h, w);
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const cpx<R> w0 = w[2 * cc], w1 = w[2 * cc + 1];
    const cpx<R> lo0 = cph<B::e0 + ph>(w[2 * cc + B::j0]);
    const cpx<R> lo1 = cph<B::e1 + ph>(w[2 * cc + B::j1]);
    if (FIRST && DIR == 0) {
      acc[4 * cc] = w0; acc[4 * cc + 1] = w1; acc[4 * cc + 2] = lo0; acc[4 * cc + 3] = lo1;
    } else if constexpr (RAW) {
      acc[4 * cc] = cfma(sc, w0, acc[4 * cc]);
      acc[4 * cc + 1] = cfma(sc, w1, acc[4 * cc + 1]);
      acc[4 * cc + 2] = cfma(sc, lo0, acc[4 * cc + 2]);
      acc[4 * cc + 3] = cfma(sc, lo1, acc[4 * cc + 3]);
    } else {
      acc[4 * cc] = cadd(acc[4 * cc], w0);
      acc[4 * cc + 1] = cadd(acc[4 * cc + 1], w1);
      acc[4 * cc + 2] = cadd(acc[4 * cc + 2], lo0);
      acc[4 * cc + 3] = cadd(acc[4 * cc + 3], lo1);
    }
  }
}

template <class R, class RL> __device__ __forceinline__ void link_cvt(const cpx<RL> u0[9], cpx<R> u[9]) {
#pragma unroll
  for (int j = 0; j < 9; ++j) u[j] = cmake((R)u0[j].re, (R)u0[j].im);
}

template <int MU, int DIR, bool DAG, bool FIRST, int L, bool NT, class Ld>
__device__ __forceinline__ void hop_term(const Geo &g, const void *gauge, const Ld &ld, const SiteC &c, int p,
                                         cpx<typename Ld::R> acc[Ld::NF][12]) {
  using R = typename Ld::R;
  const int n = nbr(g, c, MU, DIR == 0);
  cpx<R> u[9];
  {
    cpx<typename LinkIO<L>::R> u0[9];
    if (DIR == 0) LinkIO<L>::template load<NT>(gauge, p, MU, c.s, g.nb, u0);
    else LinkIO<L>::template load<NT>(gauge, 1 - p, MU, n, g.nb, u0);
    link_cvt(u0, u);
  }
#pragma unroll
  for (int r = 0; r < Ld::NF; ++r) {
    cpx<R> psi[12];
    R sc = (R)1;
    if constexpr (Ld::RAW) ld.raw(r, n, psi, sc);
    else ld(r, n, psi);
    term_acc<MU, DIR, DAG, FIRST, Ld::RAW>(u, psi, sc, acc[r]);
  }
}

// The loads of one term of a single-field loader (see FieldLd::PAIR).
template <int L, class Ld> struct TermIn {
  typename LinkIO<L>::Raw lr;
  typename Ld::Raw sr;
};

template <int MU, int DIR, int L, bool NT, class Ld>
__device__ __forceinline__ void term_fetch(const Geo &g, const void *gauge, const Ld &ld, const SiteC &c, int p,
                                           TermIn<L, Ld> &in) {
  const int n = nbr(g, c, MU, DIR == 0);
  if (DIR == 0) LinkIO<L>::template fetch<NT>(gauge, p, MU, c.s, g.nb, in.lr);
  else LinkIO<L>::template fetch<NT>(gauge, 1 - p, MU, n, g.nb, in.lr);
  ld.fetch(0, n, in.sr);
}

template <int MU, int DIR, bool DAG, bool FIRST, int L, class Ld>
__device__ __forceinline__ void term_use(const Ld &ld, const TermIn<L, Ld> &in, cpx<typename Ld::R> acc[12]) {
  using R = typename Ld::R;
  cpx<R> u[9], psi[12];
  {
    cpx<typename LinkIO<L>::R> u0[9];
    LinkIO<L>::decode(in.lr, u0);
    link_cvt(u0, u);
  }
  R sc;
  ld.decode(in.sr, psi, sc);
  term_acc<MU, DIR, DAG, FIRST, Ld::RAW>(u, psi, sc, acc);
}

template <int MU, bool DAG, bool FIRST, int L, bool NT, class Ld>
__device__ __forceinline__ void hop_mu(const Geo &g, const void *gauge, const Ld &ld, const SiteC &c, int p,
                                       cpx<typename Ld::R> acc[Ld::NF][12]) {
  if constexpr (Ld::PAIR) {
    TermIn<L, Ld> f, b;
    term_fetch<MU, 0, L, NT>(g, gauge, ld, c, p, f);
    term_fetch<MU, 1, L, NT>(g, gauge, ld, c, p, b);
    // keep the scheduler from sinking the second fetch below the first use
    __builtin_amdgcn_sched_barrier(0);
    term_use<MU, 0, DAG, FIRST, L>(ld, f, acc[0]);
    term_use<MU, 1, DAG, false, L>(ld, b, acc[0]);
  } else {
    hop_term<MU, 0, DAG, FIRST, L, NT>(g, gauge, ld, c, p, acc);
    hop_term<MU, 1, DAG, false, L, NT>(g, gauge, ld, c, p, acc);
  }
}

// acc[r] = this wave group's part of (H psi_r)(s) (DAG: H^dagger) for output
// parity p: the directions grp, grp + T, ...  grp must be wave-uniform.
template <int L, bool DAG, int T, bool NT, class Ld>
__device__ __forceinline__ void hop_wave(const Geo &g, const void *gauge, const Ld &ld, int s, int p, int grp,
                                         cpx<typename Ld::R> acc[Ld::NF][12]) {
  static_assert(T == 1 || T == 2 || T == 4, "1, 2 or 4 waves per site block");
  const SiteC c = site_c(g, s, p);
  if constexpr (T == 1) {
    hop_mu<0, DAG, true, L, NT>(g, gauge, ld, c, p, acc);
    hop_mu<1, DAG, false, L, NT>(g, gauge, ld, c, p, acc);
    hop_mu<2, DAG, false, L, NT>(g, gauge, ld, c, p, acc);
    hop_mu<3, DAG, false, L, NT>(g, gauge, ld, c, p, acc);
  } else if constexpr (T == 2) {
    if (grp == 0) {
      hop_mu<0, DAG, true, L, NT>(g, gauge, ld, c, p, acc);
      hop_mu<2, DAG, false, L, NT>(g, gauge, ld, c, p, acc);
    } else {
      hop_mu<1, DAG, true, L, NT>(g, gauge, ld, c, p, acc);
      hop_mu<3, DAG, false, L, NT>(g, gauge, ld, c, p, acc);
    }
  } else {
    if (grp == 0) hop_mu<0, DAG, true, L, NT>(g, gauge, ld, c, p, acc);
    else if (grp == 1) hop_mu<1, DAG, true, L, NT>(g, gauge, ld, c, p, acc);
    else if (grp == 2) hop_mu<2, DAG, true, L, NT>(g, gauge, ld, c, p, acc);
    else hop_mu<3, DAG, true, L, NT>(g, gauge, ld, c, p, acc);
  }
}

// LDS for wave_combine: (4/T items) x (T-1 groups) x NF fields x 24 reals x 64
// lanes, in 16-byte vectors.
template <class R> struct Vec16;
template <> struct Vec16<float> { using T = float4; static constexpr int N = 4; };
template <> struct Vec16<double> { using T = double2; static constexpr int N = 2; };
template <int T, int NF, class R> struct HopLds {
  static constexpr int PER = 24 / Vec16<R>::N;   // vectors per field
  static constexpr int VECS = T == 1 ? 1 : (4 / T) * (T - 1) * NF * PER * WAVE;
  using V = typename Vec16<R>::T;
};

template <class R> __device__ __forceinline__ void v16_put(typename Vec16<R>::T *p, const cpx<R> a[12], int j);
template <> __device__ __forceinline__ void v16_put<float>(float4 *p, const cpx<float> a[12], int j) {
  *p = make_float4(a[2 * j].re, a[2 * j].im, a[2 * j + 1].re, a[2 * j + 1].im);
}
template <> __device__ __forceinline__ void v16_put<double>(double2 *p, const cpx<double> a[12], int j) {
  *p = make_double2(a[j].re, a[j].im);
}
template <class R> __device__ __forceinline__ void v16_add(const typename Vec16<R>::T *p, cpx<R> a[12], int j);
template <> __device__ __forceinline__ void v16_add<float>(const float4 *p, cpx<float> a[12], int j) {
  const float4 v = *p;
  a[2 * j] = cadd(a[2 * j], cmake(v.x, v.y));
  a[2 * j + 1] = cadd(a[2 * j + 1], cmake(v.z, v.w));
}
template <> __device__ __forceinline__ void v16_add<double>(const double2 *p, cpx<double> a[12], int j) {
  const double2 v = *p;
  a[j] = cadd(a[j], cmake(v.x, v.y));
}

// Add the partial sums of the T wave groups of each item (in the order
// 0, 1, .., T-1, so the result does not depend on scheduling); afterwards group
// 0 holds the full sums.  Every wave of the work-group must call it (barrier).
template <int T, int NF, class R>
__device__ __forceinline__ void wave_combine(cpx<R> acc[NF][12], int slot, int grp,
                                             typename HopLds<T, NF, R>::V *lds) {
  if constexpr (T > 1) {
    constexpr int PER = HopLds<T, NF, R>::PER;
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    if (grp != 0) {
      typename HopLds<T, NF, R>::V *q = lds + (size_t)(slot * (T - 1) + grp - 1) * NF * PER * WAVE + lane;
#pragma unroll
      for (int r = 0; r < NF; ++r)
#pragma unroll
        for (int j = 0; j < PER; ++j) v16_put<R>(q + (r * PER + j) * WAVE, acc[r], j);
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int g2 = 1; g2 < T; ++g2) {
        const typename HopLds<T, NF, R>::V *q = lds + (size_t)(slot * (T - 1) + g2 - 1) * NF * PER * WAVE + lane;
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
          for (int j = 0; j < PER; ++j) v16_add<R>(q + (r * PER + j) * WAVE, acc[r], j);
      }
    }
  }
}

// The site-diagonal part of the twisted-mass operator, A = 1 + i t gamma_5
// with t = 2 kappa mu (gamma_5 = diag(1, 1, -1, -1) in the chiral basis), and
// its dagger, inverse and inverse dagger act on a spinor as one complex factor
// on the upper spins and its conjugate-sign partner on the lower ones.
enum { CHI_ONE = 0, CHI_A = 1, CHI_ADAG = 2, CHI_AINV = 3, CHI_AINVDAG = 4 };

template <class R> __device__ __forceinline__ void apply_chi(cpx<R> v[12], int mode, double t) {
  if (mode == CHI_ONE || t == 0.0) return;
  const double n = (mode == CHI_AINV || mode == CHI_AINVDAG) ? 1.0 / (1.0 + t * t) : 1.0;
  const double sg = (mode == CHI_A || mode == CHI_AINVDAG) ? 1.0 : -1.0;
  const cpx<R> cu = cmake((R)n, (R)(n * sg * t)), cl = cmake((R)n, (R)(-n * sg * t));
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = cmul((k & 3) < 2 ? cu : cl, v[k]);
}

template <int NF, class R> __device__ __forceinline__ void zero_acc(cpx<R> acc[NF][12]) {
#pragma unroll
  for (int r = 0; r < NF; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = cmake((R)0, (R)0);
}

// ---------------------------------------------------------------------------
// Reductions.  A wave sums its 64 lanes with a fixed xor butterfly and stores
// one partial per wave; a separate kernel sums a system's partials in index
// order (the kernel boundary makes them visible).  Nothing depends on
// scheduling, so repeated runs are bitwise identical.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
  return v;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

template <class R> __device__ __forceinline__ double norm12(const cpx<R> v[12]) {
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) a += (double)v[k].re * (double)v[k].re + (double)v[k].im * (double)v[k].im;
  return a;
}

// (a | b) = sum conj(a) b, accumulated in FP64
template <class R> __device__ __forceinline__ void dot12(const cpx<R> a[12], const cpx<R> b[12], double &re, double &im) {
  double r = 0.0, i = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double ar = a[k].re, ai = a[k].im, br = b[k].re, bi = b[k].im;
    r += ar * br + ai * bi;
    i += ar * bi - ai * br;
  }
  re = r;
  im = i;
}


// XCD-aware block order: the hardware hands consecutive work-group ids to the 8
// XCDs in turn; this remap gives each XCD one contiguous range of logical
// blocks, so neighbouring sites share an L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_remap(int hw, int nblocks) {
#ifdef QIRAL_NO_XCD_REMAP
  return hw;
#endif
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = hw & 7, idx = hw >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Traversal order of the 64-site blocks of a hop.  With zb > 0 (a t-slice and a
// chunk of zb z-planes are whole numbers of blocks, and zb divides Lz) logical
// block L runs over (z-tile of zb planes, t, block within the chunk of the
// tile's planes at that t), so the t-neighbours of a block were read one chunk
// earlier, not a whole t-slice earlier, and are still in the L2 of the XCD that
// takes the range.  zb = 0 is the plain lexicographic order.
__host__ __device__ inline int block_order(const Geo &g, int L, int zb) {
  if (zb <= 0) return L;
  const int P = zb * g.sz / WAVE;    // blocks per chunk (zb planes of one t-slice)
  const int Bt = g.st / WAVE;        // blocks per t-slice
  const int j = L % P, L2 = L / P;
  const int t = L2 % g.lt, zt = L2 / g.lt;
  return t * Bt + zt * P + j;
}

}  // namespace qiral
