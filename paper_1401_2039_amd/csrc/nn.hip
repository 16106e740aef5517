// Learned gauge-covariant preconditioner (an addition to the paper's method):
// a network of parallel-transport convolution layers (Lehner & Wettig,
// Phys. Rev. D 108 (2023) 034503)
//     psi_out^i(x) = sum_j sum_p W_p^{ij} [T_p psi_in^j](x),
// 9 paths p (0: identity; 1..4: +x..+t, T psi(x) = U_mu(x) psi(x+mu); 5..8:
// -x..-t, T psi(x) = U_mu(x-mu)^+ psi(x-mu)), W a complex 4x4 spin matrix,
// trained on pairs (D v, v) of Gaussian v drawn on the device (Philox4x32-10,
// Salmon et al., SC'11, with the Box-Muller transform) with Adam (Kingma & Ba
// 2015), and used as the right preconditioner of flexible GMRES(m) (Saad 1993)
// on the full operator D, with even-odd CGNR as the fallback.
//
// Fields are packed FP32 full fields (even half, odd half) per channel; the
// network runs on the FP32 reconstruct-12 links.  Weights are FP32 complex,
// layer 1 [9][H][1][4][4] then layer 2 [9][1][H][4][4].
#include <hip/hip_runtime.h>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "qiral_int.h"

using namespace qiral;

struct qiral_nn {
  qiral_lattice *lat = nullptr;
  int hidden = 0;
  int nw1 = 0, nw2 = 0;     // complex weights per layer
  float2 *w = nullptr;      // [nw1 + nw2]
  float2 *wadj = nullptr;   // adjoint-layer weights (scratch)
  float2 *kmat = nullptr;   // folded path-pair weights K, then K' (scratch)
  void *kfrag = nullptr;    // MFMA A fragments of K, then of K' (scratch)
  float *am = nullptr, *av = nullptr;   // Adam moments, [2 (nw1 + nw2)]
  double *grad = nullptr;   // dL/dRe, dL/dIm interleaved, [2 (nw1 + nw2)]
  double *part = nullptr;   // weight-gradient partials
  double *scal = nullptr;   // small reductions: [0] ||v||^2, [1] loss sum, ... ; plus partial area
  void *act = nullptr;      // hidden activations (H full F32 fields)
  void *gact = nullptr;     // gradient w.r.t. the activations (H fields)
  void *fv = nullptr, *fb = nullptr, *fy = nullptr, *fg = nullptr;   // one full F32 field each
  double *loss_dev = nullptr;   // losses of up to LOSS_CAP training steps
  long adam_step = 0;
};

namespace {

constexpr int NPATH = 9;
constexpr int WG_CHUNKS = 64;   // site chunks of the weight-gradient reduction
constexpr int LOSS_CAP = 256;    // training losses kept on the device between copies to the host

qiral_status fail(qiral_status s, const char *m) {
  set_error(m);
  return s;
}

// ---------------------------------------------------------------------------
// device helpers
__device__ __forceinline__ void path_of(int p, int &mu, bool &fwd) {
  mu = (p - 1) & 3;
  fwd = p <= 4;
}

// t = U psi (adj = false) or U^+ psi (adj = true) on the colour index of a 3x4 block.
__device__ __forceinline__ void transport(const cpx<float> u[9], const cpx<float> psi[12], cpx<float> t[12], bool adj) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      cpx<float> r;
      if (!adj) {
        r = cmul(u[3 * a], psi[s]);
        r = cmac(u[3 * a + 1], psi[4 + s], r);
        r = cmac(u[3 * a + 2], psi[8 + s], r);
      } else {
        r = cjmul(u[a], psi[s]);
        r = cjmac(u[3 + a], psi[4 + s], r);
        r = cjmac(u[6 + a], psi[8 + s], r);
      }
      t[4 * a + s] = r;
    }
  }
}

// (T_p psi)(x) for a full field: x = (par, s), psi read at the neighbour.
__device__ __forceinline__ void path_apply(const Geo &g, const void *links, const void *field, size_t hb, size_t npad,
                                           const SiteC &c, int par, int p, cpx<float> t[12]) {
  if (p == 0) {
    SpinorIO<S_F32>::load((const char *)field + par * hb, c.s, npad, t);
    return;
  }
  int mu;
  bool fwd;
  path_of(p, mu, fwd);
  const int n = nbr(g, c, mu, fwd);
  cpx<float> u[9], psi[12];
  if (fwd) LinkIO<L_F32R12>::load(links, par, mu, c.s, g.nb, u);
  else LinkIO<L_F32R12>::load(links, 1 - par, mu, n, g.nb, u);
  SpinorIO<S_F32>::load((const char *)field + (1 - par) * hb, n, npad, psi);
  transport(u, psi, t, !fwd);
}

// ---------------------------------------------------------------------------
// kernels

// One layer (training), CI output channels per pass of each thread over the
// paths.
template <int CIN, int COUT, int CI>
__global__ __launch_bounds__(256) void k_ptc_layer(Geo g, const void *__restrict__ links,
                                                   const float2 *__restrict__ w, const void *__restrict__ in,
                                                   void *__restrict__ out, size_t fstride) {
  __shared__ float2 sw[NPATH * COUT * CIN * 16];
  for (int i = threadIdx.x; i < NPATH * COUT * CIN * 16; i += blockDim.x) sw[i] = w[i];
  __syncthreads();
  const size_t npad = (size_t)g.nb * WAVE, hb = npad * SpinorIO<S_F32>::SITE_BYTES;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 2 * npad) return;
  const int par = (int)(gid / npad), s = (int)(gid % npad);
  if (s >= g.vh) return;
  const SiteC c = site_c(g, s, par);
  if constexpr (COUT == 1 && CIN > 1) {
    // Spin weights commute with the colour transport: per path, mix the CIN
    // input channels at the neighbour, then transport once.
    cpx<float> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cmake(0.f, 0.f);
#pragma unroll 1
    for (int p = 0; p < NPATH; ++p) {
      int mu = 0, n = s, lp = par;
      bool fwd = true;
      if (p > 0) {
        path_of(p, mu, fwd);
        n = nbr(g, c, mu, fwd);
        lp = 1 - par;
      }
      cpx<float> m[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) m[k] = cmake(0.f, 0.f);
#pragma unroll 1
      for (int j = 0; j < CIN; ++j) {
        cpx<float> psi[12];
        SpinorIO<S_F32>::load((const char *)in + j * fstride + lp * hb, n, npad, psi);
        const float2 *W = sw + (p * CIN + j) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const cpx<float> wr = cmake(W[4 * r + q].x, W[4 * r + q].y);
#pragma unroll
            for (int a = 0; a < 3; ++a) m[4 * a + r] = cmac(wr, psi[4 * a + q], m[4 * a + r]);
          }
      }
      if (p == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cadd(acc[k], m[k]);
      } else {
        cpx<float> u[9], t[12];
        if (fwd) LinkIO<L_F32R12>::load(links, par, mu, c.s, g.nb, u);
        else LinkIO<L_F32R12>::load(links, 1 - par, mu, n, g.nb, u);
        transport(u, m, t, !fwd);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cadd(acc[k], t[k]);
      }
    }
    SpinorIO<S_F32>::store((char *)out + par * hb, s, npad, acc);
    return;
  }
#pragma unroll 1
  for (int i0 = 0; i0 < COUT; i0 += CI) {
    cpx<float> acc[CI][12];
#pragma unroll
    for (int ii = 0; ii < CI; ++ii)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[ii][k] = cmake(0.f, 0.f);
#pragma unroll 1
    for (int p = 0; p < NPATH; ++p) {
#pragma unroll 1
      for (int j = 0; j < CIN; ++j) {
        cpx<float> t[12];
        path_apply(g, links, (const char *)in + j * fstride, hb, npad, c, par, p, t);
#pragma unroll
        for (int ii = 0; ii < CI; ++ii) {
          const float2 *W = sw + ((p * COUT + i0 + ii) * CIN + j) * 16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const cpx<float> wr = cmake(W[4 * r + q].x, W[4 * r + q].y);
#pragma unroll
              for (int a = 0; a < 3; ++a) acc[ii][4 * a + r] = cmac(wr, t[4 * a + q], acc[ii][4 * a + r]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int ii = 0; ii < CI; ++ii)
      SpinorIO<S_F32>::store((char *)out + (i0 + ii) * fstride + par * hb, s, npad, acc[ii]);
  }
}

// Adjoint-layer weights: W'[mirror(p)][j][i] = (W[p][i][j])^dagger, so that the
// forward layer with W' (CIN and COUT swapped) applies the adjoint.
__global__ void k_adj_weights(const float2 *__restrict__ w, float2 *__restrict__ wa, int cout, int cin) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = NPATH * cout * cin * 16;
  if (idx >= n) return;
  const int e = idx & 15, blk = idx >> 4;
  const int j = blk % cin, i = (blk / cin) % cout, p = blk / (cin * cout);
  const int pm = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
  const int r = e >> 2, q = e & 3;
  const float2 v = w[((p * cout + i) * cin + j) * 16 + 4 * q + r];
  wa[((pm * cin + j) * cout + i) * 16 + 4 * r + q] = make_float2(v.x, -v.y);
}

// ---------------------------------------------------------------------------
// Inference with the two layers folded.  The layers are linear and a spin
// matrix commutes with a colour transport, so
//     N = sum_{p,p'} T_p K_{pp'} T_{p'},   K_{pp'} = sum_c W2_p^c W1_{p'}^c,
// and N^dagger has the same form with K'_{pp'} = (K_{m(p') m(p)})^dagger, m the
// mirror path (T_p^dagger = T_{m(p)}).  Pass A forms m_p(y) = sum_{p'} K_{pp'}
// (T_{p'} v)(y) at every site, pass B sums out(x) = sum_p (T_p m_p)(x): one
// transport per path and a spin product per path pair, where the layers take a
// transport and H spin products per path in each layer and pass the H hidden
// fields through memory nine times.

__device__ __forceinline__ int mirror_path(int p) { return p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4); }

// K (adj = 0) or K' (adj = 1) into k[p][p'][4][4], summed over the H channels
// in FP64; one thread per entry.
__global__ void k_nn_fold(const float2 *__restrict__ w1, const float2 *__restrict__ w2, int hidden, int adj,
                          float2 *__restrict__ k) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NPATH * NPATH * 16) return;
  const int e = idx & 15, pq = idx >> 4, p = pq / NPATH, q = pq % NPATH;
  const int P = adj ? mirror_path(q) : p, Q = adj ? mirror_path(p) : q;
  const int r = adj ? e & 3 : e >> 2, c = adj ? e >> 2 : e & 3;
  double re = 0.0, im = 0.0;
  for (int h = 0; h < hidden; ++h) {
    const float2 *a = w2 + (P * hidden + h) * 16, *b = w1 + (Q * hidden + h) * 16;
    for (int j = 0; j < 4; ++j) {
      const float2 x = a[4 * r + j], y = b[4 * j + c];
      re += (double)x.x * y.x - (double)x.y * y.y;
      im += (double)x.x * y.y + (double)x.y * y.x;
    }
  }
  k[idx] = make_float2((float)re, (float)(adj ? -im : im));
}

// A spinor of a field in storage class S (F32, or F64 rounded to F32).
template <int S>
__device__ __forceinline__ void load_as_f32(const void *half, int s, size_t npad, cpx<float> v[12]) {
  if constexpr (S == S_F32) {
    SpinorIO<S_F32>::load(half, s, npad, v);
  } else {
    cpx<double> d[12];
    SpinorIO<S_F64>::load(half, s, npad, d);
    cvt12(d, v);
  }
}

// Pass A over both parities and all nine paths (vector ALU, FP32): the input's
// half-fields are in0 (even) and in1 (odd), storage SIN; m_p is written to the
// F32 half-field m + p * mstride + parity * (npad * 96 bytes).  Two waves share
// a 64-site block, each sweeping the input paths for its own PC output paths,
// so the second wave's neighbour loads hit the cache lines the first has just
// brought in.  Site blocks in the hop's XCD-mapped order (zb as block_order).
// Grid: (ceil(nb / 2), 2 parities), 256 threads: two site blocks.
template <int SIN, int PC>
__global__ __launch_bounds__(256) void k_nn_pass_a(Geo g, const void *__restrict__ links,
                                                   const float2 *__restrict__ K, const void *__restrict__ in0,
                                                   const void *__restrict__ in1, void *__restrict__ m,
                                                   size_t mstride, int zb) {
  const int ya = blockIdx.y;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int L = xcd_remap(blockIdx.x, gridDim.x) * 2 + (w >> 1);
  if (L >= g.nb) return;
  const int s = block_order(g, L, zb) * WAVE + (threadIdx.x & (WAVE - 1));
  if (s >= g.vh) return;
  const size_t npad = (size_t)g.nb * WAVE, hb = npad * SpinorIO<S_F32>::SITE_BYTES;
  const int p0 = (w & 1) * PC, p1 = min(NPATH, p0 + PC);
  const void *here = ya ? in1 : in0, *there = ya ? in0 : in1;
  const SiteC c = site_c(g, s, ya);
  cpx<float> acc[PC][12];
#pragma unroll
  for (int j = 0; j < PC; ++j)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[j][k] = cmake(0.f, 0.f);
#pragma unroll 1
  for (int q = 0; q < NPATH; ++q) {
    cpx<float> t[12];
    if (q == 0) {
      load_as_f32<SIN>(here, s, npad, t);
    } else {
      int mu;
      bool fwd;
      path_of(q, mu, fwd);
      const int n = nbr(g, c, mu, fwd);
      cpx<float> u[9], psi[12];
      if (fwd) LinkIO<L_F32R12>::load(links, ya, mu, s, g.nb, u);
      else LinkIO<L_F32R12>::load(links, 1 - ya, mu, n, g.nb, u);
      load_as_f32<SIN>(there, n, npad, psi);
      transport(u, psi, t, !fwd);
    }
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      if (p0 + j >= p1) break;
      const float2 *Kp = K + ((p0 + j) * NPATH + q) * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const cpx<float> kr = cmake(Kp[4 * r + e].x, Kp[4 * r + e].y);
#pragma unroll
          for (int a = 0; a < 3; ++a) acc[j][4 * a + r] = cmac(kr, t[4 * a + e], acc[j][4 * a + r]);
        }
    }
  }
#pragma unroll
  for (int j = 0; j < PC; ++j) {
    if (p0 + j >= p1) break;
    SpinorIO<S_F32>::store((char *)m + (size_t)(p0 + j) * mstride + ya * hb, s, npad, acc[j]);
  }
}

// Pass A of the one-parity form on the matrix cores.  With the input on
// parity P and the output kept on P, a site y of the other parity needs
// m_p(y) = sum_q K_pq t_q(y) for the eight hops p and q: per colour, a 32x32
// complex (64x64 real) matrix applied to the 64-real vector of the t_q.  Over a
// 64-site block that is a 64 x 64 x 192 product, done as 16x16x32 bf16 MFMAs
// with FP32 accumulation: rows (p, spin, re/im), columns (site, colour),
// k = (q, spin, re/im).  Each real is split into bf16 hi + lo parts and three
// products are summed (hi*hi + hi*lo + lo*hi), about 1e-5 relative: used only
// as the flexible solvers' preconditioner, which needs no exact arithmetic
// (every recurrence uses the vector the preconditioner actually returned).
//
// Four waves per 64-site block.  Per K-step of four input paths, wave w makes
// t_q for q = 1 + 4 ks + w at its lane's site and leaves its bf16 hi and lo
// parts in LDS; after a barrier every wave reads the B fragments (8 k-values of
// one column per lane) and multiplies them into its M-tile (output paths
// 1 + 2w and 2 + 2w).  The accumulator rows of lane (g, n) are two complex
// spin components of one colour of one site, which is exactly a float4 unit of
// the F32 spinor layout, so the results are stored straight from the
// accumulators.  Sites of parity P keep m_0 = K_00 v (vector ALU).  A
// fragments come from k_nn_frag.  Site blocks in the hop's XCD-mapped order.
// Grid: (nb, 2 parities), 256 threads.
//
// Each work-group does its site block for nsys systems one after the other
// (inputs istride bytes apart, path fields msys bytes apart); the links it
// reads for the first system are kept in LDS for the others.
// Path field p of a system starts at p * mstride and its parity-x half at
// x * hoff (hoff = 0: each path field holds only the parity it is used on).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// A fragments of the real form of K (or K') over the hop pairs, bf16 hi and lo:
// f[(((mt * 2 + ks) * 2 + hl) * 64 + lane) * 8 + kk]; row lane % 16 of M-tile mt
// is (p = 1 + 2 mt + row / 8, spin (row % 8) / 2, re/im row % 2); kk is (spin
// kk / 2, re/im kk % 2) of input path q = 1 + 4 ks + lane / 16.
__global__ void k_nn_frag(const float2 *__restrict__ K, __bf16 *__restrict__ f) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4 * 2 * 2 * 64 * 8) return;
  const int kk = idx & 7, lane = (idx >> 3) & 63, hl = (idx >> 9) & 1, ks = (idx >> 10) & 1, mt = idx >> 11;
  const int row = lane & 15, r = (row & 7) >> 1, c = row & 1, e = kk >> 1, ci = kk & 1;
  const int p = 1 + 2 * mt + (row >> 3), q = 1 + 4 * ks + (lane >> 4);
  const float2 k = K[(p * NPATH + q) * 16 + 4 * r + e];
  // (re, im) of the product k x: re = k.re x.re - k.im x.im, im = k.im x.re + k.re x.im
  const float v = c == 0 ? (ci == 0 ? k.x : -k.y) : (ci == 0 ? k.y : k.x);
  const __bf16 hi = (__bf16)v;
  f[idx] = hl == 0 ? hi : (__bf16)(v - (float)hi);
}

template <int SIN>
__global__ __launch_bounds__(256, 3) void k_nn_pass_a_mfma(Geo g, const void *__restrict__ links,
                                                        const float2 *__restrict__ K, const bf16x8 *__restrict__ frag,
                                                        const void *__restrict__ in, size_t istride,
                                                        void *__restrict__ m, size_t mstride, size_t hoff, size_t msys,
                                                        int nsys, int par, int zb) {
  __shared__ uint4 lds_hi[4 * 3 * WAVE], lds_lo[4 * 3 * WAVE];   // [q in K-step][colour][site]
  // each lane's two links (stored rows), kept for the systems after the first:
  // in the cache they would not outlive one system's pass over the XCD
  __shared__ float4 lds_link[2 * 3 * 256];
  const int ya = blockIdx.y;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & (WAVE - 1);
  const int sb = block_order(g, xcd_remap(blockIdx.x, gridDim.x), zb), s = sb * WAVE + lane;
  const bool live = s < g.vh;
  const size_t npad = (size_t)g.nb * WAVE;
  if (ya == par) {
    if (w != 0 || !live) return;
#pragma unroll 1
    for (int sy = 0; sy < nsys; ++sy) {
      cpx<float> v[12], o[12];
      load_as_f32<SIN>((const char *)in + sy * istride, s, npad, v);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = cmake(0.f, 0.f);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const cpx<float> kr = cmake(K[4 * r + e].x, K[4 * r + e].y);
#pragma unroll
          for (int a = 0; a < 3; ++a) o[4 * a + r] = cmac(kr, v[4 * a + e], o[4 * a + r]);
        }
      SpinorIO<S_F32>::store((char *)m + sy * msys + ya * hoff, s, npad, o);
    }
    return;
  }
  // every lane takes part in the matrix products; lanes past the last site
  // carry zeros and store nothing
  const SiteC c = site_c(g, live ? s : sb * WAVE, ya);
  bf16x8 A[2][2];   // [ks][hi, lo] of M-tile w
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int hl = 0; hl < 2; ++hl) A[ks][hl] = frag[((w * 2 + ks) * 2 + hl) * WAVE + lane];
#pragma unroll 1
  for (int sy = 0; sy < nsys; ++sy) {
    const void *in_s = (const char *)in + sy * istride;
    f32x4 D[4][3];   // [site tile][colour]
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) D[j][a] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int g4 = lane >> 4, n = lane & 15;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      cpx<float> t[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) t[k] = cmake(0.f, 0.f);
      if (live) {
        int mu;
        bool fwd;
        path_of(1 + 4 * ks + w, mu, fwd);
        const int nb_ = nbr(g, c, mu, fwd);
        cpx<float> u[9], psi[12];
        LinkIO<L_F32R12>::Raw lr;
        float4 *st = lds_link + ks * 3 * 256 + threadIdx.x;
        if (sy == 0) {
          if (fwd) LinkIO<L_F32R12>::fetch(links, ya, mu, s, g.nb, lr);
          else LinkIO<L_F32R12>::fetch(links, 1 - ya, mu, nb_, g.nb, lr);
          if (nsys > 1)
#pragma unroll
            for (int j = 0; j < 3; ++j) st[j * 256] = lr.q[j];
        } else {
#pragma unroll
          for (int j = 0; j < 3; ++j) lr.q[j] = st[j * 256];
        }
        LinkIO<L_F32R12>::decode(lr, u);
        load_as_f32<SIN>(in_s, nb_, npad, psi);
        transport(u, psi, t, !fwd);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bf16x8 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float xr = t[4 * a + e].re, xi = t[4 * a + e].im;
          const __bf16 hr = (__bf16)xr, hi = (__bf16)xi;
          h[2 * e] = hr;
          h[2 * e + 1] = hi;
          l[2 * e] = (__bf16)(xr - (float)hr);
          l[2 * e + 1] = (__bf16)(xi - (float)hi);
        }
        lds_hi[(w * 3 + a) * WAVE + lane] = __builtin_bit_cast(uint4, h);
        lds_lo[(w * 3 + a) * WAVE + lane] = __builtin_bit_cast(uint4, l);
      }
      __syncthreads();
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bf16x8 bh = __builtin_bit_cast(bf16x8, lds_hi[(g4 * 3 + a) * WAVE + 16 * j + n]);
          const bf16x8 bl = __builtin_bit_cast(bf16x8, lds_lo[(g4 * 3 + a) * WAVE + 16 * j + n]);
          D[j][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][0], bh, D[j][a], 0, 0, 0);
          D[j][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][0], bl, D[j][a], 0, 0, 0);
          D[j][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][1], bh, D[j][a], 0, 0, 0);
        }
      __syncthreads();   // the next K-step overwrites the LDS tiles
    }
    // lane (g4, n) holds rows 4 g4 .. 4 g4 + 3 of column (site 16 j + n, colour a):
    // path 1 + 2w + g4 / 2, float4 unit 2a + g4 % 2 of the F32 spinor layout
    float4 *base = (float4 *)((char *)m + sy * msys + (size_t)(1 + 2 * w + (g4 >> 1)) * mstride + ya * hoff);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (sb * WAVE + 16 * j + n >= g.vh) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const f32x4 d = D[j][a];
        base[((size_t)sb * 6 + 2 * a + (g4 & 1)) * WAVE + 16 * j + n] = make_float4(d[0], d[1], d[2], d[3]);
      }
    }
  }
}

// Pass B: out(x) = sum_p (T_p m_p)(x) at the sites of parity out_par (both if
// negative; grid (ceil(nb / 4), 1 or 2), four site blocks in the hop's
// XCD-mapped order), written in storage SOUT to out0 (even half) or out1 (odd
// half).  Path fields as in pass A; nsys systems one after the other (outputs
// ostride bytes apart), reusing the block's links from the cache.
template <int SOUT, bool MULTI>
__global__ __launch_bounds__(256) void k_nn_pass_b(Geo g, const void *__restrict__ links, const void *__restrict__ m,
                                                   size_t mstride, size_t hoff, size_t msys, void *__restrict__ out0,
                                                   void *__restrict__ out1, size_t ostride, int nsys, int out_par,
                                                   int zb) {
  const int px = out_par >= 0 ? out_par : (int)blockIdx.y;
  const int L = xcd_remap(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6);
  if (L >= g.nb) return;
  const int s = block_order(g, L, zb) * WAVE + (int)(threadIdx.x & (WAVE - 1));
  if (s >= g.vh) return;
  const size_t npad = (size_t)g.nb * WAVE;
  const SiteC c = site_c(g, s, px);
  // one system: no loop state, so the kernel keeps five waves per SIMD
  const int ns = MULTI ? nsys : 1;
#pragma unroll 1
  for (int sy = 0; sy < ns; ++sy) {
    const char *ms = (const char *)m + sy * msys;
    cpx<float> acc[12];
    SpinorIO<S_F32>::load(ms + px * hoff, s, npad, acc);
#pragma unroll 1
    for (int p = 1; p < NPATH; ++p) {
      cpx<float> t[12];
      path_apply(g, links, ms + (size_t)p * mstride, hoff, npad, c, px, p, t);
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = cadd(acc[k], t[k]);
    }
    void *dst = (char *)(px ? out1 : out0) + sy * ostride;
    if constexpr (SOUT == S_F32) {
      SpinorIO<S_F32>::store(dst, s, npad, acc);
    } else {
      cpx<double> d[12];
      cvt12(acc, d);
      SpinorIO<S_F64>::store(dst, s, npad, d);
    }
  }
}

// dL/d conj(W_p^{ij}) = sum_{x,c} g^i(x)[c][r] conj((T_p psi^j)(x)[c][s]).  One
// block row per path p and chunk of JC inputs j and IC outputs i (the link of
// p is loaded once per site for the JC transports, each g^i once for the JC
// inputs), WG_CHUNKS site chunks, partials in FP64 per (p, i, j), each over the
// same sites in the same order as with one row per pair.
template <int CIN, int COUT, int JC, int IC>
__global__ __launch_bounds__(256) void k_ptc_wgrad(Geo g, const void *__restrict__ links, const void *__restrict__ in,
                                                   const void *__restrict__ gout, size_t fstride,
                                                   double *__restrict__ part) {
  static_assert(CIN % JC == 0 && COUT % IC == 0, "k_ptc_wgrad: whole chunks");
  constexpr int NJ = CIN / JC, NI = COUT / IC;
  const int row = blockIdx.y;   // (p * NI + ib) * NJ + jb
  const int jb = row % NJ, ib = (row / NJ) % NI, p = row / (NJ * NI);
  const size_t npad = (size_t)g.nb * WAVE, hb = npad * SpinorIO<S_F32>::SITE_BYTES;
  const size_t nsite = 2 * npad;
  cpx<float> acc[IC][JC][16];
#pragma unroll
  for (int ii = 0; ii < IC; ++ii)
#pragma unroll
    for (int jj = 0; jj < JC; ++jj)
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[ii][jj][k] = cmake(0.f, 0.f);
  for (size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x; gid < nsite; gid += (size_t)gridDim.x * blockDim.x) {
    const int par = (int)(gid / npad), s = (int)(gid % npad);
    if (s >= g.vh) continue;
    const SiteC c = site_c(g, s, par);
    cpx<float> t[JC][12];
    if (p == 0) {
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
        SpinorIO<S_F32>::load((const char *)in + (size_t)(jb * JC + jj) * fstride + par * hb, s, npad, t[jj]);
    } else {
      int mu;
      bool fwd;
      path_of(p, mu, fwd);
      const int n = nbr(g, c, mu, fwd);
      cpx<float> u[9];
      if (fwd) LinkIO<L_F32R12>::load(links, par, mu, c.s, g.nb, u);
      else LinkIO<L_F32R12>::load(links, 1 - par, mu, n, g.nb, u);
#pragma unroll
      for (int jj = 0; jj < JC; ++jj) {
        cpx<float> psi[12];
        SpinorIO<S_F32>::load((const char *)in + (size_t)(jb * JC + jj) * fstride + (1 - par) * hb, n, npad, psi);
        transport(u, psi, t[jj], !fwd);
      }
    }
#pragma unroll
    for (int ii = 0; ii < IC; ++ii) {
      cpx<float> gg[12];
      SpinorIO<S_F32>::load((const char *)gout + (size_t)(ib * IC + ii) * fstride + par * hb, s, npad, gg);
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a)
              acc[ii][jj][4 * r + q] = cjmac(t[jj][4 * a + q], gg[4 * a + r], acc[ii][jj][4 * r + q]);
    }
  }
  // fixed-order block reduction, one (i, j) pair after the other
  __shared__ double red[32][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int ii = 0; ii < IC; ++ii)
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        double re = wave_sum((double)acc[ii][jj][k].re), im = wave_sum((double)acc[ii][jj][k].im);
        if (lane == 0) { red[2 * k][wv] = re; red[2 * k + 1][wv] = im; }
      }
      __syncthreads();
      if (threadIdx.x < 32) {
        const int combo = (p * COUT + ib * IC + ii) * CIN + jb * JC + jj;
        const double v = (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
        part[((size_t)combo * gridDim.x + blockIdx.x) * 32 + threadIdx.x] = v;
      }
      __syncthreads();   // red is written again for the next pair
    }
}

// grad[2 k] = dL/dRe W_k = 2 Re G_k, grad[2 k + 1] = dL/dIm W_k = 2 Im G_k.
__global__ void k_wgrad_final(const double *__restrict__ part, double *__restrict__ grad, int ncombo, int nchunk) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncombo * 32) return;
  const int combo = idx >> 5, k = idx & 31;
  double s = 0.0;
#pragma unroll 8
  for (int ch = 0; ch < nchunk; ++ch) s += part[((size_t)combo * nchunk + ch) * 32 + k];
  grad[(size_t)combo * 32 + k] = 2.0 * s;
}

// Adam on the real and imaginary parts of every weight.
__global__ void k_adam(float *__restrict__ theta, const double *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gr = (float)grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gr;
  const float vi = b2 * v[i] + (1.f - b2) * gr * gr;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Philox4x32-10 (Salmon et al. 2011): 10 rounds of the multiply-xor round with
// the published multipliers and Weyl key increments.
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const unsigned hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// Gaussian training vector: the 24 reals of canonical site `lex` come from six
// Philox blocks with counter (lex, block, step_lo, step_hi) and key (seed_lo,
// seed_hi); uniforms u = (n + 1/2) 2^-32 pair into Box-Muller normals
// sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1).  Also partial sums of ||v||^2.
__global__ __launch_bounds__(256) void k_gauss(Geo g, void *__restrict__ out, uint2 key, unsigned long long step,
                                               double *__restrict__ part) {
  const size_t npad = (size_t)g.nb * WAVE, hb = npad * SpinorIO<S_F32>::SITE_BYTES;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double nrm = 0.0;
  if (gid < 2 * npad) {
    const int par = (int)(gid / npad), s = (int)(gid % npad);
    cpx<float> v[12];
    if (s < g.vh) {
      const SiteC c = site_c(g, s, par);
      const unsigned lex = (unsigned)((((size_t)c.t * g.lz + c.z) * g.ly + c.y) * g.lx + c.x);
      float r[24];
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const uint4 u = philox(make_uint4(lex, (unsigned)b, (unsigned)step, (unsigned)(step >> 32)), key);
        const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float u0 = ((float)w[2 * h] + 0.5f) * 2.3283064365386963e-10f;
          const float u1 = ((float)w[2 * h + 1] + 0.5f) * 2.3283064365386963e-10f;
          const float rad = sqrtf(-2.f * logf(u0));
          r[4 * b + 2 * h] = rad * cosf(6.283185307179586f * u1);
          r[4 * b + 2 * h + 1] = rad * sinf(6.283185307179586f * u1);
        }
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = cmake(r[2 * k], r[2 * k + 1]);
      nrm = norm12(v);
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = cmake(0.f, 0.f);
    }
    SpinorIO<S_F32>::store((char *)out + par * hb, s, npad, v);
  }
  nrm = wave_sum(nrm);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// g = (y - v) / ||v||^2 and partials of ||y - v||^2.
__global__ __launch_bounds__(256) void k_loss_grad(Geo g, const void *__restrict__ y, const void *__restrict__ v,
                                                   void *__restrict__ gout, const double *__restrict__ vnorm,
                                                   double *__restrict__ part) {
  const size_t npad = (size_t)g.nb * WAVE, hb = npad * SpinorIO<S_F32>::SITE_BYTES;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d2 = 0.0;
  if (gid < 2 * npad) {
    const int par = (int)(gid / npad), s = (int)(gid % npad);
    cpx<float> a[12], b[12];
    SpinorIO<S_F32>::load((const char *)y + par * hb, s, npad, a);
    SpinorIO<S_F32>::load((const char *)v + par * hb, s, npad, b);
    const float inv = (float)(1.0 / vnorm[0]);
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = csub(a[k], b[k]);
    d2 = s < g.vh ? norm12(a) : 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = cscale(inv, a[k]);
    SpinorIO<S_F32>::store((char *)gout + par * hb, s, npad, a);
  }
  d2 = wave_sum(d2);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d2;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Sum of x[i], i = tid, tid + 256, ... < n, as four interleaved chains (i / 256
// mod 4) added at the end: a fixed order, with four loads in flight per thread
// where one chain would wait out a memory latency per element.
template <class T> __device__ __forceinline__ T zero_of();
template <> __device__ __forceinline__ double zero_of<double>() { return 0.0; }
template <> __device__ __forceinline__ double2 zero_of<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double add_of(double a, double b) { return a + b; }
__device__ __forceinline__ double2 add_of(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
template <class T> __device__ __forceinline__ T strided_sum(const T *__restrict__ x, int n, int tid) {
  T c0 = zero_of<T>(), c1 = c0, c2 = c0, c3 = c0;
  int i = tid;
  for (; i + 768 < n; i += 1024) {
    const T a = x[i], b = x[i + 256], c = x[i + 512], d = x[i + 768];
    c0 = add_of(c0, a);
    c1 = add_of(c1, b);
    c2 = add_of(c2, c);
    c3 = add_of(c3, d);
  }
  if (i < n) c0 = add_of(c0, x[i]);
  if (i + 256 < n) c1 = add_of(c1, x[i + 256]);
  if (i + 512 < n) c2 = add_of(c2, x[i + 512]);
  return add_of(add_of(c0, c1), add_of(c2, c3));
}

// out[0] = sum(part[0..n)) (divided by divisor[0] if given), in a fixed order
// (one work-group).
__global__ __launch_bounds__(256) void k_sum(const double *__restrict__ part, int n, double *__restrict__ out,
                                             const double *__restrict__ divisor) {
  __shared__ double red[4];
  double a = strided_sum(part, n, (int)threadIdx.x);
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    out[0] = divisor ? s / divisor[0] : s;
  }
}

// ---------------------------------------------------------------------------
// FP64 full-field vector kernels for FGMRES (both halves, padding stays zero)
// out = C in on a packed F64 half-field, C the twisted-mass site factor `mode`
// (CHI_*; a copy at mu = 0)
__global__ __launch_bounds__(256) void k_chi64(Geo g, const void *__restrict__ in, void *__restrict__ out, int mode,
                                               double tmu) {
  const size_t npad = (size_t)g.nb * WAVE;
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= npad) return;
  cpx<double> v[12];
  SpinorIO<S_F64>::load(in, (int)s, npad, v);
  apply_chi(v, mode, tmu);
  SpinorIO<S_F64>::store(out, (int)s, npad, v);
}


// Complex dots (V_i | w) for i < k, with partials per work-group.
__global__ __launch_bounds__(256) void k_mdot(const double2 *__restrict__ V, size_t vstride, int k,
                                              const double2 *__restrict__ w, size_t n, double *__restrict__ part) {
  __shared__ double red[2][4];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double2 wv = i < n ? w[i] : make_double2(0.0, 0.0);
  for (int q = 0; q < k; ++q) {
    double re = 0.0, im = 0.0;
    if (i < n) {
      const double2 v = V[q * vstride + i];
      re = v.x * wv.x + v.y * wv.y;
      im = v.x * wv.y - v.y * wv.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = re; red[1][threadIdx.x >> 6] = im; }
    __syncthreads();
    if (threadIdx.x < 2)
      part[((size_t)q * gridDim.x + blockIdx.x) * 2 + threadIdx.x] =
          (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
    __syncthreads();
  }
}

// coef[q] = sum of the partial pairs of coefficient q, one work-group per q
// (grid = k): strided sums, then a fixed-order wave and work-group reduction.
__global__ __launch_bounds__(256) void k_mdot_final(const double *__restrict__ part, int nblk,
                                                    double2 *__restrict__ coef) {
  __shared__ double red[2][4];
  const int q = blockIdx.x;
  const double2 sum = strided_sum((const double2 *)(part + (size_t)q * nblk * 2), nblk, (int)threadIdx.x);
  const double re = wave_sum(sum.x), im = wave_sum(sum.y);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = re; red[1][threadIdx.x >> 6] = im; }
  __syncthreads();
  if (threadIdx.x == 0)
    coef[q] = make_double2((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]),
                           (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
}

// w += sign * sum_q coef[q] V_q
__global__ __launch_bounds__(256) void k_maxpy(const double2 *__restrict__ V, size_t vstride, int k,
                                               const double2 *__restrict__ coef, double sign, double2 *__restrict__ w,
                                               size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 a = w[i];
  for (int q = 0; q < k; ++q) {
    const double2 c = coef[q], v = V[q * vstride + i];
    a.x += sign * (c.x * v.x - c.y * v.y);
    a.y += sign * (c.x * v.y + c.y * v.x);
  }
  w[i] = a;
}

// partial sums of |w|^2
__global__ __launch_bounds__(256) void k_norm(const double2 *__restrict__ w, size_t n, double *__restrict__ part) {
  __shared__ double red[4];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double a = 0.0;
  if (i < n) a = w[i].x * w[i].x + w[i].y * w[i].y;
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// k_norm for nsys vectors of n2 entries each (a whole number of nbk 256-entry
// blocks), optionally as two halves a and b of one field per system: grid
// (nsys * nbk, 1 or 2); part[(k * halves + half) * nbk + block], so that system
// k's partials are those k_norm gives for its field a (then b) alone.
__global__ __launch_bounds__(256) void k_norm_sys(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                                  size_t n2, int nbk, double *__restrict__ part) {
  __shared__ double red[4];
  const int k = blockIdx.x / nbk, j = blockIdx.x - k * nbk, half = blockIdx.y;
  const double2 *w = (half ? b : a) + (size_t)k * n2;
  const size_t i = (size_t)j * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n2) v = w[i].x * w[i].x + w[i].y * w[i].y;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[((size_t)k * gridDim.y + half) * nbk + j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// v = w / sqrt(nrm2[0])  (zero if the norm is zero)
__global__ __launch_bounds__(256) void k_scale(const double2 *__restrict__ w, const double *__restrict__ nrm2,
                                               double2 *__restrict__ v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
  v[i] = make_double2(w[i].x * s, w[i].y * s);
}

// r = b - r   (r holds D x on entry)
__global__ __launch_bounds__(256) void k_bminus(const double2 *__restrict__ b, double2 *__restrict__ r, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = make_double2(b[i].x - r[i].x, b[i].y - r[i].y);
}


// Right-preconditioned BiCGStab's scalars, kept on the device in coef[] so that
// an iteration needs one read by the host (||r||^2 and the breakdown flags).
enum : int {
  BQ_RHO = 40, BQ_ALPHA, BQ_OMEGA, BQ_RHO1, BQ_RV, BQ_TS, BQ_TT, BQ_RN2, BQ_FLAG,   // scalars; FLAG.x, .y below
  BQ_C_OMEGA = 50, BQ_C_BETA, BQ_C_MALPHA, BQ_C_X, BQ_C_X2, BQ_C_MOMEGA,     // coefficients of the vector kernels
  BQ_DONE = 56,            // DONE.x != 0: the system is retired; its x and r stay as they are
  BQ_BN2, BQ_TR2,          // .x: ||b||^2 of the full source, ||b - D x||^2 of the final x
  BQ_SLOTS = 64            // coefficient slots per system: system k's are coef[64 k ..]
};

// k_sum per system: coef[BQ_SLOTS k + slot].x = the sum of part[n k .. n k + n)
// in k_sum's order; one work-group per system
__global__ __launch_bounds__(256) void k_sum_sys(const double *__restrict__ part, int n, double2 *__restrict__ coef,
                                                 int slot) {
  __shared__ double red[4];
  double a = strided_sum(part + (size_t)blockIdx.x * n, n, (int)threadIdx.x);
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) coef[(size_t)blockIdx.x * BQ_SLOTS + slot].x = (red[0] + red[1]) + (red[2] + red[3]);
}
// FLAG.x: the iteration broke down before x changed (rho_new or (r~, v) zero):
// every later coefficient is 0, so x keeps its value and every vector stays
// finite; FLAG.y: omega = 0, restart after this iteration.

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// a / b by Smith's method (scaled by the larger part of b)
__device__ inline double2 zdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ inline bool zzero(double2 a) { return a.x == 0.0 && a.y == 0.0; }

// (re)start: rho = alpha = omega = 1, no flags
// The scalar steps run for nsys systems at once, one thread each, on system
// k's slots coef[BQ_SLOTS k ..].  A system marked DONE gets coefficients that
// leave x and r as they are (p = r, s = r, x += 0, r = s).
__global__ void k_bq_init(double2 *coef, int nsys) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsys) return;
  double2 *c = coef + (size_t)k * BQ_SLOTS;
  c[BQ_RHO] = c[BQ_ALPHA] = c[BQ_OMEGA] = make_double2(1.0, 0.0);
  c[BQ_FLAG] = make_double2(0.0, 0.0);
}

// beta = (rho_new / rho) (alpha / omega); coefficients of p = r + beta (p - omega v)
__global__ void k_bq_beta(double2 *coef, int nsys) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsys) return;
  double2 *c = coef + (size_t)k * BQ_SLOTS;
  const double2 rho1 = c[BQ_RHO1];
  double2 beta = make_double2(0.0, 0.0), om = make_double2(0.0, 0.0);
  if (c[BQ_DONE].x != 0.0) {
    // p = r
  } else if (zzero(rho1)) {
    c[BQ_FLAG].x = 1.0;
  } else {
    beta = zmul(zdiv(rho1, c[BQ_RHO]), zdiv(c[BQ_ALPHA], c[BQ_OMEGA]));
    om = c[BQ_OMEGA];
    c[BQ_RHO] = rho1;
  }
  c[BQ_C_OMEGA] = om;
  c[BQ_C_BETA] = beta;
}

// alpha = rho_new / (r~, v); coefficient of s = r - alpha v
__global__ void k_bq_alpha(double2 *coef, int nsys) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsys) return;
  double2 *c = coef + (size_t)k * BQ_SLOTS;
  double2 al = make_double2(0.0, 0.0);
  if (c[BQ_FLAG].x == 0.0 && c[BQ_DONE].x == 0.0) {
    if (zzero(c[BQ_RV])) c[BQ_FLAG].x = 1.0;
    else al = zdiv(c[BQ_RHO], c[BQ_RV]);   // BQ_RHO holds rho_new by now
  }
  c[BQ_ALPHA] = al;
  c[BQ_C_MALPHA] = make_double2(-al.x, -al.y);
}

// omega = (t, s) / (t, t); coefficients of x += alpha p^ + omega s^ and r = s - omega t
__global__ void k_bq_omega(double2 *coef, int nsys) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsys) return;
  double2 *c = coef + (size_t)k * BQ_SLOTS;
  const double tt = c[BQ_TT].x;
  double2 om = make_double2(0.0, 0.0), al = c[BQ_ALPHA];
  if (c[BQ_DONE].x != 0.0) {
    al = make_double2(0.0, 0.0);
  } else if (c[BQ_FLAG].x == 0.0) {
    if (tt > 0.0) om = make_double2(c[BQ_TS].x / tt, c[BQ_TS].y / tt);
    if (zzero(om)) c[BQ_FLAG].y = 1.0;
  } else {
    al = make_double2(0.0, 0.0);
  }
  c[BQ_OMEGA] = om;
  c[BQ_C_X] = al;
  c[BQ_C_X2] = om;
  c[BQ_C_MOMEGA] = make_double2(-om.x, -om.y);
}

// Fused BiCGStab vector steps over the Krylov vectors of nsys systems, one
// after the other (system k = element / n2; n2 is a whole number of 256-entry
// work-groups, so a work-group never spans two systems).
// Block partial pairs of a complex dot, (a | b) = sum conj(a) b, in the order
// of k_mdot: wave sums, then (w0 + w1) + (w2 + w3).
__device__ __forceinline__ void block_pair(double re, double im, double *__restrict__ dst) {
  __shared__ double red[2][4];
  re = wave_sum(re);
  im = wave_sum(im);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = re; red[1][threadIdx.x >> 6] = im; }
  __syncthreads();
  if (threadIdx.x < 2)
    dst[threadIdx.x] = (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
}

// Two block partial pairs at once, each summed as block_pair sums it, with one
// barrier: p0 = (re0, im0) to dst0, p1 = (re1, im1) to dst1.
__device__ __forceinline__ void block_pair2(double re0, double im0, double re1, double im1, double *__restrict__ dst0,
                                            double *__restrict__ dst1) {
  __shared__ double red[4][4];
  re0 = wave_sum(re0);
  im0 = wave_sum(im0);
  re1 = wave_sum(re1);
  im1 = wave_sum(im1);
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    red[0][w] = re0;
    red[1][w] = im0;
    red[2][w] = re1;
    red[3][w] = im1;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int t = threadIdx.x;
    const double v = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
    if (t < 2) dst0[t] = v;
    else dst1[t - 2] = v;
  }
}

__device__ __forceinline__ const double2 *sys_coef(const double2 *coef, size_t i, size_t n2) {
  return coef + (i / n2) * BQ_SLOTS;
}

// P = R + beta (P - omega V)
__global__ __launch_bounds__(256) void k_bq_p(const double2 *__restrict__ coef, const double2 *__restrict__ R,
                                              const double2 *__restrict__ V, double2 *__restrict__ P, size_t n2,
                                              size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 *c = sys_coef(coef, i, n2);
  const double2 be = c[BQ_C_BETA], om = c[BQ_C_OMEGA], r = R[i], v = V[i];
  double2 p = P[i];
  p.x -= om.x * v.x - om.y * v.y;
  p.y -= om.x * v.y + om.y * v.x;
  P[i] = make_double2(r.x + (be.x * p.x - be.y * p.y), r.y + (be.x * p.y + be.y * p.x));
}

// S = R - alpha V
__global__ __launch_bounds__(256) void k_bq_s(const double2 *__restrict__ coef, const double2 *__restrict__ V,
                                              const double2 *__restrict__ R, double2 *__restrict__ S, size_t n2,
                                              size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 a = sys_coef(coef, i, n2)[BQ_C_MALPHA], v = V[i], r = R[i];
  S[i] = make_double2(r.x + (a.x * v.x - a.y * v.y), r.y + (a.x * v.y + a.y * v.x));
}

// X += alpha PH + omega SH
__global__ __launch_bounds__(256) void k_bq_x(const double2 *__restrict__ coef, const double2 *__restrict__ PH,
                                              const double2 *__restrict__ SH, double2 *__restrict__ X, size_t n2,
                                              size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 *c = sys_coef(coef, i, n2);
  const double2 al = c[BQ_C_X], om = c[BQ_C_X2], ph = PH[i], sh = SH[i];
  double2 x = X[i];
  x.x += al.x * ph.x - al.y * ph.y;
  x.y += al.x * ph.y + al.y * ph.x;
  x.x += om.x * sh.x - om.y * sh.y;
  x.y += om.x * sh.y + om.y * sh.x;
  X[i] = x;
}

// partial pairs of (a | b): part[block * 2 + re/im]
__global__ __launch_bounds__(256) void k_dot1(const double2 *__restrict__ a, const double2 *__restrict__ b, size_t n,
                                              double *__restrict__ part) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 ab = make_double2(0.0, 0.0);
  if (i < n) {
    const double2 av = a[i], bv = b[i];
    ab = make_double2(av.x * bv.x + av.y * bv.y, av.x * bv.y - av.y * bv.x);
  }
  block_pair(ab.x, ab.y, part + (size_t)blockIdx.x * 2);
}

// partial pairs of (a | b) and (a | a): part[(q * gridDim.x + block) * 2 + re/im]
__global__ __launch_bounds__(256) void k_dot2(const double2 *__restrict__ a, const double2 *__restrict__ b, size_t n,
                                              double *__restrict__ part) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 ab = make_double2(0.0, 0.0), aa = ab;
  if (i < n) {
    const double2 av = a[i], bv = b[i];
    ab = make_double2(av.x * bv.x + av.y * bv.y, av.x * bv.y - av.y * bv.x);
    aa = make_double2(av.x * av.x + av.y * av.y, av.x * av.y - av.y * av.x);
  }
  block_pair2(ab.x, ab.y, aa.x, aa.y, part + (size_t)blockIdx.x * 2, part + ((size_t)gridDim.x + blockIdx.x) * 2);
}

// R = S - omega T, with the partial pairs of (RT | R) and (R | R), laid out as k_dot2's
__global__ __launch_bounds__(256) void k_bq_r(const double2 *__restrict__ coef, const double2 *__restrict__ S,
                                              const double2 *__restrict__ T, const double2 *__restrict__ RT,
                                              double2 *__restrict__ R, size_t n2, size_t n, double *__restrict__ part) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 rr = make_double2(0.0, 0.0), tr = rr;
  if (i < n) {
    const double2 a = sys_coef(coef, i, n2)[BQ_C_MOMEGA], sv = S[i], tv = T[i], rt = RT[i];
    const double2 r = make_double2(sv.x + (a.x * tv.x - a.y * tv.y), sv.y + (a.x * tv.y + a.y * tv.x));
    R[i] = r;
    tr = make_double2(rt.x * r.x + rt.y * r.y, rt.x * r.y - rt.y * r.x);
    rr = make_double2(r.x * r.x + r.y * r.y, 0.0);
  }
  block_pair2(tr.x, tr.y, rr.x, rr.y, part + (size_t)blockIdx.x * 2, part + ((size_t)gridDim.x + blockIdx.x) * 2);
}

// Sums of partial-pair rows: grid (nrow, nsys), row q of system k (its nbk
// work-groups of a kernel that ran over nsys * nbk) into coef[BQ_SLOTS k + slot_q].
__global__ __launch_bounds__(256) void k_pair_final(const double *__restrict__ part, int nbk,
                                                    double2 *__restrict__ coef, int slot0, int slot1) {
  __shared__ double red[2][4];
  const int q = blockIdx.x, k = blockIdx.y;
  const size_t row = ((size_t)q * gridDim.y + k) * nbk;
  const double2 sum = strided_sum((const double2 *)(part + row * 2), nbk, (int)threadIdx.x);
  const double re = wave_sum(sum.x), im = wave_sum(sum.y);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = re; red[1][threadIdx.x >> 6] = im; }
  __syncthreads();
  if (threadIdx.x == 0)
    coef[(size_t)k * BQ_SLOTS + (q == 0 ? slot0 : slot1)] =
        make_double2((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]), (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
}

// FCG step: x += alpha p, r -= alpha q, s -= alpha w (alpha = coef[0]); partial
// sums of |s|^2 per work-group
__global__ __launch_bounds__(256) void k_fcg_upd(const double2 *__restrict__ coef, const double2 *__restrict__ p,
                                                 const double2 *__restrict__ q, const double2 *__restrict__ w,
                                                 double2 *__restrict__ x, double2 *__restrict__ r,
                                                 double2 *__restrict__ sv, size_t n, double *__restrict__ part) {
  __shared__ double red[4];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double a = 0.0;
  if (i < n) {
    const double2 al = coef[0], pv = p[i], qv = q[i], wv = w[i];
    double2 xv = x[i], rv = r[i], s = sv[i];
    xv.x += al.x * pv.x - al.y * pv.y;
    xv.y += al.x * pv.y + al.y * pv.x;
    rv.x -= al.x * qv.x - al.y * qv.y;
    rv.y -= al.x * qv.y + al.y * qv.x;
    s.x -= al.x * wv.x - al.y * wv.y;
    s.y -= al.x * wv.y + al.y * wv.x;
    x[i] = xv;
    r[i] = rv;
    sv[i] = s;
    a = s.x * s.x + s.y * s.y;
  }
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// partial sums of ||f||^2 over the sites of a packed F32 full field
__global__ __launch_bounds__(256) void k_norm32(Geo g, const void *__restrict__ f, double *__restrict__ part) {
  const size_t npad = (size_t)g.nb * WAVE, hb = npad * SpinorIO<S_F32>::SITE_BYTES;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double a = 0.0;
  if (gid < 2 * npad) {
    const int par = (int)(gid / npad), s = (int)(gid % npad);
    if (s < g.vh) {
      cpx<float> v[12];
      SpinorIO<S_F32>::load((const char *)f + par * hb, s, npad, v);
      a = norm12(v);
    }
  }
  a = wave_sum(a);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

inline int nblk(size_t n) { return (int)((n + 255) / 256); }

// ---------------------------------------------------------------------------
// host helpers
size_t full_bytes32(const Geo &g) { return 2 * half_bytes(g, QIRAL_F32); }
size_t full_bytes64(const Geo &g) { return 2 * half_bytes(g, QIRAL_F64); }

hipError_t layer_launch(const qiral_nn *nn, const float2 *w, int cin, int cout, const void *in, void *out,
                        hipStream_t s) {
  const Geo &g = nn->lat->geo;
  const size_t fs = full_bytes32(g);
  const int nb = nblk(2 * npad_of(g));
  const void *links = nn->lat->g32;
  // 1 -> 8 in two passes of 4 channels (184 VGPRs): one pass of 8 (256 VGPRs, one
  // wave per SIMD) recomputes no transport but measured 12% slower
  if (cin == 1 && cout == 8)
    hipLaunchKernelGGL((k_ptc_layer<1, 8, 4>), dim3(nb), dim3(256), 0, s, g, links, w, in, out, fs);
  else if (cin == 8 && cout == 1)
    hipLaunchKernelGGL((k_ptc_layer<8, 1, 1>), dim3(nb), dim3(256), 0, s, g, links, w, in, out, fs);
  else if (cin == 1 && cout == 4)
    hipLaunchKernelGGL((k_ptc_layer<1, 4, 4>), dim3(nb), dim3(256), 0, s, g, links, w, in, out, fs);
  else if (cin == 4 && cout == 1)
    hipLaunchKernelGGL((k_ptc_layer<4, 1, 1>), dim3(nb), dim3(256), 0, s, g, links, w, in, out, fs);
  else if (cin == 1 && cout == 2)
    hipLaunchKernelGGL((k_ptc_layer<1, 2, 2>), dim3(nb), dim3(256), 0, s, g, links, w, in, out, fs);
  else if (cin == 2 && cout == 1)
    hipLaunchKernelGGL((k_ptc_layer<2, 1, 1>), dim3(nb), dim3(256), 0, s, g, links, w, in, out, fs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t wgrad_launch(const qiral_nn *nn, int cin, int cout, const void *in, const void *gout, double *grad,
                        hipStream_t s) {
  const Geo &g = nn->lat->geo;
  const size_t fs = full_bytes32(g);
  const int ncombo = NPATH * cin * cout;
  // rows of 2 (p, i, j) pairs: one transport or one g^i serves both
  dim3 grid(WG_CHUNKS, ncombo / 2);
  const void *links = nn->lat->g32;
  if (cin == 1 && cout == 8) hipLaunchKernelGGL((k_ptc_wgrad<1, 8, 1, 2>), grid, dim3(256), 0, s, g, links, in, gout, fs, nn->part);
  else if (cin == 8 && cout == 1) hipLaunchKernelGGL((k_ptc_wgrad<8, 1, 2, 1>), grid, dim3(256), 0, s, g, links, in, gout, fs, nn->part);
  else if (cin == 1 && cout == 4) hipLaunchKernelGGL((k_ptc_wgrad<1, 4, 1, 2>), grid, dim3(256), 0, s, g, links, in, gout, fs, nn->part);
  else if (cin == 4 && cout == 1) hipLaunchKernelGGL((k_ptc_wgrad<4, 1, 2, 1>), grid, dim3(256), 0, s, g, links, in, gout, fs, nn->part);
  else if (cin == 1 && cout == 2) hipLaunchKernelGGL((k_ptc_wgrad<1, 2, 1, 2>), grid, dim3(256), 0, s, g, links, in, gout, fs, nn->part);
  else if (cin == 2 && cout == 1) hipLaunchKernelGGL((k_ptc_wgrad<2, 1, 2, 1>), grid, dim3(256), 0, s, g, links, in, gout, fs, nn->part);
  else return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_wgrad_final, dim3((ncombo * 32 + 255) / 256), dim3(256), 0, s, nn->part, grad, ncombo, WG_CHUNKS);
  return hipGetLastError();
}

// K and K' of the current weights into nn->kmat, and their MFMA fragments into
// nn->kfrag (before folded inference).
hipError_t nn_fold(const qiral_nn *nn, hipStream_t s) {
  const int n = NPATH * NPATH * 16, nf = 4 * 2 * 2 * 64 * 8;
  for (int adj = 0; adj < 2; ++adj) {
    hipLaunchKernelGGL(k_nn_fold, dim3((n + 255) / 256), dim3(256), 0, s, nn->w, nn->w + nn->nw1, nn->hidden, adj,
                       nn->kmat + adj * n);
    hipLaunchKernelGGL(k_nn_frag, dim3(nf / 256), dim3(256), 0, s, (const float2 *)(nn->kmat + adj * n),
                       (__bf16 *)nn->kfrag + adj * nf);
  }
  return hipGetLastError();
}

// out = N(in) (adj = false) or N^dagger(in), folded, with the K of the last
// nn_fold.  SIO: storage of in and out (packed F32 or F64 fields), given as
// half-fields (in0, in1) and (out0, out1).  par >= 0: in is zero off parity par
// (in0 or in1 is then not read) and only that parity of out is written, and
// pass A runs on bf16 MFMA (about 1e-5 relative; the flexible solvers only).
// There nsys systems may go through in one pass each: inputs and outputs
// iostride bytes apart, their path fields in mbuf (nsys x 9 F32 half-fields;
// the network's own buffer when null, which holds one system's).
template <int SIO>
hipError_t nn_apply_folded(const qiral_nn *nn, void *out0, void *out1, const void *in0, const void *in1, bool adj,
                           hipStream_t s, int par = -1, int nsys = 1, size_t iostride = 0, void *mbuf = nullptr) {
  const Geo &g = nn->lat->geo;
  const size_t fs = full_bytes32(g), hb = fs / 2;
  const float2 *K = nn->kmat + (adj ? NPATH * NPATH * 16 : 0);
  const int zb = hop_zb(g);   // the hops' z-tiles: neighbours stay in one XCD's L2
  if (par >= 0) {
    // path field p is the one parity it is used on: m_0 on par, m_1..m_8 on 1 - par
    void *m = mbuf ? mbuf : nn->act;
    hipLaunchKernelGGL((k_nn_pass_a_mfma<SIO>), dim3(g.nb, 2), dim3(256), 0, s, g, nn->lat->g32, K,
                       (const bf16x8 *)nn->kfrag + (adj ? 4 * 2 * 2 * WAVE : 0), par ? in1 : in0, iostride, m, hb,
                       (size_t)0, NPATH * hb, nsys, par, zb);
    if (nsys > 1)
      hipLaunchKernelGGL((k_nn_pass_b<SIO, true>), dim3((g.nb + 3) / 4, 1), dim3(256), 0, s, g, nn->lat->g32,
                         (const void *)m, hb, (size_t)0, NPATH * hb, out0, out1, iostride, nsys, par, zb);
    else
      hipLaunchKernelGGL((k_nn_pass_b<SIO, false>), dim3((g.nb + 3) / 4, 1), dim3(256), 0, s, g, nn->lat->g32,
                         (const void *)m, hb, (size_t)0, NPATH * hb, out0, out1, (size_t)0, 1, par, zb);
  } else {   // all nine output paths in two waves per site block, five and four
    hipLaunchKernelGGL((k_nn_pass_a<SIO, 5>), dim3((g.nb + 1) / 2, 2), dim3(256), 0, s, g, nn->lat->g32, K, in0, in1,
                       nn->act, fs, zb);
    hipLaunchKernelGGL((k_nn_pass_b<SIO, false>), dim3((g.nb + 3) / 4, 2), dim3(256), 0, s, g, nn->lat->g32,
                       (const void *)nn->act, fs, hb, (size_t)0, out0, out1, (size_t)0, 1, par, zb);
  }
  return hipGetLastError();
}

// D on a packed full field (out = A in - kappa H in, A = 1 + 2 i kappa mu gamma_5), precision prec
hipError_t apply_D_full(const qiral_lattice *lat, int prec, void *out, const void *in, hipStream_t s) {
  const size_t hb = half_bytes(lat->geo, prec);
  const char *ie = (const char *)in, *io = ie + hb;
  char *oe = (char *)out, *oo = oe + hb;
  hipError_t e = launch_hop(lat, prec, 0, 0, 1, -lat->kappa, io, oe, ie, 1, s, CHI_ONE, CHI_A);
  if (e != hipSuccess) return e;
  return launch_hop(lat, prec, 0, 1, 1, -lat->kappa, ie, oo, io, 1, s, CHI_ONE, CHI_A);
}

// D^dagger on a packed full field (out = A^dagger in - kappa H^dagger in)
hipError_t apply_Ddag_full(const qiral_lattice *lat, int prec, void *out, const void *in, hipStream_t s) {
  const size_t hb = half_bytes(lat->geo, prec);
  const char *ie = (const char *)in, *io = ie + hb;
  char *oe = (char *)out, *oo = oe + hb;
  hipError_t e = launch_hop(lat, prec, 1, 0, 1, -lat->kappa, io, oe, ie, 1, s, CHI_ONE, CHI_ADAG);
  if (e != hipSuccess) return e;
  return launch_hop(lat, prec, 1, 1, 1, -lat->kappa, ie, oo, io, 1, s, CHI_ONE, CHI_ADAG);
}

void neumann2(int hidden, double kappa, std::vector<float2> &w) {
  // layer 1: ch0 = psi (identity path), ch1 = H psi; layer 2: psi + kappa ch1 + kappa^2 H ch1.
  // Spin matrices 1 -+ gamma_mu of the chiral basis gamma_mu = [[0, B],[B^+, 0]],
  // B_x = -i sigma_x, B_y = -i sigma_y, B_z = -i sigma_z, B_t = 1.
  const int nw1 = NPATH * hidden * 16, nw2 = NPATH * hidden * 16;
  w.assign(nw1 + nw2, make_float2(0.f, 0.f));
  typedef std::complex<double> C;
  const C I(0, 1);
  C B[4][2][2] = {{{0, -I}, {-I, 0}}, {{0, -1.0}, {1.0, 0}}, {{-I, 0}, {0, I}}, {{1.0, 0}, {0, 1.0}}};
  auto gamma = [&](int mu, int r, int c) -> C {
    if (r < 2 && c >= 2) return B[mu][r][c - 2];
    if (r >= 2 && c < 2) return std::conj(B[mu][c][r - 2]);
    return C(0, 0);
  };
  auto put = [&](int base, double scale, int mu, int sign) {   // scale (1 + sign gamma_mu); mu < 0: identity
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        C v = (r == c ? C(1, 0) : C(0, 0));
        if (mu >= 0) v += (double)sign * gamma(mu, r, c);
        v *= scale;
        w[base + 4 * r + c] = make_float2((float)v.real(), (float)v.imag());
      }
  };
  auto i1 = [&](int p, int i) { return ((p * hidden + i) * 1 + 0) * 16; };          // layer 1 [p][i][0]
  auto i2 = [&](int p, int j) { return nw1 + ((p * 1 + 0) * hidden + j) * 16; };   // layer 2 [p][0][j]
  put(i1(0, 0), 1.0, -1, 0);
  put(i2(0, 0), 1.0, -1, 0);
  if (hidden >= 2) {
    put(i2(0, 1), kappa, -1, 0);
    for (int mu = 0; mu < 4; ++mu) {
      put(i1(1 + mu, 1), 1.0, mu, -1);
      put(i1(5 + mu, 1), 1.0, mu, +1);
      put(i2(1 + mu, 1), kappa * kappa, mu, -1);
      put(i2(5 + mu, 1), kappa * kappa, mu, +1);
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
namespace {
// Offsets of the network's device memory (one caller-owned buffer).
struct NnLayout {
  size_t w, wadj, kmat, kfrag, am, av, grad, part, scal, act, gact, pairx, fv, fb, fy, fg, loss, total;
};
inline size_t al256(size_t v) { return (v + 255) / 256 * 256; }
NnLayout nn_layout(const Geo &g, int hidden) {
  NnLayout l;
  const size_t nw = (size_t)2 * NPATH * hidden * 16;
  const size_t f32 = full_bytes32(g);
  const int nblocks = nblk(2 * npad_of(g));
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = al256(o + bytes); return at; };
  l.w = take(sizeof(float2) * nw);
  l.wadj = take(sizeof(float2) * nw);
  l.kmat = take(sizeof(float2) * 2 * NPATH * NPATH * 16);
  l.kfrag = take(2 * 4 * 2 * 2 * 64 * 8 * sizeof(__bf16));
  l.am = take(sizeof(float) * 2 * nw);
  l.av = take(sizeof(float) * 2 * nw);
  l.grad = take(sizeof(double) * 2 * nw);
  l.part = take(sizeof(double) * std::max<size_t>((size_t)NPATH * hidden * WG_CHUNKS * 32, (size_t)nblocks + 64));
  l.scal = take(sizeof(double) * ((size_t)nblocks + 64));
  l.act = take(f32 * hidden);
  l.gact = take(f32 * hidden);
  // f32 is a whole number of 256-byte units, so act, gact and pairx are
  // adjacent: together they hold the nine F32 fields m_p of folded inference
  l.pairx = take(f32 * (size_t)std::max(0, NPATH - 2 * hidden));
  l.fv = take(f32);
  l.fb = take(f32);
  l.fy = take(f32);
  l.fg = take(f32);
  l.loss = take(sizeof(double) * LOSS_CAP);
  l.total = o;
  return l;
}
bool valid_hidden(int h) { return h == 2 || h == 4 || h == 8; }
}  // namespace

extern "C" size_t qiral_nn_bytes(const qiral_lattice *lat, int32_t hidden) {
  if (!lat || !valid_hidden(hidden)) return 0;
  return nn_layout(lat->geo, hidden).total;
}

extern "C" qiral_status qiral_nn_create(qiral_nn **out, qiral_lattice *lat, int32_t hidden, void *mem,
                                        size_t mem_bytes, qiral_stream_t stream) {
  if (!out || !lat) return fail(QIRAL_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (!valid_hidden(hidden)) return fail(QIRAL_ERR_UNSUPPORTED, "hidden channels must be 2, 4 or 8");
  if (!mem) return fail(QIRAL_ERR_WORKSPACE, "mem is NULL (size it with qiral_nn_bytes)");
  if (((uintptr_t)mem & 255) != 0) return fail(QIRAL_ERR_INVALID_ARG, "mem must be 256-byte aligned");
  if (!lat->g32) return fail(QIRAL_ERR_INVALID_ARG, "the network needs the lattice's FP32 links (gauge_f32)");
  const NnLayout l = nn_layout(lat->geo, hidden);
  if (mem_bytes < l.total) return fail(QIRAL_ERR_WORKSPACE, "mem_bytes is smaller than qiral_nn_bytes");
  qiral_nn *nn = new qiral_nn();
  nn->lat = lat;
  nn->hidden = hidden;
  nn->nw1 = NPATH * hidden * 16;
  nn->nw2 = NPATH * hidden * 16;
  const int nw = nn->nw1 + nn->nw2;
  char *m = (char *)mem;
  nn->w = (float2 *)(m + l.w);
  nn->wadj = (float2 *)(m + l.wadj);
  nn->kmat = (float2 *)(m + l.kmat);
  nn->kfrag = m + l.kfrag;
  nn->am = (float *)(m + l.am);
  nn->av = (float *)(m + l.av);
  nn->grad = (double *)(m + l.grad);
  nn->part = (double *)(m + l.part);
  nn->scal = (double *)(m + l.scal);
  nn->act = m + l.act;
  nn->gact = m + l.gact;
  nn->fv = m + l.fv;
  nn->fb = m + l.fb;
  nn->fy = m + l.fy;
  nn->fg = m + l.fg;
  nn->loss_dev = (double *)(m + l.loss);
  hipStream_t s = (hipStream_t)stream;
  std::vector<float2> w0;
  neumann2(hidden, lat->kappa, w0);
  hipError_t e = hipMemcpyAsync(nn->w, w0.data(), sizeof(float2) * nw, hipMemcpyHostToDevice, s);
  // Adam moments start at zero; activations too, so that padding sites stay zero
  if (e == hipSuccess) e = hipMemsetAsync(nn->am, 0, sizeof(float) * 2 * nw, s);
  if (e == hipSuccess) e = hipMemsetAsync(nn->av, 0, sizeof(float) * 2 * nw, s);
  if (e == hipSuccess) e = hipMemsetAsync(nn->act, 0, full_bytes32(lat->geo) * hidden, s);
  if (e == hipSuccess) e = hipMemsetAsync(nn->gact, 0, full_bytes32(lat->geo) * hidden, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // w0 is a host temporary
  if (e != hipSuccess) {
    delete nn;
    return hip_fail(e, "nn init");
  }
  *out = nn;
  return QIRAL_OK;
}

extern "C" qiral_status qiral_nn_destroy(qiral_nn *nn) {
  if (!nn) return fail(QIRAL_ERR_INVALID_ARG, "nn is NULL");
  delete nn;   // the device memory belongs to the caller
  return QIRAL_OK;
}

extern "C" size_t qiral_nn_num_weights(const qiral_nn *nn) { return nn ? (size_t)(nn->nw1 + nn->nw2) : 0; }

extern "C" qiral_status qiral_nn_set_weights(qiral_nn *nn, const float *w, size_t count, qiral_stream_t stream) {
  if (!nn || !w) return fail(QIRAL_ERR_INVALID_ARG, "NULL argument");
  if (count != (size_t)(nn->nw1 + nn->nw2)) return fail(QIRAL_ERR_INVALID_ARG, "count must equal qiral_nn_num_weights");
  hipStream_t s = (hipStream_t)stream;
  QIRAL_HIP(hipMemcpyAsync(nn->w, w, sizeof(float2) * count, hipMemcpyHostToDevice, s));
  QIRAL_HIP(hipStreamSynchronize(s));
  return QIRAL_OK;
}

extern "C" qiral_status qiral_nn_get_weights(const qiral_nn *nn, float *w, size_t count, qiral_stream_t stream) {
  if (!nn || !w) return fail(QIRAL_ERR_INVALID_ARG, "NULL argument");
  if (count != (size_t)(nn->nw1 + nn->nw2)) return fail(QIRAL_ERR_INVALID_ARG, "count must equal qiral_nn_num_weights");
  hipStream_t s = (hipStream_t)stream;
  QIRAL_HIP(hipMemcpyAsync(w, nn->w, sizeof(float2) * count, hipMemcpyDeviceToHost, s));
  QIRAL_HIP(hipStreamSynchronize(s));
  return QIRAL_OK;
}

// Both network calls run the folded form on packed F32 full fields.
static qiral_status nn_apply_api(const qiral_nn *nn, void *out, const void *in, bool adj, qiral_stream_t stream) {
  if (!nn || !out || !in) return fail(QIRAL_ERR_INVALID_ARG, "NULL argument");
  if (out == in) return fail(QIRAL_ERR_INVALID_ARG, "in and out must not alias");
  hipStream_t s = (hipStream_t)stream;
  const size_t hb = half_bytes(nn->lat->geo, QIRAL_F32);
  QIRAL_HIP(nn_fold(nn, s));
  QIRAL_HIP(nn_apply_folded<S_F32>(nn, out, (char *)out + hb, in, (const char *)in + hb, adj, s));
  return QIRAL_OK;
}

extern "C" qiral_status qiral_nn_apply(const qiral_nn *nn, void *out, const void *in, qiral_stream_t stream) {
  return nn_apply_api(nn, out, in, false, stream);
}

extern "C" qiral_status qiral_nn_apply_adjoint(qiral_nn *nn, void *out, const void *in, qiral_stream_t stream) {
  return nn_apply_api(nn, out, in, true, stream);
}

extern "C" qiral_status qiral_nn_sample(qiral_nn *nn, void *out, uint64_t seed, uint64_t step, double *norm2,
                                        qiral_stream_t stream) {
  if (!nn || !out) return fail(QIRAL_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const Geo &g = nn->lat->geo;
  const int nb = nblk(2 * npad_of(g));
  hipLaunchKernelGGL(k_gauss, dim3(nb), dim3(256), 0, s, g, out, make_uint2((unsigned)seed, (unsigned)(seed >> 32)),
                     (unsigned long long)step, nn->part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, nn->part, nb, nn->scal, (const double *)nullptr);
  QIRAL_HIP(hipGetLastError());
  if (norm2) {
    QIRAL_HIP(hipMemcpyAsync(norm2, nn->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    QIRAL_HIP(hipStreamSynchronize(s));
  }
  return QIRAL_OK;
}

namespace {

// Loss L = ||N(src) - target||^2 / ||target||^2 into *loss_dev and its gradient
// with respect to the real and imaginary parts of every weight into nn->grad.
hipError_t train_step(qiral_nn *nn, const void *src, const void *target, double *loss_dev, hipStream_t s) {
  const Geo &g = nn->lat->geo;
  const int H = nn->hidden;
  const int nb = nblk(2 * npad_of(g));
  hipLaunchKernelGGL(k_norm32, dim3(nb), dim3(256), 0, s, g, target, nn->part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, nn->part, nb, nn->scal, (const double *)nullptr);
  hipError_t e = layer_launch(nn, nn->w, 1, H, src, nn->act, s);
  if (e != hipSuccess) return e;
  e = layer_launch(nn, nn->w + nn->nw1, H, 1, nn->act, nn->fy, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, s, g, nn->fy, target, nn->fg, nn->scal, nn->part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, nn->part, nb, loss_dev, nn->scal);
  // layer 2: weights and the gradient w.r.t. its input (the adjoint layer)
  e = wgrad_launch(nn, H, 1, nn->act, nn->fg, nn->grad + 2 * nn->nw1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_weights, dim3((NPATH * H * 16 + 255) / 256), dim3(256), 0, s, nn->w + nn->nw1, nn->wadj, 1, H);
  e = layer_launch(nn, nn->wadj, 1, H, nn->fg, nn->gact, s);
  if (e != hipSuccess) return e;
  // layer 1 weights
  e = wgrad_launch(nn, 1, H, src, nn->gact, nn->grad, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

extern "C" qiral_status qiral_nn_grad(qiral_nn *nn, const void *src, const void *target, double *loss, double *grad,
                                      qiral_stream_t stream) {
  if (!nn || !src || !target) return fail(QIRAL_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  QIRAL_HIP(train_step(nn, src, target, nn->scal + 1, s));
  if (loss) QIRAL_HIP(hipMemcpyAsync(loss, nn->scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
  if (grad) QIRAL_HIP(hipMemcpyAsync(grad, nn->grad, sizeof(double) * 2 * (nn->nw1 + nn->nw2), hipMemcpyDeviceToHost, s));
  QIRAL_HIP(hipStreamSynchronize(s));
  return QIRAL_OK;
}

extern "C" qiral_status qiral_nn_train(qiral_nn *nn, int32_t steps, double lr, uint64_t seed, double *loss_history,
                                       qiral_stream_t stream) {
  if (!nn) return fail(QIRAL_ERR_INVALID_ARG, "nn is NULL");
  if (steps < 0) return fail(QIRAL_ERR_INVALID_ARG, "steps must be >= 0");
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(QIRAL_ERR_INVALID_ARG, "lr must be positive");
  if (steps == 0) return QIRAL_OK;
  hipStream_t s = (hipStream_t)stream;
  const Geo &g = nn->lat->geo;
  const int nb = nblk(2 * npad_of(g));
  const int nreal = 2 * (nn->nw1 + nn->nw2);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int k = 0; k < steps; ++k) {
    // training pair (D v, v) with v Gaussian; the counter is the global step
    const unsigned long long ctr = (unsigned long long)nn->adam_step;
    hipLaunchKernelGGL(k_gauss, dim3(nb), dim3(256), 0, s, g, nn->fv, make_uint2((unsigned)seed, (unsigned)(seed >> 32)),
                       ctr, nn->part);
    QIRAL_HIP(apply_D_full(nn->lat, QIRAL_F32, nn->fb, nn->fv, s));
    QIRAL_HIP(train_step(nn, nn->fb, nn->fv, nn->loss_dev + k % LOSS_CAP, s));
    nn->adam_step += 1;
    const float c1 = 1.f - powf(b1, (float)nn->adam_step), c2 = 1.f - powf(b2, (float)nn->adam_step);
    hipLaunchKernelGGL(k_adam, dim3((nreal + 255) / 256), dim3(256), 0, s, (float *)nn->w, nn->grad, nn->am, nn->av,
                       nreal, (float)lr, b1, b2, eps, c1, c2);
    QIRAL_HIP(hipGetLastError());
    // the device keeps LOSS_CAP losses: copy them out when the buffer is full
    // (the copy is ordered before the steps that overwrite it)
    const int done = k + 1;
    if (loss_history && (done % LOSS_CAP == 0 || done == steps)) {
      const int first = (done - 1) / LOSS_CAP * LOSS_CAP;
      QIRAL_HIP(hipMemcpyAsync(loss_history + first, nn->loss_dev, sizeof(double) * (done - first),
                               hipMemcpyDeviceToHost, s));
    }
  }
  QIRAL_HIP(hipStreamSynchronize(s));
  return QIRAL_OK;
}

// ---------------------------------------------------------------------------
// Flexible solvers, composed with the system they run on and a right
// preconditioner (the runtime counterpart of the right-to-left template chains
// of Sec. 2 and Sec. 3.1):
//   system: the full D x = b, or the odd-site Schur system S x_o = b_hat of the
//           "schur" template (then x_e = A^-1 (b_e + kappa H_eo x_o));
//   preconditioner M ~ A^-1: the network N (full system), its Schur
//           restriction M_S v = P_o N (0 (+) v) (the odd part of D^-1 (0 (+) v)
//           is S^-1 v), or the identity;
//   solver: FGMRES(m) with M on the right, FCG(1) on the normal equations with
//           M M^dagger, or BiCGStab with M on the right.
// Krylov vectors are packed FP64 fields (both halves, or the odd half), handled
// as flat complex arrays; the network runs in FP32.
namespace qiral {
qiral_status run_solve_cg_fallback(qiral_lattice *lat, double *x, const double *b, const qiral_solve_params *prm,
                                   void *ws, size_t ws_bytes, qiral_solve_info *info, hipStream_t s);
void import_field(const Geo &g, const double *src, void *dst, int subset, int prec, int nrhs, hipStream_t s);
void export_field(const Geo &g, double *dst, const void *src, int subset, int prec, int nrhs, hipStream_t s);

namespace {

// Krylov vectors each flexible solver keeps (beyond the common fields)
int flex_nvec(int solver, int m) {
  return solver == QIRAL_FGMRES_NN ? 2 * m + 5 : solver == QIRAL_FCG_NN ? 8 : 10;
}

bool flex_schur(const qiral_solve_params *prm) {
  if (prm->system == QIRAL_SYSTEM_SCHUR) return true;
  if (prm->system == QIRAL_SYSTEM_FULL) return false;
  return prm->solver == QIRAL_BICGSTAB_EO;   // default: BiCGStab on the Schur system, FGMRES / FCG on D
}

int flex_restart(const qiral_solve_params *prm) { return prm->restart > 0 ? prm->restart : 20; }

// The system, its preconditioner and the workspace fields of one flexible solve.
struct Flex {
  qiral_lattice *lat;
  qiral_nn *nn;        // NULL: the identity preconditioner
  bool schur;
  size_t hb64;         // bytes of an F64 half-field
  size_t vb, n2;       // bytes and complex entries of a Krylov vector
  int nbk;             // work-groups of the flat vector kernels
  double2 *BF, *XF, *RF;        // F64 full fields: b, x, the true residual
  void *tmpE;                   // F64 even half-field (Schur operator, source)
  double2 *vec;                 // the solver's Krylov vectors, vb bytes apart
  double *part, *npart, *nrm;   // partial sums
  double2 *coef;                // complex coefficients (device)
  void *mbuf;                   // path fields of the network for all systems at once (lockstep), or null
  int nsys = 1;                 // systems solved in lockstep (BiCGStab); their Krylov vectors follow one another
  double2 *v(int i) const { return (double2 *)((char *)vec + (size_t)i * vb); }
  // vector i of system k; vector i of every system is one block of nsys vectors
  double2 *slot(int i, int k) const { return (double2 *)((char *)vec + ((size_t)i * nsys + k) * vb); }
  // system k alone: its coefficients, the shared full fields and scratch
  Flex sys_view(int k) const {
    Flex f = *this;
    f.nsys = 1;
    f.coef = coef + (size_t)k * BQ_SLOTS;
    return f;
  }
};

size_t flex_bytes(const Geo &g, const qiral_solve_params *prm, bool schur, Flex *f, int nsys = 1) {
  const size_t hb64 = half_bytes(g, QIRAL_F64);
  const size_t vb = schur ? hb64 : 2 * hb64;
  const int m = flex_restart(prm);
  const int nbk = nblk(vb / 16);
  const int nv = flex_nvec(prm->solver, m);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += (bytes + 255) / 256 * 256; return at; };
  // b, x and the true residual of the system being set up or finished, and the
  // even half-fields of the Schur operator's first hop, one per system
  const size_t oBF = take(2 * hb64), oXF = take(2 * hb64), oRF = take(2 * hb64), oT = take((size_t)nsys * hb64);
  const size_t ovec = o;
  o += (size_t)nv * nsys * vb;
  const size_t opart = take(sizeof(double) * std::max<size_t>(2 * (size_t)(m + 2) * nbk, 4 * (size_t)nsys * nbk));
  // norms of full fields (begin, end) take twice the blocks of a Schur vector
  const size_t onpart = take(sizeof(double) * nblk(2 * hb64 / 16));
  const size_t onrm = take(sizeof(double) * 2 * 64), ocoef = take(sizeof(double2) * BQ_SLOTS * nsys);
  // systems in lockstep on the Schur system take the network's passes together:
  // nine F32 half-fields of path fields each
  const bool batched_net = prm->precond && schur && nsys > 1;
  const size_t om = batched_net ? take((size_t)nsys * NPATH * half_bytes(g, QIRAL_F32)) : 0;
  if (f) {
    f->nsys = nsys;
    f->hb64 = hb64;
    f->vb = vb;
    f->n2 = vb / 16;
    f->nbk = nbk;
    f->BF = (double2 *)oBF;   // offsets here; based by flex_setup
    f->XF = (double2 *)oXF;
    f->RF = (double2 *)oRF;
    f->tmpE = (void *)oT;
    f->vec = (double2 *)ovec;
    f->part = (double *)opart;
    f->npart = (double *)onpart;
    f->nrm = (double *)onrm;
    f->coef = (double2 *)ocoef;
    f->mbuf = batched_net ? (void *)om : nullptr;
  }
  return o;
}

qiral_status flex_setup(qiral_lattice *lat, const qiral_solve_params *prm, void *ws, size_t ws_bytes, Flex &f,
                        int nsys = 1) {
  f.lat = lat;
  f.nn = (qiral_nn *)prm->precond;
  if (f.nn && f.nn->lat != lat) return fail(QIRAL_ERR_INVALID_ARG, "precond must be a network made for this lattice");
  f.schur = flex_schur(prm);
  const size_t need = flex_bytes(lat->geo, prm, f.schur, &f, nsys);
  if (ws_bytes < need) return fail(QIRAL_ERR_WORKSPACE, "flexible-solver workspace too small");
  char *b = (char *)ws;
  f.BF = (double2 *)(b + (size_t)f.BF);
  f.XF = (double2 *)(b + (size_t)f.XF);
  f.RF = (double2 *)(b + (size_t)f.RF);
  f.tmpE = b + (size_t)f.tmpE;
  f.vec = (double2 *)(b + (size_t)f.vec);
  f.part = (double *)(b + (size_t)f.part);
  f.npart = (double *)(b + (size_t)f.npart);
  f.nrm = (double *)(b + (size_t)f.nrm);
  f.coef = (double2 *)(b + (size_t)f.coef);
  if (f.mbuf) f.mbuf = b + (size_t)f.mbuf;
  return QIRAL_OK;
}

// y = A x or A^dagger x in FP64 (A = D, or S = A_oo - kappa^2 H_oe A_ee^-1 H_eo)
// for nsys consecutive vectors (the Schur operator's hops take them together)
hipError_t flex_A(const Flex &f, void *y, const void *x, bool dag, hipStream_t s, int nsys = 1) {
  const qiral_lattice *lat = f.lat;
  if (!f.schur) {
    for (int k = 0; k < nsys; ++k) {
      void *yk = (char *)y + (size_t)k * f.vb;
      const void *xk = (const char *)x + (size_t)k * f.vb;
      hipError_t e = dag ? apply_Ddag_full(lat, QIRAL_F64, yk, xk, s) : apply_D_full(lat, QIRAL_F64, yk, xk, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const double k = lat->kappa;
  hipError_t e = launch_hop(lat, QIRAL_F64, dag, 0, 0, 1.0, x, f.tmpE, nullptr, nsys, s,
                            dag ? CHI_AINVDAG : CHI_AINV, CHI_ONE);
  if (e != hipSuccess) return e;
  return launch_hop(lat, QIRAL_F64, dag, 1, 1, -k * k, f.tmpE, y, x, nsys, s, CHI_ONE, dag ? CHI_ADAG : CHI_A);
}

// z = M v (or M^dagger v): the folded network in FP32 on v (full system) or on
// v placed on the odd sites, keeping the odd part of the result (Schur system:
// the passes skip the paths and sites that would only add zeros or be
// dropped, and the path-pair products run on bf16 MFMA), reading and writing
// the FP64 Krylov vectors directly; the identity without a network.  nsys
// consecutive vectors (the Schur form takes them in one pass each).
hipError_t flex_M(const Flex &f, void *z, const void *v, bool adj, hipStream_t s, int nsys = 1) {
  if (!f.nn) return hipMemcpyAsync(z, v, (size_t)nsys * f.vb, hipMemcpyDeviceToDevice, s);
  if (f.schur) {
    if (nsys > 1 && !f.mbuf) return hipErrorInvalidValue;
    return nn_apply_folded<S_F64>(f.nn, nullptr, z, nullptr, v, adj, s, 1, nsys, f.vb, nsys > 1 ? f.mbuf : nullptr);
  }
  for (int k = 0; k < nsys; ++k) {
    char *zk = (char *)z + (size_t)k * f.vb;
    const char *vk = (const char *)v + (size_t)k * f.vb;
    hipError_t e = nn_apply_folded<S_F64>(f.nn, zk, zk + f.hb64, vk, vk + f.hb64, adj, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

qiral_status flex_read(void *dst, const void *src, size_t bytes, hipStream_t s) {
  QIRAL_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  QIRAL_HIP(hipStreamSynchronize(s));
  return QIRAL_OK;
}

qiral_status flex_norm2(const Flex &f, const double2 *v, double &out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm, dim3(f.nbk), dim3(256), 0, s, v, f.n2, f.npart);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, f.npart, f.nbk, f.nrm, (const double *)nullptr);
  return flex_read(&out, f.nrm, sizeof(double), s);
}

// (a | b) on the host
qiral_status flex_dot(const Flex &f, const double2 *a, const double2 *b, std::complex<double> &out, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot, dim3(f.nbk), dim3(256), 0, s, a, f.n2, 1, b, f.n2, f.part);
  hipLaunchKernelGGL(k_mdot_final, dim3(1), dim3(256), 0, s, f.part, f.nbk, f.coef + 32);
  double2 c;
  qiral_status st = flex_read(&c, f.coef + 32, sizeof c, s);
  out = std::complex<double>(c.x, c.y);
  return st;
}

// (a | b) into coef[slot], ||v||^2 into coef[slot].x: on the device, no host read
void flex_dot_dev(const Flex &f, const double2 *a, const double2 *b, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot, dim3(f.nbk), dim3(256), 0, s, a, f.n2, 1, b, f.n2, f.part);
  hipLaunchKernelGGL(k_mdot_final, dim3(1), dim3(256), 0, s, f.part, f.nbk, f.coef + slot);
}
void flex_norm2_dev(const Flex &f, const double2 *v, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_norm, dim3(f.nbk), dim3(256), 0, s, v, f.n2, f.npart);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, f.npart, f.nbk, (double *)(f.coef + slot),
                     (const double *)nullptr);
}

qiral_status flex_set_coef(const Flex &f, const std::vector<double2> &c, hipStream_t s) {
  QIRAL_HIP(hipMemcpyAsync(f.coef, c.data(), sizeof(double2) * c.size(), hipMemcpyHostToDevice, s));
  return QIRAL_OK;
}

// Inputs: b (full) into BF, x into XF (guess or 0), and the system's right-hand
// side into rhs (b itself, or b_hat = b_o + kappa H_oe A^-1 b_e) and its x.
qiral_status flex_begin(const Flex &f, const double *x_canon, const double *b_canon, bool guess, double2 *rhs,
                        double2 *X, double &bnorm, hipStream_t s, int bn2_slot = -1, bool fold = true) {
  const qiral_lattice *lat = f.lat;
  const Geo &g = lat->geo;
  import_field(g, b_canon, f.BF, QIRAL_FULL, QIRAL_F64, 1, s);
  if (guess) import_field(g, x_canon, f.XF, QIRAL_FULL, QIRAL_F64, 1, s);
  else QIRAL_HIP(hipMemsetAsync(f.XF, 0, 2 * f.hb64, s));
  // Hops and network layers write only the lattice's sites, while the flat
  // vector kernels also sum the padding sites of the last 64-site block: every
  // field whose padding they can reach starts at zero (the Krylov vectors are
  // cleared by the solvers).
  QIRAL_HIP(hipMemsetAsync(f.RF, 0, 2 * f.hb64, s));
  if (f.nn && fold) QIRAL_HIP(nn_fold(f.nn, s));   // the network's folded weights for this solve
  const char *be = (const char *)f.BF, *bo = be + f.hb64;
  if (!f.schur) {
    QIRAL_HIP(hipMemcpyAsync(rhs, f.BF, 2 * f.hb64, hipMemcpyDeviceToDevice, s));
    QIRAL_HIP(hipMemcpyAsync(X, f.XF, 2 * f.hb64, hipMemcpyDeviceToDevice, s));
  } else {
    hipLaunchKernelGGL(k_chi64, dim3(nblk(npad_of(g))), dim3(256), 0, s, g, be, f.tmpE, (int)CHI_AINV,
                       2.0 * lat->kappa * lat->mu);
    QIRAL_HIP(launch_hop(lat, QIRAL_F64, 0, 1, 1, lat->kappa, f.tmpE, rhs, bo, 1, s, CHI_ONE, CHI_ONE));
    QIRAL_HIP(hipMemcpyAsync(X, (const char *)f.XF + f.hb64, f.hb64, hipMemcpyDeviceToDevice, s));
  }
  QIRAL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_norm, dim3(nblk(2 * f.hb64 / 16)), dim3(256), 0, s, f.BF, 2 * f.hb64 / 16, f.npart);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, f.npart, nblk(2 * f.hb64 / 16),
                     bn2_slot >= 0 ? (double *)(f.coef + bn2_slot) : f.nrm, (const double *)nullptr);
  if (bn2_slot >= 0) return QIRAL_OK;   // ||b||^2 left in coef[bn2_slot].x
  double b2 = 0;
  qiral_status st = flex_read(&b2, f.nrm, sizeof b2, s);
  bnorm = std::sqrt(b2);
  return st;
}

// x (full) from the system's solution X, its FP64 true residual ||b - D x||, export.
qiral_status flex_end(const Flex &f, const double2 *X, double *x_canon, double &rn, hipStream_t s,
                      int rn2_slot = -1) {
  const qiral_lattice *lat = f.lat;
  const Geo &g = lat->geo;
  if (!f.schur) {
    QIRAL_HIP(hipMemcpyAsync(f.XF, X, 2 * f.hb64, hipMemcpyDeviceToDevice, s));
  } else {
    char *xe = (char *)f.XF, *xo = xe + f.hb64;
    QIRAL_HIP(hipMemcpyAsync(xo, X, f.hb64, hipMemcpyDeviceToDevice, s));
    // x_e = A^-1 (b_e + kappa H_eo x_o)
    QIRAL_HIP(launch_hop(lat, QIRAL_F64, 0, 0, 1, lat->kappa, xo, xe, f.BF, 1, s, CHI_AINV, CHI_ONE));
  }
  QIRAL_HIP(apply_D_full(lat, QIRAL_F64, f.RF, f.XF, s));
  const size_t nf = 2 * f.hb64 / 16;
  hipLaunchKernelGGL(k_bminus, dim3(nblk(nf)), dim3(256), 0, s, f.BF, f.RF, nf);
  hipLaunchKernelGGL(k_norm, dim3(nblk(nf)), dim3(256), 0, s, f.RF, nf, f.npart);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, f.npart, nblk(nf),
                     rn2_slot >= 0 ? (double *)(f.coef + rn2_slot) : f.nrm, (const double *)nullptr);
  if (rn2_slot >= 0) {   // ||b - D x||^2 left in coef[rn2_slot].x; the caller reads it later
    export_field(g, x_canon, f.XF, QIRAL_FULL, QIRAL_F64, 1, s);
    QIRAL_HIP(hipGetLastError());
    return QIRAL_OK;
  }
  double r2 = 0;
  qiral_status st = flex_read(&r2, f.nrm, sizeof r2, s);
  rn = std::sqrt(r2);
  export_field(g, x_canon, f.XF, QIRAL_FULL, QIRAL_F64, 1, s);
  QIRAL_HIP(hipGetLastError());
  QIRAL_HIP(hipStreamSynchronize(s));
  return st;
}

// R = rhs - A X (rhs itself when X is known to be zero); returns ||R||
qiral_status flex_residual(const Flex &f, const double2 *rhs, const double2 *X, double2 *R, double &rn,
                           hipStream_t s, bool xzero = false, int rn2_slot = -1) {
  if (xzero) {
    QIRAL_HIP(hipMemcpyAsync(R, rhs, f.vb, hipMemcpyDeviceToDevice, s));
  } else {
    QIRAL_HIP(flex_A(f, R, X, false, s));
    hipLaunchKernelGGL(k_bminus, dim3(f.nbk), dim3(256), 0, s, rhs, R, f.n2);
  }
  if (rn2_slot >= 0) {   // ||R||^2 left in coef[rn2_slot].x
    flex_norm2_dev(f, R, rn2_slot, s);
    return QIRAL_OK;
  }
  double r2 = 0;
  qiral_status st = flex_norm2(f, R, r2, s);
  rn = std::sqrt(r2);
  return st;
}

// Fill info, and continue with even-odd CGNR from the current x when asked.
qiral_status flex_finish(qiral_lattice *lat, double *x_canon, const double *b_canon, const qiral_solve_params *prm,
                         void *ws, size_t ws_bytes, qiral_solve_info *info, int steps, long long hops, double rn,
                         double bn, bool broke, const char *name, std::chrono::steady_clock::time_point t0,
                         hipStream_t s) {
  const double target = prm->tol * bn;
  qiral_status result = QIRAL_OK;
  info->iterations = steps;
  info->reliable_updates = 0;
  info->fell_back = 0;
  info->hop_applications = hops;
  info->true_rel_resid = bn > 0 ? rn / bn : rn;
  if (!std::isfinite(rn)) {
    set_error(std::string("a NaN or Inf appeared in ") + name);
    result = QIRAL_ERR_NONFINITE;
  } else if (rn > target && prm->fallback_cg) {
    qiral_solve_params cg = *prm;
    cg.solver = QIRAL_CGNR_EO;
    cg.system = QIRAL_SYSTEM_DEFAULT;
    cg.precond = nullptr;
    cg.x0_is_guess = 1;
    qiral_solve_info ci;
    memset(&ci, 0, sizeof ci);
    result = run_solve_cg_fallback(lat, x_canon, b_canon, &cg, ws, ws_bytes, &ci, s);
    info->iterations = steps + ci.iterations;
    info->reliable_updates = ci.reliable_updates;
    info->true_rel_resid = ci.true_rel_resid;
    info->hop_applications = hops + ci.hop_applications;
    info->fell_back = 1;
  } else if (rn > target) {
    set_error(broke ? (std::string(name) + " broke down").c_str() : "tolerance not reached within maxiter");
    result = QIRAL_ERR_NOT_CONVERGED;
  }
  info->converged = (result == QIRAL_OK);
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return result;
}

// hop applications (units of V/2 sites) of one application of A
long long flex_hops(const Flex &f) { return 2; }

}  // namespace

size_t flex_ws_bytes(const qiral_lattice *lat, const qiral_solve_params *prm, int nsys) {
  // BiCGStab solves its right-hand sides in lockstep, FGMRES and FCG one after the other
  return flex_bytes(lat->geo, prm, flex_schur(prm), nullptr, prm->solver == QIRAL_BICGSTAB_EO ? nsys : 1);
}

// FGMRES(m) with M on the right: x = x0 + Z y, z_j = M v_j (Saad 1993).
qiral_status run_fgmres(qiral_lattice *lat, double *x_canon, const double *b_canon, const qiral_solve_params *prm,
                        void *ws, size_t ws_bytes, qiral_solve_info *info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  Flex f;
  qiral_status st = flex_setup(lat, prm, ws, ws_bytes, f);
  if (st != QIRAL_OK) return st;
  const int m = flex_restart(prm);
  double2 *V = f.v(0), *Z = f.v(m + 1), *B = f.v(2 * m + 1), *X = f.v(2 * m + 2), *Wv = f.v(2 * m + 3),
          *R = f.v(2 * m + 4);
  const size_t vs = f.n2;   // stride between vectors of V and Z in complex entries
  QIRAL_HIP(hipMemsetAsync(f.vec, 0, (size_t)(2 * m + 5) * f.vb, s));
  double bn = 0;
  if ((st = flex_begin(f, x_canon, b_canon, prm->x0_is_guess != 0, B, X, bn, s)) != QIRAL_OK) return st;
  const double target = prm->tol * bn;
  double rn = 0;
  const bool xzero = prm->x0_is_guess == 0;
  if ((st = flex_residual(f, B, X, R, rn, s, xzero)) != QIRAL_OK) return st;
  int steps = 0;
  long long hops = xzero ? 0 : flex_hops(f);
  double prev_cycle = rn;
  typedef std::complex<double> C;
  std::vector<C> H((m + 1) * m), cs(m), sn(m), gv(m + 1);
  bool broke = false;
  while (rn > target && steps < prm->maxiter) {
    // V0 = R / |R|
    hipLaunchKernelGGL(k_norm, dim3(f.nbk), dim3(256), 0, s, R, f.n2, f.npart);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, f.npart, f.nbk, f.nrm, (const double *)nullptr);
    hipLaunchKernelGGL(k_scale, dim3(f.nbk), dim3(256), 0, s, R, f.nrm, V, f.n2);
    std::fill(H.begin(), H.end(), C(0));
    std::fill(gv.begin(), gv.end(), C(0));
    gv[0] = rn;
    int k = 0;
    for (int j = 0; j < m && steps < prm->maxiter; ++j) {
      // Z_j = M V_j, W = A Z_j
      QIRAL_HIP(flex_M(f, Z + j * vs, V + j * vs, false, s));
      QIRAL_HIP(flex_A(f, Wv, Z + j * vs, false, s));
      hops += flex_hops(f);
      // classical Gram-Schmidt with selective reorthogonalisation (Daniel,
      // Gragg, Kaufman and Stewart 1976): a second pass only when the first
      // removed more than half of w's squared norm, i.e. when cancellation
      // may have left w short of orthogonal to V
      std::vector<C> h(j + 2, C(0));
      double w2 = 0;
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_mdot, dim3(f.nbk), dim3(256), 0, s, V, vs, j + 1, Wv, f.n2, f.part);
        hipLaunchKernelGGL(k_mdot_final, dim3(j + 1), dim3(256), 0, s, f.part, f.nbk, f.coef);
        hipLaunchKernelGGL(k_maxpy, dim3(f.nbk), dim3(256), 0, s, V, vs, j + 1, f.coef, -1.0, Wv, f.n2);
        std::vector<double2> c(j + 1);
        if ((st = flex_read(c.data(), f.coef, sizeof(double2) * (j + 1), s)) != QIRAL_OK) return st;
        double c2 = 0;
        for (int i = 0; i <= j; ++i) {
          h[i] += C(c[i].x, c[i].y);
          c2 += c[i].x * c[i].x + c[i].y * c[i].y;
        }
        if ((st = flex_norm2(f, Wv, w2, s)) != QIRAL_OK) return st;
        if (w2 > 0.5 * (w2 + c2)) break;   // ||w_after||^2 > ||w_before||^2 / 2
      }
      h[j + 1] = std::sqrt(w2);
      hipLaunchKernelGGL(k_scale, dim3(f.nbk), dim3(256), 0, s, Wv, f.nrm, V + (j + 1) * vs, f.n2);
      // Givens rotations on the new column
      for (int i = 0; i < j; ++i) {
        const C hi = h[i];
        h[i] = std::conj(cs[i]) * hi + std::conj(sn[i]) * h[i + 1];
        h[i + 1] = -sn[i] * hi + cs[i] * h[i + 1];
      }
      const double den = std::sqrt(std::norm(h[j]) + std::norm(h[j + 1]));
      cs[j] = den > 0 ? h[j] / den : C(1);
      sn[j] = den > 0 ? h[j + 1] / den : C(0);
      h[j] = den;
      h[j + 1] = 0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = std::conj(cs[j]) * gv[j];
      for (int i = 0; i <= j; ++i) H[i * m + j] = h[i];
      k = j + 1;
      ++steps;
      if (!std::isfinite(std::abs(gv[j + 1]))) break;
      if (std::abs(gv[j + 1]) <= 0.5 * target) break;
    }
    // y = R^{-1} g, X += Z y
    std::vector<C> y(k);
    for (int i = k - 1; i >= 0; --i) {
      C a = gv[i];
      for (int l = i + 1; l < k; ++l) a -= H[i * m + l] * y[l];
      // a zero pivot is a breakdown (e.g. a preconditioner returning 0): drop that direction
      y[i] = std::abs(H[i * m + i]) > 0 ? a / H[i * m + i] : C(0);
    }
    std::vector<double2> yc(k);
    for (int i = 0; i < k; ++i) yc[i] = make_double2(y[i].real(), y[i].imag());
    if ((st = flex_set_coef(f, yc, s)) != QIRAL_OK) return st;
    hipLaunchKernelGGL(k_maxpy, dim3(f.nbk), dim3(256), 0, s, Z, vs, k, f.coef, 1.0, X, f.n2);
    if ((st = flex_residual(f, B, X, R, rn, s)) != QIRAL_OK) return st;
    hops += flex_hops(f);
    if (!std::isfinite(rn)) break;
    if (rn > target && prm->fallback_cg && rn > 0.5 * prev_cycle) { broke = true; break; }   // stagnation
    prev_cycle = rn;
  }
  double rt = 0;
  if ((st = flex_end(f, X, x_canon, rt, s)) != QIRAL_OK) return st;
  hops += 2;
  if (std::isfinite(rn) && !std::isfinite(rt)) rn = rt;
  return flex_finish(lat, x_canon, b_canon, prm, ws, ws_bytes, info, steps, hops, std::isfinite(rn) ? rt : rn, bn,
                     broke, "FGMRES", t0, s);
}

// Flexible CG (Notay 2000), FCG(1), on the normal equations A^dagger A x =
// A^dagger rhs with the preconditioner z = M (M^dagger r).  M is a fixed linear
// map, so one previous direction is enough (as in preconditioned CG); the
// flexible coefficient beta = (A^dagger A p_prev | z) / (p_prev | A^dagger A p_prev)
// keeps the directions conjugate although z carries FP32 rounding.  The FP64
// residual s = rhs - A x is updated alongside the normal residual r = A^dagger s
// and decides convergence; the true residual is recomputed at the end.
qiral_status run_fcg(qiral_lattice *lat, double *x_canon, const double *b_canon, const qiral_solve_params *prm,
                     void *ws, size_t ws_bytes, qiral_solve_info *info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  Flex f;
  qiral_status st = flex_setup(lat, prm, ws, ws_bytes, f);
  if (st != QIRAL_OK) return st;
  double2 *B = f.v(0), *X = f.v(1), *Sv = f.v(2), *Wv = f.v(3), *P = f.v(4), *Z = f.v(5), *R = f.v(6), *Q = f.v(7);
  QIRAL_HIP(hipMemsetAsync(f.vec, 0, 8 * f.vb, s));
  double bn = 0;
  if ((st = flex_begin(f, x_canon, b_canon, prm->x0_is_guess != 0, B, X, bn, s)) != QIRAL_OK) return st;
  const double target = prm->tol * bn;
  // S = B - A X, R = A^dagger S; returns ||S||
  auto residuals = [&](double &sn, bool xzero) -> qiral_status {
    qiral_status r = flex_residual(f, B, X, Sv, sn, s, xzero);
    if (r != QIRAL_OK) return r;
    QIRAL_HIP(flex_A(f, R, Sv, true, s));
    return QIRAL_OK;
  };
  double sn = 0;
  const bool xzero = prm->x0_is_guess == 0;
  if ((st = residuals(sn, xzero)) != QIRAL_OK) return st;
  long long hops = (xzero ? 1 : 2) * flex_hops(f);
  int it = 0, since_best = 0;
  bool broke = false;
  double best = sn, dprev = 0;
  typedef std::complex<double> C;
  while (sn > target && it < prm->maxiter) {
    // Z = M (M^dagger R)
    QIRAL_HIP(flex_M(f, Q, R, true, s));   // Q is free until W = A P below
    QIRAL_HIP(flex_M(f, Z, Q, false, s));
    if (it > 0) {
      // Z -= ((Q_prev | Z) / (P | Q_prev)) P, then P <- Z  (Q_prev = A^dagger A P_prev lives in Wv here)
      C c;
      if ((st = flex_dot(f, Wv, Z, c, s)) != QIRAL_OK) return st;
      if ((st = flex_set_coef(f, {make_double2(-c.real() / dprev, -c.imag() / dprev)}, s)) != QIRAL_OK) return st;
      hipLaunchKernelGGL(k_maxpy, dim3(f.nbk), dim3(256), 0, s, P, f.n2, 1, f.coef, 1.0, Z, f.n2);
    }
    std::swap(P, Z);
    // Q = A P, Wv = A^dagger Q, (P | Wv) = ||Q||^2, (P | R) = conj((R | P))
    QIRAL_HIP(flex_A(f, Q, P, false, s));
    QIRAL_HIP(flex_A(f, Wv, Q, true, s));
    hops += 2 * flex_hops(f);
    C rp;
    if ((st = flex_dot(f, R, P, rp, s)) != QIRAL_OK) return st;
    double d = 0;
    if ((st = flex_norm2(f, Q, d, s)) != QIRAL_OK) return st;
    if (!(d > 0) || !std::isfinite(d)) { broke = true; break; }   // P = 0: the preconditioner returned 0
    // alpha = (P | R) / (P | A^dagger A P); X += alpha P, R -= alpha Wv, S -= alpha Q
    if ((st = flex_set_coef(f, {make_double2(rp.real() / d, -rp.imag() / d)}, s)) != QIRAL_OK) return st;
    hipLaunchKernelGGL(k_fcg_upd, dim3(f.nbk), dim3(256), 0, s, f.coef, P, Wv, Q, X, R, Sv, f.n2, f.npart);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, f.npart, f.nbk, f.nrm, (const double *)nullptr);
    double s2 = 0;
    if ((st = flex_read(&s2, f.nrm, sizeof s2, s)) != QIRAL_OK) return st;
    sn = std::sqrt(s2);
    dprev = d;
    ++it;
    if (!std::isfinite(sn)) break;
    if (sn < 0.99 * best) { best = sn; since_best = 0; }
    else if (++since_best >= 50 && prm->fallback_cg) { broke = true; break; }   // stagnation
  }
  double rt = 0;
  if ((st = flex_end(f, X, x_canon, rt, s)) != QIRAL_OK) return st;
  hops += 2;
  return flex_finish(lat, x_canon, b_canon, prm, ws, ws_bytes, info, it, hops, std::isfinite(sn) ? rt : sn, bn,
                     broke, "FCG", t0, s);
}

// BiCGStab (van der Vorst 1992) with M on the right: the directions p and s are
// preconditioned, p^ = M p, s^ = M s, and x moves along them (the preconditioned
// BiCGStab of Barrett et al., Templates, SIAM 1994); with the identity these are
// plain BiCGStab's iterates.  The nsys right-hand sides run in lockstep: one
// launch of each vector step and dot for all of them, the Schur operator's hops
// on all of them at once, the preconditioner on each system still iterating.
// The scalars of each system stay on the device (k_bq_*); the host reads them
// once per iteration, retires the systems that converged (their coefficients
// then leave x and r unchanged) and restarts those that broke down.  Every
// system takes the iterates it would take alone.
qiral_status run_bicgstab_prec(qiral_lattice *lat, double *x_canon, const double *b_canon, int nsys,
                               const qiral_solve_params *prm, void *ws, size_t ws_bytes, qiral_solve_info *info,
                               hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  Flex f;
  qiral_status st = flex_setup(lat, prm, ws, ws_bytes, f, nsys);
  if (st != QIRAL_OK) return st;
  const Geo &g = lat->geo;
  const size_t stride = (size_t)g.vh * 2 * 24;   // doubles of one canonical field
  enum { B, X, R, RT, P, V, S, T, PH, SH };
  auto blk = [&](int i) { return f.slot(i, 0); };   // vector i of every system
  // p and v start at zero; with padding sites in the last block every vector
  // does, since the vector kernels sum over them and no hop writes them
  if (g.vh % WAVE) QIRAL_HIP(hipMemsetAsync(f.vec, 0, 10 * (size_t)nsys * f.vb, s));
  else for (int i : {(int)P, (int)V}) QIRAL_HIP(hipMemsetAsync(blk(i), 0, (size_t)nsys * f.vb, s));
  std::vector<double> bn(nsys), rn(nsys), target(nsys), rt(nsys);
  std::vector<int> it(nsys, 0), restarts(nsys, 0);
  std::vector<long long> hops(nsys, 0);
  std::vector<char> active(nsys, 1), broke(nsys, 0);
  const std::vector<double2> one(nsys, make_double2(1.0, 0.0)), zero(nsys, make_double2(0.0, 0.0));
  // every system's source, x and residual, with ||b||^2 and ||r||^2 left in
  // its coefficient slots: one host read for all of them
  const bool guess = prm->x0_is_guess != 0;
  const dim3 gn1((unsigned)(nsys * f.nbk), 1), gn2((unsigned)(nsys * f.nbk), 2), gk((unsigned)nsys);
  if (f.schur) {
    // all systems at once, with the same arithmetic as flex_begin and
    // flex_residual system by system: b_e in PH and b_o in SH for now (p and v
    // stay zero for the first iteration)
    if (f.nn) QIRAL_HIP(nn_fold(f.nn, s));
    import_field(g, b_canon, blk(PH), QIRAL_EVEN, QIRAL_F64, nsys, s);
    import_field(g, b_canon, blk(SH), QIRAL_ODD, QIRAL_F64, nsys, s);
    if (guess) import_field(g, x_canon, blk(X), QIRAL_ODD, QIRAL_F64, nsys, s);
    else QIRAL_HIP(hipMemsetAsync(blk(X), 0, (size_t)nsys * f.vb, s));
    for (int k = 0; k < nsys; ++k)
      hipLaunchKernelGGL(k_chi64, dim3(nblk(npad_of(g))), dim3(256), 0, s, g, f.slot(PH, k),
                         (char *)f.tmpE + (size_t)k * f.hb64, (int)CHI_AINV, 2.0 * lat->kappa * lat->mu);
    // b^ = b_o + kappa H_oe A_ee^-1 b_e
    QIRAL_HIP(launch_hop(lat, QIRAL_F64, 0, 1, 1, lat->kappa, f.tmpE, blk(B), blk(SH), nsys, s, CHI_ONE, CHI_ONE));
    hipLaunchKernelGGL(k_norm_sys, gn2, dim3(256), 0, s, blk(PH), blk(SH), f.n2, f.nbk, f.part);
    hipLaunchKernelGGL(k_sum_sys, gk, dim3(256), 0, s, f.part, 2 * f.nbk, f.coef, (int)BQ_BN2);
    if (guess) {
      QIRAL_HIP(flex_A(f, blk(R), blk(X), false, s, nsys));
      hipLaunchKernelGGL(k_bminus, dim3((unsigned)(nsys * f.nbk)), dim3(256), 0, s, blk(B), blk(R),
                         (size_t)nsys * f.n2);
    } else {
      QIRAL_HIP(hipMemcpyAsync(blk(R), blk(B), (size_t)nsys * f.vb, hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_norm_sys, gn1, dim3(256), 0, s, blk(R), (const double2 *)nullptr, f.n2, f.nbk, f.part);
    hipLaunchKernelGGL(k_sum_sys, gk, dim3(256), 0, s, f.part, f.nbk, f.coef, (int)BQ_RN2);
    QIRAL_HIP(hipGetLastError());
  } else {
    for (int k = 0; k < nsys; ++k) {
      const Flex fk = f.sys_view(k);
      if ((st = flex_begin(fk, x_canon + k * stride, b_canon + k * stride, guess, f.slot(B, k), f.slot(X, k), bn[k],
                           s, BQ_BN2, k == 0)) != QIRAL_OK)
        return st;
      if ((st = flex_residual(fk, f.slot(B, k), f.slot(X, k), f.slot(R, k), rn[k], s, !guess, BQ_RN2)) != QIRAL_OK)
        return st;
    }
  }
  std::vector<double2> hc((size_t)nsys * BQ_SLOTS);
  if ((st = flex_read(hc.data(), f.coef, sizeof(double2) * hc.size(), s)) != QIRAL_OK) return st;
  for (int k = 0; k < nsys; ++k) {
    bn[k] = std::sqrt(hc[(size_t)k * BQ_SLOTS + BQ_BN2].x);
    rn[k] = std::sqrt(hc[(size_t)k * BQ_SLOTS + BQ_RN2].x);
    target[k] = prm->tol * bn[k];
    hops[k] = prm->x0_is_guess ? flex_hops(f) : 0;
    active[k] = rn[k] > target[k] && prm->maxiter > 0;
    QIRAL_HIP(hipMemcpyAsync(f.coef + (size_t)k * BQ_SLOTS + BQ_DONE, active[k] ? &zero[k] : &one[k], sizeof(double2),
                             hipMemcpyHostToDevice, s));
  }
  auto retire = [&](int k) -> qiral_status {   // x and r of system k stay as they are from now on
    active[k] = 0;
    QIRAL_HIP(hipMemcpyAsync(f.coef + (size_t)k * BQ_SLOTS + BQ_DONE, &one[k], sizeof(double2),
                             hipMemcpyHostToDevice, s));
    return QIRAL_OK;
  };
  auto restart = [&](int k) -> qiral_status {   // shadow residual r~ = r, rho = alpha = omega = 1, p = v = 0
    QIRAL_HIP(hipMemcpyAsync(f.slot(RT, k), f.slot(R, k), f.vb, hipMemcpyDeviceToDevice, s));
    QIRAL_HIP(hipMemsetAsync(f.slot(P, k), 0, f.vb, s));
    QIRAL_HIP(hipMemsetAsync(f.slot(V, k), 0, f.vb, s));
    hipLaunchKernelGGL(k_bq_init, dim3(1), dim3(1), 0, s, f.coef + (size_t)k * BQ_SLOTS, 1);
    flex_dot_dev(f.sys_view(k), f.slot(RT, k), f.slot(R, k), BQ_RHO1, s);
    return QIRAL_OK;
  };
  const size_t ntot = (size_t)nsys * f.n2;
  const dim3 gv((unsigned)(nsys * f.nbk)), bv(256), gs((unsigned)((nsys + 63) / 64)), bs(64);
  auto any_active = [&]() { return std::find(active.begin(), active.end(), 1) != active.end(); };
  if (any_active()) {
    QIRAL_HIP(hipMemcpyAsync(blk(RT), blk(R), (size_t)nsys * f.vb, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_bq_init, gs, bs, 0, s, f.coef, nsys);
    hipLaunchKernelGGL(k_dot1, gv, bv, 0, s, blk(RT), blk(R), ntot, f.part);
    hipLaunchKernelGGL(k_pair_final, dim3(1, nsys), dim3(256), 0, s, f.part, f.nbk, f.coef, (int)BQ_RHO1,
                       (int)BQ_RHO1);
  }
  while (any_active()) {
    hipLaunchKernelGGL(k_bq_beta, gs, bs, 0, s, f.coef, nsys);
    hipLaunchKernelGGL(k_bq_p, gv, bv, 0, s, f.coef, blk(R), blk(V), blk(P), f.n2, ntot);   // p = r + beta (p - omega v)
    QIRAL_HIP(flex_M(f, blk(PH), blk(P), false, s, nsys));
    QIRAL_HIP(flex_A(f, blk(V), blk(PH), false, s, nsys));
    hipLaunchKernelGGL(k_dot1, gv, bv, 0, s, blk(RT), blk(V), ntot, f.part);
    hipLaunchKernelGGL(k_pair_final, dim3(1, nsys), dim3(256), 0, s, f.part, f.nbk, f.coef, (int)BQ_RV, (int)BQ_RV);
    hipLaunchKernelGGL(k_bq_alpha, gs, bs, 0, s, f.coef, nsys);
    hipLaunchKernelGGL(k_bq_s, gv, bv, 0, s, f.coef, blk(V), blk(R), blk(S), f.n2, ntot);   // s = r - alpha v
    QIRAL_HIP(flex_M(f, blk(SH), blk(S), false, s, nsys));
    QIRAL_HIP(flex_A(f, blk(T), blk(SH), false, s, nsys));
    hipLaunchKernelGGL(k_dot2, gv, bv, 0, s, blk(T), blk(S), ntot, f.part);   // (t|s), ||t||^2
    hipLaunchKernelGGL(k_pair_final, dim3(2, nsys), dim3(256), 0, s, f.part, f.nbk, f.coef, (int)BQ_TS, (int)BQ_TT);
    hipLaunchKernelGGL(k_bq_omega, gs, bs, 0, s, f.coef, nsys);
    // x += alpha p^ + omega s^; r = s - omega t with (r~|r), the next rho, and ||r||^2
    hipLaunchKernelGGL(k_bq_x, gv, bv, 0, s, f.coef, blk(PH), blk(SH), blk(X), f.n2, ntot);
    hipLaunchKernelGGL(k_bq_r, gv, bv, 0, s, f.coef, blk(S), blk(T), blk(RT), blk(R), f.n2, ntot, f.part);
    hipLaunchKernelGGL(k_pair_final, dim3(2, nsys), dim3(256), 0, s, f.part, f.nbk, f.coef, (int)BQ_RHO1,
                       (int)BQ_RN2);
    if ((st = flex_read(hc.data(), f.coef, sizeof(double2) * hc.size(), s)) != QIRAL_OK) return st;
    for (int k = 0; k < nsys; ++k) {
      if (!active[k]) continue;
      const double2 *c = hc.data() + (size_t)k * BQ_SLOTS;
      bool again = c[BQ_FLAG].x != 0.0;   // broke down before x changed: the iteration does not count
      if (!again) {
        hops[k] += 2 * flex_hops(f);
        rn[k] = std::sqrt(c[BQ_RN2].x);
        ++it[k];
        if (!std::isfinite(rn[k]) || rn[k] <= target[k]) {
          if ((st = retire(k)) != QIRAL_OK) return st;
          continue;
        }
        again = c[BQ_FLAG].y != 0.0;   // omega = 0
      }
      if (it[k] >= prm->maxiter) {
        if ((st = retire(k)) != QIRAL_OK) return st;
      } else if (again) {
        // breakdown: restart from the current x with the recomputed residual
        if (++restarts[k] > 5) {
          broke[k] = 1;
          if ((st = retire(k)) != QIRAL_OK) return st;
          continue;
        }
        if ((st = flex_residual(f.sys_view(k), f.slot(B, k), f.slot(X, k), f.slot(R, k), rn[k], s)) != QIRAL_OK)
          return st;
        hops[k] += flex_hops(f);
        if (rn[k] <= target[k]) {
          if ((st = retire(k)) != QIRAL_OK) return st;
        } else if ((st = restart(k)) != QIRAL_OK) {
          return st;
        }
      }
    }
  }
  // every solution out first (a CG fallback below reuses the workspace), with
  // ||b - D x||^2 in the coefficient slots: one host read for all systems
  if (f.schur) {
    // all systems at once, with flex_end's arithmetic: b_e in V, b_o in S,
    // x_e in P, D x in T (even) and PH (odd), then b - D x there
    const double k1 = lat->kappa;
    import_field(g, b_canon, blk(V), QIRAL_EVEN, QIRAL_F64, nsys, s);
    import_field(g, b_canon, blk(S), QIRAL_ODD, QIRAL_F64, nsys, s);
    // x_e = A_ee^-1 (b_e + kappa H_eo x_o)
    QIRAL_HIP(launch_hop(lat, QIRAL_F64, 0, 0, 1, k1, blk(X), blk(P), blk(V), nsys, s, CHI_AINV, CHI_ONE));
    QIRAL_HIP(launch_hop(lat, QIRAL_F64, 0, 0, 1, -k1, blk(X), blk(T), blk(P), nsys, s, CHI_ONE, CHI_A));
    QIRAL_HIP(launch_hop(lat, QIRAL_F64, 0, 1, 1, -k1, blk(P), blk(PH), blk(X), nsys, s, CHI_ONE, CHI_A));
    const dim3 gb((unsigned)(nsys * f.nbk));
    hipLaunchKernelGGL(k_bminus, gb, dim3(256), 0, s, blk(V), blk(T), (size_t)nsys * f.n2);
    hipLaunchKernelGGL(k_bminus, gb, dim3(256), 0, s, blk(S), blk(PH), (size_t)nsys * f.n2);
    hipLaunchKernelGGL(k_norm_sys, gn2, dim3(256), 0, s, blk(T), blk(PH), f.n2, f.nbk, f.part);
    hipLaunchKernelGGL(k_sum_sys, gk, dim3(256), 0, s, f.part, 2 * f.nbk, f.coef, (int)BQ_TR2);
    export_field(g, x_canon, blk(P), QIRAL_EVEN, QIRAL_F64, nsys, s);
    export_field(g, x_canon, blk(X), QIRAL_ODD, QIRAL_F64, nsys, s);
    QIRAL_HIP(hipGetLastError());
    for (int k = 0; k < nsys; ++k) hops[k] += 2;
  } else {
    for (int k = 0; k < nsys; ++k) {
      import_field(g, b_canon + k * stride, f.BF, QIRAL_FULL, QIRAL_F64, 1, s);
      if ((st = flex_end(f.sys_view(k), f.slot(X, k), x_canon + k * stride, rt[k], s, BQ_TR2)) != QIRAL_OK)
        return st;
      hops[k] += 2;
    }
  }
  if ((st = flex_read(hc.data(), f.coef, sizeof(double2) * hc.size(), s)) != QIRAL_OK) return st;
  for (int k = 0; k < nsys; ++k) rt[k] = std::sqrt(hc[(size_t)k * BQ_SLOTS + BQ_TR2].x);
  qiral_status worst = QIRAL_OK;
  for (int k = 0; k < nsys; ++k) {
    st = flex_finish(lat, x_canon + k * stride, b_canon + k * stride, prm, ws, ws_bytes, info + k, it[k], hops[k],
                     std::isfinite(rn[k]) ? rt[k] : rn[k], bn[k], broke[k] != 0, "BiCGStab", t0, s);
    if (st != QIRAL_OK && st != QIRAL_ERR_NOT_CONVERGED) return st;
    if (st != QIRAL_OK) worst = st;
  }
  return worst;
}
}  // namespace qiral
