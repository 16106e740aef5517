// C ABI of the library: argument validation, lattice handles, packing of links
// and fields, the hopping-term and operator entry points.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>

#include "qiral_int.h"

using namespace qiral;

// ---------------------------------------------------------------------------
// errors
namespace qiral {
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
qiral_status hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return QIRAL_ERR_HIP;
}
}  // namespace qiral

extern "C" const char *qiral_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *qiral_status_string(qiral_status s) {
  switch (s) {
    case QIRAL_OK: return "ok";
    case QIRAL_ERR_INVALID_ARG: return "invalid argument";
    case QIRAL_ERR_BAD_DIMS: return "bad lattice dimensions";
    case QIRAL_ERR_UNSUPPORTED: return "unsupported";
    case QIRAL_ERR_HIP: return "HIP runtime error";
    case QIRAL_ERR_NOT_CONVERGED: return "not converged";
    case QIRAL_ERR_NONFINITE: return "non-finite value";
    case QIRAL_ERR_WORKSPACE: return "workspace allocation failed";
  }
  return "unknown status";
}

static qiral_status fail(qiral_status s, const char *msg) {
  set_error(msg);
  return s;
}

static qiral_status check_dims(const int32_t *d) {
  if (!d) return fail(QIRAL_ERR_INVALID_ARG, "dims is NULL");
  int64_t v = 1;
  for (int i = 0; i < 4; ++i) {
    if (d[i] < 2 || (d[i] & 1)) return fail(QIRAL_ERR_BAD_DIMS, "every lattice extent must be even and >= 2");
    v *= d[i];
  }
  if (v / 2 > (1ll << 30)) return fail(QIRAL_ERR_BAD_DIMS, "lattice too large (more than 2^30 sites per parity)");
  return QIRAL_OK;
}

static bool valid_prec(int p) { return p == QIRAL_F64 || p == QIRAL_F32 || p == QIRAL_F16S; }

namespace qiral {
static size_t site_bytes(int prec) {
  return prec == QIRAL_F64 ? SpinorIO<S_F64>::SITE_BYTES
       : prec == QIRAL_F32 ? SpinorIO<S_F32>::SITE_BYTES : SpinorIO<S_F16S>::SITE_BYTES;
}
size_t half_bytes(const Geo &g, int prec) { return npad_of(g) * site_bytes(prec); }
const void *links_for(const qiral_lattice *lat, int prec) {
  return prec == QIRAL_F64 ? lat->g64 : prec == QIRAL_F32 ? lat->g32 : lat->g16;
}
size_t link_store_bytes(const Geo &g, int prec) {
  const size_t link = prec == QIRAL_F64 ? LinkIO<L_F64R18>::LINK_BYTES
                    : prec == QIRAL_F32 ? LinkIO<L_F32R12>::LINK_BYTES
                    : prec == QIRAL_F16S ? LinkIO<L_F16R12>::LINK_BYTES : 0;
  return 8 * npad_of(g) * link;   // 4 forward links per site of each parity
}
}  // namespace qiral

extern "C" size_t qiral_gauge_bytes(const int32_t dims[4], qiral_prec prec, qiral_recon recon) {
  if (check_dims(dims) != QIRAL_OK || !valid_prec(prec)) return 0;
  if ((prec == QIRAL_F64) != (recon == QIRAL_RECON18)) return 0;   // F64: 18 reals; F32, F16: 12
  if (recon != QIRAL_RECON18 && recon != QIRAL_RECON12) return 0;
  return link_store_bytes(make_geo(dims), prec);
}

extern "C" size_t qiral_field_bytes(const int32_t dims[4], qiral_subset subset, qiral_prec prec, int32_t nrhs) {
  if (check_dims(dims) != QIRAL_OK || !valid_prec(prec) || nrhs < 1) return 0;
  if (subset != QIRAL_EVEN && subset != QIRAL_ODD && subset != QIRAL_FULL) return 0;
  Geo g = make_geo(dims);
  size_t h = half_bytes(g, prec);
  return (subset == QIRAL_FULL ? 2 * h : h) * (size_t)nrhs;
}

// ---------------------------------------------------------------------------
// kernels: packing
__device__ __forceinline__ void site_coords(const Geo &g, int s, int p, int &x, int &y, int &z, int &t) {
  int xh = s % g.lxh;
  int r = s / g.lxh;
  y = r % g.ly; r /= g.ly;
  z = r % g.lz;
  t = r / g.lz;
  x = 2 * xh + ((p + y + z + t) & 1);
}

__device__ __forceinline__ size_t lex_of(const Geo &g, int x, int y, int z, int t) {
  return (((size_t)t * g.lz + z) * g.ly + y) * g.lx + x;
}

template <int L>
__global__ __launch_bounds__(WG) void k_pack_gauge(Geo g, const double *__restrict__ canon, void *__restrict__ dst) {
  const size_t npad = (size_t)g.nb * WAVE;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 8 * npad) return;
  const int s = (int)(i % npad);
  const int pm = (int)(i / npad);   // parity * 4 + mu
  const int p = pm >> 2, mu = pm & 3;
  if (s >= g.vh) return;
  int x, y, z, t;
  site_coords(g, s, p, x, y, z, t);
  const double *src = canon + (lex_of(g, x, y, z, t) * 4 + mu) * 18;
  const size_t blk = (size_t)pm * g.nb + (s >> 6);
  if (L == L_F64R18) {
    double2 *d = (double2 *)dst + blk * 9 * WAVE + (s & 63);
    for (int j = 0; j < 9; ++j) d[j * WAVE] = make_double2(src[2 * j], src[2 * j + 1]);
  } else if (L == L_F32R12) {
    float4 *d = (float4 *)dst + blk * 3 * WAVE + (s & 63);
    for (int j = 0; j < 3; ++j)
      d[j * WAVE] = make_float4((float)src[4 * j], (float)src[4 * j + 1], (float)src[4 * j + 2], (float)src[4 * j + 3]);
  } else {
    uint2 *d = (uint2 *)dst + blk * 3 * WAVE + (s & 63);
    for (int j = 0; j < 3; ++j) {
      unsigned a = d2h(src[4 * j]) | ((unsigned)d2h(src[4 * j + 1]) << 16);
      unsigned b = d2h(src[4 * j + 2]) | ((unsigned)d2h(src[4 * j + 3]) << 16);
      d[j * WAVE] = make_uint2(a, b);
    }
  }
}

// FP16 links: each real is rounded FP64 -> FP16 once, to nearest even (d2h);
// FP32 links: FP64 -> FP32, to nearest even.

template <int S>
__global__ __launch_bounds__(WG) void k_import(Geo g, const double *__restrict__ canon, size_t canon_stride,
                                               void *__restrict__ dst, size_t dst_stride, int p, int nrhs) {
  using R = typename SpinorIO<S>::R;
  const size_t npad = (size_t)g.nb * WAVE;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad * nrhs) return;
  const int s = (int)(i % npad);
  const int r = (int)(i / npad);
  cpx<R> v[12];
  if (s < g.vh) {
    int x, y, z, t;
    site_coords(g, s, p, x, y, z, t);
    const double2 *src = (const double2 *)(canon + r * canon_stride) + lex_of(g, x, y, z, t) * 12;
    for (int k = 0; k < 12; ++k) { double2 q = src[k]; v[k] = cmake((R)q.x, (R)q.y); }
  } else {
    for (int k = 0; k < 12; ++k) v[k] = cmake((R)0, (R)0);
  }
  SpinorIO<S>::store((char *)dst + r * dst_stride, s, npad, v);
}

template <int S>
__global__ __launch_bounds__(WG) void k_export(Geo g, double *__restrict__ canon, size_t canon_stride,
                                               const void *__restrict__ src, size_t src_stride, int p, int nrhs) {
  using R = typename SpinorIO<S>::R;
  const size_t npad = (size_t)g.nb * WAVE;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad * nrhs) return;
  const int s = (int)(i % npad);
  const int r = (int)(i / npad);
  if (s >= g.vh) return;
  cpx<R> v[12];
  SpinorIO<S>::load((const char *)src + r * src_stride, s, npad, v);
  int x, y, z, t;
  site_coords(g, s, p, x, y, z, t);
  double2 *d = (double2 *)(canon + r * canon_stride) + lex_of(g, x, y, z, t) * 12;
  for (int k = 0; k < 12; ++k) d[k] = make_double2((double)v[k].re, (double)v[k].im);
}

// ---------------------------------------------------------------------------
// kernel: hopping term on one lattice, nrhs consecutive fields.  A work item
// is one 64-site block of a group of NR right-hand sides (each lane applies
// every link it loads to all NR of them).  Items run tile by tile: within a
// tile of at least two t-slices, every group sweeps the tile's blocks in turn,
// so a group's neighbour spinors are re-read while still cached and the tile's
// links are re-read from cache by the next group.  T waves cover an item, each
// taking 4/T directions for all 64 sites (hop_wave), and their sums are added
// in LDS (wave_combine).
template <int S, int L, bool DAG, int EPI, int T, int NR, bool NT>
__global__ __launch_bounds__(WG, HOP_MIN_WAVES(S, T, NR)) void k_hop(Geo g, const void *__restrict__ gauge,
                                                             const void *__restrict__ in, void *__restrict__ out,
                                                             const void *__restrict__ xin, size_t fstride, int nrhs,
                                                             int p, double a, int tile, int zb, int chio, int chix,
                                                             double tmu) {
  using R = typename SpinorIO<S>::R;
  using LDS = HopLds<T, NR, R>;
  __shared__ typename LDS::V lds[LDS::VECS];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
  const int slot = w / T, grp = w % T;
  const int item = wg * (4 / T) + slot;
  // item order: (tile of `tile` blocks, right-hand-side group, block in tile)
  const int ngr = (nrhs + NR - 1) / NR;
  const int per_tile = ngr * tile;
  const int ti = item / per_tile, rem = item - ti * per_tile;
  const int rg = rem / tile;
  const int sbl = ti * tile + (rem - rg * tile);
  const bool item_ok = sbl < g.nb;   // uniform over the item's waves
  const int sb = item_ok ? block_order(g, sbl, zb) : 0;
  const int r0 = rg * NR;
  const int cnt = item_ok ? min(NR, nrhs - r0) : 1;
  const int s = sb * WAVE + (int)(threadIdx.x & (WAVE - 1));
  const bool site_ok = item_ok && s < g.vh;
  const size_t npad = (size_t)g.nb * WAVE;
  FieldLd<S, NR> ld;
  ld.npad = npad;
#pragma unroll
  for (int r = 0; r < NR; ++r) ld.base[r] = (const char *)in + (size_t)(r0 + min(r, cnt - 1)) * fstride;
  cpx<R> acc[NR][12];
  if (item_ok) hop_wave<L, DAG, T, NT>(g, gauge, ld, site_ok ? s : 0, p, grp, acc);
  else zero_acc<NR>(acc);
  wave_combine<T, NR>(acc, slot, grp, lds);
  if (!site_ok || grp != 0) return;
  const R ar = (R)a;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= cnt) continue;
    if (EPI == 0) {
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[r][k] = cscale(ar, acc[r][k]);
    } else {
      cpx<R> xv[12];
      SpinorIO<S>::load((const char *)xin + (size_t)(r0 + r) * fstride, s, npad, xv);
      apply_chi(xv, chix, tmu);
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[r][k] = cadd(xv[k], cscale(ar, acc[r][k]));
    }
    apply_chi(acc[r], chio, tmu);
    SpinorIO<S>::template store_fast<NT>((char *)out + (size_t)(r0 + r) * fstride, s, npad, acc[r]);
  }
}

namespace qiral {
HopCfg hop_config(const qiral_lattice *lat, int prec, long nrhs) {
  HopCfg c;
  const long nb = lat->geo.nb;
  if (const char *e = getenv("QIRAL_HOP_NR")) c.nr = atoi(e);
  else c.nr = tuned_nr(lat, prec, (int)nrhs);
  c.nr = std::max(1, std::min(c.nr, 4));
  if (c.nr > nrhs) c.nr = (int)nrhs;
  const long nitems = nb * ((nrhs + c.nr - 1) / c.nr);
  c.t = hop_split(prec, nitems);
  const int tt = lat->tuned_t[prec][nrhs < 4 ? nrhs : 4];
  if (tt && !getenv("QIRAL_HOP_SPLIT") && hop_nr_max(prec, tt) >= 1) c.t = tt;
  c.tile = lat->tuned_tile[prec][nrhs < 4 ? nrhs : 4];
  if (c.nr > hop_nr_max(prec, c.t)) c.t = (c.t == 1 && c.nr <= hop_nr_max(prec, 2)) ? 2 : 4;
  c.nr = std::min(c.nr, hop_nr_max(prec, c.t));   // FP64 takes at most 2
  return c;
}

bool hop_stream(const Geo &g, int prec, long nrhs, long ngroups) {
  if (const char *e = getenv("QIRAL_HOP_NT")) return atoi(e) != 0;
  if (ngroups > 1) return false;   // the groups re-read the tile's links
  const double link = prec == QIRAL_F64 ? 96 : prec == QIRAL_F32 ? 48 : 24;   // bytes a hop reads per link
  const double sp = prec == QIRAL_F64 ? 192 : prec == QIRAL_F32 ? 96 : 52;
  const double bytes = (double)g.vh * (8 * link + 2 * sp * nrhs);
  return bytes > 128e6;   // half the 256 MB last-level cache
}

bool zb_valid(const Geo &g, int zb) {
  return zb > 0 && zb < g.lz && g.lz % zb == 0 && (long)zb * g.sz % WAVE == 0 && g.st % WAVE == 0;
}

int hop_zb(const Geo &g) {
  if (g.st % WAVE != 0 || (long)g.nb * WAVE != g.vh) return 0;
  if (const char *e = getenv("QIRAL_HOP_ORDER")) {   // 0: plain order; n > 0: tiles of n planes
    const int n = atoi(e);
    return zb_valid(g, n) ? n : 0;
  }
  // A lattice whose FP64 hop (1152 B per site) fits the 256 MB last-level
  // cache keeps the plain order: its hops run from that cache, and tiling them
  // cost up to 10% (FP32 at 16^3x32).
  if ((double)g.vh * 1152.0 <= 256e6) return 0;
  // As many z-tiles as XCDs (else half or a quarter as many), so that the
  // contiguous range of blocks each XCD takes (xcd_remap) is one whole tile or
  // a whole part of one: a tile's z-neighbour planes are then read twice only
  // where two XCDs meet, and a block's t-neighbours were read one chunk earlier
  // on the same XCD.  Measured on the 1-RHS hops at 64^3x128, tiles of Lz/8
  // planes ran 21% (FP64), 15% (FP32) and 8% (F16S) faster than tiles of about
  // 0.5 MB of input spinors (1, 2 and 4 planes); at 32^3x64 and 24^3x48 the
  // best tiles were Lz/8 and Lz/4 planes as well.
  for (int ntz : {NXCD, NXCD / 2, NXCD / 4})
    if (g.lz % ntz == 0 && zb_valid(g, g.lz / ntz)) return g.lz / ntz;
  return 0;   // the plain order
}

int hop_tile(const Geo &g, int ngroups, int tuned) {
  if (ngroups <= 1) return g.nb;   // one group: plain block order
  if (const char *e = getenv("QIRAL_HOP_TILE")) {
    const int n = atoi(e);
    if (n > 0) return std::min(g.nb, n);
  }
  // Each group sweeps a tile before the next group does, so the tile's links are
  // re-read from the L2 while they are still there: 16 blocks (1.2 MB of FP64
  // links) measured within a few percent of the best tile at 24^3x48 for every
  // storage class, where tiles of two t-slices (216 blocks) were 5-25% slower.
  if (tuned > 0) return std::min(g.nb, tuned);
  return std::min(g.nb, 16);
}

int hop_split(int prec, long nwork) {
  if (const char *e = getenv("QIRAL_HOP_SPLIT")) {
    const int t = atoi(e);
    if (t == 4 || (t == 2 && prec != QIRAL_F64) || (t == 1 && prec == QIRAL_F16S)) return t;
  }
  // FP64 needs 4 waves per site block (fewer spill); otherwise 4 while the
  // blocks do not fill the SIMDs (more waves hide more latency), else 2 (less
  // LDS traffic and fewer redundant coordinate computations per site).  One
  // wave per block (F16S only) is left to the tuner.
  const long simds = 1024;   // 256 compute units x 4 SIMDs
  if (prec == QIRAL_F64 || nwork <= simds) return 4;
  return 2;
}

template <int S, int L, int T, int NR, bool NT>
static hipError_t launch_hop_ttt(const HopCfg &c, const qiral_lattice *lat, int dagger, int p, int epi, double a,
                                 const void *in,
                                 void *out, const void *x, int nrhs, hipStream_t st, int chio, int chix) {
  const Geo &g = lat->geo;
  const double tmu = 2.0 * lat->kappa * lat->mu;
  const size_t fstride = half_bytes(g, S);
  const void *gauge = links_for(lat, S);
  const int tile = hop_tile(g, (nrhs + NR - 1) / NR, c.tile);
  const int zb = hop_zb(g);
  const long ntile = (g.nb + tile - 1) / tile;
  const long nitems = ntile * tile * ((nrhs + NR - 1) / NR);
  const int nwg = (int)((nitems * T + 3) / 4);
  dim3 grid(nwg), block(WG);
  if (!dagger) {
    if (epi == 0) hipLaunchKernelGGL((k_hop<S, L, false, 0, T, NR, NT>), grid, block, 0, st, g, gauge, in, out, x, fstride, nrhs, p, a, tile, zb, chio, chix, tmu);
    else hipLaunchKernelGGL((k_hop<S, L, false, 1, T, NR, NT>), grid, block, 0, st, g, gauge, in, out, x, fstride, nrhs, p, a, tile, zb, chio, chix, tmu);
  } else {
    if (epi == 0) hipLaunchKernelGGL((k_hop<S, L, true, 0, T, NR, NT>), grid, block, 0, st, g, gauge, in, out, x, fstride, nrhs, p, a, tile, zb, chio, chix, tmu);
    else hipLaunchKernelGGL((k_hop<S, L, true, 1, T, NR, NT>), grid, block, 0, st, g, gauge, in, out, x, fstride, nrhs, p, a, tile, zb, chio, chix, tmu);
  }
  return hipGetLastError();
}

template <int S, int L, int T, int NR>
static hipError_t launch_hop_tt(const HopCfg &c, const qiral_lattice *lat, int dagger, int p, int epi, double a,
                                const void *in, void *out, const void *x, int nrhs, hipStream_t st, int chio,
                                int chix) {
  if (hop_stream(lat->geo, S, nrhs, (nrhs + NR - 1) / NR))
    return launch_hop_ttt<S, L, T, NR, true>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
  return launch_hop_ttt<S, L, T, NR, false>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
}

template <int S, int L, int T>
static hipError_t launch_hop_n(const HopCfg &c, const qiral_lattice *lat, int dagger, int p, int epi, double a,
                               const void *in, void *out, const void *x, int nrhs, hipStream_t st, int chio, int chix) {
  constexpr int NM = hop_nr_max(S, T);   // shapes beyond it are excluded by hop_config and the tuner
  if constexpr (NM == 0) {
    return hipErrorInvalidValue;
  } else {
    if (c.nr > NM) return hipErrorInvalidValue;
    if constexpr (NM >= 4) if (c.nr == 4) return launch_hop_tt<S, L, T, 4>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
    if constexpr (NM >= 3) if (c.nr == 3) return launch_hop_tt<S, L, T, 3>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
    if constexpr (NM >= 2) if (c.nr == 2) return launch_hop_tt<S, L, T, 2>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
    return launch_hop_tt<S, L, T, 1>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
  }
}

template <int S, int L>
static hipError_t launch_hop_t(const HopCfg &c, const qiral_lattice *lat, int dagger, int p, int epi, double a,
                               const void *in, void *out, const void *x, int nrhs, hipStream_t st, int chio, int chix) {
  if constexpr (S == S_F64) return launch_hop_n<S, L, 4>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
  else {
    if (c.t == 4) return launch_hop_n<S, L, 4>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
    if (c.t == 1) return launch_hop_n<S, L, 1>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
    return launch_hop_n<S, L, 2>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
  }
}

hipError_t launch_hop_cfg(const HopCfg &c, const qiral_lattice *lat, int prec, int dagger, int p, int epi, double a,
                          const void *in, void *out, const void *x, int nrhs, hipStream_t st, int chio, int chix) {
  if (prec == QIRAL_F64) return launch_hop_t<S_F64, L_F64R18>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
  if (prec == QIRAL_F32) return launch_hop_t<S_F32, L_F32R12>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
  return launch_hop_t<S_F16S, L_F16R12>(c, lat, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
}

hipError_t launch_hop(const qiral_lattice *lat, int prec, int dagger, int p, int epi, double a, const void *in,
                      void *out, const void *x, int nrhs, hipStream_t st, int chio, int chix) {
  return launch_hop_cfg(hop_config(lat, prec, nrhs), lat, prec, dagger, p, epi, a, in, out, x, nrhs, st, chio, chix);
}
}  // namespace qiral

// ---------------------------------------------------------------------------
// lattice handle
static void release_handle(qiral_lattice *lat) {
  for (hipEvent_t e : lat->poll_ev) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : lat->time_ev) if (e) (void)hipEventDestroy(e);
  if (lat->pinned) (void)hipHostFree(lat->pinned);
  delete lat;
}

extern "C" qiral_status qiral_lattice_create(qiral_lattice **out, const int32_t dims[4], double kappa, double mu,
                                             const double *gauge_canon, void *gauge_f64, void *gauge_f32,
                                             void *gauge_f16, qiral_stream_t stream) {
  if (!out) return fail(QIRAL_ERR_INVALID_ARG, "lat is NULL");
  *out = nullptr;
  qiral_status st = check_dims(dims);
  if (st != QIRAL_OK) return st;
  if (!gauge_canon) return fail(QIRAL_ERR_INVALID_ARG, "gauge_canon is NULL");
  if (!gauge_f64) return fail(QIRAL_ERR_INVALID_ARG, "gauge_f64 is NULL (the FP64 store is required)");
  if (!std::isfinite(kappa) || !std::isfinite(mu)) return fail(QIRAL_ERR_INVALID_ARG, "kappa and mu must be finite");
  for (const void *p : {gauge_f64, gauge_f32, gauge_f16})
    if (((uintptr_t)p & 15) != 0) return fail(QIRAL_ERR_INVALID_ARG, "link stores must be 16-byte aligned");
  if ((gauge_f32 && (gauge_f32 == gauge_f64 || gauge_f32 == gauge_f16)) || (gauge_f16 && gauge_f16 == gauge_f64))
    return fail(QIRAL_ERR_INVALID_ARG, "the link stores must be distinct buffers");

  qiral_lattice *lat = new qiral_lattice();
  for (int i = 0; i < 4; ++i) lat->dims[i] = dims[i];
  lat->geo = make_geo(dims);
  lat->kappa = kappa;
  lat->mu = mu;
  lat->g64 = gauge_f64;
  lat->g32 = gauge_f32;
  lat->g16 = gauge_f16;
  hipStream_t s = (hipStream_t)stream;
  const Geo &g = lat->geo;
  auto cleanup = [&](qiral_status r) {
    release_handle(lat);
    return r;
  };
  hipError_t e = hipGetDevice(&lat->device);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
  // host-side resources of later solves and tuning, made once here
  e = hipHostMalloc(&lat->pinned, poll_bytes(), hipHostMallocDefault);
  if (e != hipSuccess) { lat->pinned = nullptr; return cleanup(hip_fail(e, "hipHostMalloc(state polls)")); }
  lat->pinned_bytes = poll_bytes();
  for (hipEvent_t &ev : lat->poll_ev) {
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) { ev = nullptr; return cleanup(hip_fail(e, "hipEventCreate")); }
  }
  for (hipEvent_t &ev : lat->time_ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) { ev = nullptr; return cleanup(hip_fail(e, "hipEventCreate")); }
  }
  const size_t nlinks = 8 * npad_of(g);
  const int nblk = (int)((nlinks + WG - 1) / WG);
  hipLaunchKernelGGL(k_pack_gauge<L_F64R18>, dim3(nblk), dim3(WG), 0, s, g, gauge_canon, lat->g64);
  lat->gauge_bytes = link_store_bytes(g, QIRAL_F64);
  if (gauge_f32) {
    hipLaunchKernelGGL(k_pack_gauge<L_F32R12>, dim3(nblk), dim3(WG), 0, s, g, gauge_canon, lat->g32);
    lat->gauge_bytes += link_store_bytes(g, QIRAL_F32);
  }
  if (gauge_f16) {
    hipLaunchKernelGGL(k_pack_gauge<L_F16R12>, dim3(nblk), dim3(WG), 0, s, g, gauge_canon, lat->g16);
    lat->gauge_bytes += link_store_bytes(g, QIRAL_F16S);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return cleanup(hip_fail(e, "pack links"));
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamSynchronize(lattice_create)"));
  *out = lat;
  return QIRAL_OK;
}

extern "C" qiral_status qiral_lattice_destroy(qiral_lattice *lat) {
  if (!lat) return fail(QIRAL_ERR_INVALID_ARG, "lat is NULL");
  release_handle(lat);
  return QIRAL_OK;
}

extern "C" qiral_status qiral_lattice_query(const qiral_lattice *lat, int64_t *vh, int64_t *bytes) {
  if (!lat) return fail(QIRAL_ERR_INVALID_ARG, "lat is NULL");
  if (vh) *vh = lat->geo.vh;
  if (bytes) *bytes = (int64_t)lat->gauge_bytes;
  return QIRAL_OK;
}

// ---------------------------------------------------------------------------
// field import / export
static qiral_status check_field_args(const qiral_lattice *lat, const void *a, const void *b, int subset, int prec,
                                     int nrhs) {
  if (!lat) return fail(QIRAL_ERR_INVALID_ARG, "lat is NULL");
  if (!a || !b) return fail(QIRAL_ERR_INVALID_ARG, "field pointer is NULL");
  if (subset != QIRAL_EVEN && subset != QIRAL_ODD && subset != QIRAL_FULL)
    return fail(QIRAL_ERR_INVALID_ARG, "bad subset");
  if (!valid_prec(prec)) return fail(QIRAL_ERR_INVALID_ARG, "bad precision");
  if (nrhs < 1) return fail(QIRAL_ERR_INVALID_ARG, "nrhs must be >= 1");
  return QIRAL_OK;
}

template <int S>
static void launch_import(const Geo &g, const double *src, void *dst, int subset, int nrhs, hipStream_t s) {
  const size_t canon_stride = (size_t)g.vh * 2 * 24;   // doubles per canonical field
  const size_t hb = half_bytes(g, S);
  const size_t dstride = subset == QIRAL_FULL ? 2 * hb : hb;
  const size_t n = npad_of(g) * nrhs;
  const int nblk = (int)((n + WG - 1) / WG);
  for (int p = 0; p < 2; ++p) {
    if (subset != QIRAL_FULL && subset != p) continue;
    void *d = (char *)dst + (subset == QIRAL_FULL ? p * hb : 0);
    hipLaunchKernelGGL(k_import<S>, dim3(nblk), dim3(WG), 0, s, g, src, canon_stride, d, dstride, p, nrhs);
  }
}

template <int S>
static void launch_export(const Geo &g, double *dst, const void *src, int subset, int nrhs, hipStream_t s) {
  const size_t canon_stride = (size_t)g.vh * 2 * 24;
  const size_t hb = half_bytes(g, S);
  const size_t sstride = subset == QIRAL_FULL ? 2 * hb : hb;
  const size_t n = npad_of(g) * nrhs;
  const int nblk = (int)((n + WG - 1) / WG);
  for (int p = 0; p < 2; ++p) {
    if (subset != QIRAL_FULL && subset != p) continue;
    const void *sp = (const char *)src + (subset == QIRAL_FULL ? p * hb : 0);
    hipLaunchKernelGGL(k_export<S>, dim3(nblk), dim3(WG), 0, s, g, dst, canon_stride, sp, sstride, p, nrhs);
  }
}

namespace qiral {
void import_field(const Geo &g, const double *src, void *dst, int subset, int prec, int nrhs, hipStream_t s) {
  if (prec == QIRAL_F64) launch_import<S_F64>(g, src, dst, subset, nrhs, s);
  else if (prec == QIRAL_F32) launch_import<S_F32>(g, src, dst, subset, nrhs, s);
  else launch_import<S_F16S>(g, src, dst, subset, nrhs, s);
}
void export_field(const Geo &g, double *dst, const void *src, int subset, int prec, int nrhs, hipStream_t s) {
  if (prec == QIRAL_F64) launch_export<S_F64>(g, dst, src, subset, nrhs, s);
  else if (prec == QIRAL_F32) launch_export<S_F32>(g, dst, src, subset, nrhs, s);
  else launch_export<S_F16S>(g, dst, src, subset, nrhs, s);
}
}  // namespace qiral

extern "C" qiral_status qiral_field_import(const qiral_lattice *lat, void *dst, const double *src_canon,
                                           qiral_subset subset, qiral_prec prec, int32_t nrhs, qiral_stream_t stream) {
  qiral_status st = check_field_args(lat, dst, src_canon, subset, prec, nrhs);
  if (st != QIRAL_OK) return st;
  import_field(lat->geo, src_canon, dst, subset, prec, nrhs, (hipStream_t)stream);
  QIRAL_HIP(hipGetLastError());
  return QIRAL_OK;
}

extern "C" qiral_status qiral_field_export(const qiral_lattice *lat, double *dst_canon, const void *src,
                                           qiral_subset subset, qiral_prec prec, int32_t nrhs, qiral_stream_t stream) {
  qiral_status st = check_field_args(lat, dst_canon, src, subset, prec, nrhs);
  if (st != QIRAL_OK) return st;
  export_field(lat->geo, dst_canon, src, subset, prec, nrhs, (hipStream_t)stream);
  QIRAL_HIP(hipGetLastError());
  return QIRAL_OK;
}

// ---------------------------------------------------------------------------
// operators
static qiral_status check_op_prec(const qiral_lattice *lat, int prec) {
  if (!valid_prec(prec)) return fail(QIRAL_ERR_INVALID_ARG, "bad precision");
  if (!links_for(lat, prec))
    return fail(QIRAL_ERR_INVALID_ARG, "the lattice holds no links of this precision (see lo_precs)");
  return QIRAL_OK;
}

extern "C" qiral_status qiral_dslash_eo(const qiral_lattice *lat, void *out, const void *in, int32_t out_parity,
                                        int32_t dagger, qiral_prec prec, int32_t nrhs, qiral_stream_t stream) {
  if (!lat) return fail(QIRAL_ERR_INVALID_ARG, "lat is NULL");
  if (!out || !in) return fail(QIRAL_ERR_INVALID_ARG, "field pointer is NULL");
  if (out == in) return fail(QIRAL_ERR_INVALID_ARG, "in and out must not alias");
  if (out_parity != 0 && out_parity != 1) return fail(QIRAL_ERR_INVALID_ARG, "out_parity must be 0 or 1");
  if (nrhs < 1) return fail(QIRAL_ERR_INVALID_ARG, "nrhs must be >= 1");
  qiral_status st = check_op_prec(lat, prec);
  if (st != QIRAL_OK) return st;
  QIRAL_HIP(launch_hop(lat, prec, dagger != 0, out_parity, 0, 1.0, in, out, nullptr, nrhs, (hipStream_t)stream));
  return QIRAL_OK;
}

extern "C" qiral_status qiral_apply_M(const qiral_lattice *lat, void *out, const void *in, void *tmp, qiral_op op,
                                      qiral_prec prec, int32_t nrhs, qiral_stream_t stream) {
  if (!lat) return fail(QIRAL_ERR_INVALID_ARG, "lat is NULL");
  if (!out || !in) return fail(QIRAL_ERR_INVALID_ARG, "field pointer is NULL");
  if (out == in) return fail(QIRAL_ERR_INVALID_ARG, "in and out must not alias");
  if (nrhs < 1) return fail(QIRAL_ERR_INVALID_ARG, "nrhs must be >= 1");
  if (op != QIRAL_OP_D && op != QIRAL_OP_DDAG && op != QIRAL_OP_SCHUR && op != QIRAL_OP_SCHUR_DAG)
    return fail(QIRAL_ERR_INVALID_ARG, "bad operator");
  if ((op == QIRAL_OP_SCHUR || op == QIRAL_OP_SCHUR_DAG) && (!tmp || tmp == in || tmp == out))
    return fail(QIRAL_ERR_INVALID_ARG, "the Schur operators need a separate tmp half-field");
  qiral_status st = check_op_prec(lat, prec);
  if (st != QIRAL_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const double k = lat->kappa;
  const int dag = (op == QIRAL_OP_DDAG || op == QIRAL_OP_SCHUR_DAG);
  if (op == QIRAL_OP_D || op == QIRAL_OP_DDAG) {
    // full fields: [rhs][even | odd]; handle one right-hand side per pair of launches
    const size_t hb = half_bytes(lat->geo, prec);
    // D = A - kappa H (D^dagger = A^dagger - kappa H^dagger), A = 1 + 2 i kappa mu gamma_5
    for (int r = 0; r < nrhs; ++r) {
      const char *ie = (const char *)in + 2 * hb * r, *io = ie + hb;
      char *oe = (char *)out + 2 * hb * r, *oo = oe + hb;
      const int ca = dag ? CHI_ADAG : CHI_A;
      QIRAL_HIP(launch_hop(lat, prec, dag, 0, 1, -k, io, oe, ie, 1, s, CHI_ONE, ca));
      QIRAL_HIP(launch_hop(lat, prec, dag, 1, 1, -k, ie, oo, io, 1, s, CHI_ONE, ca));
    }
  } else {
    // S = A - kappa^2 H_oe A^-1 H_eo (S^dagger: daggered hops and site factors)
    QIRAL_HIP(launch_hop(lat, prec, dag, 0, 0, 1.0, in, tmp, nullptr, nrhs, s, dag ? CHI_AINVDAG : CHI_AINV, CHI_ONE));
    QIRAL_HIP(launch_hop(lat, prec, dag, 1, 1, -k * k, tmp, out, in, nrhs, s, CHI_ONE, dag ? CHI_ADAG : CHI_A));
  }
  return QIRAL_OK;
}
