// Grouped kernels of the even-odd solvers (CGNR of Fig. "CG" on the Schur
// system of the "schur" template, and BiCGStab), plus the FP64 reliable update
// and true-residual kernels.  Every kernel takes the system table and the work
// table; see solver_dev.h.
#include "qiral_int.h"
#include "solver_dev.h"
#include "solver_kernels.h"

namespace qiral {

__device__ __forceinline__ double coef(int amode, double k) {
  return amode == A_ONE ? 1.0 : amode == A_KAPPA ? k : amode == A_MKAPPA2 ? -k * k : -k;
}

template <int S> __device__ __forceinline__ const void *links_of(const SysDesc &d) {
  return S == S_F64 ? d.g64 : d.glo;
}

// out = C_o (a H in) (EPI 0) or out = C_o (C_x x + a H in) (EPI 1), parity
// `par` out, for the (up to NR) systems of a grouped work item (they share the
// lattice, so each link is loaded once for all of them).  C_o and C_x are the
// twisted-mass site factors chio and chix (CHI_*).
// red: 0 none; 1 ||out||^2; 2 (rt | out); 3 (out | x) and ||out||^2; 4 (z | out).
// T waves per item (see hop_wave); padded lanes compute on site 0 and store
// nothing.  Every wave reaches wave_combine's barrier.
template <int S, int L, bool DAG, int EPI, int T, int NR, bool NT>
__global__ __launch_bounds__(WG, HOP_MIN_WAVES(S, T, NR)) void k_hop_sys(const SysDesc *__restrict__ sdesc,
                                                                 const uint32_t *__restrict__ work, int nwork,
                                                                 int fin_id, int fout, int fx, int par, int amode,
                                                                 int mask, int red, int slot, int chio, int chix) {
  using R = typename SpinorIO<S>::R;
  using LDS = HopLds<T, NR, R>;
  __shared__ typename LDS::V lds[LDS::VECS];
  const Item it = fetch_item<T>(work, nwork);
  bool act[NR];
  bool any = false;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    act[r] = it.active && r < it.cnt && (sdesc[it.sys + r].st->status & mask);
    any = any || act[r];
  }
  const SysDesc &d0 = sdesc[it.sys];
  const bool site_ok = it.active && it.s < d0.g.vh;
  const size_t npad = d0.npad;
  FieldLd<S, NR> ld;
  ld.npad = npad;
#pragma unroll
  for (int r = 0; r < NR; ++r) ld.base[r] = sdesc[it.sys + min(r, it.cnt - 1)].f[fin_id];
  cpx<R> acc[NR][12];
  if (any) hop_wave<L, DAG, T, NT>(d0.g, links_of<S>(d0), ld, site_ok ? it.s : 0, par, it.grp, acc);
  else zero_acc<NR>(acc);
  wave_combine<T, NR>(acc, it.slot, it.grp, lds);
  if (!any) return;
  const R a = (R)coef(amode, d0.kappa);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (!act[r]) continue;
    const SysDesc &d = sdesc[it.sys + r];
    double v[NV] = {0.0, 0.0, 0.0};
    if (site_ok && it.grp == 0) {
      if (EPI == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[r][k] = cscale(a, acc[r][k]);
        apply_chi(acc[r], chio, d0.tmu);
      } else {
        cpx<R> xv[12];
        SpinorIO<S>::load(d.f[fx], it.s, npad, xv);
        cpx<R> ax[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) ax[k] = xv[k];
        apply_chi(ax, chix, d0.tmu);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[r][k] = cadd(ax[k], cscale(a, acc[r][k]));
        apply_chi(acc[r], chio, d0.tmu);
        if (red == 3) { dot12(acc[r], xv, v[0], v[1]); v[2] = norm12(acc[r]); }
      }
      SpinorIO<S>::template store_fast<NT>(d.f[fout], it.s, npad, acc[r]);
      if (red == 1) v[0] = norm12(acc[r]);
      if (red == 2 || red == 4) {
        cpx<R> rt[12];
        SpinorIO<S>::load(d.f[red == 2 ? F_RT : F_Z], it.s, npad, rt);
        dot12(rt, acc[r], v[0], v[1]);
      }
    }
    if (red) sys_partial(d, slot, it, v);
  }
}

// The FP64 hops of the reliable update and the true residual: 4 waves per
// item, directions summed in LDS.
constexpr int T64 = 4;
using Lds64 = HopLds<T64, 1, double>;

// T64 = A^-1 H_eo (XH + X): the hop of the current solution for the FP64 residual.
template <bool HASLO>
__global__ __launch_bounds__(WG, 2) void k_hop_sum(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                                int nwork) {
  __shared__ Lds64::V lds[Lds64::VECS];
  const Item it = fetch_item<T64>(work, nwork);
  const SysDesc &d = sdesc[it.sys];
  const bool on = it.active && (d.st->status & ST_UPDATE);
  // One work item per block, so `on` is the same in every wave of the block and
  // a block with no update pending (most iterations) leaves before the barrier.
  static_assert(WG / WAVE == T64, "k_hop_sum: one work item per block");
  if (!on) return;
  const bool site_ok = it.s < d.g.vh;
  cpx<double> acc[1][12];
  SumLd ld{d.f[F_XH], HASLO ? d.f[F_X] : nullptr, d.npad};
  hop_wave<L_F64R18, false, T64, false>(d.g, d.g64, ld, site_ok ? it.s : 0, 0, it.grp, acc);
  wave_combine<T64, 1>(acc, it.slot, it.grp, lds);
  if (site_ok && it.grp == 0) {
    apply_chi(acc[0], CHI_AINV, d.tmu);
    SpinorIO<S_F64>::store(d.f[F_T64], it.s, d.npad, acc[0]);
  }
}

// Reliable update on the odd sites: y = XH + X; XH = y; X = 0;
// r_hat = BH - (A y - kappa^2 H_oe T64) in FP64; R = r_hat rounded to the iterate
// precision; reduces ||r_hat||^2 (and (rt | r_hat) for BiCGStab).
template <int SO, bool HASLO, bool BICG>
__global__ __launch_bounds__(WG, 2) void k_hop_upd(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                                int nwork) {
  using RO = typename SpinorIO<SO>::R;
  __shared__ Lds64::V lds[Lds64::VECS];
  const Item it = fetch_item<T64>(work, nwork);
  const SysDesc &d = sdesc[it.sys];
  const bool on = it.active && (d.st->status & ST_UPDATE);
  // block-uniform, as in k_hop_sum
  static_assert(WG / WAVE == T64, "k_hop_upd: one work item per block");
  if (!on) return;
  const bool site_ok = it.s < d.g.vh;
  double v[NV] = {0.0, 0.0, 0.0};
  cpx<double> acc1[1][12];
  FieldLd<S_F64, 1> ld{{d.f[F_T64]}, d.npad};
  hop_wave<L_F64R18, false, T64, false>(d.g, d.g64, ld, site_ok ? it.s : 0, 1, it.grp, acc1);
  wave_combine<T64, 1>(acc1, it.slot, it.grp, lds);
  cpx<double> *acc = acc1[0];
  if (site_ok && it.grp == 0) {
    cpx<double> y[12], b[12];
    SumLd yl{d.f[F_XH], HASLO ? d.f[F_X] : nullptr, d.npad};
    yl(0, it.s, y);
    if (HASLO) {
      SpinorIO<S_F64>::store(d.f[F_XH], it.s, d.npad, y);
      cpx<float> z[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) z[k] = cmake(0.f, 0.f);
      SpinorIO<S_F32>::store(d.f[F_X], it.s, d.npad, z);
    }
    SpinorIO<S_F64>::load(d.f[F_BH], it.s, d.npad, b);
    apply_chi(y, CHI_A, d.tmu);
    const double k2 = d.kappa * d.kappa;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cadd(csub(b[k], y[k]), cscale(k2, acc[k]));
    v[0] = norm12(acc);
    cpx<RO> r[12];
    cvt12(acc, r);
    SpinorIO<SO>::store(d.f[F_R], it.s, d.npad, r);
    if (BICG && d.st->iter > 0) {
      cpx<RO> rt[12];
      SpinorIO<SO>::load(d.f[F_RT], it.s, d.npad, rt);
      cpx<double> rtd[12];
      cvt12(rt, rtd);
      dot12(rtd, acc, v[1], v[2]);
    }
  }
  sys_partial(d, SL_UPD, it, v);
}

// ||b - D x||^2 on the sites of parity p: B_p - A X_p + kappa H X_{1-p}.
__global__ __launch_bounds__(WG, 2) void k_hop_res(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                                int nwork, int par) {
  __shared__ Lds64::V lds[Lds64::VECS];
  const Item it = fetch_item<T64>(work, nwork);
  const SysDesc &d = sdesc[it.sys];
  const int fin_id = par ? F_XE : F_XH, fb = par ? F_BO : F_BE, fx = par ? F_XH : F_XE;
  const bool site_ok = it.active && it.s < d.g.vh;
  double v[NV] = {0.0, 0.0, 0.0};
  cpx<double> acc1[1][12];
  FieldLd<S_F64, 1> ld{{d.f[fin_id]}, d.npad};
  if (it.active) hop_wave<L_F64R18, false, T64, false>(d.g, d.g64, ld, site_ok ? it.s : 0, par, it.grp, acc1);
  else zero_acc<1>(acc1);
  wave_combine<T64, 1>(acc1, it.slot, it.grp, lds);
  if (!it.active) return;
  cpx<double> *acc = acc1[0];
  if (site_ok && it.grp == 0) {
    cpx<double> x[12], b[12];
    SpinorIO<S_F64>::load(d.f[fx], it.s, d.npad, x);
    SpinorIO<S_F64>::load(d.f[fb], it.s, d.npad, b);
    apply_chi(x, CHI_A, d.tmu);
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cadd(csub(b[k], x[k]), cscale(d.kappa, acc[k]));
    v[0] = norm12(acc);
  }
  sys_partial(d, par ? SL_RES_O : SL_RES_E, it, v);
}

// Sum a system's partials of one reduction slot and run the solver's scalar
// step (one work-group of RED_WG threads per system), in the fixed order of
// red_part: the result does not depend on scheduling.
__global__ __launch_bounds__(RED_WG) void k_reduce(const SysDesc *__restrict__ sdesc, int slot, int fin,
                                                   int mask) {
  static_assert(sizeof(SysState) % 8 == 0 && sizeof(SysState) / 8 <= RED_WG, "state copy");
  constexpr int NW8 = (int)(sizeof(SysState) / 8);
  const SysDesc &d = sdesc[blockIdx.x];
  // The reliable-update reduction has nothing to do in most iterations: look at
  // the state first there (the other reductions almost always run).
  if (fin == FIN_UPDATE && !(d.st->status & mask)) return;   // uniform over the work-group
  // The system's state is copied to LDS while the partials load, so the scalar
  // step below does not wait for another round trip to memory; the whole state
  // is written back afterwards (no other kernel runs meanwhile).
  __shared__ SysState sst;
  const int tid = threadIdx.x, w = tid >> 6;
  if (tid < NW8) ((unsigned long long *)&sst)[tid] = ((const unsigned long long *)d.st)[tid];
  __shared__ double red[NV][RED_WG / WAVE];
  double sp[NV];
  red_part<NV>(part_row(d, slot, 0), (size_t)d.g.nb * 4, d.g.nb, tid, sp);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double v = wave_sum(sp[i]);
    if (lane_id() == 0) red[i][w] = v;
  }
  __syncthreads();
  if (!(sst.status & mask)) return;   // uniform over the work-group
  if (tid == 0) {
    double t[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double v = 0.0;
      for (int j = 0; j < RED_WG / WAVE; ++j) v += red[i][j];
      t[i] = v;
    }
    finalize(&sst, fin, slot, t);
  }
  __syncthreads();
  if (tid < NW8) ((unsigned long long *)d.st)[tid] = ((const unsigned long long *)&sst)[tid];
}

// ||b||^2 over both parities.
__global__ __launch_bounds__(WG) void k_bnorm(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                              int nwork) {
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  double v[NV] = {0.0, 0.0, 0.0};
  if (it.s < d.g.vh) {
    cpx<double> a[12];
    SpinorIO<S_F64>::load(d.f[F_BE], it.s, d.npad, a);
    v[0] = norm12(a);
    SpinorIO<S_F64>::load(d.f[F_BO], it.s, d.npad, a);
    v[0] += norm12(a);
  }
  sys_partial(d, SL_B, it, v);
}

// CGNR: X += alpha P; R -= alpha AP; ||R||^2.  A plain (FP64) solve leaves X
// to k_cg2, which reads P anyway: X += alpha P there, before P changes, is the
// same arithmetic one pass over the vectors cheaper; k_cg_xfin applies the last
// one when the solve stops here.
template <int S, int XS>
__global__ __launch_bounds__(WG) void k_cg1(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                            int nwork) {
  using R = typename SpinorIO<S>::R;
  using RX = typename SpinorIO<XS>::R;
  constexpr bool xhere = S != S_F64;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_RUN)) return;
  double v[NV] = {0.0, 0.0, 0.0};
  if (it.s < d.g.vh) {
    const double al = d.st->alpha;
    cpx<R> r[12], ap[12];
    if (xhere) {
      cpx<R> p[12];
      cpx<RX> x[12];
      SpinorIO<S>::load(d.f[F_P], it.s, d.npad, p);
      SpinorIO<XS>::load(d.f[F_X], it.s, d.npad, x);
#pragma unroll
      for (int k = 0; k < 12; ++k) x[k] = cadd(x[k], cscale((RX)al, cmake((RX)p[k].re, (RX)p[k].im)));
      SpinorIO<XS>::store(d.f[F_X], it.s, d.npad, x);
    }
    SpinorIO<S>::load(d.f[F_R], it.s, d.npad, r);
    SpinorIO<S>::load(d.f[F_AP], it.s, d.npad, ap);
#pragma unroll
    for (int k = 0; k < 12; ++k) r[k] = csub(r[k], cscale((R)al, ap[k]));
    SpinorIO<S>::store(d.f[F_R], it.s, d.npad, r);
    v[0] = norm12(r);
  }
  sys_partial(d, SL_R, it, v);
}

// The x += alpha p that a plain CGNR solve stopped before (status done after
// k_cg1, flag set by the residual check).
__global__ __launch_bounds__(WG) void k_cg_xfin(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                                int nwork) {
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_DONE) || !d.st->xpend || it.s >= d.g.vh) return;
  const double al = d.st->alpha;
  cpx<double> p[12], x[12];
  SpinorIO<S_F64>::load(d.f[F_P], it.s, d.npad, p);
  SpinorIO<S_F64>::load(d.f[F_X], it.s, d.npad, x);
#pragma unroll
  for (int k = 0; k < 12; ++k) x[k] = cadd(x[k], cscale(al, cmake(p[k].re, p[k].im)));
  SpinorIO<S_F64>::store(d.f[F_X], it.s, d.npad, x);
}

// Conjugate residual on S^dagger S: X += alpha P; R -= alpha U (U = S P);
// Z -= alpha Q (Q = S^dagger S P); reduces ||R||^2 (the Schur residual).
template <int S>
__global__ __launch_bounds__(WG) void k_cr1(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                            int nwork) {
  using R = typename SpinorIO<S>::R;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_RUN)) return;
  double v[NV] = {0.0, 0.0, 0.0};
  if (it.s < d.g.vh) {
    const R al = (R)d.st->alpha;
    cpx<R> p[12], x[12], a[12], b[12];
    SpinorIO<S>::load(d.f[F_P], it.s, d.npad, p);
    SpinorIO<S>::load(d.f[F_X], it.s, d.npad, x);
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = cadd(x[k], cscale(al, p[k]));
    SpinorIO<S>::store(d.f[F_X], it.s, d.npad, x);
    SpinorIO<S>::load(d.f[F_R], it.s, d.npad, a);
    SpinorIO<S>::load(d.f[F_T], it.s, d.npad, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = csub(a[k], cscale(al, b[k]));
    SpinorIO<S>::store(d.f[F_R], it.s, d.npad, a);
    v[0] = norm12(a);
    SpinorIO<S>::load(d.f[F_Z], it.s, d.npad, a);
    SpinorIO<S>::load(d.f[F_AP], it.s, d.npad, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = csub(a[k], cscale(al, b[k]));
    SpinorIO<S>::store(d.f[F_Z], it.s, d.npad, a);
  }
  sys_partial(d, SL_R, it, v);
}

// Conjugate residual: P = Z + beta P; Q = W + beta Q; U = V + beta U (INIT:
// beta = 0, old values not read); reduces ||Q||^2.
template <int S, bool INIT>
__global__ __launch_bounds__(WG) void k_cr2(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                            int nwork) {
  using R = typename SpinorIO<S>::R;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_RUN)) return;
  double v[NV] = {0.0, 0.0, 0.0};
  if (it.s < d.g.vh) {
    const R be = (R)d.st->beta;
    const int src[3] = {F_Z, F_W, F_RT}, dst[3] = {F_P, F_AP, F_T};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      cpx<R> a[12];
      SpinorIO<S>::load(d.f[src[f]], it.s, d.npad, a);
      if (!INIT) {
        cpx<R> b[12];
        SpinorIO<S>::load(d.f[dst[f]], it.s, d.npad, b);
#pragma unroll
        for (int k = 0; k < 12; ++k) a[k] = cadd(a[k], cscale(be, b[k]));
      }
      SpinorIO<S>::store(d.f[dst[f]], it.s, d.npad, a);
      if (f == 1) v[0] = norm12(a);
    }
  }
  sys_partial(d, SL_AP, it, v);
}

// CGNR: P = Z + beta P; with XUPD (plain solves, in the iterations) first
// X += alpha P with the old P (the update k_cg1 left).
template <int S, bool XUPD>
__global__ __launch_bounds__(WG) void k_cg2(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                            int nwork) {
  using R = typename SpinorIO<S>::R;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_RUN)) return;
  if (it.s >= d.g.vh) return;
  const R be = (R)d.st->beta;
  cpx<R> p[12], z[12];
  SpinorIO<S>::load(d.f[F_P], it.s, d.npad, p);
  if (XUPD) {
    const double al = d.st->alpha;
    cpx<double> x[12];
    SpinorIO<S_F64>::load(d.f[F_X], it.s, d.npad, x);
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = cadd(x[k], cscale(al, cmake((double)p[k].re, (double)p[k].im)));
    SpinorIO<S_F64>::store(d.f[F_X], it.s, d.npad, x);
  }
  SpinorIO<S>::load(d.f[F_Z], it.s, d.npad, z);
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = cadd(z[k], cscale(be, p[k]));
  SpinorIO<S>::store(d.f[F_P], it.s, d.npad, p);
}

// BiCGStab: P = R + beta (P - omega V)    (V lives in F_AP)
template <int S>
__global__ __launch_bounds__(WG) void k_bi_p(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                             int nwork) {
  using R = typename SpinorIO<S>::R;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_RUN)) return;
  if (it.s >= d.g.vh) return;
  const cpx<R> be = cmake((R)d.st->be_re, (R)d.st->be_im), om = cmake((R)d.st->om_re, (R)d.st->om_im);
  cpx<R> p[12], r[12], vv[12];
  SpinorIO<S>::load(d.f[F_P], it.s, d.npad, p);
  SpinorIO<S>::load(d.f[F_R], it.s, d.npad, r);
  SpinorIO<S>::load(d.f[F_AP], it.s, d.npad, vv);
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = cadd(r[k], cmul(be, csub(p[k], cmul(om, vv[k]))));
  SpinorIO<S>::store(d.f[F_P], it.s, d.npad, p);
}

// BiCGStab: S = R - alpha V    (S lives in F_Z)
template <int S>
__global__ __launch_bounds__(WG) void k_bi_s(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                             int nwork) {
  using R = typename SpinorIO<S>::R;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_RUN)) return;
  if (it.s >= d.g.vh) return;
  const cpx<R> al = cmake((R)d.st->al_re, (R)d.st->al_im);
  cpx<R> r[12], vv[12];
  SpinorIO<S>::load(d.f[F_R], it.s, d.npad, r);
  SpinorIO<S>::load(d.f[F_AP], it.s, d.npad, vv);
#pragma unroll
  for (int k = 0; k < 12; ++k) r[k] = csub(r[k], cmul(al, vv[k]));
  SpinorIO<S>::store(d.f[F_Z], it.s, d.npad, r);
}

// BiCGStab: X += alpha P + omega S; R = S - omega T; reduces (rt | R) and ||R||^2
template <int S, int XS>
__global__ __launch_bounds__(WG) void k_bi_xr(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                              int nwork) {
  using R = typename SpinorIO<S>::R;
  using RX = typename SpinorIO<XS>::R;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & ST_RUN)) return;
  double v[NV] = {0.0, 0.0, 0.0};
  if (it.s < d.g.vh) {
    const cpx<RX> al = cmake((RX)d.st->al_re, (RX)d.st->al_im), om = cmake((RX)d.st->om_re, (RX)d.st->om_im);
    cpx<R> p[12], s[12], t[12], rt[12];
    cpx<RX> x[12];
    SpinorIO<S>::load(d.f[F_P], it.s, d.npad, p);
    SpinorIO<S>::load(d.f[F_Z], it.s, d.npad, s);
    SpinorIO<XS>::load(d.f[F_X], it.s, d.npad, x);
#pragma unroll
    for (int k = 0; k < 12; ++k)
      x[k] = cadd(x[k], cadd(cmul(al, cmake((RX)p[k].re, (RX)p[k].im)), cmul(om, cmake((RX)s[k].re, (RX)s[k].im))));
    SpinorIO<XS>::store(d.f[F_X], it.s, d.npad, x);
    SpinorIO<S>::load(d.f[F_T], it.s, d.npad, t);
    const cpx<R> omr = cmake((R)d.st->om_re, (R)d.st->om_im);
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = csub(s[k], cmul(omr, t[k]));
    SpinorIO<S>::store(d.f[F_R], it.s, d.npad, s);
    SpinorIO<S>::load(d.f[F_RT], it.s, d.npad, rt);
    dot12(rt, s, v[0], v[1]);
    v[2] = norm12(s);
  }
  sys_partial(d, SL_BI3, it, v);
}

// copy a half-field of the iterate precision: dst = src
template <int S>
__global__ __launch_bounds__(WG) void k_copy(const SysDesc *__restrict__ sdesc, const uint32_t *__restrict__ work,
                                             int nwork, int fsrc, int fdst, int mask, int chi) {
  using R = typename SpinorIO<S>::R;
  const Item it = fetch_item<1>(work, nwork);
  if (!it.active) return;
  const SysDesc &d = sdesc[it.sys];
  if (!(d.st->status & mask)) return;
  if (it.s >= d.g.vh) return;
  cpx<R> a[12];
  SpinorIO<S>::load(d.f[fsrc], it.s, d.npad, a);
  apply_chi(a, chi, d.tmu);
  SpinorIO<S>::store(d.f[fdst], it.s, d.npad, a);
}

// BiCGStab start: rho = (r~ | r) = ||r||^2 with r~ = r, alpha = omega = 1, beta = 0.
__global__ void k_bi_init(const SysDesc *__restrict__ sdesc, int nsys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsys) return;
  SysState *st = sdesc[i].st;
  if (!(st->status & ST_RUN)) return;
  st->rho_re = st->nr; st->rho_im = 0.0;
  st->rho0_re = st->nr; st->rho0_im = 0.0;
  st->al_re = 1.0; st->al_im = 0.0;
  st->om_re = 1.0; st->om_im = 0.0;
  st->be_re = 0.0; st->be_im = 0.0;
}

// ---------------------------------------------------------------------------
// launchers
static inline dim3 grid_of(int nwork, int T = 1) { return dim3(grid_for(nwork, T)); }

template <int S, int L, int T, int NR, bool NT>
static void hop_sys_tt(const Launch &l, bool dag, int epi, int fi, int fo, int fx, int par, int amode, int mask,
                       int red, int slot) {
  const dim3 g = grid_of(l.nwork, T), b(WG);
#define QARGS l.desc, l.work, l.nwork, fi, fo, fx, par, amode, mask, red, slot, l.chio, l.chix
  if (!dag) {
    if (epi == 0) hipLaunchKernelGGL((k_hop_sys<S, L, false, 0, T, NR, NT>), g, b, 0, l.stream, QARGS);
    else hipLaunchKernelGGL((k_hop_sys<S, L, false, 1, T, NR, NT>), g, b, 0, l.stream, QARGS);
  } else {
    if (epi == 0) hipLaunchKernelGGL((k_hop_sys<S, L, true, 0, T, NR, NT>), g, b, 0, l.stream, QARGS);
    else hipLaunchKernelGGL((k_hop_sys<S, L, true, 1, T, NR, NT>), g, b, 0, l.stream, QARGS);
  }
#undef QARGS
}

template <int S, int L, int T, int NR>
static void hop_sys_t(const Launch &l, bool dag, int epi, int fi, int fo, int fx, int par, int amode, int mask, int red,
                      int slot) {
  if (l.NT) hop_sys_tt<S, L, T, NR, true>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
  else hop_sys_tt<S, L, T, NR, false>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
}

template <int S, int L, int T>
static void hop_sys_n(const Launch &l, bool dag, int epi, int fi, int fo, int fx, int par, int amode, int mask, int red,
                      int slot) {
  // l.NR never exceeds hop_nr_max(S, T): the solver takes (T, NR) from hop_config.
  constexpr int NM = hop_nr_max(S, T);
  if constexpr (NM > 0) {
    if constexpr (NM >= 4) if (l.NR == 4) return hop_sys_t<S, L, T, 4>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
    if constexpr (NM >= 3) if (l.NR == 3) return hop_sys_t<S, L, T, 3>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
    if constexpr (NM >= 2) if (l.NR == 2) return hop_sys_t<S, L, T, 2>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
    hop_sys_t<S, L, T, 1>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
  }
}

template <int S, int L>
static void hop_sys_p(const Launch &l, bool dag, int epi, int fi, int fo, int fx, int par, int amode, int mask, int red,
                      int slot) {
  if constexpr (S == S_F64) hop_sys_n<S, L, 4>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
  else if (l.T == 4) hop_sys_n<S, L, 4>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
  else hop_sys_n<S, L, 2>(l, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
}

void reduce(const Launch &l, int slot, int fin, int mask) {
  hipLaunchKernelGGL(k_reduce, dim3(l.nsys), dim3(RED_WG), 0, l.stream, l.desc, slot, fin, mask);
}

void hop_sys(const Launch &l, int prec, bool dag, int epi, int fi, int fo, int fx, int par, int amode, int mask,
             int red, int slot, int fin, int chio, int chix) {
  // the iterate-precision hop walks the grouped table; an FP64 hop of a mixed
  // solve (source, reconstruction) walks the plain one
  const bool grouped = (prec == S_F64) == (l.prec == S_F64);
  Launch lp = l;
  lp.chio = chio;
  lp.chix = chix;
  if (grouped) { lp.work = l.work_hop; lp.nwork = l.nwork_hop; lp.T = l.T; lp.NR = l.NR; lp.NT = l.NT; }
  else { lp.T = 4; lp.NR = 1; lp.NT = l.NT64; }
  if (prec == S_F64) hop_sys_p<S_F64, L_F64R18>(lp, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
  else if (prec == S_F32) hop_sys_p<S_F32, L_F32R12>(lp, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
  else hop_sys_p<S_F16S, L_F16R12>(lp, dag, epi, fi, fo, fx, par, amode, mask, red, slot);
  if (red) reduce(l, slot, fin, mask);
}

void hop_sum(const Launch &l, bool haslo) {
  const dim3 g = grid_of(l.nwork, T64), b(WG);
  if (haslo) hipLaunchKernelGGL((k_hop_sum<true>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else hipLaunchKernelGGL((k_hop_sum<false>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
}

void hop_upd(const Launch &l, int prec, bool bicg) {
  const dim3 g = grid_of(l.nwork, T64), b(WG);
#define QU(SO, LO, BI) hipLaunchKernelGGL((k_hop_upd<SO, LO, BI>), g, b, 0, l.stream, l.desc, l.work, l.nwork)
  if (prec == S_F64) { if (bicg) QU(S_F64, false, true); else QU(S_F64, false, false); }
  else if (prec == S_F32) { if (bicg) QU(S_F32, true, true); else QU(S_F32, true, false); }
  else { if (bicg) QU(S_F16S, true, true); else QU(S_F16S, true, false); }
#undef QU
  reduce(l, SL_UPD, FIN_UPDATE, ST_UPDATE);
}

void hop_res(const Launch &l, int par) {
  const dim3 g = grid_of(l.nwork, T64), b(WG);
  hipLaunchKernelGGL(k_hop_res, g, b, 0, l.stream, l.desc, l.work, l.nwork, par);
  reduce(l, par ? SL_RES_O : SL_RES_E, FIN_NONE, ST_ANY);
}

void bnorm(const Launch &l) {
  hipLaunchKernelGGL(k_bnorm, grid_of(l.nwork), dim3(WG), 0, l.stream, l.desc, l.work, l.nwork);
  reduce(l, SL_B, FIN_BNORM, ST_ANY);
}

void cg1(const Launch &l, int prec) {
  const dim3 g = grid_of(l.nwork), b(WG);
  if (prec == S_F64) hipLaunchKernelGGL((k_cg1<S_F64, S_F64>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else if (prec == S_F32) hipLaunchKernelGGL((k_cg1<S_F32, S_F32>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else hipLaunchKernelGGL((k_cg1<S_F16S, S_F32>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  reduce(l, SL_R, FIN_NR, ST_RUN);
}

void cg2(const Launch &l, int prec, bool xupd) {
  const dim3 g = grid_of(l.nwork), b(WG);
  if (prec == S_F64) {
    if (xupd) hipLaunchKernelGGL((k_cg2<S_F64, true>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
    else hipLaunchKernelGGL((k_cg2<S_F64, false>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  } else if (prec == S_F32) hipLaunchKernelGGL((k_cg2<S_F32, false>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else hipLaunchKernelGGL((k_cg2<S_F16S, false>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
}

void cg_xfin(const Launch &l) {
  hipLaunchKernelGGL(k_cg_xfin, grid_of(l.nwork), dim3(WG), 0, l.stream, l.desc, l.work, l.nwork);
}

void cr1(const Launch &l) {
  hipLaunchKernelGGL(k_cr1<S_F64>, grid_of(l.nwork), dim3(WG), 0, l.stream, l.desc, l.work, l.nwork);
  reduce(l, SL_R, FIN_NR, ST_RUN);
}

void cr2(const Launch &l, bool init) {
  if (init) hipLaunchKernelGGL((k_cr2<S_F64, true>), grid_of(l.nwork), dim3(WG), 0, l.stream, l.desc, l.work, l.nwork);
  else hipLaunchKernelGGL((k_cr2<S_F64, false>), grid_of(l.nwork), dim3(WG), 0, l.stream, l.desc, l.work, l.nwork);
  reduce(l, SL_AP, FIN_CR_ALPHA, ST_RUN);
}

void bi_p(const Launch &l, int prec) {
  const dim3 g = grid_of(l.nwork), b(WG);
  if (prec == S_F64) hipLaunchKernelGGL(k_bi_p<S_F64>, g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else if (prec == S_F32) hipLaunchKernelGGL(k_bi_p<S_F32>, g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else hipLaunchKernelGGL(k_bi_p<S_F16S>, g, b, 0, l.stream, l.desc, l.work, l.nwork);
}

void bi_s(const Launch &l, int prec) {
  const dim3 g = grid_of(l.nwork), b(WG);
  if (prec == S_F64) hipLaunchKernelGGL(k_bi_s<S_F64>, g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else if (prec == S_F32) hipLaunchKernelGGL(k_bi_s<S_F32>, g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else hipLaunchKernelGGL(k_bi_s<S_F16S>, g, b, 0, l.stream, l.desc, l.work, l.nwork);
}

void bi_xr(const Launch &l, int prec) {
  const dim3 g = grid_of(l.nwork), b(WG);
  if (prec == S_F64) hipLaunchKernelGGL((k_bi_xr<S_F64, S_F64>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else if (prec == S_F32) hipLaunchKernelGGL((k_bi_xr<S_F32, S_F32>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  else hipLaunchKernelGGL((k_bi_xr<S_F16S, S_F32>), g, b, 0, l.stream, l.desc, l.work, l.nwork);
  reduce(l, SL_BI3, FIN_BI_RHO, ST_RUN);
}

void copy_field(const Launch &l, int prec, int fsrc, int fdst, int mask, int chi) {
  const dim3 g = grid_of(l.nwork), b(WG);
  if (prec == S_F64) hipLaunchKernelGGL(k_copy<S_F64>, g, b, 0, l.stream, l.desc, l.work, l.nwork, fsrc, fdst, mask, chi);
  else if (prec == S_F32) hipLaunchKernelGGL(k_copy<S_F32>, g, b, 0, l.stream, l.desc, l.work, l.nwork, fsrc, fdst, mask, chi);
  else hipLaunchKernelGGL(k_copy<S_F16S>, g, b, 0, l.stream, l.desc, l.work, l.nwork, fsrc, fdst, mask, chi);
}

void bi_init(const Launch &l, int nsys) {
  hipLaunchKernelGGL(k_bi_init, dim3((nsys + 63) / 64), dim3(64), 0, l.stream, l.desc, nsys);
}

}  // namespace qiral
