// Device side of the solvers: per-system state, the system table, solver
// scalar updates, and the grouped (table-driven) kernels.  One launch covers
// every system of a solve (the right-hand sides of one lattice, or the
// independent lattices of a batch); a work item is one wavefront of 64 sites of
// one system, and a system whose state does not match a kernel's mask skips it.
#pragma once
#include "qiral_dev.h"

namespace qiral {

enum : int { ST_RUN = 1, ST_UPDATE = 2, ST_DONE = 4, ST_ANY = 7 };

enum : int { SL_AP = 0, SL_R, SL_Z, SL_UPD, SL_B, SL_RES_E, SL_RES_O, SL_BI1, SL_BI2, SL_BI3, NSLOT };
constexpr int NV = 3;   // values per reduction

enum : int {
  FIN_NONE = 0, FIN_BNORM, FIN_NZ_INIT, FIN_ALPHA, FIN_NR, FIN_BETA, FIN_UPDATE,
  FIN_BI_ALPHA, FIN_BI_OMEGA, FIN_BI_RHO, FIN_CR_ZW, FIN_CR_BETA, FIN_CR_ALPHA
};

enum : int { SOLVER_CG = 0, SOLVER_BICG = 1, SOLVER_CR = 2 };

// Vectors of one system.  Odd half-fields unless noted.  "it" = iterate
// precision (FP64 for a plain solve, FP32 or F16S for a mixed one).
enum : int {
  F_X = 0,   // iterated solution: FP64 (plain) or FP32 (mixed, not yet folded into XH)
  F_R,       // residual (it)
  F_P,       // search direction (it)
  F_Z,       // S^dagger r (CG, CR) / s (BiCGStab) (it)
  F_AP,      // S p (CG) / v (BiCGStab) / q = S^dagger S p (CR) (it)
  F_TMP,     // even half-field temporary (it)
  F_XH,      // FP64 solution (mixed: accumulated; plain: unused)
  F_BH,      // FP64 Schur source b_hat
  F_T64,     // FP64 even temporary
  F_BE,      // FP64 even half of b
  F_BO,      // FP64 odd half of b
  F_XE,      // FP64 even half of x
  F_RT,      // BiCGStab shadow residual / CR v = S z (it)
  F_T,       // BiCGStab t = S s / CR u = S p (it)
  F_W,       // CR w = S^dagger S z (it)
  NF
};

struct SysState {
  double tol2, thr2, bnorm2, delta2;
  double nz, nr, nAp, alpha, beta, max_nr;
  double rho_re, rho_im, rho0_re, rho0_im, al_re, al_im, om_re, om_im, be_re, be_im;
  double res[NSLOT][NV];
  int status, iter, maxiter, nupdates, nonfinite, mixed, final_update, solver;
  int xpend;   // plain CGNR stopped after k_cg1: its last x += alpha p is still to be applied
  long long hops;
};

struct SysDesc {
  Geo g;
  double kappa;
  double tmu;         // 2 kappa mu: the twisted-mass site factor A = 1 + i tmu gamma_5
  const void *g64;    // FP64 links
  const void *glo;    // links in the iterate precision (== g64 for a plain solve)
  void *f[NF];
  SysState *st;
  double *part;       // [NSLOT][NV][4 nb] per-wave partial sums
  size_t npad;
};

__device__ __forceinline__ bool cfinite(double a) { return isfinite(a); }

// Solver scalar step run by the single lane that completed a reduction.
__device__ inline void finalize(SysState *st, int fin, int slot, const double t[NV]) {
  for (int i = 0; i < NV; ++i) st->res[slot][i] = t[i];
  switch (fin) {
    case FIN_BNORM:
      st->bnorm2 = t[0];
      st->thr2 = st->tol2 * t[0];
      if (!cfinite(t[0])) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    case FIN_NZ_INIT:
      st->nz = t[0];
      st->beta = 0.0;
      st->hops += 2;
      if (!cfinite(t[0])) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    case FIN_ALPHA: {
      st->nAp = t[0];
      double a = st->nz / t[0];
      st->alpha = a;
      st->hops += 2;
      if (!cfinite(a)) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    }
    case FIN_NR: {
      const double nr = t[0];
      st->nr = nr;
      st->iter += 1;
      if (!cfinite(nr)) { st->nonfinite = 1; st->status = ST_DONE; break; }
      const bool out_of_iters = st->iter >= st->maxiter;
      if (!st->mixed) {
        if (nr <= st->thr2 || out_of_iters) {
          st->status = ST_DONE;
          if (st->solver == SOLVER_CG) st->xpend = 1;
        }
      } else {
        if (nr > st->max_nr) st->max_nr = nr;
        if (nr <= st->thr2 || nr < st->delta2 * st->max_nr || out_of_iters) {
          st->status = ST_UPDATE;
          st->final_update = out_of_iters;
        }
      }
      break;
    }
    case FIN_BETA: {
      const double b = t[0] / st->nz;
      st->beta = b;
      st->nz = t[0];
      st->hops += 2;
      if (!cfinite(b)) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    }
    case FIN_UPDATE: {
      // t[0] = ||b_hat - S x||^2 in FP64; t[1], t[2] = (r~, r) for BiCGStab
      const double nr = t[0];
      st->nr = nr;
      st->max_nr = nr;
      st->nupdates += 1;
      st->xpend = 0;
      st->hops += 2;
      if (st->solver == SOLVER_BICG && st->iter > 0) {
        // keep the recurrence consistent with the replaced residual
        const double nre = t[1], nim = t[2];
        const double ore = st->rho0_re, oim = st->rho0_im;   // rho of the previous iteration
        const double d = ore * ore + oim * oim;
        const double qre = (nre * ore + nim * oim) / d, qim = (nim * ore - nre * oim) / d;   // rho_new / rho_old
        const double od = st->om_re * st->om_re + st->om_im * st->om_im;
        const double are = (st->al_re * st->om_re + st->al_im * st->om_im) / od;
        const double aim = (st->al_im * st->om_re - st->al_re * st->om_im) / od;        // alpha / omega
        st->be_re = qre * are - qim * aim;
        st->be_im = qre * aim + qim * are;
        st->rho_re = nre;
        st->rho_im = nim;
      }
      if (!cfinite(nr)) { st->nonfinite = 1; st->status = ST_DONE; }
      else if (nr <= st->thr2 || st->final_update || st->iter >= st->maxiter) st->status = ST_DONE;
      else st->status = ST_RUN;
      break;
    }
    case FIN_CR_ZW:   // (z | S^dagger S z) of the conjugate residual start; z, v, w took 3 S
      st->nz = t[0];
      st->beta = 0.0;
      st->hops += 6;
      if (!cfinite(t[0])) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    case FIN_CR_BETA: {   // beta = (z|Mz)_new / (z|Mz)_old
      const double b = t[0] / st->nz;
      st->beta = b;
      st->nz = t[0];
      st->hops += 4;
      if (!cfinite(b)) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    }
    case FIN_CR_ALPHA: {   // alpha = (z|Mz) / (q|q), q = M p
      st->nAp = t[0];
      const double a = st->nz / t[0];
      st->alpha = a;
      if (!cfinite(a)) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    }
    case FIN_BI_ALPHA: {
      // alpha = rho / (r~, v)
      const double dre = t[0], dim = t[1];
      const double d = dre * dre + dim * dim;
      st->al_re = (st->rho_re * dre + st->rho_im * dim) / d;
      st->al_im = (st->rho_im * dre - st->rho_re * dim) / d;
      st->hops += 2;
      if (!cfinite(st->al_re) || !cfinite(st->al_im)) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    }
    case FIN_BI_OMEGA: {
      // omega = (t, s) / (t, t)
      st->om_re = t[0] / t[2];
      st->om_im = t[1] / t[2];
      st->hops += 2;
      if (!cfinite(st->om_re) || !cfinite(st->om_im)) { st->nonfinite = 1; st->status = ST_DONE; }
      break;
    }
    case FIN_BI_RHO: {
      // rho_new = (r~, r), beta = (rho_new / rho) (alpha / omega), convergence test on (r, r)
      const double nre = t[0], nim = t[1], nr = t[2];
      const double ore = st->rho_re, oim = st->rho_im;
      const double d = ore * ore + oim * oim;
      const double qre = (nre * ore + nim * oim) / d, qim = (nim * ore - nre * oim) / d;
      const double od = st->om_re * st->om_re + st->om_im * st->om_im;
      const double are = (st->al_re * st->om_re + st->al_im * st->om_im) / od;
      const double aim = (st->al_im * st->om_re - st->al_re * st->om_im) / od;
      st->be_re = qre * are - qim * aim;
      st->be_im = qre * aim + qim * are;
      st->rho0_re = ore;
      st->rho0_im = oim;
      st->rho_re = nre;
      st->rho_im = nim;
      st->nr = nr;
      st->iter += 1;
      if (!cfinite(nr) || !cfinite(st->be_re)) { st->nonfinite = 1; st->status = ST_DONE; break; }
      const bool out_of_iters = st->iter >= st->maxiter;
      if (!st->mixed) {
        if (nr <= st->thr2 || out_of_iters) st->status = ST_DONE;
      } else {
        if (nr > st->max_nr) st->max_nr = nr;
        if (nr <= st->thr2 || nr < st->delta2 * st->max_nr || out_of_iters) {
          st->status = ST_UPDATE;
          st->final_update = out_of_iters;
        }
      }
      break;
    }
    default: break;
  }
}

// The fixed summation order of a reduction over the nb block partials of a
// row: RED_WG threads; thread tid adds the pairs tid + RED_WG j (j = 0..3) +
// 4 RED_WG k into four accumulators and combines them as (a0 + a1) + (a2 + a3),
// thread 0 also adds an odd last partial; each wave adds its threads with
// wave_sum, and the wave totals are added in wave order (k_reduce).
constexpr int RED_WG = 1024;

// Thread tid's share of N rows (`stride` doubles apart, 32-byte aligned).  The
// loads of a step (4 pairs of every row) are independent, so the compiler can
// issue them together: the partials were just written by other compute units,
// and each round trip costs a full memory latency.
template <int N>
__device__ __forceinline__ void red_part(const double *p, size_t stride, int nb, int tid, double s[N]) {
  const int npair = nb >> 1;
  double a[N][4];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) a[i][j] = 0.0;
  for (int k0 = tid; k0 < npair; k0 += 4 * RED_WG) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + j * RED_WG;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double2 x = k < npair ? ((const double2 *)(p + (size_t)i * stride))[k] : make_double2(0.0, 0.0);
        a[i][j] += x.x + x.y;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    s[i] = (a[i][0] + a[i][1]) + (a[i][2] + a[i][3]);
    if (tid == 0 && (nb & 1)) s[i] += p[(size_t)i * stride + nb - 1];
  }
}

// Row i of reduction slot `slot` of a system's partials.
__device__ __forceinline__ const double *part_row(const SysDesc &d, int slot, int i) {
  const size_t stride = (size_t)d.g.nb * 4;
  return d.part + ((size_t)slot * NV + i) * stride;
}

// Per-wave context of a table-driven kernel.  A work item is one 64-site block
// of `cnt` consecutive systems that share one lattice (cnt = 1 except for the
// grouped hop table); it is encoded as (sys0 << 24) | ((cnt - 1) << 22) | block.
// T waves share an item (sub = grp = 0..T-1 picks the wave's directions) and
// a work-group of 4 waves takes 4/T items.
// A work item as one wave sees it: T waves share an item (wave group grp of
// the item in work-group slot `slot`); each lane takes site s of the block.
struct Item {
  int sys, cnt, sb, sub, s, grp, slot;
  bool active;
};

__host__ __device__ inline uint32_t work_item(int sys0, int cnt, int sb) {
  return ((uint32_t)sys0 << 24) | ((uint32_t)(cnt - 1) << 22) | (uint32_t)sb;
}
constexpr int MAX_BLOCKS = 1 << 22;   // 64-site blocks per parity a work item can address

template <int T>
__device__ __forceinline__ Item fetch_item(const uint32_t *work, int nwork) {
  Item it;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
  const int idx = wg * (4 / T) + w / T;
  it.sub = it.grp = w % T;
  it.slot = w / T;
  if (idx >= nwork) { it.active = false; it.sys = 0; it.cnt = 1; it.sb = 0; it.s = 0; return it; }
  const uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane((int)work[idx]);
  it.sys = (int)(v >> 24);
  it.cnt = (int)((v >> 22) & 3u) + 1;
  it.sb = (int)(v & 0x3fffffu);
  it.s = it.sb * WAVE + lane_id();
  it.active = true;
  return it;
}

inline int grid_for(int nwork, int T) { return (nwork * T + 3) / 4; }

// Store a work item's partial sums: one per 64-site block (index sb), each of
// the NV values in its own row; the reduce kernel sums them in index order.
// Only wave group 0 of an item writes: after wave_combine it holds the item's
// full sums.
__device__ __forceinline__ void sys_partial(const SysDesc &d, int slot, const Item &it, double v[NV]) {
  if (it.grp != 0) return;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane_id() == 0) {
    const size_t stride = (size_t)d.g.nb * 4;   // row length (room kept for 4 per block)
    double *p = d.part + (size_t)slot * NV * stride;
#pragma unroll
    for (int i = 0; i < NV; ++i) p[i * stride + it.sb] = v[i];
  }
}

}  // namespace qiral
