// Host drivers of the even-odd solvers.
//
// The goal xx = Dirac^{-1} bb with the template chain "CGNR schur" (Sec. 2) is
// run as: b_hat = b_o + kappa H_oe b_e (the Schur source), CGNR (Fig. "CG") on
// S x_o = b_hat with S = 1 - kappa^2 H_oe H_eo, x_e = b_e + kappa H_eo x_o (the
// reconstruction, with v1 = P_e b), and a final FP64 true residual
// ||b - D x|| / ||b||.  The paper's loop condition (r|r) > eps uses
// eps = (tol ||b||)^2.  BiCGStab replaces CGNR on the same Schur system.
//
// Mixed precision: the Krylov vectors live in FP32 or F16S and the operator runs
// in FP32; the solution is kept as an FP64 part plus an FP32 part, and when the
// iterated residual has dropped by delta since the last update (or claims
// convergence) the FP32 part is folded in and the residual is recomputed in
// FP64 from the FP64 operator (reliable updates, Sleijpen & van der Vorst 1996;
// Clark et al., Comput. Phys. Commun. 181 (2010) 1517).  Convergence is only
// declared on such an FP64 residual.
//
// Several systems (right-hand sides of one lattice, or different lattices) run
// in the same launches: every kernel walks one work table over all of them and
// each system carries its own scalars and state on the device.  The host only
// enqueues iterations and reads the states every few iterations.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "qiral_int.h"
#include "solver_dev.h"
#include "solver_kernels.h"

namespace qiral {

void import_field(const Geo &g, const double *src, void *dst, int subset, int prec, int nrhs, hipStream_t s);
void export_field(const Geo &g, double *dst, const void *src, int subset, int prec, int nrhs, hipStream_t s);
qiral_status run_fgmres(qiral_lattice *lat, double *x, const double *b, const qiral_solve_params *prm, void *ws,
                        size_t ws_bytes, qiral_solve_info *info, hipStream_t s);
qiral_status run_fcg(qiral_lattice *lat, double *x, const double *b, const qiral_solve_params *prm, void *ws,
                     size_t ws_bytes, qiral_solve_info *info, hipStream_t s);
qiral_status run_bicgstab_prec(qiral_lattice *lat, double *x, const double *b, int nsys, const qiral_solve_params *prm,
                               void *ws, size_t ws_bytes, qiral_solve_info *info, hipStream_t s);
size_t flex_ws_bytes(const qiral_lattice *lat, const qiral_solve_params *prm, int nsys);
}  // namespace qiral

using namespace qiral;

namespace {

struct SysIn {
  qiral_lattice *lat;
  double *x;
  const double *b;
};

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

qiral_status fail(qiral_status s, const char *msg) {
  set_error(msg);
  return s;
}

// Per-system field sizes
struct SysSizes {
  size_t hb_it, hb_x, hb64;
  size_t bytes;
};

struct Layout {
  size_t off_desc, off_work, off_state, off_part, total;
  long nwork;
  std::vector<SysSizes> sz;      // per system: field sizes
  std::vector<size_t> off_sys;   // per system: start of its fields
  std::vector<size_t> part_off;  // per system: offset of its partials (doubles) inside the partial region
};

SysSizes sys_sizes(const Geo &g, int prec, int nit) {
  SysSizes z;
  z.hb_it = align_up(half_bytes(g, prec));
  z.hb64 = align_up(half_bytes(g, QIRAL_F64));
  const bool mixed = prec != QIRAL_F64;
  z.hb_x = mixed ? align_up(half_bytes(g, QIRAL_F32)) : 0;
  // nit iterate-precision half-fields: R P Z AP TMP (+ RT T for BiCGStab, + RT T W for CR)
  // F64: BH T64, [BE|BO] full, [XE|XH] full
  z.bytes = nit * z.hb_it + z.hb_x + 2 * z.hb64 + 2 * (2 * z.hb64);
  return z;
}

// The forms run by the flexible (host-driven, one right-hand side at a time)
// solvers: FGMRES, FCG, preconditioned or full-system BiCGStab, and CGNR on the
// full system (FCG with no preconditioner takes CGNR's iterates there).
bool is_flex(const qiral_solve_params *p) {
  if (p->solver == QIRAL_FGMRES_NN || p->solver == QIRAL_FCG_NN) return true;
  if (p->solver == QIRAL_BICGSTAB_EO) return p->precond || p->system == QIRAL_SYSTEM_FULL;
  return p->solver == QIRAL_CGNR_EO && p->system == QIRAL_SYSTEM_FULL;
}

// The parameters the flexible solver runs with (CGNR on D as FCG without a preconditioner).
qiral_solve_params flex_params(const qiral_solve_params *p) {
  qiral_solve_params q = *p;
  if (p->solver == QIRAL_CGNR_EO) {
    q.solver = QIRAL_FCG_NN;
    q.precond = nullptr;
    q.system = QIRAL_SYSTEM_FULL;
  }
  return q;
}

int n_iterate_fields(const qiral_solve_params *prm) {
  return prm->solver == QIRAL_BICGSTAB_EO ? 7 : prm->solver == QIRAL_CRNR_EO ? 8 : 5;
}

// Workspace layout of one solve over the systems `sys` (the same for the size
// query and the solve itself).
Layout solve_layout(const std::vector<const qiral_lattice *> &lats, const qiral_solve_params *prm) {
  const int nsys = (int)lats.size();
  const int nit = n_iterate_fields(prm);
  Layout lay;
  long nwork = 0;
  size_t nparts = 0;
  lay.part_off.resize(nsys);
  lay.sz.resize(nsys);
  for (int i = 0; i < nsys; ++i) {
    lay.sz[i] = sys_sizes(lats[i]->geo, prm->inner_prec, nit);
    nwork += lats[i]->geo.nb;
    lay.part_off[i] = nparts;
    nparts += (size_t)NSLOT * NV * 4 * lats[i]->geo.nb;
  }
  lay.nwork = nwork;
  size_t off = 0;
  lay.off_desc = off; off = align_up(off + sizeof(SysDesc) * nsys);
  lay.off_work = off; off = align_up(off + 2 * sizeof(uint32_t) * nwork);
  lay.off_state = off; off = align_up(off + sizeof(SysState) * nsys);
  lay.off_part = off; off = align_up(off + sizeof(double) * nparts);
  lay.off_sys.resize(nsys);
  for (int i = 0; i < nsys; ++i) { lay.off_sys[i] = off; off += lay.sz[i].bytes; }
  lay.total = off;
  return lay;
}

std::vector<const qiral_lattice *> lattices_of(const std::vector<SysIn> &sys) {
  std::vector<const qiral_lattice *> l(sys.size());
  for (size_t i = 0; i < sys.size(); ++i) l[i] = sys[i].lat;
  return l;
}

qiral_status run_solve(qiral_lattice *owner, const std::vector<SysIn> &sys, const qiral_solve_params *prm,
                       void *ws_base, size_t ws_bytes, qiral_solve_info *info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int nsys = (int)sys.size();
  const int prec = prm->inner_prec;
  const bool mixed = prec != QIRAL_F64;
  const bool bicg = prm->solver == QIRAL_BICGSTAB_EO;
  const bool cr = prm->solver == QIRAL_CRNR_EO;
  const int nit = n_iterate_fields(prm);

  // ---- layout
  const Layout lay = solve_layout(lattices_of(sys), prm);
  const std::vector<SysSizes> &sz = lay.sz;
  const long nwork = lay.nwork;
  if (nwork > (1l << 30)) return fail(QIRAL_ERR_UNSUPPORTED, "too many work items");
  if (!ws_base || ws_bytes < lay.total) return fail(QIRAL_ERR_WORKSPACE, "workspace smaller than qiral_solve_workspace_bytes");
  char *ws = (char *)ws_base;
  qiral_status st = QIRAL_OK;

  // ---- system table
  std::vector<SysDesc> desc(nsys);
  for (int i = 0; i < nsys; ++i) {
    const qiral_lattice *lat = sys[i].lat;
    SysDesc &d = desc[i];
    memset(&d, 0, sizeof(d));
    d.g = lat->geo;
    d.kappa = lat->kappa;
    d.tmu = 2.0 * lat->kappa * lat->mu;
    d.g64 = lat->g64;
    d.glo = links_for(lat, prec);
    d.npad = npad_of(lat->geo);
    d.st = (SysState *)(ws + lay.off_state) + i;
    d.part = (double *)(ws + lay.off_part) + lay.part_off[i];
    char *p = ws + lay.off_sys[i];
    const int it_fields[] = {F_R, F_P, F_Z, F_AP, F_TMP, F_RT, F_T, F_W};
    for (int k = 0; k < nit; ++k) { d.f[it_fields[k]] = p; p += sz[i].hb_it; }
    if (mixed) { d.f[F_X] = p; p += sz[i].hb_x; }
    d.f[F_BH] = p; p += sz[i].hb64;
    d.f[F_T64] = p; p += sz[i].hb64;
    d.f[F_BE] = p; d.f[F_BO] = p + half_bytes(lat->geo, QIRAL_F64); p += 2 * sz[i].hb64;
    d.f[F_XE] = p; d.f[F_XH] = p + half_bytes(lat->geo, QIRAL_F64); p += 2 * sz[i].hb64;
    if (!mixed) d.f[F_X] = d.f[F_XH];
  }
  // ---- work tables.  Plain: one item per (system, block); right-hand sides of
  // one lattice interleave per block (they share links).  Grouped (the
  // iterate-precision hop): up to NR systems of one lattice per item.
  bool same_lattice = true;
  for (int i = 1; i < nsys; ++i) same_lattice = same_lattice && sys[i].lat == sys[0].lat;
  HopCfg hc;
  if (same_lattice) hc = hop_config(sys[0].lat, prec, nsys);
  else { hc.nr = 1; hc.t = hop_split(prec, nwork); }
  if (hc.t == 1) hc.t = 2;   // the solver's hop kernel carries more state: one wave per block spills
  std::vector<uint32_t> work, work_hop;
  work.reserve(nwork);
  for (int i = 0; i < nsys; ++i)
    if (sys[i].lat->geo.nb > MAX_BLOCKS) return fail(QIRAL_ERR_UNSUPPORTED, "lattice too large for the work tables");
  if (same_lattice && nsys > 1) {
    // tile by tile (see hop_tile): each system, or group of systems, sweeps the
    // tile's blocks in turn
    const Geo &g = sys[0].lat->geo;
    const int nb = g.nb;
    const int tile = hop_tile(g, (nsys + hc.nr - 1) / hc.nr, hc.tile);
    const int zb = hop_zb(g);
    for (int b0 = 0; b0 < nb; b0 += tile) {
      const int b1 = std::min(nb, b0 + tile);
      for (int i = 0; i < nsys; ++i)
        for (int b = b0; b < b1; ++b) work.push_back(work_item(i, 1, block_order(g, b, zb)));
      for (int i = 0; i < nsys; i += hc.nr)
        for (int b = b0; b < b1; ++b) work_hop.push_back(work_item(i, std::min(hc.nr, nsys - i), block_order(g, b, zb)));
    }
  } else {
    // one item per (system, block), in each system's hop block order
    for (int i = 0; i < nsys; ++i) {
      const Geo &g = sys[i].lat->geo;
      const int zb = hop_zb(g);
      for (int b = 0; b < g.nb; ++b) work.push_back(work_item(i, 1, block_order(g, b, zb)));
    }
    work_hop = work;
  }
  std::vector<SysState> hst(nsys);
  for (int i = 0; i < nsys; ++i) {
    SysState &x = hst[i];
    memset(&x, 0, sizeof(x));
    x.tol2 = prm->tol * prm->tol;
    x.delta2 = prm->delta * prm->delta;
    x.maxiter = prm->maxiter;
    x.mixed = mixed;
    x.solver = bicg ? SOLVER_BICG : cr ? SOLVER_CR : SOLVER_CG;
    x.status = ST_UPDATE;
  }
  QIRAL_HIP(hipMemcpyAsync(ws + lay.off_desc, desc.data(), sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, s));
  QIRAL_HIP(hipMemcpyAsync(ws + lay.off_work, work.data(), sizeof(uint32_t) * nwork, hipMemcpyHostToDevice, s));
  QIRAL_HIP(hipMemcpyAsync(ws + lay.off_work + sizeof(uint32_t) * nwork, work_hop.data(),
                           sizeof(uint32_t) * work_hop.size(), hipMemcpyHostToDevice, s));
  QIRAL_HIP(hipMemcpyAsync(ws + lay.off_state, hst.data(), sizeof(SysState) * nsys, hipMemcpyHostToDevice, s));

  Launch L;
  L.desc = (const SysDesc *)(ws + lay.off_desc);
  L.work = (const uint32_t *)(ws + lay.off_work);
  L.nwork = (int)nwork;
  L.work_hop = (const uint32_t *)(ws + lay.off_work) + nwork;
  L.nwork_hop = (int)work_hop.size();
  L.nsys = nsys;
  L.prec = prec;
  L.T = hc.t;
  L.NR = hc.nr;
  L.NT = hop_stream(sys[0].lat->geo, prec, same_lattice ? nsys : 1, same_lattice ? (nsys + hc.nr - 1) / hc.nr : 1);
  L.NT64 = hop_stream(sys[0].lat->geo, QIRAL_F64, 1, 1);
  L.stream = s;

  // ---- inputs
  for (int i = 0; i < nsys; ++i) {
    const SysDesc &d = desc[i];
    const Geo &g = sys[i].lat->geo;
    import_field(g, sys[i].b, d.f[F_BE], QIRAL_FULL, QIRAL_F64, 1, s);
    if (prm->x0_is_guess) import_field(g, sys[i].x, d.f[F_XE], QIRAL_FULL, QIRAL_F64, 1, s);
    else QIRAL_HIP(hipMemsetAsync(d.f[F_XH], 0, half_bytes(g, QIRAL_F64), s));
    if (mixed) QIRAL_HIP(hipMemsetAsync(d.f[F_X], 0, half_bytes(g, QIRAL_F32), s));
    QIRAL_HIP(hipMemsetAsync(d.f[F_P], 0, half_bytes(g, prec), s));
    QIRAL_HIP(hipMemsetAsync(d.f[F_AP], 0, half_bytes(g, prec), s));
  }
  bnorm(L);
  // b_hat = b_o + kappa H_oe A^-1 b_e (A = 1 without twisted mass)
  bool twisted = false;
  for (int i = 0; i < nsys; ++i) twisted = twisted || sys[i].lat->mu != 0.0;
  if (twisted) {
    copy_field(L, S_F64, F_BE, F_T64, ST_ANY, CHI_AINV);
    hop_sys(L, S_F64, false, 1, F_T64, F_BH, F_BO, 1, A_KAPPA, ST_ANY, 0, 0, FIN_NONE);
  } else {
    hop_sys(L, S_F64, false, 1, F_BE, F_BH, F_BO, 1, A_KAPPA, ST_ANY, 0, 0, FIN_NONE);
  }
  QIRAL_HIP(hipGetLastError());

  // CR: v = S z (F_RT), w = S^dagger v (F_W) with (z | w) reduced into `fin`
  auto cr_apply = [&](int fin) {
    hop_sys(L, prec, false, 0, F_Z, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINV);
    hop_sys(L, prec, false, 1, F_TMP, F_RT, F_Z, 1, A_MKAPPA2, ST_RUN, 0, 0, FIN_NONE, CHI_ONE, CHI_A);
    hop_sys(L, prec, true, 0, F_RT, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINVDAG);
    hop_sys(L, prec, true, 1, F_TMP, F_W, F_RT, 1, A_MKAPPA2, ST_RUN, 4, SL_Z, fin, CHI_ONE, CHI_ADAG);
  };
  auto start_krylov = [&]() {
    // r = b_hat - S x (FP64), then the solver's own start
    hop_sum(L, mixed);
    hop_upd(L, prec, bicg);
    if (cr) {
      // z = S^dagger r, v = S z, w = S^dagger v, (z | w); then p = z, q = w, u = v, alpha
      hop_sys(L, prec, true, 0, F_R, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINVDAG);
      hop_sys(L, prec, true, 1, F_TMP, F_Z, F_R, 1, A_MKAPPA2, ST_RUN, 0, 0, FIN_NONE, CHI_ONE, CHI_ADAG);
      cr_apply(FIN_CR_ZW);
      cr2(L, true);
    } else if (!bicg) {
      hop_sys(L, prec, true, 0, F_R, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINVDAG);
      hop_sys(L, prec, true, 1, F_TMP, F_Z, F_R, 1, A_MKAPPA2, ST_RUN, 1, SL_Z, FIN_NZ_INIT, CHI_ONE, CHI_ADAG);
      cg2(L, prec, false);   // p = z (beta = 0)
    } else {
      copy_field(L, prec, F_R, F_RT, ST_RUN);
      bi_init(L, nsys);
    }
  };
  auto iteration = [&]() {
    if (cr) {
      cr1(L);
      cr_apply(FIN_CR_BETA);
      cr2(L, false);
    } else if (!bicg) {
      hop_sys(L, prec, false, 0, F_P, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINV);
      hop_sys(L, prec, false, 1, F_TMP, F_AP, F_P, 1, A_MKAPPA2, ST_RUN, 1, SL_AP, FIN_ALPHA, CHI_ONE, CHI_A);
      cg1(L, prec);
      if (mixed) { hop_sum(L, true); hop_upd(L, prec, false); }
      hop_sys(L, prec, true, 0, F_R, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINVDAG);
      hop_sys(L, prec, true, 1, F_TMP, F_Z, F_R, 1, A_MKAPPA2, ST_RUN, 1, SL_Z, FIN_BETA, CHI_ONE, CHI_ADAG);
      cg2(L, prec, !mixed);   // a plain solve's x += alpha p comes here
    } else {
      bi_p(L, prec);
      hop_sys(L, prec, false, 0, F_P, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINV);
      hop_sys(L, prec, false, 1, F_TMP, F_AP, F_P, 1, A_MKAPPA2, ST_RUN, 2, SL_BI1, FIN_BI_ALPHA, CHI_ONE, CHI_A);
      bi_s(L, prec);
      hop_sys(L, prec, false, 0, F_Z, F_TMP, 0, 0, A_ONE, ST_RUN, 0, 0, FIN_NONE, CHI_AINV);
      hop_sys(L, prec, false, 1, F_TMP, F_T, F_Z, 1, A_MKAPPA2, ST_RUN, 3, SL_BI2, FIN_BI_OMEGA, CHI_ONE, CHI_A);
      bi_xr(L, prec);
      if (mixed) { hop_sum(L, true); hop_upd(L, prec, true); }
    }
  };

  const int chunk = prm->check_every > 0 ? prm->check_every : 4;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  const bool use_graph = prm->use_graph && s != nullptr;
  auto free_graph = [&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  };
  auto read_states = [&]() -> qiral_status {
    QIRAL_HIP(hipMemcpyAsync(hst.data(), ws + lay.off_state, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, s));
    QIRAL_HIP(hipStreamSynchronize(s));
    return QIRAL_OK;
  };
  // Two pinned copies of the states (made with the lattice handle), so that the
  // host examines the states after one chunk of iterations while the next chunk
  // already runs.
  const size_t sbytes = sizeof(SysState) * nsys;
  if (owner->pinned_bytes < 2 * sbytes) return fail(QIRAL_ERR_INVALID_ARG, "state poll buffer too small");
  SysState *hbuf[2] = {(SysState *)owner->pinned, (SysState *)owner->pinned + nsys};
  hipEvent_t *ev = owner->poll_ev;
  auto enqueue_chunk = [&](int n) -> qiral_status {
    if (use_graph) {
      // one iteration captured once, replayed n times: the same launches as
      // without the graph, enqueued by one call per iteration
      if (!gexec) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        iteration();
        e = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess) { free_graph(); return hip_fail(e, "hipStreamEndCapture"); }
        e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { free_graph(); return hip_fail(e, "hipGraphInstantiate"); }
      }
      for (int k = 0; k < n; ++k) {
        hipError_t e = hipGraphLaunch(gexec, s);
        if (e != hipSuccess) { free_graph(); return hip_fail(e, "hipGraphLaunch"); }
      }
    } else {
      for (int k = 0; k < n; ++k) iteration();
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "solver iteration");
    }
    return QIRAL_OK;
  };
  auto post_copy = [&](int k) -> qiral_status {
    QIRAL_HIP(hipMemcpyAsync(hbuf[k], ws + lay.off_state, sbytes, hipMemcpyDeviceToHost, s));
    QIRAL_HIP(hipEventRecord(ev[k], s));
    return QIRAL_OK;
  };

  int restarts = 0;
  std::vector<double> true_rel(nsys, 0.0);
  qiral_status result = QIRAL_OK;
  while (true) {
    start_krylov();
    QIRAL_HIP(hipGetLastError());
    // Iterations until every system is done.  The next chunk is queued before
    // the states after the previous one are examined, so the GPU does not wait
    // for the host; systems that are done skip the extra chunk's work.
    int cur = 0;
    if ((st = enqueue_chunk(chunk)) != QIRAL_OK) return st;
    if ((st = post_copy(cur)) != QIRAL_OK) { free_graph(); return st; }
    long enqueued = chunk;
    // With the automatic chunk, the chunk after the queued one is
    // shortened when every running system is expected to stop within the
    // queued one: the CG-type residual norms fall about geometrically, so the
    // rate over the last checks predicts the iterations left.  This only
    // decides how many iterations the host queues ahead; the device decides
    // convergence, so the iterates do not change.
    const bool adaptive = prm->check_every <= 0 && (!bicg);
    std::vector<double> prev_nr(nsys, -1.0);
    std::vector<int> prev_it(nsys, -1);
    int next = chunk;
    while (true) {
      const int ahead = next;
      if ((st = enqueue_chunk(ahead)) != QIRAL_OK) return st;
      if ((st = post_copy(1 - cur)) != QIRAL_OK) { free_graph(); return st; }
      enqueued += ahead;
      hipError_t e = hipEventSynchronize(ev[cur]);
      if (e != hipSuccess) { free_graph(); return hip_fail(e, "hipEventSynchronize"); }
      bool all_done = true;
      for (int i = 0; i < nsys; ++i) all_done = all_done && (hbuf[cur][i].status & ST_DONE);
      if (all_done) break;
      if (enqueued > (long)prm->maxiter + 4l * chunk) break;   // device stops at maxiter; safety net
      if (adaptive) {
        int need = 1;
        for (int i = 0; i < nsys; ++i) {
          const SysState &x = hbuf[cur][i];
          if (x.status & ST_DONE) continue;
          double left = 1e30;   // predicted iterations left after the examined chunk
          if (prev_it[i] >= 0 && x.iter > prev_it[i] && x.nr > x.thr2 && x.nr < prev_nr[i] && x.thr2 > 0.0) {
            const double rate = std::log(x.nr / prev_nr[i]) / (double)(x.iter - prev_it[i]);   // < 0
            left = std::log(x.thr2 / x.nr) / rate;
          }
          prev_it[i] = x.iter;
          prev_nr[i] = x.nr;
          const double after = left - (double)ahead;   // still needed after the queued chunk
          const int n = after >= (double)chunk ? chunk : std::max(1, (int)std::ceil(after));
          need = std::max(need, n);
        }
        next = need;
      }
      cur = 1 - cur;
    }
    // a plain CGNR solve that stopped after k_cg1 still owes its last x += alpha p
    if (!mixed && !bicg && !cr) cg_xfin(L);
    // reconstruct x_e, export, FP64 true residual
    hop_sys(L, S_F64, false, 1, F_XH, F_XE, F_BE, 0, A_KAPPA, ST_ANY, 0, 0, FIN_NONE, CHI_AINV);   // x_e
    hop_res(L, 0);
    hop_res(L, 1);
    QIRAL_HIP(hipGetLastError());
    st = read_states();
    if (st != QIRAL_OK) { free_graph(); return st; }
    bool again = false;
    for (int i = 0; i < nsys; ++i) {
      const SysState &x = hst[i];
      const double r2 = x.res[SL_RES_E][0] + x.res[SL_RES_O][0];
      true_rel[i] = x.bnorm2 > 0 ? std::sqrt(r2 / x.bnorm2) : std::sqrt(r2);
      if (!x.nonfinite && true_rel[i] > prm->tol && x.iter < prm->maxiter) again = true;
    }
    if (!again || restarts >= 2) break;
    ++restarts;
    for (int i = 0; i < nsys; ++i) {
      hst[i].xpend = 0;   // k_cg_xfin has applied it
      if (!hst[i].nonfinite && true_rel[i] > prm->tol && hst[i].iter < prm->maxiter) {
        hst[i].status = ST_UPDATE;
        hst[i].final_update = 0;
      }
    }
    QIRAL_HIP(hipMemcpyAsync(ws + lay.off_state, hst.data(), sizeof(SysState) * nsys, hipMemcpyHostToDevice, s));
  }
  free_graph();
  for (int i = 0; i < nsys; ++i) {
    const SysDesc &d = desc[i];
    export_field(sys[i].lat->geo, sys[i].x, d.f[F_XE], QIRAL_FULL, QIRAL_F64, 1, s);
  }
  QIRAL_HIP(hipGetLastError());
  QIRAL_HIP(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < nsys; ++i) {
    const SysState &x = hst[i];
    if (info) {
      info[i].iterations = x.iter;
      info[i].reliable_updates = mixed ? x.nupdates - 1 - restarts : 0;
      if (info[i].reliable_updates < 0) info[i].reliable_updates = 0;
      info[i].true_rel_resid = true_rel[i];
      info[i].converged = x.nonfinite ? 0 : (true_rel[i] <= prm->tol);
      info[i].fell_back = 0;
      info[i].seconds = secs;
      info[i].hop_applications = x.hops + 4 + (long long)restarts * 2;
    }
    if (x.nonfinite) result = QIRAL_ERR_NONFINITE;
    else if (true_rel[i] > prm->tol && result == QIRAL_OK) result = QIRAL_ERR_NOT_CONVERGED;
  }
  if (result == QIRAL_ERR_NONFINITE) set_error("a NaN or Inf appeared in a reduction");
  else if (result == QIRAL_ERR_NOT_CONVERGED) set_error("tolerance not reached within maxiter");
  return result;
}

qiral_status check_params(const qiral_solve_params *p) {
  if (!p) return fail(QIRAL_ERR_INVALID_ARG, "params is NULL");
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(QIRAL_ERR_INVALID_ARG, "tol must be positive");
  if (p->maxiter < 1) return fail(QIRAL_ERR_INVALID_ARG, "maxiter must be >= 1");
  if (p->solver != QIRAL_CGNR_EO && p->solver != QIRAL_BICGSTAB_EO && p->solver != QIRAL_FGMRES_NN &&
      p->solver != QIRAL_CRNR_EO && p->solver != QIRAL_FCG_NN)
    return fail(QIRAL_ERR_INVALID_ARG, "bad solver");
  if (p->inner_prec != QIRAL_F64 && p->inner_prec != QIRAL_F32 && p->inner_prec != QIRAL_F16S)
    return fail(QIRAL_ERR_INVALID_ARG, "bad inner precision");
  if (p->inner_prec != QIRAL_F64 && !(p->delta > 0.0 && p->delta < 1.0))
    return fail(QIRAL_ERR_INVALID_ARG, "delta must lie in (0, 1) for a mixed-precision solve");
  if (p->check_every < 0) return fail(QIRAL_ERR_INVALID_ARG, "check_every must be >= 0");
  if (p->solver == QIRAL_CRNR_EO && p->inner_prec != QIRAL_F64)
    return fail(QIRAL_ERR_UNSUPPORTED, "the conjugate residual solver runs in FP64 (inner_prec F64)");
  if (p->system != QIRAL_SYSTEM_DEFAULT && p->system != QIRAL_SYSTEM_SCHUR && p->system != QIRAL_SYSTEM_FULL)
    return fail(QIRAL_ERR_INVALID_ARG, "bad system");
  if ((p->solver == QIRAL_CGNR_EO || p->solver == QIRAL_CRNR_EO) && p->precond)
    return fail(QIRAL_ERR_UNSUPPORTED, "CGNR and CRNR take no preconditioner (FCG is the preconditioned CG on the "
                                       "normal equations)");
  if (p->solver == QIRAL_CRNR_EO && p->system == QIRAL_SYSTEM_FULL)
    return fail(QIRAL_ERR_UNSUPPORTED, "the conjugate residual solver runs on the Schur system");
  if (is_flex(p) && p->inner_prec != QIRAL_F64)
    return fail(QIRAL_ERR_UNSUPPORTED, "FGMRES, FCG and the preconditioned or full-system forms run in FP64 "
                                       "(inner_prec F64)");
  if (p->solver == QIRAL_FGMRES_NN && p->restart > 64) return fail(QIRAL_ERR_INVALID_ARG, "restart must be <= 64");
  return QIRAL_OK;
}

}  // namespace

namespace qiral {
size_t poll_bytes() { return 2 * (size_t)QIRAL_MAX_SYSTEMS * sizeof(SysState); }

qiral_status run_solve_cg_fallback(qiral_lattice *lat, double *x, const double *b, const qiral_solve_params *prm,
                                   void *ws, size_t ws_bytes, qiral_solve_info *info, hipStream_t s) {
  std::vector<SysIn> sys{SysIn{lat, x, b}};
  return run_solve(lat, sys, prm, ws, ws_bytes, info, s);
}
}  // namespace qiral

namespace {

// Workspace of a solve over these lattices (one system each; the right-hand
// sides of qiral_solve are systems of one lattice).  FGMRES and FCG run one
// right-hand side at a time in the same workspace, the flexible BiCGStab all of
// them in lockstep, and each may continue with even-odd CGNR (the fallback) in it.
size_t ws_need(const std::vector<const qiral_lattice *> &lats, const qiral_solve_params *p) {
  if (is_flex(p)) {
    qiral_solve_params cg = *p;
    cg.solver = QIRAL_CGNR_EO;
    cg.system = QIRAL_SYSTEM_DEFAULT;
    cg.precond = nullptr;
    const qiral_solve_params f = flex_params(p);
    return std::max(flex_ws_bytes(lats[0], &f, (int)lats.size()), solve_layout({lats[0]}, &cg).total);
  }
  return solve_layout(lats, p).total;
}

// The workspace pointer itself (before the handle is read)
qiral_status check_ws_ptr(const void *ws) {
  if (!ws) return fail(QIRAL_ERR_WORKSPACE, "ws is NULL (size it with qiral_solve_workspace_bytes)");
  if (((uintptr_t)ws & 255) != 0) return fail(QIRAL_ERR_INVALID_ARG, "ws must be 256-byte aligned");
  return QIRAL_OK;
}

qiral_status check_ws(const void *ws, size_t ws_bytes, size_t need) {
  qiral_status st = check_ws_ptr(ws);
  if (st != QIRAL_OK) return st;
  if (ws_bytes < need) return fail(QIRAL_ERR_WORKSPACE, "ws_bytes is smaller than qiral_solve_workspace_bytes");
  return QIRAL_OK;
}

}  // namespace

namespace qiral {
// The checks of qiral_solve's arguments that do not read the handle.
qiral_status check_solve_args(const qiral_lattice *lat, const double *x, const double *b, int nrhs,
                              const qiral_solve_params *params, const qiral_solve_info *info) {
  if (!lat) return fail(QIRAL_ERR_INVALID_ARG, "lat is NULL");
  if (!x || !b) return fail(QIRAL_ERR_INVALID_ARG, "field pointer is NULL");
  if (nrhs < 1 || nrhs > QIRAL_MAX_SYSTEMS) return fail(QIRAL_ERR_INVALID_ARG, "nrhs must be in [1, 255]");
  if (!info) return fail(QIRAL_ERR_INVALID_ARG, "info is NULL");
  return check_params(params);
}

// The handle holds links of the solve's inner precision.
qiral_status check_solve_links(const qiral_lattice *lat, const qiral_solve_params *params) {
  if (!links_for(lat, params->inner_prec))
    return fail(QIRAL_ERR_INVALID_ARG, "the lattice holds no links of the inner precision (gauge_f32 / gauge_f16)");
  return QIRAL_OK;
}

// qiral_solve after its argument checks, in the workspace ws.
qiral_status solve_in(qiral_lattice *lat, double *x_canon, const double *b_canon, int32_t nrhs,
                      const qiral_solve_params *params, void *ws, size_t ws_bytes, qiral_solve_info *info,
                      hipStream_t stream) {
  const size_t stride = (size_t)lat->geo.vh * 2 * 24;
  if (is_flex(params)) {
    const qiral_solve_params fp = flex_params(params);
    if (fp.solver == QIRAL_BICGSTAB_EO)   // the right-hand sides in lockstep
      return run_bicgstab_prec(lat, x_canon, b_canon, nrhs, &fp, ws, ws_bytes, info, stream);
    // one right-hand side after the other
    auto run = fp.solver == QIRAL_FGMRES_NN ? run_fgmres : run_fcg;
    qiral_status worst = QIRAL_OK;
    for (int r = 0; r < nrhs; ++r) {
      qiral_status s = run(lat, x_canon + r * stride, b_canon + r * stride, &fp, ws, ws_bytes, info + r, stream);
      if (s != QIRAL_OK && s != QIRAL_ERR_NOT_CONVERGED) return s;
      if (s != QIRAL_OK) worst = s;
    }
    return worst;
  }
  std::vector<SysIn> sys(nrhs);
  for (int r = 0; r < nrhs; ++r) sys[r] = SysIn{lat, x_canon + r * stride, b_canon + r * stride};
  return run_solve(lat, sys, params, ws, ws_bytes, info, stream);
}
}  // namespace qiral

extern "C" size_t qiral_solve_workspace_bytes(const qiral_lattice *lat, const qiral_solve_params *params,
                                              int32_t nrhs) {
  if (!lat || nrhs < 1 || nrhs > QIRAL_MAX_SYSTEMS || check_params(params) != QIRAL_OK) return 0;
  return ws_need(std::vector<const qiral_lattice *>(nrhs, lat), params);
}

extern "C" size_t qiral_solve_batch_workspace_bytes(const qiral_lattice *const *lats, int32_t nsys,
                                                    const qiral_solve_params *params) {
  if (!lats || nsys < 1 || nsys > QIRAL_MAX_SYSTEMS || check_params(params) != QIRAL_OK) return 0;
  if (is_flex(params)) return 0;
  std::vector<const qiral_lattice *> l(nsys);
  for (int i = 0; i < nsys; ++i) {
    if (!lats[i]) return 0;
    l[i] = lats[i];
  }
  return ws_need(l, params);
}

extern "C" qiral_status qiral_solve(qiral_lattice *lat, double *x_canon, const double *b_canon, int32_t nrhs,
                                    const qiral_solve_params *params, void *ws, size_t ws_bytes,
                                    qiral_solve_info *info, qiral_stream_t stream) {
  qiral_status st = check_solve_args(lat, x_canon, b_canon, nrhs, params, info);
  if (st != QIRAL_OK) return st;
  if ((st = check_ws_ptr(ws)) != QIRAL_OK) return st;
  if ((st = check_solve_links(lat, params)) != QIRAL_OK) return st;
  const size_t need = qiral_solve_workspace_bytes(lat, params, nrhs);
  if ((st = check_ws(ws, ws_bytes, need)) != QIRAL_OK) return st;
  return solve_in(lat, x_canon, b_canon, nrhs, params, ws, ws_bytes, info, (hipStream_t)stream);
}

extern "C" qiral_status qiral_solve_batch(qiral_lattice *const *lats, double *const *x_canon,
                                          const double *const *b_canon, int32_t nsys,
                                          const qiral_solve_params *params, void *ws, size_t ws_bytes,
                                          qiral_solve_info *info, qiral_stream_t stream) {
  if (!lats || !x_canon || !b_canon) return fail(QIRAL_ERR_INVALID_ARG, "array pointer is NULL");
  if (nsys < 1 || nsys > QIRAL_MAX_SYSTEMS) return fail(QIRAL_ERR_INVALID_ARG, "nsys must be in [1, 255]");
  if (!info) return fail(QIRAL_ERR_INVALID_ARG, "info is NULL");
  qiral_status st = check_params(params);
  if (st != QIRAL_OK) return st;
  if (is_flex(params))
    return fail(QIRAL_ERR_UNSUPPORTED, "FGMRES, FCG and the preconditioned or full-system forms take one lattice "
                                       "(qiral_solve)");
  if ((st = check_ws_ptr(ws)) != QIRAL_OK) return st;
  std::vector<SysIn> sys(nsys);
  for (int i = 0; i < nsys; ++i) {
    if (!lats[i] || !x_canon[i] || !b_canon[i]) return fail(QIRAL_ERR_INVALID_ARG, "a system pointer is NULL");
    if (!links_for(lats[i], params->inner_prec))
      return fail(QIRAL_ERR_INVALID_ARG, "a lattice holds no links of the inner precision (gauge_f32 / gauge_f16)");
    sys[i] = SysIn{lats[i], x_canon[i], b_canon[i]};
  }
  if ((st = check_ws(ws, ws_bytes, qiral_solve_batch_workspace_bytes(lats, nsys, params))) != QIRAL_OK) return st;
  return run_solve(lats[0], sys, params, ws, ws_bytes, info, (hipStream_t)stream);
}
