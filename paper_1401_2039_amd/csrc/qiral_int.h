// Host-side internals shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <string>
#include <vector>

#include "../../include/qiral.h"
#include "qiral_dev.h"

struct qiral_lattice {
  int32_t dims[4];
  qiral::Geo geo;
  double kappa, mu;
  // packed link stores, owned by the caller (see qiral_gauge_bytes)
  void *g64 = nullptr;   // FP64 links, all 18 reals (hops read rows 0-1)
  void *g32 = nullptr;   // FP32 reconstruct-12 links (optional)
  void *g16 = nullptr;   // FP16 reconstruct-12 links (optional)
  size_t gauge_bytes = 0;
  // made once by qiral_lattice_create, so that solves allocate nothing: the
  // pinned host buffer the solver copies its per-system states into (two
  // copies of QIRAL_MAX_SYSTEMS states), two events that mark those copies, and
  // two timing events for the autotuner
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  hipEvent_t time_ev[2] = {nullptr, nullptr};
  int device = 0;
  int tuned_nr[3][5] = {};   // autotuned right-hand sides per lane [prec][min(nrhs,4)], 0 = not tuned
  int tuned_t[3][5] = {};    // autotuned waves per site block, same index, 0 = not tuned
  int tuned_tile[3][5] = {}; // autotuned traversal tile of multi-group hops (blocks), 0 = default
};

namespace qiral {

void set_error(const std::string &msg);
qiral_status hip_fail(hipError_t e, const char *what);

#define QIRAL_HIP(call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return qiral::hip_fail(e_, #call); \
  } while (0)

inline size_t npad_of(const Geo &g) { return (size_t)g.nb * WAVE; }
size_t half_bytes(const Geo &g, int prec);
const void *links_for(const qiral_lattice *lat, int prec);

// Launch shape of a hop: t waves per 64-site block (1, 2 or 4) and nr
// right-hand sides per lane (1..4; see hop_nr_max).  hop_split picks t for `nwork` 64-site work items
// (enough waves to give every SIMD, 256 CUs x 4, a few); tuned_nr gives the
// autotuned nr of a lattice (a heuristic until tuned).  QIRAL_HOP_SPLIT and
// QIRAL_HOP_NR override.
struct HopCfg { int t = 4, nr = 1, tile = 0; };   // tile 0: hop_tile's default
// Largest number of right-hand sides per lane that a hop of storage precision
// S with T waves per site block keeps in registers; 0: the split is not built
// (FP64 needs T = 4 and spills at 3 RHS; one wave per block fits only the F16S
// hop with one RHS; FP32 on 2 waves per block spills at 3 RHS).
constexpr int hop_nr_max(int S, int T) {
  return S == 0 ? (T == 4 ? 2 : 0) : T == 1 ? (S == 2 ? 1 : 0) : (S == 1 && T == 2) ? 2 : 4;
}
int hop_split(int prec, long nwork);
// Streaming (non-temporal) link loads and output stores for hops whose working
// set exceeds half the last-level cache and whose links are read by one group
// of right-hand sides (several groups re-read each tile's links from the cache).
// QIRAL_HOP_NT=0|1 overrides.
bool hop_stream(const Geo &g, int prec, long nrhs, long ngroups);
// Planes per z-tile of the hop's block order (block_order), 0 for the plain
// order.  QIRAL_HOP_ORDER=0 forces the plain order, QIRAL_HOP_ORDER=n tiles of
// n planes where the lattice allows them.
int hop_zb(const Geo &g);
// Blocks per traversal tile of a multi-group hop (see k_hop); tuned > 0 is an
// autotuned size.
int hop_tile(const Geo &g, int ngroups, int tuned = 0);
int tuned_nr(const qiral_lattice *lat, int prec, int nrhs);
HopCfg hop_config(const qiral_lattice *lat, int prec, long nrhs);
hipError_t launch_hop_cfg(const HopCfg &c, const qiral_lattice *lat, int prec, int dagger, int out_parity, int epi,
                          double a, const void *in, void *out, const void *x, int nrhs, hipStream_t s,
                          int chio = 0, int chix = 0);

// Grid of ceil(nwaves / 4) work-groups (4 waves of 64 lanes each).
inline int wg_count(long nwaves) { return (int)((nwaves + 3) / 4); }

// Launchers implemented in api.hip (single lattice, nrhs consecutive fields).
// epi = 0: out = C_o (a * H in);  epi = 1: out = C_o (C_x x + a * H in), where
// C_o, C_x are the twisted-mass site factors selected by chio, chix (CHI_*;
// the identity for CHI_ONE or mu = 0).
hipError_t launch_hop(const qiral_lattice *lat, int prec, int dagger, int out_parity, int epi, double a,
                      const void *in, void *out, const void *x, int nrhs, hipStream_t s, int chio = 0, int chix = 0);

// The checks of qiral_solve's arguments that do not read the handle, the
// handle's links of the inner precision, and the solve itself in a workspace
// of ws_bytes >= qiral_solve_workspace_bytes (solver.hip).
qiral_status check_solve_args(const qiral_lattice *lat, const double *x, const double *b, int nrhs,
                              const qiral_solve_params *params, const qiral_solve_info *info);
qiral_status check_solve_links(const qiral_lattice *lat, const qiral_solve_params *params);
qiral_status solve_in(qiral_lattice *lat, double *x_canon, const double *b_canon, int32_t nrhs,
                      const qiral_solve_params *params, void *ws, size_t ws_bytes, qiral_solve_info *info,
                      hipStream_t stream);

// Bytes of a packed link store of the given storage precision (0: not built).
size_t link_store_bytes(const Geo &g, int prec);
// Pinned host bytes the solver's state polls need (two copies of every state).
size_t poll_bytes();

}  // namespace qiral
