// Autotuner of the hop's launch shape: waves per 64-site block (1 (F16S), 2 or
// 4), right-hand sides per lane (1..4) and, when that leaves several groups of
// right-hand sides, the traversal tile (8..64 blocks), timed with HIP events on
// the caller's stream for one
// lattice, precision and right-hand-side count.  Results live in the lattice
// handle and, if QIRAL_TUNE_CACHE names a file, in a JSON cache keyed by
// (architecture, precision, dims, nrhs) that later handles read.  The caller
// passes the two half-fields the timed hops read and write.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "qiral_int.h"

using namespace qiral;

namespace {

std::string cache_key(const qiral_lattice *lat, int prec, int nrhs) {
  std::ostringstream k;
  k << "gfx950/shape3/p" << prec << "/" << lat->dims[0] << "x" << lat->dims[1] << "x" << lat->dims[2] << "x" << lat->dims[3]
    << "/n" << nrhs;
  return k.str();
}

// The cache is a flat JSON object {"key": [t, nr, tile, us], ...}, one entry per line.
bool cache_lookup(const std::string &key, int &t, int &nr, int &tile) {
  const char *path = getenv("QIRAL_TUNE_CACHE");
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  const std::string pat = "\"" + key + "\": [";
  while (std::getline(f, line)) {
    const size_t i = line.find(pat);
    if (i == std::string::npos) continue;
    int a = 0, b = 0, c = 0;
    if (sscanf(line.c_str() + i + pat.size(), "%d, %d, %d", &a, &b, &c) == 3 && (a == 1 || a == 2 || a == 4) &&
        b >= 1 && b <= 4 && c >= 0) {
      t = a;
      nr = b;
      tile = c;
      return true;
    }
  }
  return false;
}

void cache_store(const std::string &key, int t, int nr, int tile, double us) {
  const char *path = getenv("QIRAL_TUNE_CACHE");
  if (!path) return;
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
      if (line.find('"') == std::string::npos) continue;
      if (line.find("\"" + key + "\"") != std::string::npos) continue;
      while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
      lines.push_back(line);
    }
  }
  char buf[256];
  snprintf(buf, sizeof buf, "  \"%s\": [%d, %d, %d, %.3f]", key.c_str(), t, nr, tile, us);
  lines.push_back(buf);
  std::ofstream o(path);
  o << "{\n";
  for (size_t i = 0; i < lines.size(); ++i) o << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
  o << "}\n";
}

}  // namespace

namespace qiral {
int tuned_nr(const qiral_lattice *lat, int prec, int nrhs) {
  const int idx = nrhs < 4 ? nrhs : 4;
  if (lat->tuned_nr[prec][idx]) return lat->tuned_nr[prec][idx];
  // untuned: share each link between two right-hand sides when there are several
  return nrhs >= 2 ? 2 : 1;
}
}  // namespace qiral

extern "C" qiral_status qiral_tune(qiral_lattice *lat, qiral_prec prec, int32_t nrhs, void *in, void *out,
                                   int32_t *best_t, int32_t *best_nr, double *best_us, qiral_stream_t stream) {
  if (!lat) { set_error("lat is NULL"); return QIRAL_ERR_INVALID_ARG; }
  if (!in || !out || in == out) { set_error("in and out must be two distinct half-fields"); return QIRAL_ERR_INVALID_ARG; }
  if (prec != QIRAL_F64 && prec != QIRAL_F32 && prec != QIRAL_F16S) { set_error("bad precision"); return QIRAL_ERR_INVALID_ARG; }
  if (nrhs < 1) { set_error("nrhs must be >= 1"); return QIRAL_ERR_INVALID_ARG; }
  if (!links_for(lat, prec)) { set_error("the lattice holds no links of this precision"); return QIRAL_ERR_INVALID_ARG; }
  const int idx = nrhs < 4 ? nrhs : 4;
  const std::string key = cache_key(lat, prec, nrhs);
  int t = 0, nr = 0, tile = 0;
  double us = 0.0;
  if (cache_lookup(key, t, nr, tile) && (t == 1 || t == 2 || t == 4) && nr >= 1 && nr <= hop_nr_max(prec, t)) {
    lat->tuned_t[prec][idx] = t;
    lat->tuned_nr[prec][idx] = nr;
    lat->tuned_tile[prec][idx] = tile;
  } else {
    hipStream_t s = (hipStream_t)stream;
    const size_t fb = half_bytes(lat->geo, prec) * (size_t)nrhs;
    // the values do not change the timing; zeros keep every scale finite
    QIRAL_HIP(hipMemsetAsync(in, 0, fb, s));
    hipEvent_t e0 = lat->time_ev[0], e1 = lat->time_ev[1];
    hipError_t e = hipSuccess;
    double best = 1e30;
    const int nrmax = 4;   // further limited per shape by hop_nr_max
    for (int tt : {1, 2, 4}) {
      for (int n = 1; n <= std::min(std::min(nrmax, hop_nr_max(prec, tt)), (int)nrhs) && e == hipSuccess; ++n) {
        // several groups of right-hand sides: also the traversal tile (blocks
        // each group sweeps before the next re-reads the tile's links)
        const bool groups = (nrhs + n - 1) / n > 1;
        for (int tl : {8, 16, 32, 64}) {
          if (!groups && tl != 8) break;
          HopCfg c;
          c.t = tt;
          c.nr = n;
          c.tile = groups ? tl : 0;
          const int reps = 10;
          for (int w = 0; w < 2; ++w) (void)launch_hop_cfg(c, lat, prec, 0, 0, 0, 1.0, in, out, nullptr, nrhs, s);
          (void)hipEventRecord(e0, s);
          for (int r = 0; r < reps; ++r) (void)launch_hop_cfg(c, lat, prec, 0, 0, 0, 1.0, in, out, nullptr, nrhs, s);
          (void)hipEventRecord(e1, s);
          e = hipEventSynchronize(e1);
          if (e != hipSuccess) break;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          const double u = 1e3 * ms / reps;
          if (u < best) { best = u; t = tt; nr = n; tile = c.tile; }
        }
      }
    }
    if (e != hipSuccess) return hip_fail(e, "tuning launch");
    lat->tuned_t[prec][idx] = t;
    lat->tuned_nr[prec][idx] = nr;
    lat->tuned_tile[prec][idx] = tile;
    us = best;
    cache_store(key, t, nr, tile, us);
  }
  if (best_t) *best_t = t;
  if (best_nr) *best_nr = nr;
  if (best_us) *best_us = us;
  return QIRAL_OK;
}
