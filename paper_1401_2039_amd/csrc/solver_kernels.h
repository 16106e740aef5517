// Launchers of the grouped solver kernels (solver_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qiral {

struct SysDesc;

struct Launch {
  const SysDesc *desc;       // device system table
  const uint32_t *work;      // device work table, one item per (system, 64-site block)
  int nwork;
  const uint32_t *work_hop;  // grouped table for the iterate-precision hop: items cover
  int nwork_hop;             //   up to NR systems of one lattice
  int nsys;
  int prec;                  // iterate precision (S_F64, S_F32, S_F16S)
  int T;                     // waves per site block of the iterate-precision hop (2 or 4)
  int NR;                    // systems per item of the grouped table
  int NT;                    // streaming accesses in the iterate-precision hop (see hop_stream)
  int NT64;                  // ... and in the FP64 hops of a mixed solve
  int chio = 0, chix = 0;    // twisted-mass site factors of the hop's epilogue (set by hop_sys)
  hipStream_t stream;
};

enum : int { A_ONE = 0, A_KAPPA = 1, A_MKAPPA2 = 2, A_MKAPPA = 3 };

// The hop over the system table (see k_hop_sys); chio / chix select the
// twisted-mass site factors applied to the output and to x (CHI_*).
void hop_sys(const Launch &l, int prec, bool dag, int epi, int fi, int fo, int fx, int par, int amode, int mask,
             int red, int slot, int fin, int chio = CHI_ONE, int chix = CHI_ONE);
void hop_sum(const Launch &l, bool haslo);
void hop_upd(const Launch &l, int prec, bool bicg);
void hop_res(const Launch &l, int par);
void bnorm(const Launch &l);
void cg1(const Launch &l, int prec);
void cg2(const Launch &l, int prec, bool xupd);
void cg_xfin(const Launch &l);
// Conjugate residual on S^dagger S (FP64): the x, r, z update with ||r||^2, and
// the p, q, u update with ||q||^2 (init: p = z, q = w, u = v).
void cr1(const Launch &l);
void cr2(const Launch &l, bool init);
void bi_p(const Launch &l, int prec);
void bi_s(const Launch &l, int prec);
void bi_xr(const Launch &l, int prec);
void copy_field(const Launch &l, int prec, int fsrc, int fdst, int mask, int chi = CHI_ONE);
void bi_init(const Launch &l, int nsys);

}  // namespace qiral
