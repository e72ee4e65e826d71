// Host side of the C ABI declared in include/qmc.h: validation, device
// allocation of system and walker state, and the launch sequences of the
// evaluation, move and Metropolis calls.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "lrdmc.h"

using namespace qmc;

namespace {
thread_local std::string g_err;

qmc_status fail(qmc_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

qmc_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return QMC_ERR_HIP;
}

#define HIP_TRY(expr, where)                          \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, count * sizeof(T) + 256);
}
}  // namespace

struct qmc_system {
  SysDev d{};
  int device = 0;
  long generation = 0;   // bumped by qmc_system_set_params
  std::vector<void*> allocs;
  ~qmc_system() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

// Event-pair timers for the kernels launched on behalf of one walker set.
struct Timers {
  bool on = false;
  uint32_t mask = 0;   // timers that record (bit k: timer k)
  double ms[QMC_TIMER_COUNT] = {};
  int64_t n[QMC_TIMER_COUNT] = {};
  struct Pair { hipEvent_t a, b; int id; };
  std::vector<Pair> pending;
  std::vector<Pair> spare;
  int open_id = -1;
  hipEvent_t open_a = nullptr;

  hipError_t fold() {   // wait for pending pairs and accumulate them
    for (auto& p : pending) {
      hipError_t e = hipEventSynchronize(p.b);
      if (e != hipSuccess) return e;
      float t = 0.f;
      e = hipEventElapsedTime(&t, p.a, p.b);
      if (e != hipSuccess) return e;
      ms[p.id] += t;
      n[p.id] += 1;
      spare.push_back(p);
    }
    pending.clear();
    return hipSuccess;
  }
  hipError_t begin(int id, hipStream_t st) {
    if (!on || !((mask >> id) & 1u)) return hipSuccess;
    if (pending.size() >= 8192) {
      hipError_t e = fold();
      if (e != hipSuccess) return e;
    }
    Pair p;
    if (!spare.empty()) { p = spare.back(); spare.pop_back(); }
    else {
      hipError_t e = hipEventCreate(&p.a);
      if (e == hipSuccess) e = hipEventCreate(&p.b);
      if (e != hipSuccess) return e;
    }
    p.id = id;
    open_id = id;
    open_a = p.a;
    pending.push_back(p);
    return hipEventRecord(p.a, st);
  }
  hipError_t end(hipStream_t st) {
    if (!on || open_id < 0) return hipSuccess;
    open_id = -1;
    return hipEventRecord(pending.back().b, st);
  }
  // A pair for a kernel that records it in its own dispatch (hipExtLaunchKernelGGL):
  // both null when this timer is off.
  hipError_t begin_ext(int id, hipEvent_t* a, hipEvent_t* b) {
    *a = *b = nullptr;
    if (!on || !((mask >> id) & 1u)) return hipSuccess;
    hipError_t e = begin_pair(id);
    if (e != hipSuccess) return e;
    *a = pending.back().a;
    *b = pending.back().b;
    return hipSuccess;
  }
  hipError_t begin_pair(int id) {
    if (pending.size() >= 8192) {
      hipError_t e = fold();
      if (e != hipSuccess) return e;
    }
    Pair p;
    if (!spare.empty()) { p = spare.back(); spare.pop_back(); }
    else {
      hipError_t e = hipEventCreate(&p.a);
      if (e == hipSuccess) e = hipEventCreate(&p.b);
      if (e != hipSuccess) return e;
    }
    p.id = id;
    pending.push_back(p);
    return hipSuccess;
  }
  void destroy() {
    (void)fold();
    for (auto& p : spare) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    spare.clear();
  }
};

struct qmc_walkers {
  qmc_system* sys = nullptr;
  WalkDev d{};
  std::vector<void*> allocs;
  int pending_e = -1;
  long attempts = 0;
  int since = 0;        // attempted moves since the last refresh
  int buf_spin = -1;    // spin of the moves in the delayed-update buffer (-1: empty)
  double* rd_scratch = nullptr;   // [Wk][2][kb][n] materialised-inverse work (read-out, drift check)
  double* res_x = nullptr;        // [Wk][n][n] refresh check: the inverse being replaced
  double* res_p = nullptr;        // [Wk][n][n] W times it
  double* res_v = nullptr;        // [Wk] max |W X - I| of the last checked refresh
  double drift_tol = 1e-6;        // status 3 when the checked residual exceeds this
  bool evaluated = false;
  bool P_up_valid = false, P_dn_valid = false;
  // (QMC_REFINED) parameter generation at which each P half's rows were last
  // built with their positions recorded (-1: never): a later build of that
  // half may take only the rows whose electron has moved
  long P_gen[2] = {-1, -1};
  // lattice-regularised DMC: the cofactor rows Yt hold for the positions of
  // the last evaluation until a move; hops computed for them (lr_ready)
  LrdmcDev lr{};
  LrdmcParams lr_p{};
  bool yt_valid = false, lr_ready = false;
  Timers tm;
  AdjWork aw{};
  bool aw_ready = false;
  long generation = -1;  // system generation of the last evaluation
  ~qmc_walkers() {
    tm.destroy();
    for (void* p : allocs) (void)hipFree(p);
  }
};

// Launch `expr` between the begin/end events of timer `id` (when timing is on).
// hipError_t-returning variant for helpers
#define TIMED_E(wk, id, st, expr)                                   \
  do {                                                              \
    hipError_t te_ = (wk)->tm.begin((id), (st));                    \
    if (te_ == hipSuccess) te_ = (expr);                            \
    if (te_ == hipSuccess) te_ = (wk)->tm.end((st));                \
    if (te_ != hipSuccess) return te_;                              \
  } while (0)

#define TIMED(wk, id, st, expr, where)                    \
  do {                                                    \
    HIP_TRY((wk)->tm.begin((id), (st)), "timer begin");   \
    HIP_TRY((expr), where);                               \
    HIP_TRY((wk)->tm.end((st)), "timer end");             \
  } while (0)

qmc_status qmc::set_error(qmc_status st, const char* msg) { return fail(st, msg); }

extern "C" int32_t qmc_abi_version(void) { return QMC_ABI_VERSION; }

extern "C" const char* qmc_last_error(void) { return g_err.c_str(); }

extern "C" qmc_status qmc_system_create(const qmc_system_desc* desc, qmc_system** out) {
  if (!desc || !out) return fail(QMC_ERR_ARG, "null argument");
  *out = nullptr;
  const qmc_system_desc& q = *desc;
  if (q.n_nuc <= 0 || q.n_nuc > kMaxNuc || !q.R || !q.Z) return fail(QMC_ERR_ARG, "bad nuclei");
  if (q.n_basis <= 0 || !q.center || !q.l || !q.m || !q.zeta || !q.lambda)
    return fail(QMC_ERR_ARG, "bad basis");
  if (q.n_up <= 0 || q.n_dn < 0) return fail(QMC_ERR_ARG, "bad electron counts");
  const bool pf = q.pairing == 1;
  if (q.pairing != 0 && !pf) return fail(QMC_ERR_ARG, "pairing must be 0 or 1");
  if (pf) {
    if (q.precision != QMC_FP64 && q.precision != QMC_REFINED)
      return fail(QMC_ERR_UNSUPPORTED, "the Pfaffian is built in FP64 and QMC_REFINED only");
    if (q.pf_k < 0) return fail(QMC_ERR_ARG, "pf_k must be >= 0");
    if ((q.n_up + q.n_dn + q.pf_k) % 2) return fail(QMC_ERR_ARG, "N + pf_k must be even");
    if (q.n_up + q.n_dn + q.pf_k > kLuRowMax) return fail(QMC_ERR_UNSUPPORTED, "Pfaffian of dimension > 96");
    if (!q.pf_uu || !q.pf_dd) return fail(QMC_ERR_ARG, "Pfaffian same-spin blocks missing");
    if (q.pf_k > 0 && (!q.unpaired || !q.pf_unpaired_dn)) return fail(QMC_ERR_ARG, "unpaired orbitals missing");
  } else {
    if (q.n_up < q.n_dn) return fail(QMC_ERR_UNSUPPORTED, "n_up < n_dn: label the majority spin up");
    if (q.n_up > q.n_dn && !q.unpaired) return fail(QMC_ERR_ARG, "n_up > n_dn needs the unpaired orbitals");
  }
  if (q.n_up > kBigMaxN) return fail(QMC_ERR_UNSUPPORTED, "n_up > 1024 is not built");
  if (q.precision < QMC_FP64 || q.precision > QMC_REFINED || q.precision == QMC_W_BF16 ||
      q.precision == QMC_W_FP8)
    return fail(QMC_ERR_UNSUPPORTED, "precision not built");
  if (q.refresh_every < 1) return fail(QMC_ERR_ARG, "refresh_every must be >= 1");
  if (q.j1_form < 0 || q.j1_form > 2 || (q.j1_form && !q.j1_b)) return fail(QMC_ERR_ARG, "bad j1");
  if (q.j2_form < 0 || q.j2_form > 2) return fail(QMC_ERR_ARG, "bad j2 form");
  if (q.j2_form == 1 && (q.n_j2 != 2 || !q.j2)) return fail(QMC_ERR_ARG, "j2 form 1 needs 2 params");
  if (q.j2_form == 2 && (q.n_j2 != 8 || !q.j2)) return fail(QMC_ERR_ARG, "j2 form 2 needs 8 params");
  const int Lb = q.n_basis;                       // basis functions (primitives when contracted)
  const int Lc = q.n_contracted;
  if (Lc < 0) return fail(QMC_ERR_ARG, "n_contracted must be >= 0");
  if (Lc > 0) {
    if (!q.con_ptr || !q.con_idx || !q.con_coef) return fail(QMC_ERR_ARG, "contraction arrays missing");
    if (Lb > kMaxLq) return fail(QMC_ERR_UNSUPPORTED, "contracted basis of more than 2048 primitives");
    if (q.con_ptr[0] != 0) return fail(QMC_ERR_ARG, "con_ptr[0] must be 0");
    if (q.con_ptr[Lc] <= 0) return fail(QMC_ERR_ARG, "contraction without coefficients");
    for (int c = 0; c < Lc; ++c)
      if (q.con_ptr[c + 1] < q.con_ptr[c]) return fail(QMC_ERR_ARG, "con_ptr must be non-decreasing");
    for (int k = 0; k < q.con_ptr[Lc]; ++k)
      if (q.con_idx[k] < 0 || q.con_idx[k] >= Lb) return fail(QMC_ERR_ARG, "con_idx out of range");
  }
  const int L = Lc > 0 ? Lc : Lb;                 // orbitals of the geminal
  std::vector<int> kind(Lb);
  for (int mu = 0; mu < Lb; ++mu) {
    if (q.radial && q.radial[mu] != 0 && q.radial[mu] != 1) return fail(QMC_ERR_ARG, "radial must be 0 or 1");
    if (q.center[mu] < 0 || q.center[mu] >= q.n_nuc) return fail(QMC_ERR_ARG, "basis center out of range");
    const int l = q.l[mu], m = q.m[mu];
    if (l < 0 || l > 2) return fail(QMC_ERR_UNSUPPORTED, "l > 2 not built");
    if (m < 0 || m >= 2 * l + 1) return fail(QMC_ERR_ARG, "component index out of range");
    kind[mu] = ((l == 0) ? 0 : (l == 1 ? 1 + m : 4 + m)) | ((q.radial && q.radial[mu] == 1) ? kSlaterBit : 0);
  }
  std::vector<int> cptr(q.n_nuc + 1, 0), cmu(Lb);
  for (int mu = 0; mu < Lb; ++mu) cptr[q.center[mu] + 1]++;
  for (int a = 0; a < q.n_nuc; ++a) cptr[a + 1] += cptr[a];
  {
    std::vector<int> fill(cptr.begin(), cptr.end() - 1);
    for (int mu = 0; mu < Lb; ++mu) cmu[fill[q.center[mu]]++] = mu;
  }
  auto* s = new qmc_system();
  SysDev& d = s->d;
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
  d.n_nuc = q.n_nuc; d.L = L; d.Lp = round_up(L, 32);
  d.nu = q.n_up; d.nd = q.n_dn; d.N = q.n_up + q.n_dn; d.nk = pf ? 0 : q.n_up - q.n_dn;
  d.pairing = pf ? 1 : 0; d.pk = pf ? q.pf_k : 0; d.npf = pf ? d.N + q.pf_k : 0;
  d.j1_form = q.j1_form; d.j2_form = q.j2_form;
  for (int k = 0; k < 8; ++k) d.j2[k] = (q.j2 && k < q.n_j2) ? q.j2[k] : 0.0;
  d.precision = q.precision; d.refresh_every = q.refresh_every;
  d.np = round_up(d.nu, 64);
  // Jastrow basis (onebody_J_inh, threebody_jastrow)
  const int LJ = q.n_jbasis;
  if (LJ < 0 || LJ > kMaxLJ) return fail(QMC_ERR_UNSUPPORTED, "Jastrow basis of more than 1024 functions");
  std::vector<double> jb4(4 * (size_t)LJ), M3((size_t)4 * LJ * LJ), jm(2 * (size_t)LJ);
  std::vector<int> jkind(LJ);
  if (LJ > 0) {
    if (!q.jb_center || !q.jb_l || !q.jb_m || !q.jb_zeta || !q.j1_inh || !q.j3)
      return fail(QMC_ERR_ARG, "Jastrow basis arrays missing");
    for (int k = 0; k < LJ; ++k) {
      const int c = q.jb_center[k], l = q.jb_l[k], m = q.jb_m[k], rad = q.jb_radial ? q.jb_radial[k] : 0;
      if (c < 0 || c >= q.n_nuc) return fail(QMC_ERR_ARG, "Jastrow basis center out of range");
      if (l < 0 || l > 2) return fail(QMC_ERR_UNSUPPORTED, "Jastrow basis l > 2 not built");
      if (m < 0 || m >= 2 * l + 1) return fail(QMC_ERR_ARG, "Jastrow basis component out of range");
      if (rad != 0 && rad != 1) return fail(QMC_ERR_ARG, "Jastrow basis radial must be 0 or 1");
      jkind[k] = ((l == 0) ? 0 : (l == 1 ? 1 + m : 4 + m)) | (rad ? kSlaterBit : 0);
      jb4[4 * k] = q.R[3 * c]; jb4[4 * k + 1] = q.R[3 * c + 1]; jb4[4 * k + 2] = q.R[3 * c + 2];
      jb4[4 * k + 3] = q.jb_zeta[k];
    }
    const double* Muu = q.j3;
    const double* Mdd = q.j3 + (size_t)LJ * LJ;
    const double* Mud = q.j3 + 2 * (size_t)LJ * LJ;
    double mx = 0.0;
    for (size_t k = 0; k < 2 * (size_t)LJ * LJ; ++k) mx = std::max(mx, std::fabs(q.j3[k]));
    for (int a = 0; a < LJ; ++a)
      for (int b = 0; b < LJ; ++b) {
        if (std::fabs(Muu[a * LJ + b] - Muu[b * LJ + a]) > 1e-12 * mx ||
            std::fabs(Mdd[a * LJ + b] - Mdd[b * LJ + a]) > 1e-12 * mx)
          return fail(QMC_ERR_ARG, "same-spin three/four-body matrices must be symmetric");
        const size_t n2 = 2 * (size_t)LJ;
        M3[a * n2 + b] = Muu[a * LJ + b];
        M3[(LJ + a) * n2 + LJ + b] = Mdd[a * LJ + b];
        M3[a * n2 + LJ + b] = Mud[a * LJ + b];
        M3[(LJ + b) * n2 + a] = Mud[a * LJ + b];
      }
    for (int k = 0; k < 2 * LJ; ++k) jm[k] = q.j1_inh[k];
  }
  const int Lp = d.Lp, A = q.n_nuc;
  std::vector<double> lam((size_t)Lp * Lp, 0.0), lamT((size_t)Lp * Lp, 0.0);
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      lam[(size_t)i * Lp + j] = q.lambda[(size_t)i * L + j];
      lamT[(size_t)j * Lp + i] = q.lambda[(size_t)i * L + j];
    }
  std::vector<double> j1b(A, 1.0);
  if (q.j1_form) for (int a = 0; a < A; ++a) j1b[a] = q.j1_b[a];
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dst, bytes + 256);
    if (e != hipSuccess) return e;
    s->allocs.push_back(*dst);
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  if (!e) e = up((void**)&d.R, q.R, sizeof(double) * 3 * A);
  if (!e) e = up((void**)&d.Z, q.Z, sizeof(double) * A);
  if (!e) e = up((void**)&d.j1_b, j1b.data(), sizeof(double) * A);
  if (!e) e = up((void**)&d.j2d, d.j2, sizeof(double) * 8);
  if (!e) e = up((void**)&d.center, q.center, sizeof(int) * Lb);
  if (!e) e = up((void**)&d.kind, kind.data(), sizeof(int) * Lb);
  if (!e) e = up((void**)&d.zeta, q.zeta, sizeof(double) * Lb);
  if (!e) e = up((void**)&d.lam, lam.data(), sizeof(double) * lam.size());
  if (!e) e = up((void**)&d.lamT, lamT.data(), sizeof(double) * lamT.size());
  if (!e) e = up((void**)&d.cptr, cptr.data(), sizeof(int) * cptr.size());
  if (!e) e = up((void**)&d.cmu, cmu.data(), sizeof(int) * cmu.size());
  d.LJ = LJ;
  if (!e && LJ > 0) {
    e = up((void**)&d.jbfn, jb4.data(), sizeof(double) * jb4.size());
    if (!e) e = up((void**)&d.jkind, jkind.data(), sizeof(int) * jkind.size());
    if (!e) e = up((void**)&d.jm, jm.data(), sizeof(double) * jm.size());
    if (!e) e = up((void**)&d.M3, M3.data(), sizeof(double) * M3.size());
    std::vector<int> jc(LJ), jptr(q.n_nuc + 1, 0), jmu(LJ);
    for (int k = 0; k < LJ; ++k) { jc[k] = q.jb_center[k]; jptr[jc[k] + 1]++; }
    for (int a = 0; a < q.n_nuc; ++a) jptr[a + 1] += jptr[a];
    std::vector<int> fill(jptr.begin(), jptr.end() - 1);
    for (int k = 0; k < LJ; ++k) jmu[fill[jc[k]]++] = k;
    if (!e) e = up((void**)&d.jcenter, jc.data(), sizeof(int) * LJ);
    if (!e) e = up((void**)&d.jcptr, jptr.data(), sizeof(int) * jptr.size());
    if (!e) e = up((void**)&d.jcmu, jmu.data(), sizeof(int) * LJ);
  }
  d.Lq = Lc > 0 ? Lb : 0;
  d.nnz_con = Lc > 0 ? q.con_ptr[Lc] : 0;
  if (!e && Lc > 0) {
    const int nnz = q.con_ptr[Lc];
    // the same matrix by primitive: pri_* (counting sort of the entries by primitive)
    std::vector<int> pptr(Lb + 1, 0), pidx(nnz);
    std::vector<double> pcoef(nnz);
    for (int k = 0; k < nnz; ++k) pptr[q.con_idx[k] + 1]++;
    for (int mu = 0; mu < Lb; ++mu) pptr[mu + 1] += pptr[mu];
    std::vector<int> fill(pptr.begin(), pptr.end() - 1);
    for (int c = 0; c < Lc; ++c)
      for (int k = q.con_ptr[c]; k < q.con_ptr[c + 1]; ++k) {
        const int at = fill[q.con_idx[k]]++;
        pidx[at] = c;
        pcoef[at] = q.con_coef[k];
      }
    e = up((void**)&d.con_ptr, q.con_ptr, sizeof(int) * (Lc + 1));
    if (!e) e = up((void**)&d.con_idx, q.con_idx, sizeof(int) * nnz);
    if (!e) e = up((void**)&d.con_coef, q.con_coef, sizeof(double) * nnz);
    if (!e) e = up((void**)&d.pri_ptr, pptr.data(), sizeof(int) * (Lb + 1));
    if (!e) e = up((void**)&d.pri_idx, pidx.data(), sizeof(int) * nnz);
    if (!e) e = up((void**)&d.pri_coef, pcoef.data(), sizeof(double) * nnz);
  }
  if (!e) {
    std::vector<double> bf(4 * (size_t)Lb);
    for (int mu = 0; mu < Lb; ++mu) {
      const int c = q.center[mu];
      bf[4 * mu] = q.R[3 * c]; bf[4 * mu + 1] = q.R[3 * c + 1]; bf[4 * mu + 2] = q.R[3 * c + 2];
      bf[4 * mu + 3] = q.zeta[mu];
    }
    e = up((void**)&d.bfn, bf.data(), sizeof(double) * bf.size());
  }
  if (!e && pf) {
    // K^{s s'} = (A^{s s'})^T, zero padded; unpaired rows per spin
    const double* Auu = q.pf_uu;
    const double* Add = q.pf_dd;
    double mx = 0.0;
    for (size_t k = 0; k < (size_t)L * L; ++k) mx = std::max(mx, std::max(std::fabs(Auu[k]), std::fabs(Add[k])));
    for (int a = 0; a < L && !e; ++a)
      for (int b = 0; b < L; ++b)
        if (std::fabs(Auu[(size_t)a * L + b] + Auu[(size_t)b * L + a]) > 1e-12 * mx ||
            std::fabs(Add[(size_t)a * L + b] + Add[(size_t)b * L + a]) > 1e-12 * mx) {
          delete s;
          return fail(QMC_ERR_ARG, "Pfaffian same-spin blocks must be skew-symmetric");
        }
    std::vector<double> kuu((size_t)Lp * Lp, 0.0), kud(kuu), kdu(kuu), kdd(kuu);
    for (int a = 0; a < L; ++a)
      for (int b = 0; b < L; ++b) {
        kuu[(size_t)b * Lp + a] = Auu[(size_t)a * L + b];
        kdd[(size_t)b * Lp + a] = Add[(size_t)a * L + b];
        kud[(size_t)b * Lp + a] = q.lambda[(size_t)a * L + b];
        kdu[(size_t)a * Lp + b] = -q.lambda[(size_t)a * L + b];
      }
    std::vector<double> kcu((size_t)Lp * 2 * Lp), kcd((size_t)Lp * 2 * Lp);
    for (int r = 0; r < Lp; ++r)
      for (int c = 0; c < Lp; ++c) {
        kcu[(size_t)r * 2 * Lp + c] = kuu[(size_t)r * Lp + c];
        kcu[(size_t)r * 2 * Lp + Lp + c] = kdu[(size_t)r * Lp + c];
        kcd[(size_t)r * 2 * Lp + c] = kud[(size_t)r * Lp + c];
        kcd[(size_t)r * 2 * Lp + Lp + c] = kdd[(size_t)r * Lp + c];
      }
    e = up((void**)&d.Kcat_u, kcu.data(), sizeof(double) * kcu.size());
    if (!e) e = up((void**)&d.Kcat_d, kcd.data(), sizeof(double) * kcd.size());
    if (!e) e = up((void**)&d.Kuu, kuu.data(), sizeof(double) * kuu.size());
    if (!e) e = up((void**)&d.Kud, kud.data(), sizeof(double) * kud.size());
    if (!e) e = up((void**)&d.Kdu, kdu.data(), sizeof(double) * kdu.size());
    if (!e) e = up((void**)&d.Kdd, kdd.data(), sizeof(double) * kdd.size());
    const int k = q.pf_k;
    std::vector<double> upf(2 * (size_t)(k > 0 ? k : 1) * Lp, 0.0);
    for (int l = 0; l < k; ++l)
      for (int mu = 0; mu < L; ++mu) {
        upf[(size_t)l * Lp + mu] = q.unpaired[(size_t)mu * k + l];
        upf[((size_t)k + l) * Lp + mu] = q.pf_unpaired_dn[(size_t)mu * k + l];
      }
    if (!e) e = up((void**)&d.Upf, upf.data(), sizeof(double) * upf.size());
  }
  if (!e && d.nk > 0) {
    // unpaired orbital l as a fixed row: Uph[l][mu] = unpaired[mu][l]
    std::vector<double> uph((size_t)d.nk * Lp, 0.0);
    for (int l = 0; l < d.nk; ++l)
      for (int mu = 0; mu < L; ++mu) uph[(size_t)l * Lp + mu] = q.unpaired[(size_t)mu * d.nk + l];
    e = up((void**)&d.Uph, uph.data(), sizeof(double) * uph.size());
    if (!e && d.f32()) {
      std::vector<float> u32(uph.begin(), uph.end());
      e = up((void**)&d.Uph32, u32.data(), sizeof(float) * u32.size());
    }
    if (!e) {
      if (!d.f32()) {
        d.UphS = d.Uph;
      } else if (q.precision == QMC_MIXED_BF16) {
        void* u16 = nullptr;
        e = hipMalloc(&u16, sizeof(uint16_t) * uph.size() + 256);
        if (!e) {
          s->allocs.push_back(u16);
          e = launch_downcast(d.Uph, u16, true, (long)uph.size(), nullptr);
          if (!e) e = hipStreamSynchronize(nullptr);
        }
        d.UphS = u16;
      } else {
        d.UphS = d.Uph32;
      }
    }
  }
  if (!e && d.f32()) {
    std::vector<float> l32(lam.begin(), lam.end()), lT32(lamT.begin(), lamT.end());
    e = up((void**)&d.lam32, l32.data(), sizeof(float) * l32.size());
    if (!e) e = up((void**)&d.lamT32, lT32.data(), sizeof(float) * lT32.size());
  }
  if (!e && d.bf16()) {
    // BF16 hi / lo pairs of Lambda^T and Lambda, [n][k] with k contiguous:
    // the operands of the BF16 matrix-core P rebuilds
    const size_t pl = (size_t)Lp * Lp;
    std::vector<uint16_t> b(4 * pl);
    for (size_t h = 0; h < 2; ++h) {
      const std::vector<double>& src = h == 0 ? lamT : lam;
      for (size_t k = 0; k < pl; ++k) {
        const bf16s hi(src[k]);
        const bf16s lo(src[k] - (double)hi);
        b[(2 * h) * pl + k] = hi.x;
        b[(2 * h + 1) * pl + k] = lo.x;
      }
    }
    e = up((void**)&d.lamB, b.data(), sizeof(uint16_t) * b.size());
  }
  if (!e) {
    const size_t mb = (size_t)((Lp + kLamTileK - 1) / kLamTileK) * ((Lp + kLamTileN - 1) / kLamTileN);
    std::vector<uint8_t> ones(mb, 1);
    e = up((void**)&d.lam_mask, ones.data(), mb);
    if (!e) e = up((void**)&d.lamT_mask, ones.data(), mb);
    if (!e) e = launch_lam_mask(d, nullptr);
    if (!e) e = hipStreamSynchronize(nullptr);
  }
  if (!e && (d.refined() || d.screened()) && !pf) {
    // int8 digits of Lambda for the error-free P products of the evaluation
    d.oz_s = kOzSlices;
    const size_t plane = (size_t)oz_plane_bytes(Lp, Lp);
    std::vector<int8_t> z8(2 * (size_t)d.oz_s * plane, 0);
    std::vector<int> z4(2 * (size_t)Lp, 0);
    e = up((void**)&d.oz_lam, z8.data(), z8.size());
    if (!e) e = up((void**)&d.oz_elam, z4.data(), sizeof(int) * z4.size());
    if (!e) e = launch_oz_lambda(d, nullptr);
    if (!e) e = hipStreamSynchronize(nullptr);
  }
  if (!e && d.pf_refined()) {
    // int8 digits of the four K^T for the error-free B rows of the evaluation
    d.oz_s = kOzSlices;
    const size_t plane = (size_t)oz_plane_bytes(Lp, Lp);
    std::vector<int8_t> z8(4 * (size_t)d.oz_s * plane, 0);
    std::vector<int> z4(4 * (size_t)Lp, 0);
    std::vector<double> zt((size_t)Lp * Lp, 0.0);
    e = up((void**)&d.oz_lam, z8.data(), z8.size());
    if (!e) e = up((void**)&d.oz_elam, z4.data(), sizeof(int) * z4.size());
    if (!e) e = up((void**)&d.oz_tmp, zt.data(), sizeof(double) * zt.size());
    if (!e) e = launch_oz_pf_K(d, nullptr);
    if (!e) e = hipStreamSynchronize(nullptr);
  }
  if (e != hipSuccess) {
    delete s;
    return e == hipErrorOutOfMemory ? fail(QMC_ERR_OOM, "device allocation failed") : hip_fail(e, "system_create");
  }
  *out = s;
  return QMC_OK;
}

extern "C" qmc_status qmc_system_destroy(qmc_system* sys) {
  if (!sys) return fail(QMC_ERR_ARG, "null system");
  (void)hipDeviceSynchronize();
  delete sys;
  return QMC_OK;
}

// Device layout of one walker set: every array of the evaluation and move
// state, and (flag QMC_WALKERS_ADJOINT) the reverse-pass workspace, carved out
// of one buffer at 256-byte boundaries (each array keeps 256 spare bytes past
// its end, so 16-byte vector loads of a padded row never leave it).  Run once
// with base == nullptr to size the buffer, then with the buffer to place the
// arrays.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  void take(T** p, size_t bytes) {
    off = (off + 255) / 256 * 256;
    if (base) *p = reinterpret_cast<T*>(base + off);
    off += bytes + 256;
  }
};

static void walker_layout(const SysDev& s, int n_walkers, bool adjoint, Carver& c, qmc_walkers& wk) {
  WalkDev& d = wk.d;
  d.Wk = n_walkers;
  const size_t Wk = n_walkers, N = s.N, Lp = s.Lp;
  const size_t nmax = s.nu > s.nd ? s.nu : s.nd;
  const size_t esz = s.bf16() ? sizeof(uint16_t) : (s.f32() ? sizeof(float) : sizeof(double));
  c.take(&d.r, sizeof(double) * Wk * N * 3);
  c.take(&d.phi, esz * Wk * N * Lp);
  c.take(&d.P, esz * Wk * N * Lp);
  const size_t nsq = s.pairing ? (size_t)s.npf * s.npf : (size_t)s.nu * s.nu;   // G~ or W
  c.take(&d.W, sizeof(double) * Wk * nsq);
  c.take(&d.A, sizeof(double) * Wk * nsq);
  c.take(&d.Yt, sizeof(double) * Wk * N * Lp);
  c.take(&d.D, sizeof(double) * Wk * N * 4);
  c.take(&d.logdet, sizeof(double) * Wk);
  c.take(&d.detsign, sizeof(double) * Wk);
  c.take(&d.singular, sizeof(int) * Wk);
  c.take(&d.logabs, sizeof(double) * Wk);
  c.take(&d.sign, sizeof(double) * Wk);
  c.take(&d.J, sizeof(double) * Wk);
  c.take(&d.psi_new, sizeof(double) * Wk * Lp);
  c.take(&d.w_new, sizeof(double) * Wk * (s.pairing ? std::max(nmax, (size_t)s.npf) : nmax));
  c.take(&d.rdet, sizeof(double) * Wk);
  c.take(&d.dJ, sizeof(double) * Wk);
  c.take(&d.r_new, sizeof(double) * Wk * 3);
  c.take(&d.ratio, sizeof(double) * Wk);
  c.take(&d.acc, sizeof(uint8_t) * Wk);
  const size_t S = (nmax + kPropRowsMin - 1) / kPropRowsMin;
  c.take(&d.rdet_part, sizeof(double) * Wk * S);
  c.take(&d.gdet_part, sizeof(double) * Wk * S * 3);
  c.take(&d.gJ_new, sizeof(double) * Wk * 3);
  c.take(&d.gpsi_new, sizeof(double) * Wk * 3 * Lp);
  c.take(&d.gJ, sizeof(double) * Wk * N * 4);
  c.take(&d.drift, sizeof(double) * Wk * N * 3);
  if (s.refined()) {
    c.take(&d.phi64, sizeof(double) * Wk * N * s.Lp);
    c.take(&d.P64, sizeof(double) * Wk * N * s.Lp);
  }
  if ((s.refined() || s.screened() || s.pf_refined()) && s.oz_s > 0) {
    c.take(&d.oz_phi, (size_t)oz_phi_bytes(s, (long)Wk));
    c.take(&d.oz_ephi, sizeof(int) * Wk * N);
  }
  if (s.screened()) {
    c.take(&d.PT, sizeof(double) * Wk * s.pt_ld() * s.Lp);
    c.take(&d.cmax, sizeof(double) * Wk * 2 * s.Lp);
    c.take(&d.muk, sizeof(int) * Wk * s.Lp);
    c.take(&d.psk, sizeof(double) * Wk * s.Lp);
    c.take(&d.nkeep, sizeof(int) * Wk);
    c.take(&d.oz_ephi_c, sizeof(int) * Wk * N);
  }
  if (!s.refined() && !s.pairing) {   // P builds of the moved rows only (FP64, FP32, QMC_REFINED)
    c.take(&d.rpos_P, sizeof(double) * Wk * N * 3);
    c.take(&d.dirty_idx, sizeof(int) * Wk * N);
    c.take(&d.dirty_cnt, sizeof(int) * 2);
    c.take(&d.dirty_blk, sizeof(int) * ((size_t)Wk * N / 256 + 2));
  }
  if (s.nu > kLuRowMax) {
    const size_t np = s.np;
    c.take(&d.T, sizeof(double) * Wk * np * np);
    c.take(&d.Tsave, sizeof(double) * Wk * kGjPanel * np);
    c.take(&d.rowk, sizeof(int) * Wk * np);
    c.take(&d.prow, sizeof(int) * Wk * np);
    c.take(&d.pivv, sizeof(double) * Wk * np);
  }
  d.kb = wb_cap(s);
  {
    const size_t n = s.nu, kb = d.kb;
    c.take(&d.wm, sizeof(int) * Wk);
    c.take(&d.wv, sizeof(double) * Wk * kb * n);
    c.take(&d.wd, sizeof(double) * Wk * kb * n);
    c.take(&d.wS, sizeof(double) * Wk * kb * kb);
    c.take(&d.cvec, sizeof(double) * Wk * n);
    c.take(&d.v0, sizeof(double) * Wk * n);
    c.take(&d.tz, sizeof(double) * Wk * 2 * kb);
    c.take(&wk.rd_scratch, sizeof(double) * Wk * 2 * kb * n);
    // refresh residual check: the inverse being replaced and W times it
    c.take(&wk.res_x, sizeof(double) * Wk * nsq);
    c.take(&wk.res_p, sizeof(double) * Wk * nsq);
    c.take(&wk.res_v, sizeof(double) * Wk);
  }
  if (s.LJ > 0) {
    const size_t LJ = s.LJ;
    c.take(&d.chi, sizeof(double) * Wk * N * LJ);
    c.take(&d.hv, sizeof(double) * Wk * N * LJ);
    c.take(&d.G3, sizeof(double) * Wk * 2 * LJ);
    c.take(&d.chi_new, sizeof(double) * Wk * LJ);
    c.take(&d.j3e, sizeof(double) * Wk * N * 5);
  }
  if (s.Lq > 0) c.take(&d.qbuf, sizeof(double) * Wk * 4 * s.Lq);
  if (s.pairing) {
    c.take(&d.Bd, sizeof(double) * Wk * N * Lp);
    c.take(&d.pfB, sizeof(double) * Wk * 2 * Lp);
    c.take(&d.pfT, sizeof(double) * Wk * N * Lp);
  }
  c.take(&wk.lr.ratio, sizeof(double) * Wk * N * kHops);
  c.take(&wk.lr.ah, sizeof(double) * Wk * N);
  c.take(&wk.lr.terms, sizeof(double) * Wk * kLrTerms);
  c.take(&wk.lr.ekin, sizeof(double) * Wk);
  c.take(&wk.lr.eloc, sizeof(double) * Wk);
  if (!adjoint) return;
  // reverse pass (qmc_forces)
  const size_t n = s.nu, L = s.L, A = s.n_nuc;
  const size_t nj = A + (s.j2_form == 1 ? 2 : (s.j2_form == 2 ? 8 : 0));
  AdjWork& a = wk.aw;
  a.chunk_walkers = (int)((Wk + 63) / 64);
  a.chunks = (int)((Wk + a.chunk_walkers - 1) / a.chunk_walkers);
  const size_t f8 = sizeof(double);
  c.take(&a.SU, f8 * Wk * 2 * n * Lp);
  c.take(&a.SD, f8 * Wk * 2 * n * Lp);
  c.take(&a.VQ, f8 * Wk * n * n);
  c.take(&a.T1, f8 * Wk * n * n);
  c.take(&a.M, f8 * Wk * n * n);
  c.take(&a.GG, f8 * Wk * 2 * n * n);
  c.take(&a.GGt, f8 * Wk * 2 * n * n);
  c.take(&a.XZ, f8 * Wk * 2 * n * Lp);
  c.take(&a.XD, f8 * Wk * n * Lp);
  c.take(&a.PB, f8 * Wk * N * Lp);
  const size_t Lb = s.Lq ? (size_t)s.Lq : L;   // basis functions (primitives of a contracted basis)
  c.take(&a.tmu, f8 * Wk * Lb * 3);
  c.take(&a.Rbar, f8 * Wk * A * 3);
  c.take(&a.zbar, f8 * Wk * Lb);
  if (s.pairing) {
    const size_t np = s.npf;
    c.take(&a.pfT, f8 * Wk * np * np);
    c.take(&a.pfZ1, f8 * Wk * np * np);
    c.take(&a.pfZ, f8 * Wk * np * np);
    c.take(&a.pfBb, f8 * Wk * N * 2 * Lp);
    c.take(&a.pfY, f8 * Wk * N * Lp);
    const size_t per = 3 * L * L + 2 * L * (size_t)s.pk;
    c.take(&a.pfD, f8 * Wk * per);
    c.take(&a.pfS, f8 * per);
  }
  if (s.Lq) {
    const size_t lqp = (s.Lq + 31) / 32 * 32;
    c.take(&a.dcw, f8 * Wk * (size_t)s.nnz_con);
    c.take(&a.PBq, f8 * Wk * N * lqp);
    c.take(&a.Ytq, f8 * Wk * N * lqp);
  }
  if (s.LJ) {
    const size_t LJ = s.LJ, LJp = (LJ + 31) / 32 * 32;
    a.LJp = (int)LJp;
    c.take(&a.ju, f8 * Wk * N * LJp);
    c.take(&a.jgv, f8 * Wk * N * LJp);
    c.take(&a.jac, f8 * Wk * N * LJp);
    c.take(&a.jpb, f8 * Wk * N * LJp);
    c.take(&a.jhu, f8 * Wk * N * LJp);
    c.take(&a.jX, f8 * Wk * 4 * LJ);
    c.take(&a.jH, f8 * Wk * 2 * LJ);
    c.take(&a.jdm, f8 * Wk * 2 * LJ);
    c.take(&a.jC, f8 * Wk * 2 * LJ * LJ);
    c.take(&a.jdM, f8 * Wk * 3 * LJ * LJ);
    c.take(&a.jzbar, f8 * Wk * LJ);
    c.take(&a.jtmu, f8 * Wk * LJ * 3);
    c.take(&a.drift4, f8 * Wk * N * 4);
  }
  c.take(&a.jbar, f8 * Wk * nj);
  c.take(&a.dr, f8 * Wk * N * 3);
  c.take(&a.lam_part, f8 * (size_t)a.chunks * L * L);
}

static qmc_status check_walker_args(qmc_system* sys, int32_t n_walkers, int32_t flags) {
  if (!sys) return fail(QMC_ERR_ARG, "null system");
  if (n_walkers <= 0) return fail(QMC_ERR_ARG, "n_walkers must be positive");
  if (flags & ~QMC_WALKERS_ADJOINT) return fail(QMC_ERR_ARG, "unknown walker flags");
  return QMC_OK;
}

extern "C" qmc_status qmc_workspace_size(const qmc_system* sys, int32_t n_walkers, int32_t flags, size_t* bytes) {
  if (!bytes) return fail(QMC_ERR_ARG, "null bytes");
  *bytes = 0;
  qmc_status c = check_walker_args(const_cast<qmc_system*>(sys), n_walkers, flags);
  if (c) return c;
  qmc_walkers probe;
  Carver cv{nullptr};
  walker_layout(sys->d, n_walkers, (flags & QMC_WALKERS_ADJOINT) != 0, cv, probe);
  *bytes = cv.off;
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_create(qmc_system* sys, int32_t n_walkers, int32_t flags, void* ws, size_t ws_bytes,
                                         qmc_walkers** out) {
  if (!out) return fail(QMC_ERR_ARG, "null argument");
  *out = nullptr;
  qmc_status c = check_walker_args(sys, n_walkers, flags);
  if (c) return c;
  const bool adjoint = (flags & QMC_WALKERS_ADJOINT) != 0;
  size_t need = 0;
  c = qmc_workspace_size(sys, n_walkers, flags, &need);
  if (c) return c;
  if (ws && ((uintptr_t)ws % 256 != 0)) return fail(QMC_ERR_ARG, "workspace must be 256-byte aligned");
  if (ws && ws_bytes < need) return fail(QMC_ERR_ARG, "workspace smaller than qmc_workspace_size");
  auto* wk = new qmc_walkers();
  wk->sys = sys;
  void* base = ws;
  if (!base) {
    hipError_t e = hipMalloc(&base, need);
    if (e != hipSuccess) {
      delete wk;
      return e == hipErrorOutOfMemory ? fail(QMC_ERR_OOM, "device allocation failed") : hip_fail(e, "walkers_create");
    }
    wk->allocs.push_back(base);
  }
  Carver cv{(char*)base};
  walker_layout(sys->d, n_walkers, adjoint, cv, *wk);
  wk->aw_ready = adjoint;
  hipError_t e = hipMemset(base, 0, need);
  if (e == hipSuccess && sys->d.screened() && sys->d.nk > 0) {   // the unpaired orbitals' transposed rows
    e = launch_pt_unpaired(sys->d, wk->d, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  }
  if (e != hipSuccess) {
    delete wk;
    return hip_fail(e, "walkers_create");
  }
  *out = wk;
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_destroy(qmc_walkers* wk) {
  if (!wk) return fail(QMC_ERR_ARG, "null walkers");
  (void)hipDeviceSynchronize();
  delete wk;
  return QMC_OK;
}

static qmc_status check_pair(qmc_system* sys, qmc_walkers* wk) {
  if (!sys || !wk) return fail(QMC_ERR_ARG, "null handle");
  if (wk->sys != sys) return fail(QMC_ERR_ARG, "walkers belong to another system");
  return QMC_OK;
}

extern "C" qmc_status qmc_eval_batch(qmc_system* sys, qmc_walkers* wk, const double* r, double* logabs,
                                     double* sign, double* drift, double* e_kin, double* e_loc,
                                     int32_t* status, hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!r && !wk->evaluated) return fail(QMC_ERR_STATE, "no current positions: evaluate at given positions first");
  const SysDev& s = sys->d;
  WalkDev& d = wk->d;
  if (r) HIP_TRY(hipMemcpyAsync(d.r, r, sizeof(double) * d.Wk * s.N * 3, hipMemcpyDeviceToDevice, stream), "copy r");
  // At the current positions, the P rows of a spin none of whose electrons
  // has moved since they were built (the rebuild between the two halves of a
  // sweep) are still Phi Lambda: the FP64, FP32 and int8-refined builds skip
  // them (the rebuilds between moves compute exactly what this build would).
  int halves = 3;
  if (!r && wk->generation == sys->generation && !s.refined() && !s.pairing) {
    if (wk->P_up_valid) halves &= ~1;
    if (wk->P_dn_valid) halves &= ~2;
  }
  // QMC_MIXED evaluates through the FP64 kernels on the FP64 work arrays, then
  // stores the FP32 basis and P rows the moves stream.
  const bool refine = s.refined();
  SysDev se = s;
  WalkDev de = d;
  if (refine) {
    se.precision = QMC_FP64;
    de.phi = d.phi64;
    de.P = d.P64;
  }
  // the FP32 / BF16 copies of Phi and P are written by the producing kernels
  // the int8 digits of the refined products take their row scales from here
  const bool oz = (refine || s.screened()) && s.oz_s > 0;
  int* ephi = (oz && s.Lq == 0) ? d.oz_ephi : nullptr;
  TIMED(wk, QMC_T_BASIS, stream, launch_basis_values(se, de, stream, refine ? d.phi : nullptr, s.bf16(), ephi),
        "basis");
  if (s.pairing) {
    TIMED(wk, QMC_T_P_BUILD, stream, s.pf_refined() ? launch_pf_B_build_oz(s, d, stream) : launch_pf_B_build(s, d, stream),
          "Pfaffian B rows");
    TIMED(wk, QMC_T_W_BUILD, stream, launch_pf_G_build(s, d, stream), "Pfaffian G");
    TIMED(wk, QMC_T_LU, stream, launch_pf_factor(s, d, stream), "Pfaffian and inverse");
    TIMED(wk, QMC_T_Y_BUILD, stream, launch_pf_Y_build(s, d, stream), "Pfaffian Y build");
  } else {
  if (oz) {
    // reduced-precision digits on the int8 matrix cores, refined to the FP64
    // product (see ozaki.hip); the moves' FP32 / BF16 rows (refined modes) or
    // the transposed rows of the screened proposals are written beside
    if (halves) {
      // (QMC_REFINED) a half built before at these parameters: only the rows
      // whose electron has moved since
      int dirty = 0;
      if (s.screened() && d.rpos_P)
        for (int h = 0; h < 2; ++h)
          if (wk->P_gen[h] == sys->generation) dirty |= 1 << h;
      TIMED(wk, QMC_T_P_BUILD, stream,
            launch_P_build_oz(s, d, halves, de.phi == d.phi64 ? d.phi64 : (const double*)d.phi,
                              refine ? d.P64 : (double*)d.P, refine ? d.P : nullptr, s.bf16(), stream,
                              ephi != nullptr, s.screened() ? d.PT : nullptr, dirty & halves),
            "P build");
      if (s.screened())
        for (int h = 0; h < 2; ++h)
          if ((halves >> h) & 1) wk->P_gen[h] = sys->generation;
      if (s.screened())
        TIMED(wk, QMC_T_OTHER, stream, launch_screen_colmax(s, d, halves, stream), "column maxima");
    }
  } else if (halves) {
    // (FP64, FP32) a half built before at these parameters: only the rows
    // whose electron has moved since
    int dirty = 0;
    if (d.rpos_P)
      for (int h = 0; h < 2; ++h)
        if (((halves >> h) & 1) && wk->P_gen[h] == sys->generation) dirty |= 1 << h;
    TIMED(wk, QMC_T_P_BUILD, stream,
          launch_P_build(se, de, halves, stream, refine ? d.P : nullptr, s.bf16(), dirty), "P build");
    if (d.rpos_P)
      for (int h = 0; h < 2; ++h)
        if ((halves >> h) & 1) wk->P_gen[h] = sys->generation;
  }
  TIMED(wk, QMC_T_W_BUILD, stream, launch_W_build(se, de, stream), "W build");
  TIMED(wk, QMC_T_LU, stream, launch_lu_inverse(se, de, stream), "LU");
  TIMED(wk, QMC_T_Y_BUILD, stream, launch_Y_build(se, de, stream), "Y build");
  }
  TIMED(wk, QMC_T_ROWDOT, stream, launch_rowdots(s, d, stream), "row dots");
  if (s.LJ) TIMED(wk, QMC_T_ASSEMBLE, stream, launch_jastrow3_eval(s, d, stream), "Jastrow basis terms");
  // E_kin and E_loc stay with the walkers (the LRDMC step reads them)
  TIMED(wk, QMC_T_ASSEMBLE, stream,
        launch_jastrow_assemble(s, d, logabs, sign, drift, wk->lr.ekin, wk->lr.eloc, status, stream), "assemble");
  if (e_kin)
    HIP_TRY(hipMemcpyAsync(e_kin, wk->lr.ekin, sizeof(double) * d.Wk, hipMemcpyDeviceToDevice, stream), "e_kin");
  if (e_loc)
    HIP_TRY(hipMemcpyAsync(e_loc, wk->lr.eloc, sizeof(double) * d.Wk, hipMemcpyDeviceToDevice, stream), "e_loc");
  wk->evaluated = true;
  wk->yt_valid = true;
  wk->lr_ready = false;
  wk->generation = sys->generation;
  wk->P_up_valid = wk->P_dn_valid = true;
  wk->attempts = 0;
  wk->since = 0;
  wk->buf_spin = -1;
  wk->pending_e = -1;
  return QMC_OK;
}

// P rows of the spin opposite to electron e must match the current basis rows.
static hipError_t rebuild_P(qmc_walkers* wk, int halves, hipStream_t stream) {
  const SysDev& s = wk->sys->d;
  const WalkDev& d = wk->d;
  if (!s.screened()) {
    int dirty = 0;
    if (d.rpos_P)
      for (int h = 0; h < 2; ++h)
        if (((halves >> h) & 1) && wk->P_gen[h] == wk->sys->generation) dirty |= 1 << h;
    hipError_t e = launch_P_build(s, d, halves, stream, nullptr, false, dirty);
    if (e == hipSuccess && d.rpos_P)
      for (int h = 0; h < 2; ++h)
        if ((halves >> h) & 1) wk->P_gen[h] = wk->sys->generation;
    return e;
  }
  // refined int8 products from the FP64 rows the accepts maintain (only the
  // rows whose electron has moved since the half was last built), with the
  // transposed rows and column maxima of the screened proposals
  int dirty = 0;
  for (int h = 0; h < 2; ++h)
    if (((halves >> h) & 1) && wk->P_gen[h] == wk->sys->generation) dirty |= 1 << h;
  hipError_t e = launch_P_build_oz(s, d, halves, (const double*)d.phi, (double*)d.P, nullptr, false, stream, false,
                                   d.PT, dirty);
  if (e == hipSuccess) e = launch_screen_colmax(s, d, halves, stream);
  if (e == hipSuccess)
    for (int h = 0; h < 2; ++h)
      if ((halves >> h) & 1) wk->P_gen[h] = wk->sys->generation;
  return e;
}

static qmc_status ensure_P(qmc_walkers* wk, int e, hipStream_t stream) {
  const SysDev& s = wk->sys->d;
  const bool up = e < s.nu;
  if (up && !wk->P_dn_valid) {
    TIMED(wk, QMC_T_P_REBUILD, stream, rebuild_P(wk, 2, stream), "P_dn rebuild");
    wk->P_dn_valid = true;
  } else if (!up && !wk->P_up_valid) {
    TIMED(wk, QMC_T_P_REBUILD, stream, rebuild_P(wk, 1, stream), "P_up rebuild");
    wk->P_up_valid = true;
  }
  return QMC_OK;
}

static qmc_status before_propose(qmc_walkers* wk, int e, hipStream_t stream);

extern "C" qmc_status qmc_propose_move(qmc_system* sys, qmc_walkers* wk, int32_t electron,
                                       const double* r_new, double* ratio, double* drift_new,
                                       hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  const SysDev& s = sys->d;
  if (!wk->evaluated) return fail(QMC_ERR_STATE, "propose before eval_batch");
  if (wk->generation != sys->generation) return fail(QMC_ERR_STATE, "parameters changed since the last eval_batch");
  if (electron < 0 || electron >= s.N) return fail(QMC_ERR_ARG, "electron index out of range");
  if (!r_new) return fail(QMC_ERR_ARG, "null r_new");
  // (a pending proposal is simply replaced)
  if (s.pairing) {
    wk->yt_valid = wk->lr_ready = false;
    TIMED(wk, QMC_T_PROPOSE, stream,
          launch_pf_propose(s, wk->d, electron, r_new, nullptr, ratio, drift_new, stream), "Pfaffian proposal");
    wk->pending_e = electron;
    return QMC_OK;
  }
  c = before_propose(wk, electron, stream);
  if (c) return c;
  c = ensure_P(wk, electron, stream);
  if (c) return c;
  TIMED(wk, QMC_T_PROPOSE_PREP, stream,
        launch_propose_prep(s, wk->d, electron, r_new, nullptr, drift_new != nullptr, stream), "propose prep");
{
    hipEvent_t ea, eb;
    HIP_TRY(wk->tm.begin_ext(QMC_T_PROPOSE, &ea, &eb), "timer begin");
    if (s.screened() && !drift_new)
      HIP_TRY(launch_propose_screened(s, wk->d, electron, ratio, true, stream, ea, eb), "screened proposal");
    else
      HIP_TRY(launch_propose_rows(s, wk->d, electron, ratio, drift_new, true, stream, ea, eb), "propose rows");
  }
  wk->pending_e = electron;
  return QMC_OK;
}

// Refresh schedule (the same for one system and for a multi-system member):
// the delayed-update buffer holds moves of one spin and at most wb_cap(s)
// moves, so a proposal of the other spin refreshes first, and the move that
// fills the buffer refreshes after its accept.  A refresh is the FP64 inverse
// of the maintained W, which also resets log|Psi| and the sign.
struct Sched {
  long attempts;
  int since, buf_spin;
};
static bool sched_before(const SysDev& s, Sched& q, int e) {   // true: refresh before proposing e
  const int spin = e < s.nu ? 0 : 1;
  const bool pre = q.since > 0 && spin != q.buf_spin;
  if (pre) q.since = 0;
  q.buf_spin = spin;
  return pre;
}
static bool sched_after(const SysDev& s, Sched& q) {           // true: refresh after this accept
  q.attempts += 1;
  q.since += 1;
  if (q.since < wb_cap(s)) return false;
  q.since = 0;
  return true;
}

// With a status array the refresh also measures how far the inverse it
// replaces had drifted: X = the maintained inverse (delayed form materialised,
// or the Pfaffian's G~^{-1}), res = max |W X - I|, status 3 above drift_tol.
static hipError_t residual_before(const SysDev& s, qmc_walkers* wk, hipStream_t stream) {
  const int n = s.pairing ? s.npf : s.nu;
  const long nn = (long)n * n;
  if (s.pairing) {
    TIMED_E(wk, QMC_T_OTHER, stream,
            hipMemcpyAsync(wk->res_x, wk->d.A, sizeof(double) * nn * wk->d.Wk, hipMemcpyDeviceToDevice, stream));
  } else {
    TIMED_E(wk, QMC_T_OTHER, stream,
            launch_materialize_inverse(s, wk->d, wk->buf_spin == 1, wk->rd_scratch, wk->res_x, stream));
  }
  GemmArgs g = gemm_args(n, n, n);
  g.A = wk->d.W; g.lda = n; g.a_bs = nn;
  g.B = wk->res_x; g.ldb = n; g.b_bs = nn;
  g.C = wk->res_p; g.ldc = n; g.c_bs = nn;
  g.batch = wk->d.Wk;
  TIMED_E(wk, QMC_T_OTHER, stream, gemm_f64(g, false, false, false, stream));
  return hipSuccess;
}

static hipError_t refresh(const SysDev& s, qmc_walkers* wk, int32_t* status, hipStream_t stream) {
  const bool check = status && wk->drift_tol >= 0.0;
  if (check) {
    hipError_t e = residual_before(s, wk, stream);
    if (e != hipSuccess) return e;
  }
  TIMED_E(wk, QMC_T_LU, stream, launch_lu_inverse(s, wk->d, stream));
  TIMED_E(wk, QMC_T_OTHER, stream, launch_refresh_finish(s, wk->d, status, stream));
  if (check) {
    const int n = s.pairing ? s.npf : s.nu;
    TIMED_E(wk, QMC_T_OTHER, stream,
            launch_refresh_residual(wk->res_p, n, wk->d.Wk, wk->drift_tol, wk->res_v, status, stream));
  }
  return hipSuccess;
}

static qmc_status before_propose(qmc_walkers* wk, int e, hipStream_t stream) {
  const SysDev& s = wk->sys->d;
  wk->yt_valid = wk->lr_ready = false;
  Sched q{wk->attempts, wk->since, wk->buf_spin};
  if (sched_before(s, q, e)) HIP_TRY(refresh(s, wk, nullptr, stream), "spin-switch refresh");
  wk->since = q.since;
  wk->buf_spin = q.buf_spin;
  return QMC_OK;
}

static qmc_status after_accept(qmc_walkers* wk, int e, int32_t* status, hipStream_t stream) {
  const SysDev& s = wk->sys->d;
  if (e < s.nu) wk->P_up_valid = false; else wk->P_dn_valid = false;
  wk->pending_e = -1;
  Sched q{wk->attempts, wk->since, wk->buf_spin};
  const bool post = sched_after(s, q);
  wk->attempts = q.attempts;
  wk->since = q.since;
  if (post) HIP_TRY(refresh(s, wk, status, stream), "refresh");
  return QMC_OK;
}

// Pfaffian moves: the rank-2 updates of G~^{-1} are exact in exact arithmetic;
// the inverse, log|Psi| and the sign are recomputed from the maintained G~
// every refresh_every moves.
static qmc_status pf_after_accept(qmc_walkers* wk, int32_t* status, hipStream_t stream) {
  const SysDev& s = wk->sys->d;
  wk->pending_e = -1;
  wk->attempts += 1;
  if (++wk->since < s.refresh_every) return QMC_OK;
  wk->since = 0;
  const bool check = status && wk->drift_tol >= 0.0;
  if (check) HIP_TRY(residual_before(s, wk, stream), "refresh residual");
  TIMED(wk, QMC_T_LU, stream, launch_pf_factor(s, wk->d, stream), "Pfaffian refresh");
  TIMED(wk, QMC_T_OTHER, stream, launch_refresh_finish(s, wk->d, status, stream), "refresh finish");
  if (check)
    TIMED(wk, QMC_T_OTHER, stream,
          launch_refresh_residual(wk->res_p, s.npf, wk->d.Wk, wk->drift_tol, wk->res_v, status, stream),
          "refresh residual");
  return QMC_OK;
}

extern "C" qmc_status qmc_accept_move(qmc_system* sys, qmc_walkers* wk, int32_t electron,
                                      const uint8_t* accept, int32_t* status, hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!accept) return fail(QMC_ERR_ARG, "null accept");
  if (wk->pending_e < 0 || wk->pending_e != electron)
    return fail(QMC_ERR_STATE, "no pending proposal for this electron");
  if (sys->d.pairing) {
    TIMED(wk, QMC_T_ACCEPT, stream, launch_pf_accept(sys->d, wk->d, electron, accept, nullptr, nullptr, stream),
          "Pfaffian accept");
    return pf_after_accept(wk, status, stream);
  }
  TIMED(wk, QMC_T_ACCEPT, stream, launch_accept(sys->d, wk->d, electron, accept, stream), "accept");
  return after_accept(wk, electron, status, stream);
}

// The accept of e can run fused with the set-up of the next proposal e2 when
// neither a refresh (after the accept, or before proposing e2) nor a P rebuild
// (for e2) falls between them, and psi(r') fits the kernel's LDS stage.
// The host's move bookkeeping (refresh schedule and P validity), stepped
// without launching anything.
struct MoveState {
  Sched q;
  bool up_ok, dn_ok;
};
// fusable on state m; on success m becomes the state after the accept of e,
// the refresh check before e2 and its P check (none of which then launches).
static bool fuse_step(const qmc_walkers* wk, MoveState& m, int e, int e2) {
  const SysDev& s = wk->sys->d;
  if (s.Lp > kFuseMaxLp || s.nu > kBigMaxN || !wk->d.wv || e2 == e || s.LJ > 0 || s.Lq > 0) return false;
  MoveState t = m;
  if (sched_after(s, t.q)) return false;
  if (sched_before(s, t.q, e2)) return false;
  if (e < s.nu) t.up_ok = false; else t.dn_ok = false;
  if (!(e2 < s.nu ? t.dn_ok : t.up_ok)) return false;
  m = t;
  return true;
}
static bool fusable(const qmc_walkers* wk, int e, int e2) {
  MoveState m{Sched{wk->attempts, wk->since, wk->buf_spin}, wk->P_up_valid, wk->P_dn_valid};
  return fuse_step(wk, m, e, e2);
}
// Moves t, t + 1, ..., t + k - 1 of a vmc_steps call whose accepts, all but
// the last, are fusable with the next set-up: the k of the run starting at t.
static int fused_run(const qmc_walkers* wk, int e_start, int t, int n_steps) {
  const int N = wk->sys->d.N;
  MoveState m{Sched{wk->attempts, wk->since, wk->buf_spin}, wk->P_up_valid, wk->P_dn_valid};
  int k = 1;
  while (t + k < n_steps &&
         fuse_step(wk, m, (int)((e_start + (long)t + k - 1) % N), (int)((e_start + (long)t + k) % N)))
    ++k;
  return k;
}

extern "C" qmc_status qmc_vmc_steps(qmc_system* sys, qmc_walkers* wk, int32_t e_start, int32_t n_steps,
                                    const double* disp, const double* unif, int32_t* accept_count,
                                    hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  const SysDev& s = sys->d;
  if (!wk->evaluated) return fail(QMC_ERR_STATE, "vmc_steps before eval_batch");
  if (wk->generation != sys->generation) return fail(QMC_ERR_STATE, "parameters changed since the last eval_batch");
  if (!disp || !unif) return fail(QMC_ERR_ARG, "null random arrays");
  if (n_steps < 0 || e_start < 0) return fail(QMC_ERR_ARG, "negative step count or electron");
  if (s.pairing) {
    wk->yt_valid = wk->lr_ready = false;
    for (int t = 0; t < n_steps; ++t) {
      const int e = (int)((e_start + (long)t) % s.N);
      TIMED(wk, QMC_T_PROPOSE, stream,
            launch_pf_propose(s, wk->d, e, nullptr, disp + (long)t * wk->d.Wk * 3, nullptr, nullptr, stream),
            "Pfaffian proposal");
      TIMED(wk, QMC_T_ACCEPT, stream,
            launch_pf_accept(s, wk->d, e, nullptr, unif + (long)t * wk->d.Wk, accept_count, stream),
            "Pfaffian Metropolis");
      c = pf_after_accept(wk, nullptr, stream);
      if (c) return c;
    }
    return QMC_OK;
  }
  const long Wk = wk->d.Wk;
  bool prepped = false;   // the set-up of step t ran in step t-1's fused accept
  for (int t = 0; t < n_steps; ++t) {
    const int e = (int)((e_start + (long)t) % s.N);
    if (!prepped) {
      c = before_propose(wk, e, stream);
      if (c) return c;
      c = ensure_P(wk, e, stream);
      if (c) return c;
      TIMED(wk, QMC_T_PROPOSE_PREP, stream,
            launch_propose_prep(s, wk->d, e, nullptr, disp + (long)t * Wk * 3, false, stream), "propose prep");
      // a run of fusable moves from here: one persistent launch, then the
      // bookkeeping of its fused steps (which launches nothing) and a plain
      // accept of its last proposal
      const int k = sweep_segment_ok(s, wk->d, e) ? fused_run(wk, e_start, t, n_steps) : 1;
      if (k >= 2) {
        hipEvent_t ea, eb;
        HIP_TRY(wk->tm.begin_ext(QMC_T_SWEEP, &ea, &eb), "timer begin");
        HIP_TRY(launch_sweep_segment(s, wk->d, e, k, disp + (long)t * Wk * 3, unif + (long)t * Wk, accept_count,
                                     wk->since, stream, ea, eb),
                "persistent sweep");
        for (int j = 0; j + 1 < k; ++j) {
          const int ej = (int)((e_start + (long)t + j) % s.N), ej2 = (int)((e_start + (long)t + j + 1) % s.N);
          c = after_accept(wk, ej, nullptr, stream);
          if (c) return c;
          c = before_propose(wk, ej2, stream);
          if (c) return c;
          c = ensure_P(wk, ej2, stream);
          if (c) return c;
        }
        const long tl = t + k - 1;
        TIMED(wk, QMC_T_ACCEPT, stream,
              launch_metropolis_accept(s, wk->d, (int)((e_start + tl) % s.N), unif + tl * Wk, accept_count, stream),
              "metropolis");
        c = after_accept(wk, (int)((e_start + tl) % s.N), nullptr, stream);
        if (c) return c;
        t += k - 1;
        continue;
      }
    }
{
      hipEvent_t ea, eb;
      HIP_TRY(wk->tm.begin_ext(QMC_T_PROPOSE, &ea, &eb), "timer begin");
      if (s.screened())
        HIP_TRY(launch_propose_screened(s, wk->d, e, nullptr, false, stream, ea, eb), "screened proposal");
      else
        HIP_TRY(launch_propose_rows(s, wk->d, e, nullptr, nullptr, false, stream, ea, eb), "propose rows");
    }
    const int e2 = (int)((e_start + (long)t + 1) % s.N);
    prepped = t + 1 < n_steps && fusable(wk, e, e2);
    if (prepped) {
      // no refresh and no P rebuild fall between the two: the bookkeeping of
      // after_accept, before_propose and ensure_P below launches nothing
      TIMED(wk, QMC_T_ACCEPT, stream,
            launch_metropolis_accept_prep(s, wk->d, e, unif + (long)t * Wk, accept_count, e2,
                                          disp + (long)(t + 1) * Wk * 3, wk->since, stream),
            "metropolis + next set-up");
      c = after_accept(wk, e, nullptr, stream);
      if (c) return c;
      c = before_propose(wk, e2, stream);
      if (c) return c;
      c = ensure_P(wk, e2, stream);
      if (c) return c;
    } else {
      TIMED(wk, QMC_T_ACCEPT, stream,
            launch_metropolis_accept(s, wk->d, e, unif + (long)t * Wk, accept_count, stream), "metropolis");
      c = after_accept(wk, e, nullptr, stream);
      if (c) return c;
    }
  }
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_read(qmc_walkers* wk, int32_t item, double* dst, hipStream_t stream) {
  if (!wk || !dst) return fail(QMC_ERR_ARG, "null argument");
  const SysDev& s = wk->sys->d;
  const WalkDev& d = wk->d;
  const size_t Wk = d.Wk;
  const void* src = nullptr;
  size_t bytes = 0;
  switch (item) {
    case QMC_STATE_R: src = d.r; bytes = sizeof(double) * Wk * s.N * 3; break;
    case QMC_STATE_LOGABS: src = d.logabs; bytes = sizeof(double) * Wk; break;
    case QMC_STATE_SIGN: src = d.sign; bytes = sizeof(double) * Wk; break;
    case QMC_STATE_W:
      src = d.W;
      bytes = sizeof(double) * Wk * (s.pairing ? (size_t)s.npf * s.npf : (size_t)s.nu * s.nu);
      break;
    case QMC_STATE_AINV:   // A0 combined with the delayed updates
      if (s.pairing) { src = d.A; bytes = sizeof(double) * Wk * s.npf * s.npf; break; }
      HIP_TRY(launch_materialize_inverse(s, d, wk->buf_spin == 1, wk->rd_scratch, dst, stream), "read inverse");
      return QMC_OK;
    case QMC_STATE_PHI:
      HIP_TRY(launch_export_phi(s, d, dst, stream), "export phi");
      return QMC_OK;
    case QMC_STATE_RESIDUAL: src = wk->res_v; bytes = sizeof(double) * Wk; break;
    case QMC_STATE_KEPT:
      if (!s.screened()) return fail(QMC_ERR_ARG, "QMC_STATE_KEPT needs a QMC_REFINED system");
      HIP_TRY(launch_export_kept(d, dst, stream), "export kept counts");
      return QMC_OK;
    default: return fail(QMC_ERR_ARG, "unknown state item");
  }
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream), "read state");
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_set_drift_tol(qmc_walkers* wk, double tol) {
  if (!wk) return fail(QMC_ERR_ARG, "null walkers");
  if (tol != tol) return fail(QMC_ERR_ARG, "tolerance is not a number");
  wk->drift_tol = tol;
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_set_timing_mask(qmc_walkers* wk, uint32_t mask) {
  if (!wk) return fail(QMC_ERR_ARG, "null walkers");
  HIP_TRY(wk->tm.fold(), "timer fold");
  for (int k = 0; k < QMC_TIMER_COUNT; ++k) { wk->tm.ms[k] = 0.0; wk->tm.n[k] = 0; }
  wk->tm.mask = mask & ((1u << QMC_TIMER_COUNT) - 1u);
  wk->tm.on = wk->tm.mask != 0;
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_set_timing(qmc_walkers* wk, int32_t enable) {
  return qmc_walkers_set_timing_mask(wk, enable ? ~0u : 0u);
}

extern "C" qmc_status qmc_walkers_timing(qmc_walkers* wk, double* ms, int64_t* launches) {
  if (!wk || !ms || !launches) return fail(QMC_ERR_ARG, "null argument");
  HIP_TRY(wk->tm.fold(), "timer fold");
  for (int k = 0; k < QMC_TIMER_COUNT; ++k) { ms[k] = wk->tm.ms[k]; launches[k] = wk->tm.n[k]; }
  return QMC_OK;
}

extern "C" qmc_status qmc_forces(qmc_system* sys, qmc_walkers* wk, const double* r, int32_t per_walker,
                                 const double* gbar_logpsi, const double* gbar_eloc, const qmc_grads* out,
                                 hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!r || !out) return fail(QMC_ERR_ARG, "null positions or output block");
  const SysDev& s = sys->d;
  if (s.precision != QMC_FP64) return fail(QMC_ERR_UNSUPPORTED, "forces are built for the FP64 path");
  if (!s.pairing && (out->dpf_uu || out->dpf_dd || out->dunpaired_dn))
    return fail(QMC_ERR_ARG, "dpf_uu, dpf_dd and dunpaired_dn are outputs of Pfaffian systems");
  if (s.n_nuc > kMaxNucBack) return fail(QMC_ERR_UNSUPPORTED, "forces need <= 256 nuclei");
  if (!wk->aw_ready)
    return fail(QMC_ERR_STATE, "walkers created without QMC_WALKERS_ADJOINT (no reverse-pass workspace)");
  c = qmc_eval_batch(sys, wk, r, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, stream);
  if (c) return c;
  HIP_TRY(launch_forces(s, wk->d, wk->aw, gbar_logpsi, gbar_eloc, per_walker, out->dR, out->dzeta,
                        out->dlambda, out->djas, out->dr, s.LJ ? out->dj1_inh : nullptr, s.LJ ? out->dj3 : nullptr,
                        s.LJ ? out->djb_zeta : nullptr, (s.nk || s.pk) ? out->dunpaired : nullptr,
                        s.Lq ? out->dcon_coef : nullptr, out->dpf_uu, out->dpf_dd,
                        s.pk ? out->dunpaired_dn : nullptr, stream), "forces");
  return QMC_OK;
}

// ---------------------------------------------------------------------------
// lattice-regularised diffusion Monte Carlo
// ---------------------------------------------------------------------------

extern "C" qmc_status qmc_lrdmc_hops(qmc_system* sys, qmc_walkers* wk, const qmc_lrdmc_params* params,
                                     double* ratios, double* terms, hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!params) return fail(QMC_ERR_ARG, "null parameters");
  const qmc_lrdmc_params& q = *params;
  if (!(q.a > 0.0) || !std::isfinite(q.a)) return fail(QMC_ERR_ARG, "hop length a must be positive");
  const bool dbl = q.a_valence > 0.0;
  if (dbl && (!std::isfinite(q.a_valence) || !(q.tf_scale > 0.0) || !std::isfinite(q.tf_scale)))
    return fail(QMC_ERR_ARG, "double grid needs a finite a_valence and a positive tf_scale");
  if (!(q.gamma >= 0.0) || !std::isfinite(q.gamma)) return fail(QMC_ERR_ARG, "gamma must be >= 0");
  if (!wk->evaluated || !wk->yt_valid)
    return fail(QMC_ERR_STATE, "lattice hops need an evaluation since the last move");
  if (wk->generation != sys->generation) return fail(QMC_ERR_STATE, "parameters changed since the last eval_batch");
  const SysDev& s = sys->d;
  const WalkDev& d = wk->d;
  const LrdmcParams p{q.a, dbl ? q.a_valence : 0.0, q.tf_scale, q.gamma};
  TIMED(wk, QMC_T_LRDMC_HOPS, stream, launch_lrdmc_hops(s, d, wk->lr, p, stream), "lattice hops");
  if (ratios)
    HIP_TRY(hipMemcpyAsync(ratios, wk->lr.ratio, sizeof(double) * d.Wk * s.N * kHops, hipMemcpyDeviceToDevice,
                           stream), "copy ratios");
  if (terms)
    HIP_TRY(hipMemcpyAsync(terms, wk->lr.terms, sizeof(double) * d.Wk * kLrTerms, hipMemcpyDeviceToDevice,
                           stream), "copy terms");
  wk->lr_p = p;
  wk->lr_ready = true;
  return QMC_OK;
}

extern "C" qmc_status qmc_lrdmc_advance(qmc_system* sys, qmc_walkers* wk, const double* xi, double* weight,
                                        double* tau_left, double* r_next, int32_t* hop, hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!xi || !weight || !tau_left || !r_next) return fail(QMC_ERR_ARG, "null argument");
  if (!wk->lr_ready || !wk->yt_valid) return fail(QMC_ERR_STATE, "qmc_lrdmc_hops has not run for these positions");
  if (wk->generation != sys->generation) return fail(QMC_ERR_STATE, "parameters changed since the last eval_batch");
  TIMED(wk, QMC_T_LRDMC_STEP, stream,
        launch_lrdmc_advance(sys->d, wk->d, wk->lr, wk->lr_p, xi, weight, tau_left, r_next, hop, stream),
        "lattice step");
  return QMC_OK;
}

// ---------------------------------------------------------------------------
// estimators
// ---------------------------------------------------------------------------

extern "C" qmc_status qmc_swct(qmc_system* sys, int32_t n_walkers, const double* r, const double* dR,
                               const double* dr, int32_t jacobian, double* out, hipStream_t stream) {
  if (!sys || !r || !dR || !dr || !out) return fail(QMC_ERR_ARG, "null argument");
  if (n_walkers <= 0) return fail(QMC_ERR_ARG, "n_walkers must be positive");
  if (sys->d.N > 1024) return fail(QMC_ERR_UNSUPPORTED, "space warp built for N <= 1024");
  HIP_TRY(launch_swct(sys->d, n_walkers, r, dR, dr, jacobian ? 1 : 0, out, stream), "space warp");
  return QMC_OK;
}

extern "C" qmc_status qmc_reweight(qmc_system* sys, qmc_walkers* wk, double theta, double eps, double* R,
                                   double* weight, hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!R) return fail(QMC_ERR_ARG, "null output");
  if (!(theta > 0.0) || !(eps >= 0.0)) return fail(QMC_ERR_ARG, "theta > 0 and eps >= 0 required");
  if (!wk->evaluated || !wk->yt_valid)
    return fail(QMC_ERR_STATE, "the reweighting factor needs an evaluation since the last move");
  HIP_TRY(launch_reweight(sys->d, wk->d, theta, eps, R, weight, stream), "reweight");
  return QMC_OK;
}

extern "C" qmc_status qmc_jastrow_basis_logderiv(qmc_system* sys, qmc_walkers* wk, double* d_j1_inh, double* d_j3,
                                                 hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (sys->d.LJ <= 0) return fail(QMC_ERR_ARG, "the system has no Jastrow basis");
  if (!wk->evaluated) return fail(QMC_ERR_STATE, "log-derivatives before eval_batch");
  if (wk->generation != sys->generation) return fail(QMC_ERR_STATE, "parameters changed since the last eval_batch");
  if (!d_j1_inh && !d_j3) return QMC_OK;
  HIP_TRY(launch_jastrow3_logderiv(sys->d, wk->d, d_j1_inh, d_j3, stream), "Jastrow-basis log-derivatives");
  return QMC_OK;
}

extern "C" qmc_status qmc_pfaffian_logderiv(qmc_system* sys, qmc_walkers* wk, double* d_uu, double* d_dd,
                                            double* d_ud, double* d_unpaired_up, double* d_unpaired_dn,
                                            hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!sys->d.pairing) return fail(QMC_ERR_ARG, "the system is not a Pfaffian");
  if (!wk->evaluated) return fail(QMC_ERR_STATE, "log-derivatives before eval_batch");
  if (wk->generation != sys->generation) return fail(QMC_ERR_STATE, "parameters changed since the last eval_batch");
  HIP_TRY(launch_pf_logderiv(sys->d, wk->d, d_uu, d_dd, d_ud, d_unpaired_up, d_unpaired_dn, stream),
          "Pfaffian log-derivatives");
  return QMC_OK;
}

extern "C" size_t qmc_sr_workspace_size(int32_t n_samples, int64_t n_params) {
  if (n_samples <= 0 || n_params <= 0) return 0;
  return sizeof(double) * sr_workspace_doubles(n_samples, (long)n_params);
}

extern "C" qmc_status qmc_sr_step(int32_t n_samples, int64_t n_params, const double* O, const double* e_loc,
                                  const double* weights, double eps, int32_t max_iter, double tol, double* delta,
                                  double* force, double* residual, void* work, size_t work_bytes,
                                  hipStream_t stream) {
  if (!O || !e_loc || !delta || !work) return fail(QMC_ERR_ARG, "null argument");
  if (n_samples <= 0 || n_params <= 0 || max_iter < 0) return fail(QMC_ERR_ARG, "bad sizes");
  if (!(eps >= 0.0) || !(tol >= 0.0)) return fail(QMC_ERR_ARG, "eps and tol must be >= 0");
  if (work_bytes < qmc_sr_workspace_size(n_samples, n_params)) return fail(QMC_ERR_ARG, "workspace too small");
  HIP_TRY(launch_sr_step(n_samples, (long)n_params, O, e_loc, weights, eps, max_iter, tol, delta, force, residual,
                         (double*)work, stream), "SR step");
  return QMC_OK;
}

extern "C" qmc_status qmc_system_set_jastrow_basis(qmc_system* sys, const double* j1_inh, const double* j3,
                                                   const double* jb_zeta, hipStream_t stream) {
  if (!sys) return fail(QMC_ERR_ARG, "null system");
  const SysDev& d = sys->d;
  if (d.LJ <= 0) return fail(QMC_ERR_ARG, "the system has no Jastrow basis");
  HIP_TRY(launch_set_jastrow_basis(d, j1_inh, j3, jb_zeta, stream), "set Jastrow basis");
  sys->generation += 1;
  return QMC_OK;
}

extern "C" qmc_status qmc_system_set_pfaffian(qmc_system* sys, const double* pf_uu, const double* pf_dd,
                                               const double* unpaired, const double* unpaired_dn, hipStream_t stream) {
  if (!sys) return fail(QMC_ERR_ARG, "null system");
  if (!sys->d.pairing) return fail(QMC_ERR_ARG, "the system is not a Pfaffian");
  HIP_TRY(launch_pf_set(sys->d, nullptr, pf_uu, pf_dd, sys->d.pk ? unpaired : nullptr,
                        sys->d.pk ? unpaired_dn : nullptr, stream), "set Pfaffian");
  if ((pf_uu || pf_dd) && sys->d.pf_refined()) HIP_TRY(launch_oz_pf_K(sys->d, stream), "K digits");
  sys->generation += 1;
  return QMC_OK;
}

extern "C" qmc_status qmc_system_set_params(qmc_system* sys, const double* R, const double* zeta,
                                            const double* lambda, const double* jas, hipStream_t stream) {
  if (!sys) return fail(QMC_ERR_ARG, "null system");
  SysDev& d = sys->d;
  if (R) HIP_TRY(hipMemcpyAsync(d.R, R, sizeof(double) * 3 * d.n_nuc, hipMemcpyDeviceToDevice, stream), "set R");
  if (zeta)   // one exponent per basis function (per primitive of a contracted basis)
    HIP_TRY(hipMemcpyAsync(d.zeta, zeta, sizeof(double) * d.nprim(), hipMemcpyDeviceToDevice, stream), "set zeta");
  if (lambda && d.pairing) HIP_TRY(launch_pf_set(d, lambda, nullptr, nullptr, nullptr, nullptr, stream), "set A^ud");
  if (lambda && d.pf_refined()) HIP_TRY(launch_oz_pf_K(d, stream), "K digits");
  if (lambda && !d.pairing) HIP_TRY(launch_set_lambda(d, lambda, stream), "set lambda");
  if (lambda && !d.pairing) HIP_TRY(launch_lam_mask(d, stream), "lambda mask");
  if (lambda && !d.pairing && d.oz_s > 0) HIP_TRY(launch_oz_lambda(d, stream), "lambda digits");
  if (R || zeta) HIP_TRY(launch_pack_basis(d, stream), "pack basis");
  if (jas) {
    HIP_TRY(hipMemcpyAsync(d.j1_b, jas, sizeof(double) * d.n_nuc, hipMemcpyDeviceToDevice, stream), "set j1");
    const int n2 = d.j2_form == 1 ? 2 : (d.j2_form == 2 ? 8 : 0);
    if (n2)
      HIP_TRY(hipMemcpyAsync(const_cast<double*>(d.j2d), jas + d.n_nuc, sizeof(double) * n2, hipMemcpyDeviceToDevice,
                             stream), "set j2");
  }
  sys->generation += 1;
  return QMC_OK;
}

// ===========================================================================
// multi-system groups
// ===========================================================================
struct qmc_multi {
  int n = 0;
  std::vector<qmc_system*> sys;
  std::vector<qmc_walkers*> wk;
  std::vector<SysDev> h_sys;
  std::vector<WalkDev> h_wk;
  std::vector<long long> h_steps;
  std::vector<const double*> h_disp, h_unif;
  std::vector<int> order;        // members by decreasing cost
  std::vector<int> rows;         // rows per proposal item, per member
  SysDev* d_sys = nullptr;
  WalkDev* d_wk = nullptr;
  long long* d_steps = nullptr;
  int* d_rows = nullptr;
  const double** d_disp = nullptr;
  const double** d_unif = nullptr;
  int2* d_items = nullptr;
  int n_items = 0;
  int4* d_rows_items = nullptr;
  int n_rows_items = 0, rows_cap = 0;
  int grid_rows = 2048, grid_items = 1024;
  int nc = 1;
  int store = 0;        // 0 FP64, 1 FP32, 2 BF16 rows
  size_t scr_lds = 0;   // QMC_REFINED members: dynamic LDS of the screened streams (0: other modes)
  hipStream_t own = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string gkey;
  std::vector<void*> allocs;
  ~qmc_multi() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    if (own) { (void)hipStreamSynchronize(own); (void)hipStreamDestroy(own); }
    for (void* p : allocs) (void)hipFree(p);
  }
};

static hipError_t multi_build_rows(qmc_multi* m) {
  std::vector<int4> items;
  for (int k : m->order) {
    const SysDev& s = m->h_sys[k];
    // (QMC_REFINED: one screened stream per walker)
    const int S = s.screened() ? 1 : (s.nu + m->rows[k] - 1) / m->rows[k];
    for (int w = 0; w < m->h_wk[k].Wk; ++w)
      for (int sb = 0; sb < S; ++sb) items.push_back(make_int4(k, w, sb, S));
  }
  if ((int)items.size() > m->rows_cap) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(int4) * items.size());
    if (e != hipSuccess) return e;
    m->allocs.push_back(p);
    m->d_rows_items = (int4*)p;
    m->rows_cap = (int)items.size();
  }
  m->n_rows_items = (int)items.size();
  hipError_t e = hipMemcpy(m->d_rows_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(m->d_rows, m->rows.data(), sizeof(int) * m->n, hipMemcpyHostToDevice);
}

extern "C" qmc_status qmc_multi_create(int32_t n_members, qmc_system* const* systems, qmc_walkers* const* walkers,
                                       qmc_multi** out) {
  if (!systems || !walkers || !out) return fail(QMC_ERR_ARG, "null argument");
  if (n_members < 1 || n_members > 32) return fail(QMC_ERR_ARG, "1..32 members");
  *out = nullptr;
  auto* m = new qmc_multi();
  m->n = n_members;
  for (int k = 0; k < n_members; ++k) {
    if (check_pair(systems[k], walkers[k])) { delete m; return QMC_ERR_ARG; }
    const SysDev& s = systems[k]->d;
    if (s.precision != systems[0]->d.precision) { delete m; return fail(QMC_ERR_ARG, "members differ in precision"); }
    // unpaired orbitals, a Jastrow basis and contracted orbitals run in the
    // per-item bodies every member shares with the one-system kernels
    if (s.nu > kLuMaxN) { delete m; return fail(QMC_ERR_UNSUPPORTED, "members need n_up <= 128"); }
    if (s.pairing) { delete m; return fail(QMC_ERR_UNSUPPORTED, "Pfaffian members are not built"); }
    m->sys.push_back(systems[k]);
    m->wk.push_back(walkers[k]);
    m->h_sys.push_back(s);
    m->h_wk.push_back(walkers[k]->d);
    m->rows.push_back(s.prop_rows());
  }
  m->store = systems[0]->d.store();
  if (systems[0]->d.screened()) {
    // the largest LDS any member's blocked screened stream needs (both spins);
    // at least the 1 KiB granule, so that the screened kernel is chosen
    m->scr_lds = 1024;
    for (int k = 0; k < n_members; ++k) {
      const SysDev& s = m->h_sys[k];
      for (int e : {0, s.N - 1}) m->scr_lds = std::max(m->scr_lds, screened_stream_lds(s, m->h_wk[k], e));
    }
  }
  m->order.resize(n_members);
  std::iota(m->order.begin(), m->order.end(), 0);
  std::stable_sort(m->order.begin(), m->order.end(), [&](int a, int b) {
    const SysDev &x = m->h_sys[a], &y = m->h_sys[b];
    return (long)x.L * x.nu > (long)y.L * y.nu;
  });
  const int vec = 64 * (m->store == 0 ? 2 : (m->store == 1 ? 4 : 8));
  std::vector<int2> items;
  for (int k : m->order) {
    const SysDev& s = m->h_sys[k];
    m->nc = std::max(m->nc, (s.Lp + vec - 1) / vec);
    for (int w = 0; w < m->h_wk[k].Wk; ++w) items.push_back(make_int2(k, w));
  }
  if (m->nc > 8) { delete m; return fail(QMC_ERR_UNSUPPORTED, "members need L <= 1024 (FP64) or 2048 (FP32)"); }
  m->n_items = (int)items.size();
  m->grid_items = std::min(m->n_items, 2048);
  hipError_t e = hipSuccess;
  auto al = [&](void** p, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(p, bytes);
    if (e == hipSuccess) m->allocs.push_back(*p);
  };
  al((void**)&m->d_sys, sizeof(SysDev) * n_members);
  al((void**)&m->d_wk, sizeof(WalkDev) * n_members);
  al((void**)&m->d_steps, sizeof(long long) * n_members);
  al((void**)&m->d_rows, sizeof(int) * n_members);
  al((void**)&m->d_disp, sizeof(double*) * n_members);
  al((void**)&m->d_unif, sizeof(double*) * n_members);
  al((void**)&m->d_items, sizeof(int2) * items.size());
  if (!e) e = hipMemcpy(m->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(m->d_wk, m->h_wk.data(), sizeof(WalkDev) * n_members, hipMemcpyHostToDevice);
  if (!e) e = multi_build_rows(m);
  if (!e) e = hipStreamCreateWithFlags(&m->own, hipStreamNonBlocking);
  if (!e) e = hipEventCreateWithFlags(&m->ev_a, hipEventDisableTiming);
  if (!e) e = hipEventCreateWithFlags(&m->ev_b, hipEventDisableTiming);
  m->grid_rows = std::min(m->n_rows_items, 2048);
  if (e != hipSuccess) { delete m; return hip_fail(e, "multi_create"); }
  *out = m;
  return QMC_OK;
}

extern "C" qmc_status qmc_multi_destroy(qmc_multi* m) {
  if (!m) return fail(QMC_ERR_ARG, "null group");
  delete m;
  return QMC_OK;
}

// Refresh the device copies of the member descriptors and move counters on
// the group's stream (not part of any captured graph).
static hipError_t multi_upload(qmc_multi* m) {
  m->h_steps.resize(m->n);
  for (int k = 0; k < m->n; ++k) {
    m->h_sys[k] = m->sys[k]->d;
    m->h_steps[k] = m->wk[k]->attempts;
  }
  hipError_t e = hipMemcpyAsync(m->d_sys, m->h_sys.data(), sizeof(SysDev) * m->n, hipMemcpyHostToDevice, m->own);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_steps, m->h_steps.data(), sizeof(long long) * m->n, hipMemcpyHostToDevice, m->own);
  return e;
}

// Enqueue n_steps steps on the group's stream; P validity of the members is
// simulated in up/dn (and returned), so a captured graph and a direct run
// follow the same schedule.
// Per-member schedule state carried through a call (and into the captured graph).
struct MemberState {
  Sched q;
  char up_ok, dn_ok;   // P halves valid
};

// One member's host-side plan for its next step: electron, P half to rebuild
// (0 none, 1 up, 2 down), refreshes before the proposal and after the accept.
// The same rules as the one-system path (sched_before / ensure_P / sched_after).
static void plan_member(const SysDev& s, MemberState& st, int& pbuild, bool& pre, bool& post) {
  const int e = (int)(st.q.attempts % s.N);
  pre = sched_before(s, st.q, e);
  pbuild = 0;
  if (e < s.nu && !st.dn_ok) { pbuild = 2; st.dn_ok = 1; }
  else if (e >= s.nu && !st.up_ok) { pbuild = 1; st.up_ok = 1; }
  if (e < s.nu) st.up_ok = 0; else st.dn_ok = 0;
  post = sched_after(s, st.q);
}

static hipError_t multi_refresh(qmc_multi* m, unsigned mask) {
  for (int k = 0; k < m->n; ++k) {
    if (!((mask >> k) & 1u)) continue;
    hipError_t r = launch_lu_inverse(m->h_sys[k], m->h_wk[k], m->own);
    if (r == hipSuccess) r = launch_refresh_finish(m->h_sys[k], m->h_wk[k], nullptr, m->own);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

static hipError_t multi_enqueue(qmc_multi* m, int n_steps, bool explicit_draws, unsigned long long seed,
                                double sigma, std::vector<MemberState>& st) {
  MultiArgs a{m->d_sys, m->d_wk, m->d_steps, m->d_rows, explicit_draws ? m->d_disp : nullptr,
              explicit_draws ? m->d_unif : nullptr, 0, seed, sigma};
  for (int t = 0; t < n_steps; ++t) {
    a.t = t;
    unsigned pre_mask = 0, post_mask = 0;
    for (int k = 0; k < m->n; ++k) {
      int pb;
      bool pre, post;
      plan_member(m->h_sys[k], st[k], pb, pre, post);
      if (pb) {
        const SysDev& sk = m->h_sys[k];
        const WalkDev& wkd = m->h_wk[k];
        hipError_t r;
        if (sk.screened()) {   // the refined rows with their transposes and column maxima
          r = launch_P_build_oz(sk, wkd, pb, (const double*)wkd.phi, (double*)wkd.P, nullptr, false, m->own, false,
                                wkd.PT, 0);
          if (r == hipSuccess) r = launch_screen_colmax(sk, wkd, pb, m->own);
        } else {
          r = launch_P_build(sk, wkd, pb, m->own);
        }
        if (r != hipSuccess) return r;
      }
      if (pre) pre_mask |= 1u << k;
      if (post) post_mask |= 1u << k;
    }
    // refreshes: the one-system LU per member, so results match a lone run bitwise
    hipError_t r = multi_refresh(m, pre_mask);
    if (r == hipSuccess) r = launch_multi_prep(a, m->d_items, m->n_items, m->grid_items, m->own);
    if (r == hipSuccess)
      r = launch_multi_rows(a, m->store, m->nc, m->d_rows_items, m->n_rows_items, m->grid_rows, m->own, m->scr_lds);
    if (r == hipSuccess) r = launch_multi_accept(a, m->store, m->d_items, m->n_items, m->grid_items, m->own);
    if (r == hipSuccess) r = multi_refresh(m, post_mask);
    if (r == hipSuccess) r = launch_multi_advance(m->d_steps, m->n, m->own);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

extern "C" qmc_status qmc_multi_vmc_steps(qmc_multi* m, int32_t n_steps, const double* const* disp,
                                          const double* const* unif, uint64_t seed, double sigma, int32_t use_graph,
                                          hipStream_t stream) {
  if (!m) return fail(QMC_ERR_ARG, "null group");
  if (n_steps < 0) return fail(QMC_ERR_ARG, "negative step count");
  if ((disp == nullptr) != (unif == nullptr)) return fail(QMC_ERR_ARG, "give both draw arrays or neither");
  const bool expl = disp != nullptr;
  if (expl && use_graph) return fail(QMC_ERR_ARG, "graphs are built for the Philox draws");
  for (int k = 0; k < m->n; ++k) {
    qmc_walkers* w = m->wk[k];
    if (!w->evaluated) return fail(QMC_ERR_STATE, "member not evaluated");
    if (w->generation != m->sys[k]->generation) return fail(QMC_ERR_STATE, "member parameters changed");
    if (w->pending_e >= 0) return fail(QMC_ERR_STATE, "member has a pending proposal");
    if (expl && (!disp[k] || !unif[k])) return fail(QMC_ERR_ARG, "null draw array");
  }
  if (n_steps == 0) return QMC_OK;
  for (int k = 0; k < m->n; ++k) m->wk[k]->yt_valid = m->wk[k]->lr_ready = false;
  HIP_TRY(hipEventRecord(m->ev_a, stream), "event");
  HIP_TRY(hipStreamWaitEvent(m->own, m->ev_a, 0), "wait");
  HIP_TRY(multi_upload(m), "upload");
  if (expl) {
    m->h_disp.assign(disp, disp + m->n);
    m->h_unif.assign(unif, unif + m->n);
    HIP_TRY(hipMemcpyAsync(m->d_disp, m->h_disp.data(), sizeof(double*) * m->n, hipMemcpyHostToDevice, m->own), "ptrs");
    HIP_TRY(hipMemcpyAsync(m->d_unif, m->h_unif.data(), sizeof(double*) * m->n, hipMemcpyHostToDevice, m->own), "ptrs");
  }
  std::vector<MemberState> st(m->n);
  for (int k = 0; k < m->n; ++k) {
    const qmc_walkers* w = m->wk[k];
    st[k] = MemberState{Sched{w->attempts, w->since, w->buf_spin}, (char)w->P_up_valid, (char)w->P_dn_valid};
  }
  if (use_graph) {
    // the captured schedule is determined by each member's electron phase,
    // refresh state and valid P halves
    std::string key = std::to_string(n_steps) + ":" + std::to_string(seed) + ":" + std::to_string(sigma) + ":" +
                      std::to_string(m->grid_rows);
    for (int k = 0; k < m->n; ++k) {
      const SysDev& s = m->h_sys[k];
      key += ":" + std::to_string(st[k].q.attempts % s.N) + "," + std::to_string(st[k].q.since) + "," +
             std::to_string(st[k].q.buf_spin) + "," + std::to_string((int)st[k].up_ok) +
             std::to_string((int)st[k].dn_ok) + "," + std::to_string(m->rows[k]);
    }
    std::vector<MemberState> st2 = st;
    if (!m->gexec || key != m->gkey) {
      if (m->gexec) { (void)hipGraphExecDestroy(m->gexec); m->gexec = nullptr; }
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(m->own, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t r = multi_enqueue(m, n_steps, false, seed, sigma, st2);
      hipError_t r2 = hipStreamEndCapture(m->own, &g);
      if (r != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(r, "capture"); }
      HIP_TRY(r2, "end capture");
      r = hipGraphInstantiate(&m->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP_TRY(r, "instantiate");
      m->gkey = key;
    } else {
      // replay: the schedule is the captured one; advance the host state the same way
      for (int t = 0; t < n_steps; ++t)
        for (int k = 0; k < m->n; ++k) {
          int pb;
          bool pre, post;
          plan_member(m->h_sys[k], st2[k], pb, pre, post);
        }
    }
    HIP_TRY(hipGraphLaunch(m->gexec, m->own), "graph launch");
    st = st2;
  } else {
    HIP_TRY(multi_enqueue(m, n_steps, expl, seed, sigma, st), "multi steps");
  }
  for (int k = 0; k < m->n; ++k) {
    qmc_walkers* w = m->wk[k];
    w->attempts = st[k].q.attempts;
    w->since = st[k].q.since;
    w->buf_spin = st[k].q.buf_spin;
    w->P_up_valid = st[k].up_ok;
    w->P_dn_valid = st[k].dn_ok;
  }
  HIP_TRY(hipEventRecord(m->ev_b, m->own), "event");
  HIP_TRY(hipStreamWaitEvent(stream, m->ev_b, 0), "wait");
  return QMC_OK;
}

extern "C" qmc_status qmc_multi_autotune(qmc_multi* m, int32_t* rows_out, int32_t* grid_out, hipStream_t stream) {
  if (!m) return fail(QMC_ERR_ARG, "null group");
  for (int k = 0; k < m->n; ++k)
    if (!m->wk[k]->evaluated) return fail(QMC_ERR_STATE, "member not evaluated");
  HIP_TRY(hipStreamSynchronize(stream), "sync");
  HIP_TRY(multi_upload(m), "upload");
  MultiArgs a{m->d_sys, m->d_wk, m->d_steps, m->d_rows, nullptr, nullptr, 0, 12345ULL, 0.3};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "event");
  HIP_TRY(hipEventCreate(&e1), "event");
  const int cand_rows[3] = {8, 16, 32};
  const int cand_grid[4] = {512, 1024, 2048, 4096};
  float best = 1e30f;
  int best_r = m->rows.empty() ? 16 : m->rows[0], best_g = m->grid_rows;
  hipError_t err = hipSuccess;
  for (int r : cand_rows) {
    for (int k = 0; k < m->n; ++k) m->rows[k] = r;
    err = multi_build_rows(m);
    if (err != hipSuccess) break;
    err = launch_multi_prep(a, m->d_items, m->n_items, m->grid_items, m->own);
    if (err != hipSuccess) break;
    for (int g : cand_grid) {
      const int grid = std::min(g, m->n_rows_items);
      err = launch_multi_rows(a, m->store, m->nc, m->d_rows_items, m->n_rows_items, grid, m->own, m->scr_lds);
      if (err == hipSuccess) err = hipEventRecord(e0, m->own);
      for (int rep = 0; rep < 5 && err == hipSuccess; ++rep)
        err = launch_multi_rows(a, m->store, m->nc, m->d_rows_items, m->n_rows_items, grid, m->own, m->scr_lds);
      if (err == hipSuccess) err = hipEventRecord(e1, m->own);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) break;
      if (ms < best) { best = ms; best_r = r; best_g = grid; }
    }
    if (err != hipSuccess) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(err, "autotune");
  for (int k = 0; k < m->n; ++k) m->rows[k] = best_r;
  HIP_TRY(multi_build_rows(m), "rows table");
  m->grid_rows = std::min(best_g, m->n_rows_items);
  if (m->gexec) { (void)hipGraphExecDestroy(m->gexec); m->gexec = nullptr; }
  if (rows_out) *rows_out = best_r;
  if (grid_out) *grid_out = m->grid_rows;
  return QMC_OK;
}

extern "C" qmc_status qmc_philox_draws(uint64_t seed, int32_t member, int32_t n_walkers, uint64_t step, double sigma,
                                       double* disp, double* unif, hipStream_t stream) {
  if (!disp || !unif || n_walkers <= 0 || member < 0) return fail(QMC_ERR_ARG, "bad argument");
  HIP_TRY(launch_philox_draws(seed, member, n_walkers, step, sigma, disp, unif, stream), "philox");
  return QMC_OK;
}
