// Host side of the C ABI declared in include/qmc.h: validation, device
// allocation of system and walker state, and the launch sequences of the
// evaluation, move and Metropolis calls.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

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
    if (!on) return hipSuccess;
    if (pending.size() >= 2048) {
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
  bool evaluated = false;
  bool P_up_valid = false, P_dn_valid = false;
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
#define TIMED(wk, id, st, expr, where)                    \
  do {                                                    \
    HIP_TRY((wk)->tm.begin((id), (st)), "timer begin");   \
    HIP_TRY((expr), where);                               \
    HIP_TRY((wk)->tm.end((st)), "timer end");             \
  } while (0)

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
  if (q.n_up != q.n_dn) return fail(QMC_ERR_UNSUPPORTED, "only n_up == n_dn is built");
  if (q.n_up > kLuMaxN) return fail(QMC_ERR_UNSUPPORTED, "n_up > 128 needs the blocked LU");
  if (q.precision != QMC_FP64 && q.precision != QMC_W_FP32)
    return fail(QMC_ERR_UNSUPPORTED, "precision not built");
  if (q.refresh_every < 1) return fail(QMC_ERR_ARG, "refresh_every must be >= 1");
  if (q.j1_form < 0 || q.j1_form > 2 || (q.j1_form && !q.j1_b)) return fail(QMC_ERR_ARG, "bad j1");
  if (q.j2_form < 0 || q.j2_form > 2) return fail(QMC_ERR_ARG, "bad j2 form");
  if (q.j2_form == 1 && (q.n_j2 != 2 || !q.j2)) return fail(QMC_ERR_ARG, "j2 form 1 needs 2 params");
  if (q.j2_form == 2 && (q.n_j2 != 8 || !q.j2)) return fail(QMC_ERR_ARG, "j2 form 2 needs 8 params");
  const int L = q.n_basis;
  std::vector<int> kind(L);
  for (int mu = 0; mu < L; ++mu) {
    if (q.radial && q.radial[mu] != 0) return fail(QMC_ERR_UNSUPPORTED, "only Gaussian functions are built");
    if (q.center[mu] < 0 || q.center[mu] >= q.n_nuc) return fail(QMC_ERR_ARG, "basis center out of range");
    const int l = q.l[mu], m = q.m[mu];
    if (l < 0 || l > 2) return fail(QMC_ERR_UNSUPPORTED, "l > 2 not built");
    if (m < 0 || m >= 2 * l + 1) return fail(QMC_ERR_ARG, "component index out of range");
    kind[mu] = (l == 0) ? 0 : (l == 1 ? 1 + m : 4 + m);
  }
  std::vector<int> cptr(q.n_nuc + 1, 0), cmu(L);
  for (int mu = 0; mu < L; ++mu) cptr[q.center[mu] + 1]++;
  for (int a = 0; a < q.n_nuc; ++a) cptr[a + 1] += cptr[a];
  {
    std::vector<int> fill(cptr.begin(), cptr.end() - 1);
    for (int mu = 0; mu < L; ++mu) cmu[fill[q.center[mu]]++] = mu;
  }
  auto* s = new qmc_system();
  SysDev& d = s->d;
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
  d.n_nuc = q.n_nuc; d.L = L; d.Lp = round_up(L, 32);
  d.nu = q.n_up; d.nd = q.n_dn; d.N = q.n_up + q.n_dn;
  d.j1_form = q.j1_form; d.j2_form = q.j2_form;
  for (int k = 0; k < 8; ++k) d.j2[k] = (q.j2 && k < q.n_j2) ? q.j2[k] : 0.0;
  d.precision = q.precision; d.refresh_every = q.refresh_every;
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
  if (!e) e = up((void**)&d.center, q.center, sizeof(int) * L);
  if (!e) e = up((void**)&d.kind, kind.data(), sizeof(int) * L);
  if (!e) e = up((void**)&d.zeta, q.zeta, sizeof(double) * L);
  if (!e) e = up((void**)&d.lam, lam.data(), sizeof(double) * lam.size());
  if (!e) e = up((void**)&d.lamT, lamT.data(), sizeof(double) * lamT.size());
  if (!e) e = up((void**)&d.cptr, cptr.data(), sizeof(int) * cptr.size());
  if (!e) e = up((void**)&d.cmu, cmu.data(), sizeof(int) * cmu.size());
  if (!e && q.precision == QMC_W_FP32) {
    std::vector<float> l32(lam.begin(), lam.end()), lT32(lamT.begin(), lamT.end());
    e = up((void**)&d.lam32, l32.data(), sizeof(float) * l32.size());
    if (!e) e = up((void**)&d.lamT32, lT32.data(), sizeof(float) * lT32.size());
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

extern "C" qmc_status qmc_walkers_create(qmc_system* sys, int32_t n_walkers, qmc_walkers** out) {
  if (!sys || !out) return fail(QMC_ERR_ARG, "null argument");
  if (n_walkers <= 0) return fail(QMC_ERR_ARG, "n_walkers must be positive");
  *out = nullptr;
  const SysDev& s = sys->d;
  auto* wk = new qmc_walkers();
  wk->sys = sys;
  WalkDev& d = wk->d;
  d.Wk = n_walkers;
  const size_t Wk = n_walkers, N = s.N, Lp = s.Lp;
  const size_t nmax = s.nu > s.nd ? s.nu : s.nd;
  const size_t esz = s.precision == QMC_W_FP32 ? sizeof(float) : sizeof(double);
  hipError_t e = hipSuccess;
  auto al = [&](void** p, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(p, bytes + 256);
    if (e == hipSuccess) {
      wk->allocs.push_back(*p);
      e = hipMemset(*p, 0, bytes + 256);
    }
  };
  al((void**)&d.r, sizeof(double) * Wk * N * 3);
  al(&d.phi, esz * Wk * N * Lp);
  al(&d.P, esz * Wk * N * Lp);
  al((void**)&d.W, sizeof(double) * Wk * s.nu * s.nd);
  al((void**)&d.A, sizeof(double) * Wk * s.nd * s.nu);
  al((void**)&d.Yt, sizeof(double) * Wk * N * Lp);
  al((void**)&d.D, sizeof(double) * Wk * N * 4);
  al((void**)&d.logdet, sizeof(double) * Wk);
  al((void**)&d.detsign, sizeof(double) * Wk);
  al((void**)&d.singular, sizeof(int) * Wk);
  al((void**)&d.logabs, sizeof(double) * Wk);
  al((void**)&d.sign, sizeof(double) * Wk);
  al((void**)&d.J, sizeof(double) * Wk);
  al((void**)&d.psi_new, sizeof(double) * Wk * Lp);
  al((void**)&d.w_new, sizeof(double) * Wk * nmax);
  al((void**)&d.rdet, sizeof(double) * Wk);
  al((void**)&d.dJ, sizeof(double) * Wk);
  al((void**)&d.r_new, sizeof(double) * Wk * 3);
  al((void**)&d.ratio, sizeof(double) * Wk);
  al((void**)&d.acc, sizeof(uint8_t) * Wk);
  const size_t S = propose_splits(s);
  al((void**)&d.rdet_part, sizeof(double) * Wk * S);
  al((void**)&d.gdet_part, sizeof(double) * Wk * S * 3);
  al((void**)&d.gJ_new, sizeof(double) * Wk * 3);
  al((void**)&d.gpsi_new, sizeof(double) * Wk * 3 * Lp);
  al((void**)&d.gJ, sizeof(double) * Wk * N * 4);
  al((void**)&d.drift, sizeof(double) * Wk * N * 3);
  if (e != hipSuccess) {
    delete wk;
    return e == hipErrorOutOfMemory ? fail(QMC_ERR_OOM, "device allocation failed") : hip_fail(e, "walkers_create");
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
  if (!r) return fail(QMC_ERR_ARG, "null positions");
  const SysDev& s = sys->d;
  WalkDev& d = wk->d;
  HIP_TRY(hipMemcpyAsync(d.r, r, sizeof(double) * d.Wk * s.N * 3, hipMemcpyDeviceToDevice, stream), "copy r");
  TIMED(wk, QMC_T_BASIS, stream, launch_basis_values(s, d, stream), "basis");
  TIMED(wk, QMC_T_P_BUILD, stream, launch_P_build(s, d, 3, stream), "P build");
  TIMED(wk, QMC_T_W_BUILD, stream, launch_W_build(s, d, stream), "W build");
  TIMED(wk, QMC_T_LU, stream, launch_lu_inverse(s, d, stream), "LU");
  TIMED(wk, QMC_T_Y_BUILD, stream, launch_Y_build(s, d, stream), "Y build");
  TIMED(wk, QMC_T_ROWDOT, stream, launch_rowdots(s, d, stream), "row dots");
  TIMED(wk, QMC_T_ASSEMBLE, stream,
        launch_jastrow_assemble(s, d, logabs, sign, drift, e_kin, e_loc, status, stream), "assemble");
  wk->evaluated = true;
  wk->generation = sys->generation;
  wk->P_up_valid = wk->P_dn_valid = true;
  wk->attempts = 0;
  wk->pending_e = -1;
  return QMC_OK;
}

// P rows of the spin opposite to electron e must match the current basis rows.
static qmc_status ensure_P(qmc_walkers* wk, int e, hipStream_t stream) {
  const SysDev& s = wk->sys->d;
  const bool up = e < s.nu;
  if (up && !wk->P_dn_valid) {
    TIMED(wk, QMC_T_P_BUILD, stream, launch_P_build(s, wk->d, 2, stream), "P_dn rebuild");
    wk->P_dn_valid = true;
  } else if (!up && !wk->P_up_valid) {
    TIMED(wk, QMC_T_P_BUILD, stream, launch_P_build(s, wk->d, 1, stream), "P_up rebuild");
    wk->P_up_valid = true;
  }
  return QMC_OK;
}

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
  c = ensure_P(wk, electron, stream);
  if (c) return c;
  TIMED(wk, QMC_T_PROPOSE_PREP, stream,
        launch_propose_prep(s, wk->d, electron, r_new, nullptr, drift_new != nullptr, stream), "propose prep");
  TIMED(wk, QMC_T_PROPOSE, stream, launch_propose_rows(s, wk->d, electron, ratio, drift_new, true, stream),
        "propose rows");
  wk->pending_e = electron;
  return QMC_OK;
}

static qmc_status after_accept(qmc_walkers* wk, int e, int32_t* status, hipStream_t stream) {
  const SysDev& s = wk->sys->d;
  if (e < s.nu) wk->P_up_valid = false; else wk->P_dn_valid = false;
  wk->pending_e = -1;
  wk->attempts += 1;
  if (wk->attempts % s.refresh_every == 0) {
    TIMED(wk, QMC_T_LU, stream, launch_lu_inverse(s, wk->d, stream), "refresh LU");
    TIMED(wk, QMC_T_OTHER, stream, launch_refresh_finish(s, wk->d, status, stream), "refresh finish");
  }
  return QMC_OK;
}

extern "C" qmc_status qmc_accept_move(qmc_system* sys, qmc_walkers* wk, int32_t electron,
                                      const uint8_t* accept, int32_t* status, hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!accept) return fail(QMC_ERR_ARG, "null accept");
  if (wk->pending_e < 0 || wk->pending_e != electron)
    return fail(QMC_ERR_STATE, "no pending proposal for this electron");
  TIMED(wk, QMC_T_ACCEPT, stream, launch_accept(sys->d, wk->d, electron, accept, stream), "accept");
  return after_accept(wk, electron, status, stream);
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
  const long Wk = wk->d.Wk;
  for (int t = 0; t < n_steps; ++t) {
    const int e = (int)((e_start + (long)t) % s.N);
    c = ensure_P(wk, e, stream);
    if (c) return c;
    TIMED(wk, QMC_T_PROPOSE_PREP, stream,
          launch_propose_prep(s, wk->d, e, nullptr, disp + (long)t * Wk * 3, false, stream), "propose prep");
    TIMED(wk, QMC_T_PROPOSE, stream, launch_propose_rows(s, wk->d, e, nullptr, nullptr, false, stream),
          "propose rows");
    TIMED(wk, QMC_T_ACCEPT, stream,
          launch_metropolis_accept(s, wk->d, e, unif + (long)t * Wk, accept_count, stream), "metropolis");
    c = after_accept(wk, e, nullptr, stream);
    if (c) return c;
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
    case QMC_STATE_W: src = d.W; bytes = sizeof(double) * Wk * s.nu * s.nd; break;
    case QMC_STATE_AINV: src = d.A; bytes = sizeof(double) * Wk * s.nd * s.nu; break;
    case QMC_STATE_PHI:
      HIP_TRY(launch_export_phi(s, d, dst, stream), "export phi");
      return QMC_OK;
    default: return fail(QMC_ERR_ARG, "unknown state item");
  }
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream), "read state");
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_set_timing(qmc_walkers* wk, int32_t enable) {
  if (!wk) return fail(QMC_ERR_ARG, "null walkers");
  HIP_TRY(wk->tm.fold(), "timer fold");
  for (int k = 0; k < QMC_TIMER_COUNT; ++k) { wk->tm.ms[k] = 0.0; wk->tm.n[k] = 0; }
  wk->tm.on = enable != 0;
  return QMC_OK;
}

extern "C" qmc_status qmc_walkers_timing(qmc_walkers* wk, double* ms, int64_t* launches) {
  if (!wk || !ms || !launches) return fail(QMC_ERR_ARG, "null argument");
  HIP_TRY(wk->tm.fold(), "timer fold");
  for (int k = 0; k < QMC_TIMER_COUNT; ++k) { ms[k] = wk->tm.ms[k]; launches[k] = wk->tm.n[k]; }
  return QMC_OK;
}

// Allocate the reverse-pass workspace of a walker set (first qmc_forces call).
static hipError_t alloc_adjoint(qmc_walkers* wk) {
  if (wk->aw_ready) return hipSuccess;
  const SysDev& s = wk->sys->d;
  const size_t Wk = wk->d.Wk, n = s.nu, Lp = s.Lp, L = s.L, N = s.N, A = s.n_nuc;
  const size_t nj = A + (s.j2_form == 1 ? 2 : (s.j2_form == 2 ? 8 : 0));
  AdjWork& a = wk->aw;
  a.chunk_walkers = (int)((Wk + 63) / 64);
  a.chunks = (int)((Wk + a.chunk_walkers - 1) / a.chunk_walkers);
  hipError_t e = hipSuccess;
  auto al = [&](double** p, size_t count) {
    if (e != hipSuccess) return;
    e = hipMalloc((void**)p, count * sizeof(double) + 256);
    if (e == hipSuccess) {
      wk->allocs.push_back(*p);
      e = hipMemset(*p, 0, count * sizeof(double) + 256);
    }
  };
  al(&a.SU, Wk * 2 * n * Lp);
  al(&a.SD, Wk * 2 * n * Lp);
  al(&a.VQ, Wk * n * n);
  al(&a.T1, Wk * n * n);
  al(&a.M, Wk * n * n);
  al(&a.GG, Wk * 2 * n * n);
  al(&a.GGt, Wk * 2 * n * n);
  al(&a.XZ, Wk * 2 * n * Lp);
  al(&a.XD, Wk * n * Lp);
  al(&a.PB, Wk * N * Lp);
  al(&a.tmu, Wk * L * 3);
  al(&a.Rbar, Wk * A * 3);
  al(&a.zbar, Wk * L);
  al(&a.jbar, Wk * nj);
  al(&a.dr, Wk * N * 3);
  al(&a.lam_part, (size_t)a.chunks * L * L);
  if (e == hipSuccess) wk->aw_ready = true;
  return e;
}

extern "C" qmc_status qmc_forces(qmc_system* sys, qmc_walkers* wk, const double* r, int32_t per_walker,
                                 const double* gbar_logpsi, const double* gbar_eloc, const qmc_grads* out,
                                 hipStream_t stream) {
  qmc_status c = check_pair(sys, wk);
  if (c) return c;
  if (!r || !out) return fail(QMC_ERR_ARG, "null positions or output block");
  const SysDev& s = sys->d;
  if (s.precision != QMC_FP64) return fail(QMC_ERR_UNSUPPORTED, "forces are built for the FP64 path");
  if (s.N > 2 * kLuMaxN || s.n_nuc > kMaxNucBack)
    return fail(QMC_ERR_UNSUPPORTED, "forces need N <= 256 electrons and <= 256 nuclei");
  hipError_t e = alloc_adjoint(wk);
  if (e != hipSuccess)
    return e == hipErrorOutOfMemory ? fail(QMC_ERR_OOM, "adjoint workspace allocation failed") : hip_fail(e, "forces workspace");
  c = qmc_eval_batch(sys, wk, r, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, stream);
  if (c) return c;
  HIP_TRY(launch_forces(s, wk->d, wk->aw, gbar_logpsi, gbar_eloc, per_walker, out->dR, out->dzeta,
                        out->dlambda, out->djas, out->dr, stream), "forces");
  return QMC_OK;
}

extern "C" qmc_status qmc_system_set_params(qmc_system* sys, const double* R, const double* zeta,
                                            const double* lambda, const double* jas, hipStream_t stream) {
  if (!sys) return fail(QMC_ERR_ARG, "null system");
  SysDev& d = sys->d;
  if (R) HIP_TRY(hipMemcpyAsync(d.R, R, sizeof(double) * 3 * d.n_nuc, hipMemcpyDeviceToDevice, stream), "set R");
  if (zeta) HIP_TRY(hipMemcpyAsync(d.zeta, zeta, sizeof(double) * d.L, hipMemcpyDeviceToDevice, stream), "set zeta");
  if (lambda) HIP_TRY(launch_set_lambda(d, lambda, stream), "set lambda");
  if (jas) {
    HIP_TRY(hipMemcpyAsync(d.j1_b, jas, sizeof(double) * d.n_nuc, hipMemcpyDeviceToDevice, stream), "set j1");
    const int n2 = d.j2_form == 1 ? 2 : (d.j2_form == 2 ? 8 : 0);
    if (n2) {
      double h[8];
      HIP_TRY(hipMemcpyAsync(h, jas + d.n_nuc, sizeof(double) * n2, hipMemcpyDeviceToHost, stream), "get j2");
      HIP_TRY(hipStreamSynchronize(stream), "sync j2");
      for (int k = 0; k < n2; ++k) d.j2[k] = h[k];
    }
  }
  sys->generation += 1;
  return QMC_OK;
}
