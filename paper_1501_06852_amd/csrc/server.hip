// Continuous-batching server for PFC Rosenbrock requests.
//
// A library-owned thread keeps the active requests resident on the GPU: each
// active request owns an instance (its matrices, Krylov basis and state stay
// in HBM for the life of the request) and a team of workgroups in the solver
// launch.  Every replay of the captured launch graph advances all active
// requests by a fixed number of phases; between replays finished requests are
// retired (state copied to the host, instance returned to a pool) and pending
// requests are admitted while a slot is free and their footprint fits the
// memory budget.  Requests that join do not disturb the ones in flight: their
// state machines simply continue with a rebuilt team table.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "host.h"
#include "solver.h"

namespace pfc {

struct Request {
  uint64_t id = 0;
  pfc_mesh* mesh = nullptr;
  double r = 0, psibar = 0, tau = 0;
  std::vector<double> psi0;
  int n_steps = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  pfc_instance* inst = nullptr;
  int status = PFC_OK;
  bool fresh = false;
  double* state_out = nullptr;
  pfc_solve_info* infos_out = nullptr;
};

}  // namespace pfc

using namespace pfc;

struct pfc_server {
  pfc_server_opts o{};
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_idle;
  std::deque<Request*> pending;
  std::vector<Request*> active;
  std::deque<Request*> done;
  std::vector<pfc_instance*> pool;
  size_t used = 0;
  bool stop = false;
  int device = 0;
  hipStream_t stream = nullptr;
  Group grp;
  std::chrono::steady_clock::time_point t0;
  int error = PFC_OK;
  long long resident_rows = 0;  // rows one round of resident workgroups covers (CUs x workgroup size)
  std::string error_msg;  // pfc_last_error() of the server thread at the error
  double clock() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

pfc_opts server_instance_opts(const pfc_server* S, const pfc_mesh* m, int rpt) {
  pfc_opts o;
  pfc_opts_default(&o);
  o.precision = S->o.precision;
  o.ticks_per_graph = S->o.ticks_per_graph;
  o.rows_per_thread = rpt;
  // a request shares its launches with whichever requests are resident, and the
  // set changes between launches while it runs.  The 2D block form of two PCG
  // iterations per launch runs in any launch set (every launch that holds such
  // an instance has it) and gives the same bits in any of them; the other
  // two-iteration forms need launches that serve the instance alone, so those
  // requests run one iteration per launch, which is valid in every launch set.
  // A server with a single slot runs every request alone and keeps every form.
  o.pcg_steps_per_launch = (S->o.max_slots == 1 || block_form_applies(m, o)) ? 2 : 1;
  return o;
}

// Rows per thread of a request's instance.  Fixed by the server options, or
// (0) taken from the autotuning table's entry for mixed batches of the number
// of active requests including this one (option `tuned`, where the table has
// such an entry), or else chosen at admission from the load: one row per thread while the active
// requests and this one fit into one round of resident workgroups (the
// shortest time per request), two once they do not (fewer, longer
// workgroups: more throughput when the GPU is full).
int choose_rpt(const pfc_server* S, const Request* q) {
  if (S->o.rows_per_thread > 0) return S->o.rows_per_thread;
  // requests that take the 2D block form at one row per thread keep it
  if (S->o.max_slots > 1 && block_form_applies(q->mesh, server_instance_opts(S, q->mesh, 1))) return 1;
  if (S->o.tuned) {
    const int t = tuned_mix_rows_per_thread(S->o.precision, (int)S->active.size() + 1);
    if (t > 0) return t;
  }
  long long rows = q->mesh->n;
  for (const Request* a : S->active) rows += a->mesh->n;
  return rows > S->resident_rows ? 2 : 1;
}

// take an instance for req: reuse a pooled one on the same mesh, else create
// one within the budget (evicting pooled instances if needed)
int acquire(pfc_server* S, Request* q, bool& ok) {
  ok = false;
  const int rpt = choose_rpt(S, q);
  for (size_t k = 0; k < S->pool.size(); ++k)
    if (S->pool[k]->mesh == q->mesh && S->pool[k]->opts.rows_per_thread == rpt) {
      q->inst = S->pool[k];
      S->pool.erase(S->pool.begin() + k);
      ok = true;
      return PFC_OK;
    }
  pfc_opts o = server_instance_opts(S, q->mesh, rpt);
  const size_t need = pfc_instance_footprint(q->mesh, &o);
  while (S->used + need > S->o.hbm_budget && !S->pool.empty()) {
    pfc_instance* v = S->pool.back();
    S->pool.pop_back();
    S->used -= v->bytes;
    pfc_instance_destroy(v);
  }
  if (S->used + need > S->o.hbm_budget) return PFC_OK;  // wait for retirements
  pfc_instance* I = nullptr;
  int rc = pfc_instance_create(q->mesh, &o, &I);
  if (rc) return rc;
  S->used += I->bytes;
  q->inst = I;
  ok = true;
  return PFC_OK;
}

int start_request(pfc_server* S, Request* q) {
  pfc_instance* I = q->inst;
  InstDev& h = I->h;
  const int n = I->mesh->n;
  std::vector<double> st((size_t)3 * n, 0.0);
  std::copy(q->psi0.begin(), q->psi0.end(), st.begin() + n);
  PFC_HIP(hipMemcpy(h.xk, st.data(), sizeof(double) * st.size(), hipMemcpyHostToDevice));
  int rcm = set_mobility_mean(I, h.xk + n, S->stream);
  if (rcm) return rcm;
  set_params(h, q->r, q->tau, 1.0 / ROS_GAMMA);
  h.replay = 0;
  h.job = JOB_RB;
  h.n_steps = q->n_steps;
  h.init_mode = PFC_INIT_CONSISTENT;
  // per-tau operator values
  int rc = prep_ops_public(I, S->stream);
  if (rc) return rc;
  q->fresh = true;
  return PFC_OK;
}

int retire(pfc_server* S, Request* q) {
  pfc_instance* I = q->inst;
  const int n = I->mesh->n;
  q->state_out = (double*)std::malloc(sizeof(double) * 3 * (size_t)n);
  q->infos_out = (pfc_solve_info*)std::calloc((size_t)std::max(1, 3 * q->n_steps), sizeof(pfc_solve_info));
  if (!q->state_out || !q->infos_out) return PFC_ERR_OOM;
  PFC_HIP(hipMemcpy(q->state_out, I->h.xk, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToHost));
  std::vector<InfoDev> f((size_t)3 * q->n_steps);
  if (!f.empty()) PFC_HIP(hipMemcpy(f.data(), I->h.info, sizeof(InfoDev) * f.size(), hipMemcpyDeviceToHost));
  State fin;
  PFC_HIP(hipMemcpy(&fin, I->h.st, sizeof(State), hipMemcpyDeviceToHost));
  int worst = fin.status < 0 ? fin.status : PFC_OK;
  for (size_t k = 0; k < f.size(); ++k) {
    fill_info(&q->infos_out[k], f[k]);
    if (f[k].status < 0) worst = f[k].status;
    else if (worst >= 0 && f[k].status > worst) worst = f[k].status;
  }
  q->status = worst;
  S->pool.push_back(I);
  q->inst = nullptr;
  return PFC_OK;
}

int rebuild(pfc_server* S) {
  S->grp.release();
  if (S->active.empty()) return PFC_OK;
  std::vector<int> ts;
  for (Request* q : S->active) ts.push_back(q->inst->team_size);
  int rc = S->grp.alloc(ts);
  if (rc) return rc;
  for (size_t i = 0; i < S->active.size(); ++i) S->grp.h_descs[i] = S->active[i]->inst->h;
  const int ticks = S->o.ticks_per_graph > 0 ? S->o.ticks_per_graph : 64;
  rc = S->grp.build(S->active[0]->inst->capture, S->o.precision, ticks + (ticks & 1));
  if (rc) return rc;
  PFC_HIP(hipMemcpyAsync(S->grp.d_descs, S->grp.h_descs, sizeof(InstDev) * S->active.size(), hipMemcpyHostToDevice,
                         S->stream));
  // only requests that just joined start from PH_START; the others continue
  for (size_t i = 0; i < S->active.size(); ++i) {
    Request* q = S->active[i];
    if (!q->fresh) continue;
    State st;
    std::memset(&st, 0, sizeof(st));
    st.phase = PH_START;
    st.job = JOB_RB;
    S->grp.h_states[i] = st;
    PFC_HIP(hipMemcpyAsync(q->inst->h.st, S->grp.h_states + i, sizeof(State), hipMemcpyHostToDevice, S->stream));
    q->fresh = false;
  }
  PFC_HIP(hipStreamSynchronize(S->stream));
  return PFC_OK;
}

// the loop stops after an error; callers read the code under the mutex
void fail(pfc_server* S, int code) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->error = code;
  S->error_msg = pfc_last_error();
}

// report the server's error to the calling thread (caller holds the mutex)
int server_error(const pfc_server* S) {
  if (S->error) set_error("server stopped after an error: " + S->error_msg);
  return S->error;
}

void loop(pfc_server* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    bool changed = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop) break;
      if (S->active.empty() && S->pending.empty()) {
        S->cv_idle.notify_all();
        S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        if (S->stop) break;
      }
      while (!S->pending.empty() && (int)S->active.size() < S->o.max_slots) {
        Request* q = S->pending.front();
        bool ok = false;
        int rc = acquire(S, q, ok);
        if (!rc && ok) rc = start_request(S, q);
        if (rc) {
          q->status = rc;
          q->t_admit = q->t_done = S->clock();
          q->state_out = nullptr;
          S->pending.pop_front();
          S->done.push_back(q);
          continue;
        }
        if (!ok) break;
        S->pending.pop_front();
        q->t_admit = S->clock();
        S->active.push_back(q);
        changed = true;
      }
    }
    if (changed && rebuild(S)) { fail(S, PFC_ERR_HIP); break; }
    if (S->active.empty()) continue;
    if (hipGraphLaunch(S->grp.exec, S->stream) != hipSuccess || hipStreamSynchronize(S->stream) != hipSuccess) {
      fail(S, PFC_ERR_HIP);
      break;
    }
    // finished requests move to `done`; every other one (also one whose
    // retirement failed) stays in `active`, so each request sits in exactly
    // one list and pfc_server_destroy frees it once
    std::vector<Request*> still;
    bool retired = false;
    int err = PFC_OK;
    for (size_t i = 0; i < S->active.size(); ++i) {
      Request* q = S->active[i];
      if (!err && ((volatile int*)S->grp.h_flags)[i] == PH_DONE) {
        const int rc = retire(S, q);
        if (rc) { err = rc; still.push_back(q); continue; }
        q->t_done = S->clock();
        std::lock_guard<std::mutex> lk(S->mu);
        S->done.push_back(q);
        retired = true;
      } else {
        still.push_back(q);
      }
    }
    if (retired || err) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->active.swap(still);
    }
    if (err) { fail(S, err); break; }
    if (retired && rebuild(S)) { fail(S, PFC_ERR_HIP); break; }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->cv_idle.notify_all();
}

}  // namespace

extern "C" {

int pfc_server_create(const pfc_server_opts* o, pfc_server** out) {
  if (!o || !out || o->struct_size != (int)sizeof(pfc_server_opts) || o->max_slots < 1 || o->hbm_budget == 0 ||
      (o->precision != PFC_FP64 && o->precision != PFC_MIXED) || o->ticks_per_graph < 0 || o->ticks_per_graph > 4096 ||
      o->rows_per_thread < 0 || o->rows_per_thread > 8 || (o->tuned != 0 && o->tuned != 1)) {
    set_error("pfc_server_create: invalid options");
    return PFC_ERR_ARG;
  }
  *out = nullptr;
  pfc_server* S = new pfc_server();
  S->o = *o;
  S->t0 = std::chrono::steady_clock::now();
  int cus = 0;
  if (hipGetDevice(&S->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device) != hipSuccess ||
      hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
    delete S;
    set_error("pfc_server_create: HIP setup failed");
    return PFC_ERR_HIP;
  }
  S->resident_rows = (long long)cus * PFC_WG;
  S->th = std::thread(loop, S);
  *out = S;
  return PFC_OK;
}

int pfc_server_submit(pfc_server* S, pfc_mesh* mesh, double r, double psibar, double tau, const double* psi0,
                      int n_steps, uint64_t req_id) {
  if (!S || !mesh || !psi0 || n_steps < 1 || !(tau > 0.0) || !std::isfinite(tau) || !std::isfinite(r) ||
      !std::isfinite(psibar)) {
    set_error("pfc_server_submit: invalid arguments");
    return PFC_ERR_ARG;
  }
  pfc_opts o = server_instance_opts(S, mesh, 1);  // the largest team: an upper bound of the footprint
  if (n_steps > o.max_run_steps) { set_error("pfc_server_submit: too many steps"); return PFC_ERR_ARG; }
  if (pfc_instance_footprint(mesh, &o) > S->o.hbm_budget) {
    set_error("pfc_server_submit: request footprint exceeds the server's memory budget");
    return PFC_ERR_ADMISSION;
  }
  Request* q = new Request();
  q->id = req_id; q->mesh = mesh; q->r = r; q->psibar = psibar; q->tau = tau; q->n_steps = n_steps;
  q->psi0.assign(psi0, psi0 + mesh->n);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error) { delete q; return server_error(S); }
    q->t_submit = S->clock();
    S->pending.push_back(q);
  }
  S->cv_work.notify_one();
  return PFC_OK;
}

int pfc_server_poll(pfc_server* S, pfc_result* out, int max, int* n_out) {
  if (!S || !out || max < 0 || !n_out) { set_error("pfc_server_poll: invalid arguments"); return PFC_ERR_ARG; }
  std::lock_guard<std::mutex> lk(S->mu);
  int k = 0;
  while (k < max && !S->done.empty()) {
    Request* q = S->done.front();
    S->done.pop_front();
    pfc_result& r = out[k++];
    r.req_id = q->id; r.status = q->status; r.n_stages = 3 * q->n_steps;
    r.t_submit = q->t_submit; r.t_admit = q->t_admit; r.t_done = q->t_done;
    r.state = q->state_out; r.infos = q->infos_out;
    delete q;
  }
  *n_out = k;
  return server_error(S);
}

void pfc_result_free(pfc_result* r) {
  if (!r) return;
  std::free(r->state);
  std::free(r->infos);
  r->state = nullptr;
  r->infos = nullptr;
}

int pfc_server_drain(pfc_server* S) {
  if (!S) { set_error("pfc_server_drain: null server"); return PFC_ERR_ARG; }
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_idle.wait(lk, [&] { return S->error || (S->pending.empty() && S->active.empty()); });
  return server_error(S);
}

double pfc_server_clock(const pfc_server* S) { return S ? S->clock() : 0.0; }

void pfc_server_destroy(pfc_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->th.joinable()) S->th.join();
  S->grp.release();
  for (Request* q : S->active) {
    if (q->inst) pfc_instance_destroy(q->inst);
    std::free(q->state_out);
    std::free(q->infos_out);
    delete q;
  }
  for (Request* q : S->pending) delete q;
  for (Request* q : S->done) { std::free(q->state_out); std::free(q->infos_out); delete q; }
  for (pfc_instance* I : S->pool) pfc_instance_destroy(I);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
