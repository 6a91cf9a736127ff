// Autotuner of the solver's launch configuration.
//
// The solver kernel's launch shape has knobs whose best values depend on the
// mesh, the precision and how many instances share a launch: rows per thread
// (team size), whether the columns of a periodic grid are computed or read,
// whether the M + c K operators are stored or formed on the fly, the PCG
// iterations per launch of a lone instance, and the launches captured per
// graph.  pfc_autotune times whole Rosenbrock steps of `count` instances on
// synthetic states for candidate configurations (coordinate descent from the
// defaults, one knob at a time) and keeps the fastest in a process-wide table
// keyed by (device architecture, dim, n, entries per row, precision, count).
// The table is read from and written to a JSON file.  pfc_batch_run takes its
// launches per graph from the table.  pfc_autotune_mix tunes one rows-per-thread
// value for batches that mix several meshes (key dim = n = z = 0): a server
// created with `tuned` gives every request it admits the value for the number
// of requests then active, since a launch lasts as long as its slowest
// workgroup and per-mesh choices that differ would leave some workgroups far
// longer than the rest.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"
#include "solver.h"

namespace pfc {

namespace {

std::mutex g_tune_mu;
std::vector<pfc_tune_entry> g_table;

bool same_key(const pfc_tune_entry& e, const char* arch, int dim, int n, int z, int precision) {
  return std::strncmp(e.arch, arch, sizeof(e.arch)) == 0 && e.dim == dim && e.n == n && e.z == z &&
         e.precision == precision;
}

// Entry for `count` instances: the largest tuned count <= count with the same
// key, or nullptr.  Caller holds g_tune_mu.
const pfc_tune_entry* find_entry(const char* arch, int dim, int n, int z, int precision, int count) {
  const pfc_tune_entry* best = nullptr;
  for (const pfc_tune_entry& e : g_table)
    if (same_key(e, arch, dim, n, z, precision) && e.count <= count && (!best || e.count > best->count)) best = &e;
  return best;
}

void put_entry(const pfc_tune_entry& e) {
  for (pfc_tune_entry& x : g_table)
    if (same_key(x, e.arch, e.dim, e.n, e.z, e.precision) && x.count == e.count) { x = e; return; }
  g_table.push_back(e);
}

int current_arch(char* out, size_t cap) {
  int d = 0;
  hipDeviceProp_t p;
  PFC_HIP(hipGetDevice(&d));
  PFC_HIP(hipGetDeviceProperties(&p, d));
  // the architecture without its feature suffixes ("gfx950:sramecc+:xnack-" -> "gfx950")
  std::string a(p.gcnArchName);
  a = a.substr(0, a.find(':'));
  std::snprintf(out, cap, "%s", a.c_str());
  return PFC_OK;
}

// entries per row of a mesh: the common slice width, else the mean rounded
int mesh_z(const pfc_mesh* m) {
  if (m->uniform_width > 0) return m->uniform_width;
  return m->n > 0 ? (int)std::lround((double)m->nnz / m->n) : 0;
}

// ---- the cache file: {"format": "pfc-tune-1", "entries": [ {flat object}, ... ]}
std::string entry_json(const pfc_tune_entry& e) {
  char b[512];
  std::snprintf(b, sizeof(b),
                "{\"arch\": \"%s\", \"dim\": %d, \"n\": %d, \"z\": %d, \"precision\": %d, \"count\": %d, "
                "\"rows_per_thread\": %d, \"ticks_per_graph\": %d, \"pcg_steps_per_launch\": %d, \"grid_columns\": %d, "
                "\"shared_ops\": %d, \"ms_per_step\": %.6g, \"ms_default\": %.6g, \"candidates\": %d}",
                e.arch, e.dim, e.n, e.z, e.precision, e.count, e.rows_per_thread, e.ticks_per_graph,
                e.pcg_steps_per_launch, e.grid_columns, e.shared_ops, e.ms_per_step, e.ms_default, e.candidates);
  return b;
}

// Parse the flat objects of the "entries" array.  Returns false on any syntax
// the writer above does not produce.
bool parse_cache(const std::string& s, std::vector<pfc_tune_entry>& out) {
  size_t p = s.find("\"entries\"");
  if (p == std::string::npos) return false;
  p = s.find('[', p);
  if (p == std::string::npos) return false;
  ++p;
  auto skip = [&]() { while (p < s.size() && std::isspace((unsigned char)s[p])) ++p; };
  for (;;) {
    skip();
    if (p >= s.size()) return false;
    if (s[p] == ']') return true;
    if (s[p] == ',') { ++p; continue; }
    if (s[p] != '{') return false;
    ++p;
    pfc_tune_entry e;
    std::memset(&e, 0, sizeof(e));
    e.struct_size = (int)sizeof(pfc_tune_entry);
    int seen = 0;
    for (;;) {
      skip();
      if (p >= s.size()) return false;
      if (s[p] == '}') { ++p; break; }
      if (s[p] == ',') { ++p; continue; }
      if (s[p] != '"') return false;
      const size_t k1 = s.find('"', p + 1);
      if (k1 == std::string::npos) return false;
      const std::string key = s.substr(p + 1, k1 - p - 1);
      p = s.find(':', k1);
      if (p == std::string::npos) return false;
      ++p;
      skip();
      if (p < s.size() && s[p] == '"') {
        const size_t v1 = s.find('"', p + 1);
        if (v1 == std::string::npos) return false;
        if (key == "arch") { std::snprintf(e.arch, sizeof(e.arch), "%s", s.substr(p + 1, v1 - p - 1).c_str()); ++seen; }
        p = v1 + 1;
      } else {
        const char* c0 = s.c_str() + p;
        char* c1 = nullptr;
        const double v = std::strtod(c0, &c1);
        if (c1 == c0) return false;
        p += (size_t)(c1 - c0);
        const int iv = (int)v;
        if (key == "dim") { e.dim = iv; ++seen; }
        else if (key == "n") { e.n = iv; ++seen; }
        else if (key == "z") { e.z = iv; ++seen; }
        else if (key == "precision") { e.precision = iv; ++seen; }
        else if (key == "count") { e.count = iv; ++seen; }
        else if (key == "rows_per_thread") e.rows_per_thread = iv;
        else if (key == "ticks_per_graph") e.ticks_per_graph = iv;
        else if (key == "pcg_steps_per_launch") e.pcg_steps_per_launch = iv;
        else if (key == "grid_columns") e.grid_columns = iv;
        else if (key == "shared_ops") e.shared_ops = iv;
        else if (key == "ms_per_step") e.ms_per_step = v;
        else if (key == "ms_default") e.ms_default = v;
        else if (key == "candidates") e.candidates = iv;
      }
    }
    if (seen != 6) return false;  // every key field present
    out.push_back(e);
  }
}

// Synthetic state of tuning instance k: psi = -0.3 + 0.01 (2u - 1) with u from
// SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", 2014) of the node's counter; mu, omega from consistent values.
double splitmix_u01(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  x ^= x >> 31;
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

struct Candidate {
  int rpt, ticks, pcg, grid, shared;
  bool operator==(const Candidate& o) const {
    return rpt == o.rpt && ticks == o.ticks && pcg == o.pcg && grid == o.grid && shared == o.shared;
  }
};

// Milliseconds of one Rosenbrock step of `count` instances with candidate c
// (best of two timed steps after a consistent initialisation and a warm-up
// step), or a negative status.
double time_candidate(pfc_mesh* const* ms, int n_meshes, int precision, int count, const Candidate& c, hipStream_t s,
                      int* status) {
  *status = PFC_OK;
  pfc_opts o;
  pfc_opts_default(&o);
  o.precision = precision;
  o.rows_per_thread = c.rpt;
  o.ticks_per_graph = c.ticks;
  o.pcg_steps_per_launch = c.pcg;
  o.grid_columns = c.grid;
  o.shared_ops = c.shared;
  o.max_run_steps = 4;
  // a mix is timed as the server runs it: instances that take the 2D block form
  // at one row per thread keep it, one iteration per launch for the others
  std::vector<pfc_opts> om(n_meshes, o);
  if (n_meshes > 1)
    for (int k = 0; k < n_meshes; ++k) {
      pfc_opts b = o;
      b.rows_per_thread = 1;
      b.pcg_steps_per_launch = 2;
      if (block_form_applies(ms[k], b)) om[k] = b;
      else om[k].pcg_steps_per_launch = 1;
    }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { *status = PFC_ERR_HIP; return -1; }
  double need = 0.0;
  for (int k = 0; k < count; ++k) {
    const size_t fp = pfc_instance_footprint(ms[k % n_meshes], &om[k % n_meshes]);
    if (fp == 0) { *status = PFC_ERR_ARG; return -1; }
    need += (double)fp;
  }
  if (need > 0.8 * (double)free_b) { *status = PFC_ERR_OOM; return -1; }
  std::vector<pfc_instance*> insts(count, nullptr);
  std::vector<double*> states(count, nullptr);
  std::vector<double> r(count, -0.35), pb(count, -0.3), tau(count, 0.5);
  int rc = PFC_OK;
  double best = 1e300;
  std::vector<double> h;
  for (int k = 0; k < count && !rc; ++k) {
    pfc_mesh* m = ms[k % n_meshes];
    const int n = m->n;
    rc = pfc_instance_create(m, &om[k % n_meshes], &insts[k]);
    if (rc) break;
    if (hipMalloc((void**)&states[k], sizeof(double) * 3 * (size_t)n) != hipSuccess) { rc = PFC_ERR_OOM; break; }
    h.assign((size_t)3 * n, 0.0);
    for (int i = 0; i < n; ++i) h[(size_t)n + i] = -0.3 + 0.01 * (2.0 * splitmix_u01((uint64_t)k * n + i) - 1.0);
    if (hipMemcpy(states[k], h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice) != hipSuccess) rc = PFC_ERR_HIP;
  }
  if (!rc) rc = pfc_batch_run(insts.data(), count, states.data(), r.data(), pb.data(), tau.data(), 0,
                              PFC_INIT_CONSISTENT, nullptr, s);
  for (int rep = 0; rep < 3 && rc >= 0; ++rep) {
    const auto t0 = std::chrono::steady_clock::now();
    if (count == 1) rc = pfc_rosenbrock_run(insts[0], states[0], r[0], pb[0], tau[0], 1, PFC_INIT_GIVEN, nullptr,
                                            nullptr, s);
    else rc = pfc_batch_run(insts.data(), count, states.data(), r.data(), pb.data(), tau.data(), 1, PFC_INIT_GIVEN,
                            nullptr, s);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep > 0) best = std::min(best, ms);  // the first step warms up (graph build, caches)
  }
  for (int k = 0; k < count; ++k) {
    if (insts[k]) pfc_instance_destroy(insts[k]);
    if (states[k]) (void)hipFree(states[k]);
  }
  if (rc < 0) { *status = rc; return -1; }
  return best;
}

// Coordinate descent from the defaults over the launch knobs for `count`
// instances on the meshes ms (round robin); the result, key fields from e, goes
// into the table and to out.
int tune_search(pfc_mesh* const* ms, int n_meshes, int precision, int count, hipStream_t s, pfc_tune_entry e,
                pfc_tune_entry* out) {
  bool grid = true;
  for (int k = 0; k < n_meshes; ++k) grid = grid && ms[k]->dev.gN > 0 && ms[k]->uniform_width >= 1;
  const bool mix = n_meshes > 1;
  // defaults: one row per thread, 64 launches per graph, two PCG iterations per
  // launch where they apply, computed columns on grids, stored operators
  Candidate best{1, 64, 2, 1, 0};
  std::vector<std::pair<Candidate, double>> seen;
  int status = PFC_OK;
  auto measure = [&](const Candidate& c) -> double {
    for (const auto& x : seen)
      if (x.first == c) return x.second;
    int st = PFC_OK;
    const double t = time_candidate(ms, n_meshes, precision, count, c, s, &st);
    if (st == PFC_ERR_OOM) { seen.push_back({c, 1e300}); return 1e300; }  // does not fit: never chosen
    if (st < 0) { status = st; return 1e300; }
    seen.push_back({c, t});
    return t;
  };
  double tbest = measure(best);
  if (status) return status;
  if (tbest >= 1e299) { set_error("pfc_autotune: the instances do not fit the free device memory"); return PFC_ERR_OOM; }
  e.ms_default = tbest;
  auto axis = [&](auto set, const std::vector<int>& values) {
    for (int v : values) {
      Candidate c = best;
      set(c, v);
      const double t = measure(c);
      if (status) return;
      if (t < tbest) { tbest = t; best = c; }
    }
  };
  axis([](Candidate& c, int v) { c.rpt = v; }, {1, 2, 4, 8});
  if (!mix) {  // a mix is tuned for the server, whose instances keep the other defaults
    if (!status && grid) axis([](Candidate& c, int v) { c.grid = v; }, {1, 0});
    if (!status && count > 1) axis([](Candidate& c, int v) { c.shared = v; }, {0, 1});
    // the two-iteration form needs one row per thread
    if (!status && best.rpt <= 1) axis([](Candidate& c, int v) { c.pcg = v; }, {2, 1});
    if (!status) axis([](Candidate& c, int v) { c.ticks = v; }, {32, 64, 128});
  }
  if (status) return status;
  e.rows_per_thread = best.rpt;
  e.ticks_per_graph = best.ticks;
  e.pcg_steps_per_launch = best.pcg;
  e.grid_columns = best.grid;
  e.shared_ops = best.shared;
  e.ms_per_step = tbest;
  e.candidates = (int)seen.size();
  e.from_cache = 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    put_entry(e);
  }
  *out = e;
  return PFC_OK;
}

}  // namespace

// launches per graph the table holds for a batch of these instances (0: none)
int tuned_ticks(const pfc_mesh* m, int precision, int count) {
  char arch[32];
  if (current_arch(arch, sizeof(arch))) { (void)hipGetLastError(); return 0; }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const pfc_tune_entry* e = find_entry(arch, m->dim, m->n, mesh_z(m), precision, count);
  return e ? e->ticks_per_graph : 0;
}

// rows per thread the table holds for `count` instances of a mix of meshes, as
// tuned by pfc_autotune_mix (0: none)
int tuned_mix_rows_per_thread(int precision, int count) {
  char arch[32];
  if (current_arch(arch, sizeof(arch))) { (void)hipGetLastError(); return 0; }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const pfc_tune_entry* e = find_entry(arch, 0, 0, 0, precision, count);
  return e ? e->rows_per_thread : 0;
}

}  // namespace pfc

using namespace pfc;

extern "C" {

int pfc_tune_load(const char* path) {
  if (!path) { set_error("pfc_tune_load: null path"); return PFC_ERR_ARG; }
  FILE* f = std::fopen(path, "rb");
  if (!f) { set_error(std::string("pfc_tune_load: cannot open ") + path); return PFC_ERR_ARG; }
  std::string s;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
  std::fclose(f);
  std::vector<pfc_tune_entry> es;
  if (!parse_cache(s, es)) { set_error(std::string("pfc_tune_load: not a tuning cache: ") + path); return PFC_ERR_ARG; }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const pfc_tune_entry& e : es) put_entry(e);
  return PFC_OK;
}

int pfc_tune_save(const char* path) {
  if (!path) { set_error("pfc_tune_save: null path"); return PFC_ERR_ARG; }
  std::string s = "{\"format\": \"pfc-tune-1\", \"entries\": [\n";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (size_t i = 0; i < g_table.size(); ++i) s += " " + entry_json(g_table[i]) + (i + 1 < g_table.size() ? ",\n" : "\n");
  }
  s += "]}\n";
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) { set_error(std::string("pfc_tune_save: cannot write ") + tmp); return PFC_ERR_ARG; }
  const bool ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
  if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
    set_error(std::string("pfc_tune_save: cannot write ") + path);
    return PFC_ERR_ARG;
  }
  return PFC_OK;
}

void pfc_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_table.clear();
}

int pfc_tune_lookup(const char* arch, int dim, int n, int z, int precision, int count, pfc_tune_entry* out) {
  if (!out || count < 1) { set_error("pfc_tune_lookup: invalid arguments"); return PFC_ERR_ARG; }
  char a[32];
  if (arch) std::snprintf(a, sizeof(a), "%s", arch);
  else if (int rc = current_arch(a, sizeof(a))) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const pfc_tune_entry* e = find_entry(a, dim, n, z, precision, count);
  if (!e) { set_error("pfc_tune_lookup: no entry for this key"); return PFC_ERR_STATE; }
  *out = *e;
  out->from_cache = 1;
  return PFC_OK;
}

int pfc_autotune(pfc_mesh* m, int precision, int count, int force, pfc_tune_entry* out, void* stream) {
  if (!m || !out || count < 1 || (precision != PFC_FP64 && precision != PFC_MIXED)) {
    set_error("pfc_autotune: invalid arguments");
    return PFC_ERR_ARG;
  }
  pfc_tune_entry e;
  std::memset(&e, 0, sizeof(e));
  e.struct_size = (int)sizeof(pfc_tune_entry);
  if (int rc = current_arch(e.arch, sizeof(e.arch))) return rc;
  e.dim = m->dim; e.n = m->n; e.z = mesh_z(m); e.precision = precision; e.count = count;
  if (!force) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const pfc_tune_entry& x : g_table)
      if (same_key(x, e.arch, e.dim, e.n, e.z, e.precision) && x.count == count) {
        *out = x;
        out->from_cache = 1;
        return PFC_OK;
      }
  }
  return tune_search(&m, 1, precision, count, (hipStream_t)stream, e, out);
}

int pfc_autotune_mix(pfc_mesh* const* meshes, int n_meshes, int precision, int count, int force, pfc_tune_entry* out,
                     void* stream) {
  if (!meshes || n_meshes < 1 || !out || count < 1 || (precision != PFC_FP64 && precision != PFC_MIXED)) {
    set_error("pfc_autotune_mix: invalid arguments");
    return PFC_ERR_ARG;
  }
  for (int k = 0; k < n_meshes; ++k)
    if (!meshes[k]) { set_error("pfc_autotune_mix: null mesh"); return PFC_ERR_ARG; }
  pfc_tune_entry e;
  std::memset(&e, 0, sizeof(e));
  e.struct_size = (int)sizeof(pfc_tune_entry);
  if (int rc = current_arch(e.arch, sizeof(e.arch))) return rc;
  e.dim = 0; e.n = 0; e.z = 0; e.precision = precision; e.count = count;  // the mix key
  if (!force) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const pfc_tune_entry& x : g_table)
      if (same_key(x, e.arch, 0, 0, 0, precision) && x.count == count) {
        *out = x;
        out->from_cache = 1;
        return PFC_OK;
      }
  }
  return tune_search(meshes, n_meshes, precision, count, (hipStream_t)stream, e, out);
}

}  // extern "C"
