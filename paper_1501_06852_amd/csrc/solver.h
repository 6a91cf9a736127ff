// Host-side solver objects: launch groups (teams of workgroups, captured
// graph of solver launches, pinned status flags) and instances.
#pragma once
#include <vector>

#include "host.h"

struct pfc_instance;

namespace pfc {

struct Group {
  int count = 0, n_wg = 0, graph_ticks = 0;
  TeamEntry* d_teams = nullptr;
  std::vector<TeamEntry> h_teams;
  int cols = 0;                 // where the launches take the P1 columns from (PFC_COL_*)
  InstDev* d_descs = nullptr;
  InstDev* h_descs = nullptr;   // pinned staging of the descriptors
  State* h_states = nullptr;    // pinned staging of the initial states
  int* h_flags = nullptr;       // pinned, mapped: phase of each instance after each replay
  int* d_flags = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  long long graphs_run = 0;
  int alloc(const std::vector<int>& team_sizes);
  int build(hipStream_t capture, int precision, int ticks);
  int run(hipStream_t s, const std::vector<State*>& dev_states, double timeout_s);
  void release();
};

size_t carve(InstDev& h, char* base, const pfc_mesh* m, const pfc_opts& o, int team_size);
int team_size_for(int n_slices, int rows_per_thread);
// whether an instance with these options on this mesh takes the 2D block form of
// two PCG iterations per launch (with pcg_steps_per_launch = 2)
bool block_form_applies(const pfc_mesh* m, const pfc_opts& o);
void set_params(InstDev& h, double r, double tau, double m11);
int set_mobility_mean(pfc_instance* I, const double* psi, hipStream_t s);
int prep_ops_public(pfc_instance* I, hipStream_t s);
// autotuning table (tune.hip), 0 where it has no entry: launches per graph for
// `count` instances of a mesh; rows per thread for `count` instances of a mix
int tuned_ticks(const pfc_mesh* m, int precision, int count);
int tuned_mix_rows_per_thread(int precision, int count);
// public result record of a solve from the device's record
void fill_info(pfc_solve_info* dst, const InfoDev& s);

}  // namespace pfc

struct pfc_instance {
  pfc_mesh* mesh = nullptr;
  pfc_opts opts{};
  int team_size = 0;
  int ticks = 64;
  size_t bytes = 0;
  char* arena = nullptr;
  InstDev h{};
  hipStream_t capture = nullptr;
  pfc::Group grp;
  double ops_tau_s = -1.0;
  int* d_sched = nullptr;
  size_t sched_bytes = 0;
  int last_applies = 0;
  double timeout_s = 600.0;
};
