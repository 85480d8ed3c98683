// Plans: persistent, graph-replayed evaluation of a fixed batch of uneven pulses, with a
// launch shape chosen by timing the candidates on the batch itself.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"

using namespace po;

struct po_plan {
  int n = 0;
  int device = 0;
  std::vector<po_pulse_spec> specs;
  std::vector<po_grid> grids;
  Batch b;
  std::vector<PulseDev> h_desc;
  EvolveConfig cfg;
  int workgroups = 0;
  int n_items = 0;
  PulseDev* d_desc = nullptr;
  int2* d_queue = nullptr;
  int* d_counter = nullptr;
  double* d_ranges = nullptr;  // table range per chunk
  double* d_units = nullptr;
  double* d_A = nullptr;
  double* d_edge = nullptr;
  double* d_spec = nullptr;
  double* d_part = nullptr;
  double* d_scale = nullptr;
  double* d_probe = nullptr;  // coefficients used while autotuning
  double* d_Jprobe = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key_coeff = nullptr;
  const void* key_J = nullptr;
  const void* key_f = nullptr;
};

namespace {

void free_all(po_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  void* bufs[] = {p->d_desc, p->d_queue, p->d_counter, p->d_ranges, p->d_units, p->d_A, p->d_edge,
                  p->d_spec, p->d_part, p->d_scale, p->d_probe, p->d_Jprobe};
  for (void* q : bufs)
    if (q) (void)hipFree(q);
  if (p->cap) (void)hipStreamDestroy(p->cap);
}

template <class T>
po_status dalloc(T** out, size_t count) {
  void* q = nullptr;
  PO_HIP(hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)));
  *out = static_cast<T*>(q);
  return PO_OK;
}

bool valid_config(const EvolveConfig& c) {
  const bool t = c.threads == 64 || c.threads == 128 || c.threads == 256;
  const bool m = c.mpl == 1 || c.mpl == 2;
  if (!t || !m) return false;
  if (!c.persistent && (c.threads != kItem || c.mpl != 1)) return false;
  return true;
}

// Work items of cfg.threads * cfg.mpl modes, longest pulse (largest nt) first.
po_status build_queue(po_plan* p, hipStream_t s) {
  const int per = p->cfg.threads * p->cfg.mpl;
  std::vector<int> order(p->n);
  for (int i = 0; i < p->n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return p->specs[a].nt > p->specs[c].nt; });
  std::vector<int2> q;
  for (int i : order) {
    const int64_t m = int64_t(p->grids[i].n[0]) * p->grids[i].n[1] * p->grids[i].n[2];
    for (int64_t first = 0; first < m; first += per) q.push_back(make_int2(i, int(first)));
  }
  p->n_items = int(q.size());
  if (p->d_queue) PO_HIP(hipFree(p->d_queue));
  p->d_queue = nullptr;
  PO_TRY(dalloc(&p->d_queue, q.size()));
  PO_HIP(hipMemcpyAsync(p->d_queue, q.data(), sizeof(int2) * q.size(), hipMemcpyHostToDevice, s));
  PO_HIP(hipStreamSynchronize(s));
  int cus = 0;
  PO_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
  p->workgroups = p->workgroups > 0 ? p->workgroups : cus * evolve_workgroups_per_cu(p->cfg);
  return PO_OK;
}

// synthesis (when coefficients are given) -> series selection -> evolution -> yield
po_status enqueue(po_plan* p, const double* d_coeff, const double* d_A, const double* d_edge, double* d_J, double* d_f,
                  hipStream_t s) {
  if (d_coeff) {
    PO_TRY(launch_synth(p->b, p->d_desc, d_coeff, p->d_spec, p->d_part, p->d_scale, p->d_A, nullptr, p->d_edge,
                        nullptr, s));
    d_A = p->d_A;
    d_edge = p->d_edge;
  }
  PO_TRY(launch_chunk_ranges(p->b, p->d_desc, d_A, p->d_ranges, s));
  double* units = d_J ? p->d_units : nullptr;
  if (p->cfg.persistent)
    PO_TRY(launch_evolve_persistent(p->cfg, p->n, p->d_desc, d_A, d_edge, p->d_ranges, p->d_queue, p->n_items,
                                    p->workgroups, p->d_counter, d_f, units, s));
  else
    PO_TRY(launch_evolve_grid(p->b, p->d_desc, d_A, d_edge, p->d_ranges, d_f, units, s));
  if (d_J) PO_TRY(launch_yield_from_units(p->b, p->d_desc, p->d_units, d_J, s));
  return PO_OK;
}

uint64_t fnv(uint64_t h, const void* data, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

std::string cache_key(const po_plan* p) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
  uint64_t h = 1469598103934665603ull;
  for (int i = 0; i < p->n; ++i) {
    h = fnv(h, &p->specs[i].nt, sizeof(int32_t));
    h = fnv(h, p->grids[i].n, sizeof(p->grids[i].n));
  }
  std::ostringstream os;
  os << arch << ":" << p->n << ":" << std::hex << h;
  return os.str();
}

bool cache_lookup(const char* path, const std::string& key, EvolveConfig* out) {
  if (!path) return false;
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    std::istringstream is(line);
    std::string k;
    EvolveConfig c;
    if (is >> k >> c.threads >> c.mpl >> c.persistent && k == key && valid_config(c)) {
      *out = c;
      found = true;
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const EvolveConfig& c) {
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << key << " " << c.threads << " " << c.mpl << " " << c.persistent << "\n";
}

po_status time_config(po_plan* p, hipStream_t s, float* ms) {
  PO_TRY(build_queue(p, s));
  hipEvent_t e0, e1;
  PO_HIP(hipEventCreate(&e0));
  PO_HIP(hipEventCreate(&e1));
  po_status st = enqueue(p, p->d_probe, nullptr, nullptr, p->d_Jprobe, nullptr, s);  // warm-up
  if (st == PO_OK) {
    (void)hipEventRecord(e0, s);
    st = enqueue(p, p->d_probe, nullptr, nullptr, p->d_Jprobe, nullptr, s);
    (void)hipEventRecord(e1, s);
  }
  if (st == PO_OK) {
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e != hipSuccess) st = device_error(e, "autotune timing");
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

po_status autotune(po_plan* p, const po_plan_config* req, hipStream_t s) {
  std::vector<EvolveConfig> cands;
  const int ths[3] = {256, 128, 64};
  for (int pers = 0; pers <= 1; ++pers)
    for (int t : ths)
      for (int m = 1; m <= 2; ++m) {
        EvolveConfig c{t, m, pers};
        if (!valid_config(c)) continue;
        if (req->threads && req->threads != t) continue;
        if (req->modes_per_lane && req->modes_per_lane != m) continue;
        if (req->persistent >= 0 && req->persistent != pers) continue;
        cands.push_back(c);
      }
  if (cands.empty()) return set_error(PO_ERR_INVALID, "no launch shape satisfies the requested config");
  float best = 1e30f;
  EvolveConfig pick = cands[0];
  const int wg_req = p->workgroups;
  for (const EvolveConfig& c : cands) {
    p->cfg = c;
    p->workgroups = wg_req;
    float ms = 0.0f;
    PO_TRY(time_config(p, s, &ms));
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  p->cfg = pick;
  p->workgroups = wg_req;
  return build_queue(p, s);
}

po_status plan_create(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const po_plan_config* cfg,
                      const char* cache_path, hipStream_t s, po_plan* p) {
  p->n = n;
  PO_HIP(hipGetDevice(&p->device));
  p->specs.assign(specs, specs + n);
  p->grids.assign(grids, grids + n);
  p->h_desc.resize(n);
  PO_TRY(build_batch(n, specs, grids, p->h_desc.data(), &p->b));
  PO_TRY(dalloc(&p->d_desc, n));
  PO_HIP(hipMemcpy(p->d_desc, p->h_desc.data(), sizeof(PulseDev) * n, hipMemcpyHostToDevice));
  PO_TRY(dalloc(&p->d_counter, 1));
  PO_TRY(dalloc(&p->d_ranges, 4 * size_t(p->b.total_chunks)));
  PO_TRY(dalloc(&p->d_units, size_t(p->b.total_units)));
  PO_TRY(dalloc(&p->d_A, size_t(2 * p->b.total_rows)));
  PO_TRY(dalloc(&p->d_edge, size_t(4 * n)));
  PO_TRY(dalloc(&p->d_spec, size_t(p->b.total_spec)));
  PO_TRY(dalloc(&p->d_part, size_t(std::max(1, p->b.max_stat_blocks)) * n));
  PO_TRY(dalloc(&p->d_scale, size_t(n)));
  PO_TRY(dalloc(&p->d_Jprobe, size_t(n)));
  PO_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));

  po_plan_config req = cfg ? *cfg : po_plan_config{0, 0, -1, 0};
  p->workgroups = req.workgroups > 0 ? req.workgroups : 0;
  EvolveConfig fixed{req.threads, req.modes_per_lane, req.persistent};
  if (req.threads && req.modes_per_lane && req.persistent >= 0) {
    if (!valid_config(fixed)) return set_error(PO_ERR_INVALID, "unsupported plan config");
    p->cfg = fixed;
    return build_queue(p, s);
  }
  const std::string key = cache_key(p);
  EvolveConfig cached;
  if (cache_lookup(cache_path, key, &cached) && (!req.threads || req.threads == cached.threads) &&
      (!req.modes_per_lane || req.modes_per_lane == cached.mpl) &&
      (req.persistent < 0 || req.persistent == cached.persistent)) {
    p->cfg = cached;
    return build_queue(p, s);
  }
  // deterministic probe coefficients: amplitudes alternate 0.5 / -0.25, phases 0
  std::vector<double> probe(size_t(std::max<int64_t>(p->b.total_coeff, 1)));
  for (int i = 0; i < n; ++i) {
    const int ns = specs[i].n_s;
    double* c = probe.data() + p->h_desc[i].coeff_off;
    for (int l = 0; l < 2; ++l)
      for (int k = 0; k < ns; ++k) {
        c[(l * 2 + 0) * ns + k] = (k + l) % 2 ? -0.25 : 0.5;
        c[(l * 2 + 1) * ns + k] = -1.0;
      }
  }
  PO_TRY(dalloc(&p->d_probe, probe.size()));
  PO_HIP(hipMemcpy(p->d_probe, probe.data(), sizeof(double) * probe.size(), hipMemcpyHostToDevice));
  PO_TRY(autotune(p, &req, s));
  cache_store(cache_path, key, p->cfg);
  return PO_OK;
}

po_status check_plan_match(const po_plan* p, int32_t n, const po_pulse_spec* specs, const po_grid* grids) {
  if (n != p->n) return set_error(PO_ERR_INVALID, "plan was made for %d pulses, not %d", p->n, n);
  for (int i = 0; i < n; ++i) {
    if (specs[i].nt != p->specs[i].nt || specs[i].T != p->specs[i].T)
      return set_error(PO_ERR_INVALID, "pulse %d: nt/T differ from the plan's", i);
    if (std::memcmp(&grids[i], &p->grids[i], sizeof(po_grid)) != 0)
      return set_error(PO_ERR_INVALID, "pulse %d: grid differs from the plan's", i);
  }
  int dev = -1;
  PO_HIP(hipGetDevice(&dev));
  if (dev != p->device) return set_error(PO_ERR_INVALID, "plan belongs to device %d, current is %d", p->device, dev);
  return PO_OK;
}

}  // namespace

namespace po {
// Used by po_evolve_modes when a plan is passed: the plan's launch shape on the caller's tables.
po_status plan_evolve(const po_plan* cp, int32_t n, const po_pulse_spec* specs, const po_grid* grids,
                      const double* d_A, const double* d_edge, double* d_f, double* d_J, hipStream_t s) {
  po_plan* p = const_cast<po_plan*>(cp);
  PO_TRY(check_plan_match(p, n, specs, grids));
  PO_TRY(enqueue(p, nullptr, d_A, d_edge, d_J, d_f, s));
  return timer_count(p->n, p->d_desc, p->d_ranges, s);
}

bool plan_matches(const po_plan* p, int32_t n, const po_pulse_spec* specs, const po_grid* grids) {
  return check_plan_match(p, n, specs, grids) == PO_OK;
}
}  // namespace po

extern "C" {

po_status po_plan_create(int32_t n, const po_pulse_spec* specs, const po_grid* grids, const po_plan_config* cfg,
                         const char* cache_path, void* stream, struct po_plan** out) {
  if (!out) return set_error(PO_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1) return set_error(PO_ERR_INVALID, "n_pulses must be >= 1");
  if (!specs || !grids) return set_error(PO_ERR_INVALID, "specs and grids are required");
  for (int i = 0; i < n; ++i) {
    PO_TRY(validate_spec(specs[i], i));
    PO_TRY(validate_grid(grids[i], i));
  }
  if (cfg) {
    if (cfg->threads && cfg->threads != 64 && cfg->threads != 128 && cfg->threads != 256)
      return set_error(PO_ERR_INVALID, "threads must be 0, 64, 128 or 256");
    if (cfg->modes_per_lane && cfg->modes_per_lane != 1 && cfg->modes_per_lane != 2)
      return set_error(PO_ERR_INVALID, "modes_per_lane must be 0, 1 or 2");
    if (cfg->persistent < -1 || cfg->persistent > 1) return set_error(PO_ERR_INVALID, "persistent must be -1, 0 or 1");
    if (cfg->workgroups < 0) return set_error(PO_ERR_INVALID, "workgroups must be >= 0");
  }
  po_plan* p = new (std::nothrow) po_plan();
  if (!p) return set_error(PO_ERR_NOMEM, "plan allocation failed");
  const po_status st = plan_create(n, specs, grids, cfg, cache_path, static_cast<hipStream_t>(stream), p);
  if (st != PO_OK) {
    free_all(p);
    delete p;
    return st;
  }
  *out = p;
  return PO_OK;
}

po_status po_plan_get_config(const struct po_plan* p, po_plan_config* out) {
  if (!p || !out) return set_error(PO_ERR_INVALID, "plan and out are required");
  *out = po_plan_config{p->cfg.threads, p->cfg.mpl, p->cfg.persistent, p->workgroups};
  return PO_OK;
}

po_status po_plan_evaluate(struct po_plan* p, const double* d_coeff, double* d_J, double* d_f, void* stream) {
  if (!p) return set_error(PO_ERR_INVALID, "plan is NULL");
  int dev = -1;
  PO_HIP(hipGetDevice(&dev));
  if (dev != p->device) return set_error(PO_ERR_INVALID, "plan belongs to device %d, current is %d", p->device, dev);
  PO_TRY(check_device_range(d_coeff, sizeof(double) * p->b.total_coeff, 8, "d_coeff"));
  PO_TRY(check_device_range(d_J, sizeof(double) * p->n, 8, "d_J"));
  if (d_f) PO_TRY(check_device_range(d_f, sizeof(double) * p->b.total_modes, 8, "d_f"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!p->exec || p->key_coeff != d_coeff || p->key_J != d_J || p->key_f != d_f) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    PO_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    const po_status st = enqueue(p, d_coeff, nullptr, nullptr, d_J, d_f, p->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (st != PO_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return device_error(e, "hipStreamEndCapture");
    p->graph = g;
    PO_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->key_coeff = d_coeff;
    p->key_J = d_J;
    p->key_f = d_f;
  }
  hipEvent_t e0 = nullptr;
  const bool timed = timer_start(s, &e0);
  PO_HIP(hipGraphLaunch(p->exec, s));
  if (timed) {
    timer_stop(s, e0);
    PO_TRY(timer_count(p->n, p->d_desc, p->d_ranges, s));
  }
  return PO_OK;
}

void po_plan_destroy(struct po_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  free_all(p);
  delete p;
}

}  // extern "C"
