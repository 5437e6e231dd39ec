// Batched solves of independent problems (host side): every stage of the
// multigrid cycle and of the Krylov iteration runs for all problems in one
// packed launch (packed.hpp), and the whole batched preconditioning cycle is
// one HIP graph launch.
//
// Packing: each problem's cycle is recorded as a list of launch functors,
// tagged by stage (the depth below its finest level and the phase of
// Algorithm 1, see EngineT::cycle_t).  Stages are run in tag order; within a
// stage, problems whose stage has the same sequence of kernels (the kernel
// variant follows the level size) form a group, and launch k of the group is
// one packed launch over the group's problems.  A problem's own launches keep
// their order, and problems share no data, so the result of every problem
// is that of its own cycle.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "engine.hpp"
#include "packed.hpp"
#include "vec_kernels.hpp"

namespace smg {

struct PackedLaunch {
  const void *kernel = nullptr;
  unsigned threads = 0, grid = 0;
  const void *table = nullptr;       // device: n functors
  const uint32_t *first = nullptr;   // device: first block of each
  const uint32_t *count = nullptr;   // device: block count of each
  int n = 0;
};

// A sequence of packed launches and the device memory of their tables.
struct PackedPlan {
  std::vector<PackedLaunch> launches;
  std::vector<char *> bufs;
  PackedPlan() = default;
  PackedPlan(const PackedPlan &) = delete;
  PackedPlan &operator=(const PackedPlan &) = delete;
  ~PackedPlan() {
    for (char *b : bufs) (void)hipFree(b);
  }
  void run(hipStream_t s) const {
    for (const PackedLaunch &p : launches) {
      const void *tab = p.table;
      const void *first = p.first;
      const void *count = p.count;
      int n = p.n;
      void *args[] = {(void *)&tab, (void *)&first, (void *)&count, (void *)&n};
      SMG_HIP(hipLaunchKernel(p.kernel, dim3(p.grid), dim3(p.threads), args, 0, s));
    }
  }
  // append another plan's launches (taking over its tables)
  void append(PackedPlan &&o) {
    launches.insert(launches.end(), o.launches.begin(), o.launches.end());
    bufs.insert(bufs.end(), o.bufs.begin(), o.bufs.end());
    o.launches.clear();
    o.bufs.clear();
  }
};

// One packed launch per list entry: entries[k] = the functors (all of one
// kernel) to run together.
inline std::unique_ptr<PackedPlan> make_plan(const std::vector<std::vector<const LaunchRec *>> &entries) {
  auto plan = std::make_unique<PackedPlan>();
  std::vector<char> host;
  struct Off {
    size_t table, first, count;
  };
  std::vector<Off> offs;
  auto align = [&](size_t a) {
    while (host.size() % a) host.push_back(0);
  };
  for (const auto &group : entries) {
    if (group.empty()) continue;
    PackedLaunch p;
    p.kernel = group[0]->kernel;
    p.threads = group[0]->threads;
    p.n = (int)group.size();
    const size_t sz = group[0]->bytes.size();
    Off o;
    align(256);
    o.table = host.size();
    for (const LaunchRec *r : group) {
      if (r->kernel != p.kernel || r->bytes.size() != sz || r->threads != p.threads)
        throw Error{SMG_EINVAL, "internal: mixed kernels in a packed launch"};
      host.insert(host.end(), r->bytes.begin(), r->bytes.end());
    }
    std::vector<uint32_t> first(group.size()), count(group.size());
    uint32_t total = 0;
    for (size_t e = 0; e < group.size(); ++e) {
      first[e] = total;
      count[e] = group[e]->nblocks;
      total += (group[e]->nblocks + 7u) / 8u * 8u;   // keep each entry's block 0 on XCD 0
    }
    p.grid = total;
    align(16);
    o.first = host.size();
    host.insert(host.end(), (const char *)first.data(), (const char *)(first.data() + first.size()));
    align(16);
    o.count = host.size();
    host.insert(host.end(), (const char *)count.data(), (const char *)(count.data() + count.size()));
    plan->launches.push_back(p);
    offs.push_back(o);
  }
  if (!host.empty()) {
    char *d = nullptr;
    SMG_HIP(hipMalloc(&d, host.size()));
    plan->bufs.push_back(d);
    SMG_HIP(hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice));
    for (size_t k = 0; k < plan->launches.size(); ++k) {
      plan->launches[k].table = d + offs[k].table;
      plan->launches[k].first = (const uint32_t *)(d + offs[k].first);
      plan->launches[k].count = (const uint32_t *)(d + offs[k].count);
    }
  }
  return plan;
}

// Merge the recorded launch lists of the problems into packed launches (see
// the head of this file).
inline std::unique_ptr<PackedPlan> merge_recordings(const std::vector<Recorder> &recs) {
  // per problem: tag -> its launches of that stage, in order
  std::vector<std::map<int, std::vector<const LaunchRec *>>> by_tag(recs.size());
  std::vector<int> tags;
  for (size_t i = 0; i < recs.size(); ++i)
    for (const LaunchRec &r : recs[i].recs) {
      by_tag[i][r.tag].push_back(&r);
      tags.push_back(r.tag);
    }
  std::sort(tags.begin(), tags.end());
  tags.erase(std::unique(tags.begin(), tags.end()), tags.end());
  std::vector<std::vector<const LaunchRec *>> entries;
  for (int tag : tags) {
    // groups of problems with the same kernel sequence in this stage
    std::vector<std::pair<std::vector<const void *>, std::vector<size_t>>> groups;
    for (size_t i = 0; i < recs.size(); ++i) {
      auto it = by_tag[i].find(tag);
      if (it == by_tag[i].end()) continue;
      std::vector<const void *> sig;
      for (const LaunchRec *r : it->second) sig.push_back(r->kernel);
      auto g = std::find_if(groups.begin(), groups.end(), [&](const auto &x) { return x.first == sig; });
      if (g == groups.end()) groups.push_back({sig, {i}});
      else g->second.push_back(i);
    }
    for (const auto &g : groups)
      for (size_t k = 0; k < g.first.size(); ++k) {
        std::vector<const LaunchRec *> e;
        for (size_t i : g.second) e.push_back(by_tag[i][tag][k]);
        entries.push_back(std::move(e));
      }
  }
  return make_plan(entries);
}

// Functor as a launch record (for the driver's own packed launches).
template <class L>
LaunchRec as_record(const L &l, unsigned nb) {
  static_assert(std::is_trivially_copyable<L>::value, "launch functors are copied as bytes");
  LaunchRec r;
  r.kernel = (const void *)&k_packed<L>;
  r.nblocks = nb;
  r.threads = L::THREADS;
  r.align = alignof(L);
  r.bytes.resize(sizeof(L));
  std::memcpy(r.bytes.data(), &l, sizeof(L));
  return r;
}

class BatchDriver {
 public:
  std::vector<EngineBase *> eng;
  std::vector<BatchView> bv;
  hipStream_t stream = nullptr;
  int precision = 0;           // SMG_PRECOND_F64 / F32 (the same for every problem)
  int restart = 0;             // the smallest Krylov basis of the problems
  // batched preconditioning cycle: packed plan, captured in a graph
  std::unique_ptr<PackedPlan> cycle_plan;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  // per Krylov index j: copies in/out of the cycle, K z_j, the two
  // Gram-Schmidt passes and the normalisation
  std::vector<std::unique_ptr<PackedPlan>> iter_in, iter_out;
  // reductions: per problem RS doubles on the device, mirrored in pinned memory
  static constexpr int RS = 1024;
  double *dres = nullptr, *hres = nullptr;
  double *dy = nullptr;        // correction coefficients, per problem `restart` entries
  double *hy = nullptr;

  ~BatchDriver() { release(); }
  void release() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    if (dres) (void)hipFree(dres);
    if (dy) (void)hipFree(dy);
    if (hres) (void)hipHostFree(hres);
    if (hy) (void)hipHostFree(hy);
    dres = dy = hres = hy = nullptr;
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    iter_in.clear();
    iter_out.clear();
    cycle_plan.reset();
  }

  void init(const std::vector<EngineBase *> &e) {
    eng = e;
    bv.clear();
    restart = 1 << 30;
    for (EngineBase *x : eng) {
      bv.push_back(x->batch_view());
      restart = std::min(restart, bv.back().restart);
    }
    precision = bv[0].precision;
    for (const BatchView &v : bv)
      if (v.precision != precision) throw Error{SMG_EINVAL, "batched problems must use one preconditioner precision"};
    const size_t n = eng.size();
    SMG_HIP(hipMalloc(&dres, sizeof(double) * RS * n));
    SMG_HIP(hipHostMalloc(&hres, sizeof(double) * RS * n, hipHostMallocDefault));
    SMG_HIP(hipMalloc(&dy, sizeof(double) * (size_t)restart * n));
    SMG_HIP(hipHostMalloc(&hy, sizeof(double) * (size_t)restart * n, hipHostMallocDefault));
    if (!cap_stream) SMG_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  }

  // The batched cycle: recorded, packed and captured into one graph.
  void build_cycle() {
    drop_graph();
    const int dt = precision == SMG_PRECOND_F32 ? SMG_F32 : SMG_F64;
    std::vector<Recorder> recs(eng.size());
    for (size_t i = 0; i < eng.size(); ++i) eng[i]->record_cycle(dt, recs[i]);
    cycle_plan = merge_recordings(recs);
    SMG_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      cycle_plan->run(cap_stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    SMG_HIP(hipStreamEndCapture(cap_stream, &graph));
    SMG_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
  }

  size_t n() const { return eng.size(); }
  double *res(size_t i) const { return dres + (size_t)RS * i; }

  // copy-in / copy-out plans of the cycle for Krylov index j (z_j = M^-1 v_j)
  const PackedPlan &plan_in(int j) {
    if ((int)iter_in.size() <= j) iter_in.resize(j + 1);
    if (!iter_in[j]) {
      std::vector<LaunchRec> r;
      for (size_t i = 0; i < n(); ++i) {
        const BatchView &v = bv[i];
        const double *vj = v.V + (int64_t)j * v.N;
        if (precision == SMG_PRECOND_F32) r.push_back(as_record(LCopy<float, double>{v.b32, vj, (i64)v.N}, grid_for_n(v.N)));
        else r.push_back(as_record(LCopy<double, double>{v.b64, vj, (i64)v.N}, grid_for_n(v.N)));
      }
      iter_in[j] = plan_of(r);
    }
    return *iter_in[j];
  }
  const PackedPlan &plan_out(int j) {
    if ((int)iter_out.size() <= j) iter_out.resize(j + 1);
    if (!iter_out[j]) {
      // z_j = cycle output; w = K z_j (= v_{j+1} before orthogonalisation);
      // two Gram-Schmidt passes against v_0..v_j; ||w||^2; w /= ||w||
      std::vector<Recorder> rv(n());
      std::vector<LaunchRec> copy, p1a, p1b, p1c, p2a, p2b, p2c, nra, nrb, nrc;
      for (size_t i = 0; i < n(); ++i) {
        const BatchView &v = bv[i];
        double *zj = v.Z + (int64_t)j * v.N, *w = v.V + (int64_t)(j + 1) * v.N;
        if (precision == SMG_PRECOND_F32) copy.push_back(as_record(LCopy<double, float>{zj, v.x32, (i64)v.N}, grid_for_n(v.N)));
        else copy.push_back(as_record(LCopy<double, double>{zj, v.x64, (i64)v.N}, grid_for_n(v.N)));
        eng[i]->record_vmult(rv[i], zj, w);
        double *r = res(i);
        p1a.push_back(as_record(LMultidotPartial<double>{v.V, (i64)v.N, j + 1, w, (i64)v.N, v.partial}, RB));
        p1b.push_back(as_record(LPartialFinish{v.partial, RB, j + 1, r}, (unsigned)(j + 1)));
        p1c.push_back(as_record(LMultiAxpy<double>{w, v.V, (i64)v.N, j + 1, r, -1.0, (i64)v.N}, grid_for_n(v.N)));
        p2a.push_back(as_record(LMultidotPartial<double>{v.V, (i64)v.N, j + 1, w, (i64)v.N, v.partial}, RB));
        p2b.push_back(as_record(LPartialFinish{v.partial, RB, j + 1, r + 256}, (unsigned)(j + 1)));
        p2c.push_back(as_record(LMultiAxpy<double>{w, v.V, (i64)v.N, j + 1, r + 256, -1.0, (i64)v.N}, grid_for_n(v.N)));
        nra.push_back(as_record(LMultidotPartial<double>{w, 0, 1, w, (i64)v.N, v.partial}, RB));
        nrb.push_back(as_record(LPartialFinish{v.partial, RB, 1, r + 512}, 1));
        nrc.push_back(as_record(LScaleInvSqrt<double>{w, r + 512, (i64)v.N}, grid_for_n(v.N)));
      }
      std::vector<std::vector<const LaunchRec *>> entries;
      auto add = [&](const std::vector<LaunchRec> &l) {
        std::vector<const LaunchRec *> e;
        for (const LaunchRec &x : l) e.push_back(&x);
        entries.push_back(e);
      };
      add(copy);
      std::unique_ptr<PackedPlan> plan = make_plan(entries);
      // the operator: merged like a cycle stage (kernel variants may differ)
      plan->append(std::move(*merge_recordings(rv)));
      entries.clear();
      add(p1a), add(p1b), add(p1c), add(p2a), add(p2b), add(p2c), add(nra), add(nrb), add(nrc);
      plan->append(std::move(*make_plan(entries)));
      iter_out[j] = std::move(plan);
    }
    return *iter_out[j];
  }

  std::unique_ptr<PackedPlan> plan_of(const std::vector<LaunchRec> &r) {
    std::vector<const LaunchRec *> e;
    for (const LaunchRec &x : r) e.push_back(&x);
    return make_plan({e});
  }
  // z_i = M_i^-1 v_i for every problem: packed copies in, the cycle graph,
  // packed copies out (no operator, no Gram-Schmidt); for tests.
  void precondition(const double *const *v, double *const *z) {
    std::vector<LaunchRec> in, out;
    for (size_t i = 0; i < n(); ++i) {
      const BatchView &b = bv[i];
      if (precision == SMG_PRECOND_F32) {
        in.push_back(as_record(LCopy<float, double>{b.b32, v[i], (i64)b.N}, grid_for_n(b.N)));
        out.push_back(as_record(LCopy<double, float>{z[i], b.x32, (i64)b.N}, grid_for_n(b.N)));
      } else {
        in.push_back(as_record(LCopy<double, double>{b.b64, v[i], (i64)b.N}, grid_for_n(b.N)));
        out.push_back(as_record(LCopy<double, double>{z[i], b.x64, (i64)b.N}, grid_for_n(b.N)));
      }
    }
    auto pi = plan_of(in), po = plan_of(out);
    if (!gexec) build_cycle();
    pi->run(stream);
    SMG_HIP(hipGraphLaunch(gexec, stream));
    po->run(stream);
    SMG_HIP(hipStreamSynchronize(stream));
  }

  smg_status solve(double *const *x, const double *const *b, double rtol, int maxit, smg_solve_info *infos);
};

// FGMRES(m) for every problem, in lockstep: the problems keep their own
// Krylov bases, coefficients, residual estimates and stopping decisions (the
// iteration of EngineT::solve, without its look-ahead), while each device step
// -- residual, norms, the copies around the preconditioner, the batched cycle,
// the operator, both Gram-Schmidt passes and the normalisation -- is one
// packed launch (the cycle: one graph launch) for all problems, and the
// coefficients of all problems come back in one copy per iteration.  A
// problem that has converged keeps being carried through the launches of its
// cycle's remaining iterations; what they write is not used.
inline smg_status BatchDriver::solve(double *const *x, const double *const *b, double rtol, int maxit,
                                     smg_solve_info *infos) {
  const auto t0 = std::chrono::steady_clock::now();
  const size_t nn = n();
  const int m = restart;
  if (!gexec) build_cycle();
  // r = b - K x into v_0; ||b||^2 -> res + 768, ||r||^2 -> res + 769; v_0 /= ||r||
  std::unique_ptr<PackedPlan> resplan, bnplan, rnplan, scaleplan;
  {
    std::vector<Recorder> rv(nn);
    std::vector<LaunchRec> a, af, c, cf, sc;
    for (size_t i = 0; i < nn; ++i) {
      const BatchView &v = bv[i];
      eng[i]->record_residual(rv[i], x[i], b[i], v.V);
      a.push_back(as_record(LMultidotPartial<double>{b[i], 0, 1, b[i], (i64)v.N, v.partial}, RB));
      af.push_back(as_record(LPartialFinish{v.partial, RB, 1, res(i) + 768}, 1));
      c.push_back(as_record(LMultidotPartial<double>{v.V, 0, 1, v.V, (i64)v.N, v.partial}, RB));
      cf.push_back(as_record(LPartialFinish{v.partial, RB, 1, res(i) + 769}, 1));
      sc.push_back(as_record(LScaleInvSqrt<double>{v.V, res(i) + 769, (i64)v.N}, grid_for_n(v.N)));
    }
    resplan = merge_recordings(rv);
    auto ptrs = [](const std::vector<LaunchRec> &l) {
      std::vector<const LaunchRec *> e;
      for (const LaunchRec &r : l) e.push_back(&r);
      return e;
    };
    bnplan = make_plan({ptrs(a), ptrs(af)});
    rnplan = make_plan({ptrs(c), ptrs(cf)});
    scaleplan = make_plan({ptrs(sc)});
  }
  auto fetch = [&]() {
    SMG_HIP(hipMemcpyAsync(hres, dres, sizeof(double) * RS * nn, hipMemcpyDeviceToHost, stream));
    SMG_HIP(hipStreamSynchronize(stream));
  };
  resplan->run(stream);
  bnplan->run(stream);
  rnplan->run(stream);
  fetch();
  struct State {
    double bnorm = 0, beta = 0, rel = 0;
    int it = 0, hist = 0, jdone = 0;
    bool active = false, in_cycle = false;
    smg_status st = SMG_OK;
    std::vector<double> H, cs, sn, gv;
  };
  std::vector<State> S(nn);
  auto record = [&](size_t i, double v) {
    smg_solve_info *inf = infos ? &infos[i] : nullptr;
    if (inf && inf->history && S[i].hist < inf->history_capacity) inf->history[S[i].hist] = v;
    ++S[i].hist;
  };
  std::vector<LaunchRec> zero;
  for (size_t i = 0; i < nn; ++i) {
    State &q = S[i];
    q.bnorm = std::sqrt(hres[RS * i + 768]);
    q.beta = std::sqrt(hres[RS * i + 769]);
    q.H.assign((size_t)(m + 1) * m, 0.0);
    q.cs.assign(m, 0.0);
    q.sn.assign(m, 0.0);
    q.gv.assign(m + 1, 0.0);
    if (q.bnorm == 0.0) {
      zero.push_back(as_record(LSet<double>{x[i], 0.0, (i64)bv[i].N}, grid_for_n(bv[i].N)));
      q.rel = 0.0;
      record(i, 0.0);
    } else {
      q.rel = q.beta / q.bnorm;
      record(i, q.rel);
      q.active = q.rel > rtol && std::isfinite(q.rel);
      if (!std::isfinite(q.rel)) q.st = SMG_EBREAKDOWN;
    }
  }
  if (!zero.empty()) {
    std::vector<const LaunchRec *> e;
    for (const LaunchRec &r : zero) e.push_back(&r);
    make_plan({e})->run(stream);
  }
  int it = 0;
  auto any_active = [&]() {
    for (const State &q : S)
      if (q.active) return true;
    return false;
  };
  while (it < maxit && any_active()) {
    scaleplan->run(stream);
    for (State &q : S) {
      std::fill(q.H.begin(), q.H.end(), 0.0);
      std::fill(q.gv.begin(), q.gv.end(), 0.0);
      q.gv[0] = q.beta;
      q.jdone = 0;
      q.in_cycle = q.active;
    }
    for (int j = 0; j < m; ++j) {
      plan_in(j).run(stream);
      SMG_HIP(hipGraphLaunch(gexec, stream));
      plan_out(j).run(stream);
      fetch();
      ++it;
      bool more = false;
      for (size_t i = 0; i < nn; ++i) {
        State &q = S[i];
        if (!q.in_cycle) continue;
        const double *hb = hres + RS * i;
        for (int r = 0; r <= j; ++r) q.H[(size_t)r * m + j] += hb[r] + hb[256 + r];
        const double hn = std::sqrt(std::max(hb[512], 0.0));
        q.H[(size_t)(j + 1) * m + j] = hn;
        if (!std::isfinite(hn)) {
          q.st = SMG_EBREAKDOWN;
          q.active = q.in_cycle = false;
          continue;
        }
        for (int r = 0; r < j; ++r) {
          const double t = q.cs[r] * q.H[(size_t)r * m + j] + q.sn[r] * q.H[(size_t)(r + 1) * m + j];
          q.H[(size_t)(r + 1) * m + j] = -q.sn[r] * q.H[(size_t)r * m + j] + q.cs[r] * q.H[(size_t)(r + 1) * m + j];
          q.H[(size_t)r * m + j] = t;
        }
        const double den = std::hypot(q.H[(size_t)j * m + j], q.H[(size_t)(j + 1) * m + j]);
        q.cs[j] = q.H[(size_t)j * m + j] / den;
        q.sn[j] = q.H[(size_t)(j + 1) * m + j] / den;
        q.H[(size_t)j * m + j] = den;
        q.H[(size_t)(j + 1) * m + j] = 0.0;
        q.gv[j + 1] = -q.sn[j] * q.gv[j];
        q.gv[j] = q.cs[j] * q.gv[j];
        ++q.it;
        q.jdone = j + 1;
        q.rel = std::fabs(q.gv[j + 1]) / q.bnorm;
        if (!std::isfinite(q.rel)) {
          q.st = SMG_EBREAKDOWN;
          q.active = q.in_cycle = false;
          continue;
        }
        record(i, q.rel);
        if (q.rel <= rtol || it >= maxit) q.in_cycle = false;
        else more = true;
      }
      if (!more) break;
    }
    // x += Z y for every problem that iterated in this cycle
    std::vector<LaunchRec> upd;
    for (size_t i = 0; i < nn; ++i) {
      State &q = S[i];
      if (!q.active || q.jdone == 0) continue;
      double *y = hy + (size_t)m * i;
      for (int r = q.jdone - 1; r >= 0; --r) {
        double s = q.gv[r];
        for (int c = r + 1; c < q.jdone; ++c) s -= q.H[(size_t)r * m + c] * y[c];
        y[r] = s / q.H[(size_t)r * m + r];
      }
      upd.push_back(as_record(LMultiAxpy<double>{x[i], bv[i].Z, (i64)bv[i].N, q.jdone, dy + (size_t)m * i, 1.0,
                                                 (i64)bv[i].N},
                              grid_for_n(bv[i].N)));
    }
    SMG_HIP(hipMemcpyAsync(dy, hy, sizeof(double) * (size_t)m * nn, hipMemcpyHostToDevice, stream));
    if (!upd.empty()) {
      std::vector<const LaunchRec *> e;
      for (const LaunchRec &r : upd) e.push_back(&r);
      make_plan({e})->run(stream);
    }
    // true residuals of every problem (v_0 of the next cycle)
    resplan->run(stream);
    rnplan->run(stream);
    fetch();
    for (size_t i = 0; i < nn; ++i) {
      State &q = S[i];
      if (!q.active) continue;
      q.beta = std::sqrt(hres[RS * i + 769]);
      q.rel = q.beta / q.bnorm;
      if (!std::isfinite(q.rel)) {
        q.st = SMG_EBREAKDOWN;
        q.active = false;
        continue;
      }
      smg_solve_info *inf = infos ? &infos[i] : nullptr;
      if (q.hist > 0 && inf && inf->history && q.hist - 1 < inf->history_capacity) inf->history[q.hist - 1] = q.rel;
      if (q.rel <= rtol) q.active = false;
    }
  }
  // pressure normalisation and per-problem results
  smg_status first_err = SMG_OK;
  for (size_t i = 0; i < nn; ++i) {
    hipStream_t saved = eng[i]->stream;
    eng[i]->stream = stream;
    try {
      eng[i]->normalize_solution(x[i]);
    } catch (...) {
      eng[i]->stream = saved;
      throw;
    }
    eng[i]->stream = saved;
  }
  SMG_HIP(hipStreamSynchronize(stream));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (size_t i = 0; i < nn; ++i) {
    State &q = S[i];
    if (q.st == SMG_OK && q.rel > rtol) q.st = SMG_ENOTCONV;
    if (first_err == SMG_OK && q.st != SMG_OK) first_err = q.st;
    if (infos) {
      infos[i].iterations = q.it;
      infos[i].rel_residual = q.rel;
      infos[i].rate_q = 0.0;
      infos[i].history_len = std::min(q.hist, infos[i].history_capacity);
      infos[i].t_solve_ms = ms;
      infos[i].t_setup_ms = eng[i]->t_setup_ms;
    }
  }
  return first_err;
}

}  // namespace smg
