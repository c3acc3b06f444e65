// Call sequences of the engine's batch and plan tests, run on the host
// emulation (see hip/hip_runtime.h) under ASan/UBSan.  Every kernel runs on
// the CPU; every pass and table launch is range-checked against the memory
// registered here for its problem; each batch member must come out bitwise
// equal to the same problem propagated alone by a plan, as on the GPU.
//
// Usage: drive <scenario>   (scenarios listed in main)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "brahms.h"
#include "emu.hpp"

namespace {

struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 0x9e3779b97f4a7c15ull + 1) {}
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform(double a, double b) { return a + (b - a) * double(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct Problem {
  int nx, ny, nt, nf, nz;
  brahms_params prm{};
  std::vector<double> dk;
  std::vector<std::vector<float2>> init;
  int order = 0;
};

Problem make_problem(Rng& r, int nx, int ny, int nt, int nf, int nz, bool profile, double dk_const) {
  Problem p{nx, ny, nt, nf, nz};
  p.prm.dz = 1.0 / nz;
  p.prm.dk_const = dk_const;
  for (int j = 0; j < nf; ++j) {
    brahms_field_params& f = p.prm.field[j];
    f.kappa = 1.0 + 0.2 * j;
    f.diffraction = r.uniform(0.5, 2.0);
    f.tan_rho = r.uniform(-0.5, 0.5);
    f.delay = r.uniform(-1, 1);
    f.k2 = r.uniform(-2, 2);
  }
  if (profile) {
    p.dk.resize(size_t(nz));
    for (double& v : p.dk) v = 1.5 + r.uniform(-1, 1);
  }
  const size_t n = size_t(nx) * ny * nt;
  p.init.assign(size_t(nf), std::vector<float2>(n));
  for (auto& f : p.init)
    for (auto& v : f) v = make_float2(float(r.uniform(-0.7, 0.7)), float(r.uniform(-0.7, 0.7)));
  return p;
}

void set_profile(Problem& p) {
  p.prm.dk = p.dk.empty() ? nullptr : p.dk.data();
  p.prm.n_dk = int(p.dk.size());
}

#define OK(call)                                                                               \
  do {                                                                                         \
    brahms_status st_ = (call);                                                                \
    if (st_ != BRAHMS_OK) emu::die(std::string(#call) + " -> " + std::to_string(st_) + ": " + \
                                   brahms_last_error());                                       \
  } while (0)

struct Fields {
  std::vector<float2*> ptr;   // problem-major
  std::vector<size_t> bytes;
};

Fields upload(std::vector<Problem>& ps) {
  Fields f;
  for (Problem& p : ps)
    for (auto& h : p.init) {
      const size_t b = h.size() * sizeof(float2);
      auto* d = static_cast<float2*>(emu::device_alloc(b));
      std::memcpy(d, h.data(), b);
      f.ptr.push_back(d);
      f.bytes.push_back(b);
    }
  return f;
}

void release(Fields& f) {
  for (float2* p : f.ptr) emu::device_free(p);
  f.ptr.clear();
}

// One problem alone through a plan with the given schedule.
std::vector<std::vector<float2>> run_alone(Problem& p, int order, int merge, int fuse, int graph = 0,
                                           int wide = 0) {
  set_profile(p);
  std::vector<Problem> one{p};
  Fields f = upload(one);
  brahms_plan plan = nullptr;
  OK(brahms_plan_create(p.nx, p.ny, p.nt, p.nf, &p.prm, nullptr, &plan));
  brahms_schedule sc{};
  sc.pass_order = order;
  sc.merge_halves = merge;
  sc.fuse_steps = fuse;
  sc.graph = graph;
  sc.wide = wide;
  size_t ws_bytes = 0;
  OK(brahms_plan_workspace_size(plan, &ws_bytes));
  void* ws = emu::device_alloc(ws_bytes);
  emu::clear_regions();
  for (size_t k = 0; k < f.ptr.size(); ++k) emu::register_region(f.ptr[k], f.bytes[k], 0, "field");
  emu::register_region(ws, ws_bytes, 0, "plan workspace");
  OK(brahms_plan_set_schedule(plan, &sc));
  std::vector<void*> fp(f.ptr.begin(), f.ptr.end());
  OK(brahms_plan_bind(plan, fp.data(), ws));
  OK(brahms_step(plan, p.nz));
  OK(hipDeviceSynchronize() == hipSuccess ? BRAHMS_OK : BRAHMS_E_DEVICE);
  std::vector<std::vector<float2>> out;
  for (size_t k = 0; k < f.ptr.size(); ++k)
    out.emplace_back(f.ptr[k], f.ptr[k] + f.bytes[k] / sizeof(float2));
  OK(brahms_plan_destroy(plan));
  emu::device_free(ws);
  release(f);
  emu::clear_regions();
  return out;
}

struct BatchRun {
  std::vector<std::vector<std::vector<float2>>> out;   // [problem][field]
};

// The sequence of the batch tests: create, schedule calls, bind, run, wait,
// destroy, with the workspace and fields released after the destroy.
BatchRun run_batch(std::vector<Problem>& ps, int group_max, const std::vector<int>* orders,
                   const std::vector<int>* limits, int merge, int fuse, int runs = 1, int streams = 1) {
  const int n = int(ps.size());
  std::vector<int> shapes, steps;
  std::vector<brahms_params> prm;
  for (Problem& p : ps) {
    set_profile(p);
    shapes.insert(shapes.end(), {p.nx, p.ny, p.nt, p.nf});
    steps.push_back(p.nz);
    prm.push_back(p.prm);
  }
  brahms_batch b = nullptr;
  OK(brahms_batch_create(n, shapes.data(), prm.data(), steps.data(), nullptr, &b));
  OK(brahms_batch_set_schedule(b, group_max, orders ? orders->data() : nullptr));
  if (limits) OK(brahms_batch_set_group_limits(b, limits->data()));
  if (merge) OK(brahms_batch_set_merge_halves(b, 1));
  if (fuse) OK(brahms_batch_set_fuse_steps(b, 1));
  if (streams != 1) OK(brahms_batch_set_streams(b, streams > 0 ? streams : -streams, streams < 0));
  Fields f = upload(ps);
  size_t ws_bytes = 0;
  OK(brahms_batch_workspace_size(b, &ws_bytes));
  char* ws = static_cast<char*>(emu::device_alloc(ws_bytes));
  // the batch lays the problems' plan workspaces out one after the other
  // (each rounded up to 256 bytes), then its descriptors
  emu::clear_regions();
  size_t off = 0, fi = 0;
  for (int i = 0; i < n; ++i) {
    brahms_plan tmp = nullptr;
    OK(brahms_plan_create(ps[i].nx, ps[i].ny, ps[i].nt, ps[i].nf, &prm[i], nullptr, &tmp));
    size_t wsz = 0;
    OK(brahms_plan_workspace_size(tmp, &wsz));
    OK(brahms_plan_destroy(tmp));
    emu::register_region(ws + off, wsz, i, "member workspace");
    off = (off + wsz + 255) / 256 * 256;
    for (int j = 0; j < ps[i].nf; ++j, ++fi) emu::register_region(f.ptr[fi], f.bytes[fi], i, "member field");
  }
  if (off > ws_bytes) emu::die("member workspaces exceed the batch workspace");
  emu::register_region(ws + off, ws_bytes - off, -1, "batch descriptors");
  std::vector<void*> fp(f.ptr.begin(), f.ptr.end());
  OK(brahms_batch_bind(b, fp.data(), ws));
  for (int r = 0; r < runs; ++r) {
    if (r > 0) {
      // a replay from the entrance fields again
      fi = 0;
      for (Problem& p : ps)
        for (auto& h : p.init) std::memcpy(f.ptr[fi++], h.data(), h.size() * sizeof(float2));
    }
    OK(brahms_batch_run(b));
    OK(hipDeviceSynchronize() == hipSuccess ? BRAHMS_OK : BRAHMS_E_DEVICE);
  }
  OK(brahms_batch_destroy(b));
  BatchRun res;
  fi = 0;
  for (int i = 0; i < n; ++i) {
    res.out.emplace_back();
    for (int j = 0; j < ps[i].nf; ++j, ++fi)
      res.out.back().emplace_back(f.ptr[fi], f.ptr[fi] + f.bytes[fi] / sizeof(float2));
  }
  emu::device_free(ws);
  release(f);
  emu::clear_regions();
  return res;
}

void expect_equal(const std::vector<std::vector<float2>>& a, const std::vector<std::vector<float2>>& b,
                  const std::string& what) {
  if (a.size() != b.size()) emu::die(what + ": field count");
  for (size_t j = 0; j < a.size(); ++j)
    if (a[j].size() != b[j].size() || std::memcmp(a[j].data(), b[j].data(), a[j].size() * sizeof(float2)) != 0)
      emu::die(what + ": batch member differs from the plan run (field " + std::to_string(j) + ")");
}

// _problems() of the batch tests: mixed shapes and field counts.
std::vector<Problem> mixed_problems(uint64_t seed, bool profiles) {
  Rng r(seed);
  const int spec[7][5] = {{32, 32, 16, 2, 23}, {32, 32, 16, 2, 9}, {16, 64, 32, 3, 17}, {32, 32, 16, 2, 40},
                          {96, 96, 4, 2, 12},  {16, 64, 32, 3, 5}, {64, 8, 8, 2, 70}};
  std::vector<Problem> ps;
  for (auto& s : spec)
    ps.push_back(make_problem(r, s[0], s[1], s[2], s[3], s[4], profiles && (s[4] % 2 == 1), r.uniform(-3, 3)));
  return ps;
}

std::vector<Problem> long_tau_problems(uint64_t seed) {
  Rng r(seed);
  const int spec[5][5] = {{8, 4, 1024, 2, 9}, {4, 4, 4096, 3, 7}, {8, 4, 1024, 2, 5}, {16, 8, 512, 3, 11},
                          {16, 16, 16, 2, 8}};
  std::vector<Problem> ps;
  for (auto& s : spec) ps.push_back(make_problem(r, s[0], s[1], s[2], s[3], s[4], false, 0.7));
  return ps;
}

void compare_with_plans(std::vector<Problem>& ps, const BatchRun& br, const std::vector<int>& orders, int merge,
                        int fuse, const std::string& what) {
  for (size_t i = 0; i < ps.size(); ++i) {
    const bool long_tau = ps[i].nt > 256;
    const auto alone = run_alone(ps[i], orders.empty() ? 0 : orders[i], merge, long_tau ? 0 : fuse);
    expect_equal(br.out[i], alone, what + " problem " + std::to_string(i));
  }
}

// test_batch_equals_plain_runs_bitwise (per-step dk profiles, orders k % 4)
void scenario_plain_batches() {
  for (int gm : {0, 2, 1, -1}) {
    auto ps = mixed_problems(11, true);
    std::vector<int> orders;
    for (size_t k = 0; k < ps.size(); ++k) orders.push_back(int(k % 4));
    std::vector<int> limits;
    if (gm == -1)
      for (size_t k = 0; k < ps.size(); ++k) limits.push_back(int(k % 3));
    const BatchRun br = run_batch(ps, gm < 0 ? 0 : gm, &orders, gm == -1 ? &limits : nullptr, 0, 0, 2);
    compare_with_plans(ps, br, orders, 0, 0, "plain batch gm=" + std::to_string(gm));
    std::printf("plain batches group_max=%d: ok\n", gm);
  }
}

// test_merged_batch_equals_plain_runs_and_oracle (skipped on the GPU)
void scenario_merged_batches() {
  for (int gm : {0, 1})
    for (int fuse : {0, 1}) {
      auto ps = mixed_problems(13, false);
      std::vector<int> orders;
      for (size_t k = 0; k < ps.size(); ++k) orders.push_back(int((k + 1) % 4));
      const BatchRun br = run_batch(ps, gm, &orders, nullptr, 1, fuse);
      compare_with_plans(ps, br, orders, 1, fuse, "merged batch");
      std::printf("merged batches group_max=%d fuse=%d: ok\n", gm, fuse);
    }
  // a batch with dk profiles refuses merging
  auto ps = mixed_problems(13, true);
  ps.resize(2);
  std::vector<int> shapes, steps;
  std::vector<brahms_params> prm;
  for (Problem& p : ps) {
    set_profile(p);
    shapes.insert(shapes.end(), {p.nx, p.ny, p.nt, p.nf});
    steps.push_back(p.nz);
    prm.push_back(p.prm);
  }
  brahms_batch b = nullptr;
  OK(brahms_batch_create(2, shapes.data(), prm.data(), steps.data(), nullptr, &b));
  if (brahms_batch_set_merge_halves(b, 1) != BRAHMS_E_UNSUPPORTED) emu::die("merging with a profile accepted");
  if (brahms_batch_set_fuse_steps(b, 1) != BRAHMS_E_INVALID_ARG) emu::die("fusing without merging accepted");
  OK(brahms_batch_destroy(b));
}

// test_long_tau_in_batches (skipped on the GPU)
void scenario_long_tau_batches() {
  for (int gm : {0, 1})
    for (int merge : {0, 1}) {
      auto ps = long_tau_problems(21);
      const BatchRun br = run_batch(ps, gm, nullptr, nullptr, merge, 0);
      compare_with_plans(ps, br, {}, merge, 0, "long tau batch");
      std::printf("long tau batches group_max=%d merge=%d: ok\n", gm, merge);
    }
}

// long tau problems beside a fused group of an ordinary shape (fused step
// pairs in such batches are refused by the library; a build without that
// refusal runs them)
void scenario_long_tau_fused() {
  for (int gm : {0, 1}) {
    auto ps = long_tau_problems(23);
    std::vector<int> shapes, steps;
    std::vector<brahms_params> prm;
    for (Problem& p : ps) {
      shapes.insert(shapes.end(), {p.nx, p.ny, p.nt, p.nf});
      steps.push_back(p.nz);
      prm.push_back(p.prm);
    }
    brahms_batch b = nullptr;
    OK(brahms_batch_create(int(ps.size()), shapes.data(), prm.data(), steps.data(), nullptr, &b));
    OK(brahms_batch_set_merge_halves(b, 1));
    const brahms_status st = brahms_batch_set_fuse_steps(b, 1);
    OK(brahms_batch_destroy(b));
    if (st == BRAHMS_E_UNSUPPORTED) {
      std::printf("long tau fused batches: refused by this build\n");
      return;
    }
    OK(st);
    const BatchRun br = run_batch(ps, gm, nullptr, nullptr, 1, 1);
    compare_with_plans(ps, br, {}, 1, 1, "long tau fused batch");
    std::printf("long tau fused batches group_max=%d: ok\n", gm);
  }
}

// test_three_field_merged_batch_of_one_shape
void scenario_three_field_one_shape() {
  for (int fuse : {0, 1}) {
    Rng r(31);
    std::vector<Problem> ps;
    for (int nz : {12, 7, 16}) ps.push_back(make_problem(r, 16, 32, 32, 3, nz, false, r.uniform(-3, 3)));
    std::vector<int> orders(ps.size(), 2);
    const BatchRun br = run_batch(ps, 0, &orders, nullptr, 1, fuse);
    compare_with_plans(ps, br, orders, 1, fuse, "three-field batch");
    std::printf("three-field batch fuse=%d: ok\n", fuse);
  }
}

// reduced dimensions: CW (nt = 1) and plane-wave (nx = ny = 1) problems
void scenario_reduced_dims() {
  Rng r(41);
  std::vector<Problem> ps;
  for (int k = 0; k < 5; ++k) ps.push_back(make_problem(r, 16, 16, 1, 2, 9 + k, false, r.uniform(-4, -2)));
  for (int k = 0; k < 3; ++k) ps.push_back(make_problem(r, 1, 1, 64, 2, 11 + k, false, 0.3));
  for (int merge : {0, 1}) {
    const BatchRun br = run_batch(ps, 0, nullptr, nullptr, merge, 0);
    compare_with_plans(ps, br, {}, merge, 0, "reduced-dimension batch");
    std::printf("reduced dims merge=%d: ok\n", merge);
  }
}

// the second register/lane splits: plans with every axis on its second split
// and batches with per-problem splits
void scenario_splits() {
  Rng r(83);
  std::vector<Problem> ps;
  const int spec[4][5] = {{64, 16, 32, 2, 9}, {64, 16, 32, 2, 7}, {48, 24, 8, 3, 6}, {8, 12, 64, 3, 5}};
  for (auto& s : spec) ps.push_back(make_problem(r, s[0], s[1], s[2], s[3], s[4], false, r.uniform(-3, 3)));
  const std::vector<int> splits = {7, 1, 5, 6};
  // and 512-thread linear x and y passes on some problems (bitwise the plan
  // without them)
  const std::vector<int> wide = {3, 0, 2, 1};
  for (int merge : {0, 1}) {
    const int n = int(ps.size());
    std::vector<int> shapes, steps;
    std::vector<brahms_params> prm;
    for (Problem& p : ps) {
      shapes.insert(shapes.end(), {p.nx, p.ny, p.nt, p.nf});
      steps.push_back(p.nz);
      prm.push_back(p.prm);
    }
    brahms_batch b = nullptr;
    OK(brahms_batch_create(n, shapes.data(), prm.data(), steps.data(), nullptr, &b));
    OK(brahms_batch_set_splits(b, splits.data()));
    OK(brahms_batch_set_wide(b, wide.data()));
    if (merge) {
      OK(brahms_batch_set_merge_halves(b, 1));
      OK(brahms_batch_set_fuse_steps(b, 1));
    }
    Fields f = upload(ps);
    size_t ws_bytes = 0;
    OK(brahms_batch_workspace_size(b, &ws_bytes));
    void* ws = emu::device_alloc(ws_bytes);
    emu::clear_regions();
    emu::register_region(ws, ws_bytes, -1, "batch workspace");
    for (size_t k = 0; k < f.ptr.size(); ++k) emu::register_region(f.ptr[k], f.bytes[k], -1, "field");
    std::vector<void*> fp(f.ptr.begin(), f.ptr.end());
    OK(brahms_batch_bind(b, fp.data(), ws));
    OK(brahms_batch_run(b));
    OK(hipDeviceSynchronize() == hipSuccess ? BRAHMS_OK : BRAHMS_E_DEVICE);
    OK(brahms_batch_destroy(b));
    size_t fi = 0;
    for (int i = 0; i < n; ++i) {
      std::vector<std::vector<float2>> got;
      for (int j = 0; j < ps[i].nf; ++j, ++fi) got.emplace_back(f.ptr[fi], f.ptr[fi] + f.bytes[fi] / sizeof(float2));
      // a plan with the same split
      set_profile(ps[i]);
      std::vector<Problem> one{ps[i]};
      Fields g = upload(one);
      brahms_plan plan = nullptr;
      OK(brahms_plan_create(ps[i].nx, ps[i].ny, ps[i].nt, ps[i].nf, &ps[i].prm, nullptr, &plan));
      brahms_schedule sc{};
      sc.merge_halves = merge;
      sc.fuse_steps = merge;
      sc.split = splits[size_t(i)];
      OK(brahms_plan_set_schedule(plan, &sc));
      size_t pw = 0;
      OK(brahms_plan_workspace_size(plan, &pw));
      void* pws = emu::device_alloc(pw);
      emu::clear_regions();
      for (size_t k = 0; k < g.ptr.size(); ++k) emu::register_region(g.ptr[k], g.bytes[k], 0, "field");
      emu::register_region(pws, pw, 0, "plan workspace");
      std::vector<void*> gp(g.ptr.begin(), g.ptr.end());
      OK(brahms_plan_bind(plan, gp.data(), pws));
      OK(brahms_step(plan, ps[i].nz));
      OK(hipDeviceSynchronize() == hipSuccess ? BRAHMS_OK : BRAHMS_E_DEVICE);
      std::vector<std::vector<float2>> want;
      for (size_t k = 0; k < g.ptr.size(); ++k) want.emplace_back(g.ptr[k], g.ptr[k] + g.bytes[k] / sizeof(float2));
      expect_equal(got, want, "split batch problem " + std::to_string(i));
      OK(brahms_plan_destroy(plan));
      emu::device_free(pws);
      release(g);
    }
    emu::device_free(ws);
    release(f);
    emu::clear_regions();
    std::printf("splits merge=%d: ok\n", merge);
  }
}

// runs on several streams (a linear graph per stream) instead of one graph
void scenario_stream_graphs() {
  for (int streams : {2, 4, -3})   // negative: the largest group alone after the others
    for (int merge : {0, 1}) {
      auto ps = mixed_problems(19, false);
      std::vector<int> orders;
      for (size_t k = 0; k < ps.size(); ++k) orders.push_back(int((k + 2) % 4));
      const BatchRun br = run_batch(ps, 1, &orders, nullptr, merge, merge, 2, streams);
      compare_with_plans(ps, br, orders, merge, merge, "streams batch");
      std::printf("streams=%d merge=%d: ok\n", streams, merge);
    }
}

// axis lengths 3 * 2^a and 9 * 2^a in batches and plans
void scenario_three_lengths() {
  Rng r(61);
  std::vector<Problem> ps;
  const int spec[7][5] = {{24, 12, 6, 3, 9}, {24, 12, 6, 3, 5}, {192, 3, 4, 2, 7}, {6, 48, 12, 2, 11},
                          {18, 9, 36, 3, 5}, {72, 4, 9, 2, 4}, {9, 144, 2, 2, 3}};
  for (auto& s : spec) ps.push_back(make_problem(r, s[0], s[1], s[2], s[3], s[4], false, r.uniform(-3, 3)));
  for (int merge : {0, 1}) {
    std::vector<int> orders;
    for (size_t k = 0; k < ps.size(); ++k) orders.push_back(int(k % 4));
    const BatchRun br = run_batch(ps, 0, &orders, nullptr, merge, merge);
    compare_with_plans(ps, br, orders, merge, merge, "3 * 2^a and 9 * 2^a batch");
    std::printf("3 * 2^a and 9 * 2^a lengths merge=%d: ok\n", merge);
  }
}

// the autotuner's sequence on one batch: repeated schedule changes, binds and
// runs before the final destroy
void scenario_tuner_sequence() {
  auto ps = mixed_problems(17, false);
  const int n = int(ps.size());
  std::vector<int> shapes, steps;
  std::vector<brahms_params> prm;
  for (Problem& p : ps) {
    set_profile(p);
    shapes.insert(shapes.end(), {p.nx, p.ny, p.nt, p.nf});
    steps.push_back(p.nz);
    prm.push_back(p.prm);
  }
  brahms_batch b = nullptr;
  OK(brahms_batch_create(n, shapes.data(), prm.data(), steps.data(), nullptr, &b));
  Fields f = upload(ps);
  std::vector<void*> fp(f.ptr.begin(), f.ptr.end());
  std::vector<int> lim(size_t(n), 1);
  std::vector<int> ord(size_t(n), 3);
  void* ws = nullptr;
  size_t have = 0;
  auto rebind = [&]() {
    size_t need = 0;
    OK(brahms_batch_workspace_size(b, &need));
    if (need > have) {
      if (ws) emu::device_free(ws);
      ws = emu::device_alloc(need);
      have = need;
    }
    emu::clear_regions();
    emu::register_region(ws, have, -1, "batch workspace");   // ownership not tracked here
    for (size_t k = 0; k < f.ptr.size(); ++k) emu::register_region(f.ptr[k], f.bytes[k], -1, "field");
    OK(brahms_batch_bind(b, fp.data(), ws));
    OK(brahms_batch_run(b));
  };
  for (int gm : {0, 1, 1 << 30}) {
    OK(brahms_batch_set_schedule(b, gm, nullptr));
    rebind();
  }
  OK(brahms_batch_set_group_limits(b, lim.data()));
  rebind();
  OK(brahms_batch_set_group_limits(b, nullptr));
  OK(brahms_batch_set_schedule(b, 0, ord.data()));
  OK(brahms_batch_set_merge_halves(b, 1));
  rebind();
  OK(brahms_batch_set_fuse_steps(b, 1));
  rebind();
  OK(hipDeviceSynchronize() == hipSuccess ? BRAHMS_OK : BRAHMS_E_DEVICE);
  OK(brahms_batch_destroy(b));
  emu::device_free(ws);
  release(f);
  emu::clear_regions();
  std::printf("tuner sequence: ok\n");
}

// plans: every schedule, graph replays against eager stepping, and the
// no-allocation entry point
void scenario_plans() {
  Rng r(51);
  Problem p = make_problem(r, 16, 8, 32, 3, 70, false, 0.9);
  for (int order = 0; order < 4; ++order) {
    const auto eager = run_alone(p, order, 1, 1, 0);
    const auto graph = run_alone(p, order, 1, 1, 1);
    expect_equal(eager, graph, "graph replay order " + std::to_string(order));
  }
  Problem lt = make_problem(r, 4, 8, 512, 2, 70, false, 0.9);
  expect_equal(run_alone(lt, 0, 1, 1, 0), run_alone(lt, 0, 1, 1, 1), "long tau graph replay");
  Problem prof = make_problem(r, 8, 16, 16, 2, 66, true, 0.0);
  expect_equal(run_alone(prof, 1, 0, 0, 0), run_alone(prof, 1, 0, 0, 1), "profile graph replay");
  // 512-thread linear passes on every axis, in every order, merged and
  // fused (partial blocks: 16 x 8 x 32 has 128 y lines and 128 tau lines)
  for (int order = 0; order < 4; ++order)
    for (int fuse = 0; fuse < 2; ++fuse)
      expect_equal(run_alone(p, order, 1, fuse, 0, 7), run_alone(p, order, 1, fuse, 0, 0),
                   "wide linear passes order " + std::to_string(order));
  std::printf("plans: ok\n");
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: drive <scenario>\n");
    return 2;
  }
  const std::string s = argv[1];
  if (s == "plain_batches") scenario_plain_batches();
  else if (s == "merged_batches") scenario_merged_batches();
  else if (s == "long_tau_batches") scenario_long_tau_batches();
  else if (s == "three_field") scenario_three_field_one_shape();
  else if (s == "long_tau_fused") scenario_long_tau_fused();
  else if (s == "reduced_dims") scenario_reduced_dims();
  else if (s == "tuner_sequence") scenario_tuner_sequence();
  else if (s == "plans") scenario_plans();
  else if (s == "three_lengths") scenario_three_lengths();
  else if (s == "stream_graphs") scenario_stream_graphs();
  else if (s == "splits") scenario_splits();
  else {
    std::fprintf(stderr, "unknown scenario %s\n", s.c_str());
    return 2;
  }
  std::printf("launches %lld, checked passes %lld, checked tables %lld\n", emu::g_launches,
              emu::g_checked_passes, emu::g_checked_tables);
  return 0;
}
