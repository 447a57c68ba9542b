// Drives the host runtime through plan creation, passes and destruction for
// every kind of plan and launch shape (general, baseline K = 1..3, derived
// bin counts, shared histograms, both point sources, shared timestamps), and
// through the other entry points (stored-S peaks, FP64 comparator, bins hook,
// phase entropy, profiled passes, autotune with its cache file, the captured
// pass cache cycling through more output buffers than it keeps) and the
// default chunk rule, for use
// with the HIP stand-ins in hip_stub.cpp under the sanitizers.  argv[1]: a
// scratch path for the autotune cache.  Prints "failures: 0" when every call
// returned what it should.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fpw.h"

extern "C" void stub_fail(int kind, long nth);  // hip_stub.cpp: the nth call of a kind fails
extern "C" int stub_failed(void);

namespace {

int failures = 0;
int plans = 0;

void expect(fpw_status got, fpw_status want, const char* what) {
  if (got != want) {
    std::printf("FAIL %s: status %d (want %d) %s\n", what, got, want, fpw_last_error());
    ++failures;
  }
}

struct Batch {
  std::vector<int64_t> off;
  std::vector<double> t, y, dy, f;
};

Batch make_batch(int C, int n_freq) {
  Batch b;
  b.off.assign(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    const int n = 1 + (c * 37) % 260;
    for (int i = 0; i < n; ++i) {
      b.t.push_back(i * 3.7 + c);
      b.y.push_back(std::sin(i * 0.3));
      b.dy.push_back(0.02 + 0.001 * i);
    }
    b.off[c + 1] = (int64_t)b.t.size();
  }
  b.f.resize(n_freq);
  for (int i = 0; i < n_freq; ++i) b.f[i] = 0.05 + i * 0.025;
  return b;
}

// device buffers are host memory under the stand-ins
template <class T>
std::vector<T> buf(size_t n) {
  return std::vector<T>(n ? n : 1);
}

void passes(fpw_plan_t p, const fpw_options& o, int64_t C, int64_t F, int nvar) {
  auto S = buf<float>((size_t)nvar * C * F);
  auto idx = buf<int32_t>((size_t)nvar * C * 16);
  auto val = buf<float>((size_t)nvar * C * 16);
  for (int r = 0; r < 3; ++r)
    expect(fpw_eval_batch(p, S.data(), o.topk ? idx.data() : nullptr, o.topk ? val.data() : nullptr, nullptr), FPW_OK,
           "eval");
  if (o.topk) expect(fpw_eval_batch(p, nullptr, idx.data(), val.data(), nullptr), FPW_OK, "eval without S");
  if (o.profile) {
    float ms[3], wide = -1.f;
    expect(fpw_pass_timings(p, ms), FPW_OK, "timings");
    expect(fpw_pass_wide_ms(p, &wide), FPW_OK, "wide-kernel time");
  }
}

void run(const Batch& b, const fpw_options& o, const char* what) {
  const int64_t C = (int64_t)b.off.size() - 1, F = (int64_t)b.f.size();
  fpw_plan_t p = nullptr;
  fpw_status st = fpw_plan(&p, C, b.off.data(), b.t.data(), b.y.data(), b.dy.data(), F, b.f.data(), &o, nullptr);
  expect(st, FPW_OK, what);
  if (st != FPW_OK) return;
  ++plans;
  fpw_plan_info info;
  expect(fpw_get_plan_info(p, &info), FPW_OK, "info");
  passes(p, o, C, F, info.n_variants);
  for (int v = 0; v < info.n_variants; ++v) {
    int32_t m, off;
    expect(fpw_variant(p, v, &m, &off), FPW_OK, "variant");
  }
  auto S = buf<float>((size_t)C * F);
  auto idx = buf<int32_t>((size_t)C * 4);
  auto val = buf<float>((size_t)C * 4);
  expect(fpw_topk(p, S.data(), 4, idx.data(), val.data(), nullptr), FPW_OK, "topk");
  auto S64 = buf<double>((size_t)C * F);
  expect(fpw_eval_fp64(p, S64.data(), nullptr), o.baseline_terms ? FPW_EUNSUPPORTED : FPW_OK, "fp64");
  auto bins = buf<int32_t>((size_t)(b.off[C] - b.off[C - 1]) * 7);
  expect(fpw_debug_bins(p, o.phase, C - 1, 3, 10, bins.data(), nullptr), FPW_OK, "bins");
  auto H = buf<float>((size_t)C * 2), E = buf<float>((size_t)C * 2), V = buf<float>((size_t)C * 2);
  auto fi = buf<int32_t>((size_t)C * 2);
  expect(fpw_phase_entropy(p, fi.data(), 2, H.data(), E.data(), V.data(), nullptr), FPW_OK, "entropy");
  fpw_plan_destroy(p);
}

// The default chunk of a three-kernel plan of C curves of N observations and
// F frequencies, M = 20 (two waves per histogram), under the stand-ins' 256
// CUs x 4 groups: 1024 consumers.
void expect_chunk(int C, int N, int F, int want, const char* what) {
  Batch b;
  b.off.assign(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    for (int i = 0; i < N; ++i) {
      b.t.push_back(i * 1.9 + c);
      b.y.push_back(std::cos(i * 0.2));
      b.dy.push_back(0.03);
    }
    b.off[c + 1] = (int64_t)b.t.size();
  }
  for (int i = 0; i < F; ++i) b.f.push_back(0.05 + i * 0.005);
  fpw_options o;
  fpw_options_default(&o);
  o.n_bins = 20;
  o.topk = 5;
  o.fuse_prepare = -1;
  o.hist_share = 2;  // plans this small would take four waves per histogram by default
  fpw_plan_t p = nullptr;
  fpw_status st = fpw_plan(&p, C, b.off.data(), b.t.data(), b.y.data(), b.dy.data(), F, b.f.data(), &o, nullptr);
  expect(st, FPW_OK, what);
  if (st != FPW_OK) return;
  ++plans;
  fpw_plan_info info;
  expect(fpw_get_plan_info(p, &info), FPW_OK, "info");
  if (info.hist_share != 2 || info.chunk_freqs != want) {
    std::printf("FAIL %s: share %d chunk %d (want 2, %d)\n", what, info.hist_share, info.chunk_freqs, want);
    ++failures;
  }
  fpw_plan_destroy(p);
}

// A batch in which curve c (of `kinds`) holds its own weight pattern:
// 0 ordinary lognormal-like errors, 1 one point 1e4 times more precise than
// the rest (equal errors otherwise), 2 errors spread over 1e-5..1, 3 over
// 1e-9..1 (beyond every format).
Batch weight_batch(const std::vector<int>& kinds, int n_freq) {
  Batch b;
  b.off.assign(kinds.size() + 1, 0);
  for (size_t c = 0; c < kinds.size(); ++c) {
    const int n = 300;
    for (int i = 0; i < n; ++i) {
      double dy = 0.02 * std::exp(0.4 * std::sin(1.7 * i + (double)c));
      if (kinds[c] == 1) dy = i == n / 2 ? 2e-6 : 0.02;
      if (kinds[c] == 2) dy = std::pow(10.0, -5.0 * ((i * 37) % n) / (double)(n - 1));
      if (kinds[c] == 3) dy = std::pow(10.0, -9.0 * ((i * 37) % n) / (double)(n - 1));
      b.t.push_back(i * 4.1 + (double)c);
      b.y.push_back(dy * std::sin(i * 0.9));
      b.dy.push_back(dy);
    }
    b.off[c + 1] = (int64_t)b.t.size();
  }
  for (int i = 0; i < n_freq; ++i) b.f.push_back(0.05 + i * 0.02);
  return b;
}

fpw_status plan_of(const Batch& b, const fpw_options& o, fpw_plan_t* p) {
  const int64_t C = (int64_t)b.off.size() - 1;
  return fpw_plan(p, C, b.off.data(), b.t.data(), b.y.data(), b.dy.data(), (int64_t)b.f.size(), b.f.data(), &o, nullptr);
}

// Per-bin sum formats: curves are routed by their weights, plans that need
// the narrow format everywhere refuse wide curves, weights beyond both
// formats are refused.
void sum_formats() {
  fpw_options o;
  const Batch mixed = weight_batch({0, 1, 0, 2, 0, 1}, 300);
  for (int M : {1, 7, 20, 64}) {
    for (int topk : {0, 5}) {
      fpw_options_default(&o);
      o.n_bins = M;
      o.topk = topk;
      fpw_plan_t p = nullptr;
      expect(plan_of(mixed, o, &p), FPW_OK, "mixed-weight plan");
      if (!p) continue;
      ++plans;
      fpw_plan_info info;
      expect(fpw_get_plan_info(p, &info), FPW_OK, "info");
      if (info.n_wide_curves != 3 || info.fuse_prepare != 0) {
        std::printf("FAIL mixed-weight plan M=%d: %d wide curves, fused %d (want 3, 0)\n", M, info.n_wide_curves,
                    info.fuse_prepare);
        ++failures;
      }
      passes(p, o, 6, 300, 1);
      fpw_plan_destroy(p);
    }
  }
  // every curve wide on request, ordinary weights included; a profiled pass
  fpw_options_default(&o);
  o.n_bins = 20;
  o.topk = 3;
  o.sum_format = FPW_SUMS_WIDE;
  o.profile = 1;
  fpw_plan_t p = nullptr;
  expect(plan_of(mixed, o, &p), FPW_OK, "all-wide plan");
  if (p) {
    ++plans;
    fpw_plan_info info;
    expect(fpw_get_plan_info(p, &info), FPW_OK, "info");
    if (info.n_wide_curves != 6) {
      std::printf("FAIL all-wide plan: %d wide curves\n", info.n_wide_curves);
      ++failures;
    }
    passes(p, o, 6, 300, 1);
    fpw_plan_destroy(p);
  }
  // plans that keep every curve narrow refuse the wide ones
  struct Refusal {
    int terms, derived, phase, fuse, M;
    const char* what;
  };
  for (const Refusal& r : {Refusal{2, 0, 0, 0, 20, "baseline"}, Refusal{0, 10, 0, 0, 20, "derived bins"},
                           Refusal{0, 0, 2, 0, 20, "df32"}, Refusal{0, 0, 3, 0, 20, "fp32"},
                           Refusal{0, 0, 0, 1, 20, "forced fused pass"}, Refusal{0, 0, 0, 0, 157, "M above wide max"}}) {
    fpw_options_default(&o);
    o.n_bins = r.M;
    o.baseline_terms = r.terms;
    o.derived_bins[0] = r.derived;
    o.phase = r.phase;
    o.fuse_prepare = r.fuse;
    p = nullptr;
    expect(plan_of(mixed, o, &p), FPW_EUNSUPPORTED, r.what);
    if (p) fpw_plan_destroy(p);
  }
  fpw_options_default(&o);
  o.n_bins = 20;
  o.sum_format = FPW_SUMS_WIDE;
  o.baseline_terms = 1;
  p = nullptr;
  expect(plan_of(weight_batch({0}, 50), o, &p), FPW_EUNSUPPORTED, "wide baseline");
  if (p) fpw_plan_destroy(p);
  // beyond both formats, and weights that are not finite normal doubles
  fpw_options_default(&o);
  o.n_bins = 20;
  p = nullptr;
  expect(plan_of(weight_batch({0, 3}, 50), o, &p), FPW_EUNSUPPORTED, "weights beyond the wide format");
  if (p) fpw_plan_destroy(p);
  Batch tiny = weight_batch({0}, 50);
  tiny.dy[7] = 1e-170;
  expect(plan_of(tiny, o, &p), FPW_EUNSUPPORTED, "1/dy^2 overflows");
  tiny.dy[7] = 1e160;
  expect(plan_of(tiny, o, &p), FPW_EUNSUPPORTED, "1/dy^2 underflows");
  // a shared-timestamp plan with a wide curve: the matrix-core kernel refuses, auto takes the general one
  const int C = 5, N = 64, F = 100;
  std::vector<double> t(N), y((size_t)C * N), dy((size_t)C * N, 0.02), f(F);
  for (int i = 0; i < N; ++i) t[i] = i * 7.3;
  for (size_t i = 0; i < y.size(); ++i) y[i] = 0.02 * std::cos(0.7 * (double)i);
  dy[2 * N + 10] = 2e-6;
  for (int i = 0; i < F; ++i) f[i] = 0.1 + 0.03 * i;
  for (int kernel : {0, 2}) {
    fpw_options_default(&o);
    o.n_bins = 20;
    o.shared_kernel = kernel;
    p = nullptr;
    fpw_status st = fpw_plan_shared(&p, C, N, t.data(), y.data(), dy.data(), F, f.data(), &o, nullptr);
    expect(st, kernel == 2 ? FPW_EUNSUPPORTED : FPW_OK, "shared plan with a wide curve");
    if (!p) continue;
    ++plans;
    fpw_plan_info info;
    expect(fpw_get_plan_info(p, &info), FPW_OK, "info");
    if (info.kernel != 0 || info.n_wide_curves != 1) {
      std::printf("FAIL shared plan with a wide curve: kernel %d, %d wide\n", info.kernel, info.n_wide_curves);
      ++failures;
    }
    fpw_plan_destroy(p);
  }
}

// Error paths: the n-th allocation, copy, launch or capture fails, for every
// n up to the calls a plan and a pass make.  A failed call returns its status
// (FPW_ENOMEM for allocations, FPW_EHIP otherwise; a failed capture only
// turns the graph off), leaves no plan behind, sets a message, and leaks
// nothing (AddressSanitizer's leak check runs at exit).
void failure_paths() {
  struct Case {
    const char* what;
    int kind;
  };
  const Batch small = make_batch(6, 300);
  const Batch mixed = weight_batch({0, 1, 0}, 300);
  fpw_options o;
  for (int plan_kind = 0; plan_kind < 4; ++plan_kind) {
    fpw_options_default(&o);
    o.n_bins = 20;
    o.topk = 3;
    if (plan_kind == 1) o.baseline_terms = 2;
    if (plan_kind == 2) o.fuse_prepare = 1;
    const Batch& b = plan_kind == 3 ? mixed : small;
    for (const Case& cs : {Case{"alloc", 1}, Case{"copy", 2}, Case{"launch", 3}, Case{"capture", 4}}) {
      for (long n = 1; n < 400; ++n) {
        stub_fail(cs.kind, n);
        fpw_plan_t p = nullptr;
        fpw_status st = plan_of(b, o, &p);
        const bool in_plan = stub_failed() != 0;
        if (in_plan) {
          const fpw_status want = cs.kind == 1 ? FPW_ENOMEM : (cs.kind == 4 ? FPW_OK : FPW_EHIP);
          if (cs.kind != 4) {
            expect(st, want, cs.what);
            if (p != nullptr || fpw_last_error()[0] == 0) {
              std::printf("FAIL %s %ld in plan: plan left behind or no message\n", cs.what, n);
              ++failures;
            }
          }
          if (p) fpw_plan_destroy(p);
          continue;
        }
        expect(st, FPW_OK, "plan before the failure");
        if (!p) break;
        // the failure falls in the passes: each pass either succeeds or reports it
        auto S = buf<float>(6 * 300);
        auto idx = buf<int32_t>(6 * 3);
        auto val = buf<float>(6 * 3);
        bool any = false;
        for (int r = 0; r < 3; ++r) {
          const bool before = stub_failed() != 0;
          st = fpw_eval_batch(p, S.data(), idx.data(), val.data(), nullptr);
          const bool now = stub_failed() != 0 && !before;
          if (now && cs.kind != 4 && st == FPW_OK) {
            // a failure while capturing is retried as direct launches
          } else if (now && cs.kind != 4) {
            expect(st, cs.kind == 1 ? FPW_ENOMEM : FPW_EHIP, cs.what);
            if (fpw_last_error()[0] == 0) {
              std::printf("FAIL %s %ld in a pass: no message\n", cs.what, n);
              ++failures;
            }
          } else {
            expect(st, FPW_OK, "pass");
          }
          any = any || now;
        }
        fpw_plan_destroy(p);
        if (!any) break;  // n is past every call a plan and its passes make
      }
    }
  }
  stub_fail(0, 0);
}

// fpw_eval_static: argument checks, shapes over sizes, refusal beyond its scratch.
void static_pass() {
  fpw_options o;
  for (int nf : {1, 2, 64, 65, 129, 10000})
    for (int M : {1, 10, 20, 156})
      for (int k : {0, 5}) {
        const Batch b = make_batch(7, nf);
        fpw_options_default(&o);
        o.n_bins = M;
        o.topk = std::min(k, nf);
        auto S = buf<float>((size_t)7 * nf);
        auto idx = buf<int32_t>(7 * 5);
        auto val = buf<float>(7 * 5);
        expect(fpw_eval_static(7, b.off.data(), b.off[7], b.t.data(), b.y.data(), b.dy.data(), nf, b.f.data(), &o,
                               S.data(), o.topk ? idx.data() : nullptr, o.topk ? val.data() : nullptr, nullptr),
               FPW_OK, "static pass");
      }
  const Batch b = make_batch(7, 300);
  auto S = buf<float>(7 * 300);
  auto idx = buf<int32_t>(7 * 5);
  auto val = buf<float>(7 * 5);
  struct Bad {
    const char* what;
    fpw_status want;
    int phase, derived, terms, share, M;
    bool no_out, idx_only, npts_short;
  };
  for (const Bad& c : {Bad{"df32", FPW_EUNSUPPORTED, 2, 0, 0, 0, 20, false, false, false},
                       Bad{"derived", FPW_EUNSUPPORTED, 0, 10, 0, 0, 20, false, false, false},
                       Bad{"baseline", FPW_EUNSUPPORTED, 0, 0, 1, 0, 20, false, false, false},
                       Bad{"share override", FPW_EUNSUPPORTED, 0, 0, 0, 2, 20, false, false, false},
                       Bad{"M above wide max", FPW_EUNSUPPORTED, 0, 0, 0, 0, 157, false, false, false},
                       Bad{"no output", FPW_EINVAL, 0, 0, 0, 0, 20, true, false, false},
                       Bad{"idx without val", FPW_EINVAL, 0, 0, 0, 0, 20, false, true, false},
                       Bad{"fewer points than curves", FPW_EINVAL, 0, 0, 0, 0, 20, false, false, true}}) {
    fpw_options_default(&o);
    o.n_bins = c.M;
    o.topk = 3;
    o.phase = c.phase;
    o.derived_bins[0] = c.derived;
    o.baseline_terms = c.terms;
    o.hist_share = c.share;
    expect(fpw_eval_static(7, b.off.data(), c.npts_short ? 6 : b.off[7], b.t.data(), b.y.data(), b.dy.data(), 300,
                           b.f.data(), &o, c.no_out ? nullptr : S.data(), c.no_out ? nullptr : idx.data(),
                           c.no_out || c.idx_only ? nullptr : val.data(), nullptr),
           c.want, c.what);
  }
  // beyond the static scratch: 1e6 points need 32 MB of records
  Batch big;
  big.off = {0, 1000000};
  big.t.assign(1000000, 1.0);
  big.y.assign(1000000, 0.0);
  big.dy.assign(1000000, 0.1);
  big.f.assign(100, 1.0);
  fpw_options_default(&o);
  expect(fpw_eval_static(1, big.off.data(), 1000000, big.t.data(), big.y.data(), big.dy.data(), 100, big.f.data(),
                         &o, S.data(), nullptr, nullptr, nullptr),
         FPW_EUNSUPPORTED, "beyond the static scratch");
}

}  // namespace

int main(int argc, char** argv) {
  static_pass();
  sum_formats();
  failure_paths();
  const Batch b = make_batch(10, 477);
  fpw_options o;
  // general and baseline plans over bin counts, waves per histogram and point sources
  for (int K : {0, 1, 2, 3})
    for (int M : {1, 7, 20, 40, 64})
      for (int share : {0, 1, 2, 4})
        for (int src : {0, 1, 2}) {
          fpw_options_default(&o);
          o.n_bins = M;
          o.baseline_terms = K;
          o.hist_share = share;
          o.point_source = src;
          o.topk = K ? 3 : 5;
          run(b, o, "plan");
        }
  // derived bin counts, every offset, shared and private
  for (int M : {20, 40, 64})
    for (int share : {0, 1, 2, 4}) {
      fpw_options_default(&o);
      o.n_bins = M;
      o.derived_bins[0] = M / 2;
      o.derived_bins[1] = M / 4;
      o.all_offsets = M == 40;
      o.hist_share = share;
      o.topk = 4;
      run(b, o, "multi-M plan");
    }
  // other phase modes, launch overrides, profiling
  for (int phase : {1, 2, 3}) {
    fpw_options_default(&o);
    o.n_bins = 20;
    o.phase = phase;
    o.topk = 2;
    o.profile = 1;
    run(b, o, "phase plan");
  }
  // the fused pass: forced, refused, with a chunk override, two phase modes
  for (int single : {-1, 0, 1})
    for (int phase : {0, 3})
      for (int chunk : {0, 100}) {
        fpw_options_default(&o);
        o.n_bins = 20;
        o.phase = phase;
        o.fuse_prepare = single;
        o.chunk_freqs = chunk;
        o.topk = 4;
        o.profile = chunk != 0;
        run(b, o, "fused plan");
      }
  fpw_options_default(&o);
  o.n_bins = 20;
  o.freqs_per_lane = 2;
  o.waves_per_group = 4;
  o.chunk_freqs = 100;
  o.topk = 16;
  run(b, o, "override plan");
  // autotune, then a second plan that finds the shape in the cache
  if (argc > 1) {
    for (int r = 0; r < 2; ++r) {
      fpw_options_default(&o);
      o.n_bins = 40;
      o.topk = 5;
      o.autotune = 1;
      o.tune_cache = argv[1];
      run(b, o, "autotune plan");
    }
  }
  // the captured-pass cache: more output buffer sets than it keeps, in turn
  {
    fpw_options_default(&o);
    o.n_bins = 20;
    o.topk = 3;
    const int64_t C = 10, F = 477;
    fpw_plan_t p = nullptr;
    expect(fpw_plan(&p, C, b.off.data(), b.t.data(), b.y.data(), b.dy.data(), F, b.f.data(), &o, nullptr), FPW_OK,
           "graph plan");
    std::vector<std::vector<float>> Ss(6, buf<float>(C * F));
    std::vector<std::vector<int32_t>> is(6, buf<int32_t>(C * 3));
    std::vector<std::vector<float>> vs(6, buf<float>(C * 3));
    for (int r = 0; r < 20; ++r) {
      const int k = (r * 5) % 6;
      expect(fpw_eval_batch(p, Ss[k].data(), is[k].data(), vs[k].data(), nullptr), FPW_OK, "graph eval");
    }
    fpw_plan_destroy(p);
  }
  // shared timestamps: matrix-core and general kernels, and a baseline on a shared plan
  // (kernel: 0 auto, 1 general, 2 matrix; the auto plan with a baseline takes the general path)
  for (int mode : {0, 1, 2, 3})
    for (int M : {1, 20, 64}) {
      const int kernel = mode == 3 ? 0 : mode;
      const int C = 21, N = 37, F = 300;
      std::vector<double> t(N), y((size_t)C * N), dy((size_t)C * N, 0.03), f(F);
      for (int i = 0; i < N; ++i) t[i] = i * 11.3;
      for (size_t i = 0; i < y.size(); ++i) y[i] = std::cos(0.7 * (double)i);
      for (int i = 0; i < F; ++i) f[i] = 0.1 + 0.03 * i;
      fpw_options_default(&o);
      o.n_bins = M;
      o.shared_kernel = kernel;
      o.topk = 3;
      o.baseline_terms = mode == 3 ? 2 : 0;
      fpw_plan_t p = nullptr;
      fpw_status st = fpw_plan_shared(&p, C, N, t.data(), y.data(), dy.data(), F, f.data(), &o, nullptr);
      expect(st, FPW_OK, "shared plan");
      if (st != FPW_OK) continue;
      ++plans;
      passes(p, o, C, F, 1);
      fpw_plan_destroy(p);
    }
  // default chunks: ~12 items per consumer, raised to >= 1.2e5 evaluations per wave and item (550 / 2
  // observations per wave: 437 frequencies) unless that leaves consumers idle, in sweeps of 64
  expect_chunk(64, 550, 10000, 448, "chunk floor");        // 12 per consumer: 53; floor 437
  expect_chunk(16, 550, 10000, 192, "chunk fill cap");     // floor 437 > 16 * 1e4 / 1024 = 157
  expect_chunk(4000, 4, 4096, 16000, "chunk tiny curves");  // floor 6e4 > fill cap 4096 * 4000 / 1024 = 16000
  expect_chunk(1200, 550, 40000, 3968, "chunk 12 per consumer");  // 4e4 / (12 * 1024 / 1200) = 3907 > 437
  expect_chunk(3000, 550, 1000, 448, "chunk floor over 12 per consumer");  // 1000 / (12 * 1024 / 3000) = 245 < 437
  std::printf("plans: %d, failures: %d\n", plans, failures);
  return failures != 0;
}
