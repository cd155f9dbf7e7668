// C ABI entry points: argument checks, context and plan caches, the host half
// of the single-pulse search (joining tile fragments, ordering), grouping.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "gsp_internal.h"

namespace gsp {

void fail(int status, const std::string &msg) { throw Error{status, msg}; }

void check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) fail(GSP_ENOMEM, std::string(what) + ": out of device memory");
  fail(GSP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DevBuf::~DevBuf() {
  if (ptr) {
    (void)hipSetDevice(device);
    (void)hipFree(ptr);
  }
}

void DevBuf::reserve(size_t n) {
  if (n <= bytes && ptr) return;
  if (ptr) {
    check_hip(hipFree(ptr), "free scratch");
    ptr = nullptr;
    bytes = 0;
  }
  check_hip(hipMalloc(&ptr, n ? n : 1), "allocate scratch");
  bytes = n;
}

static hipEvent_t pool_event(gsp_ctx *ctx) {
  if (!ctx->prof_pool.empty()) {
    hipEvent_t e = ctx->prof_pool.back();
    ctx->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  check_hip(hipEventCreate(&e), "create event");
  return e;
}

ProfScope::ProfScope(gsp_ctx *c, const char *name, hipStream_t s, double work) : ctx(c), st(s), idx(SIZE_MAX) {
  if (!ctx || !ctx->prof) return;
  ProfRec r{name, pool_event(ctx), pool_event(ctx), work};
  check_hip(hipEventRecord(r.start, st), "record event");
  idx = ctx->prof_recs.size();
  ctx->prof_recs.push_back(r);
}

ProfScope::~ProfScope() {
  if (idx != SIZE_MAX) (void)hipEventRecord(ctx->prof_recs[idx].stop, st);
}

RowTables &row_tables(gsp_ctx *ctx, const gsp_dmt_desc *desc, const double *freqs, int32_t s) {
  const std::string key = plan_key(desc, freqs);
  auto it = ctx->plans.find(key);
  if (it == ctx->plans.end()) {
    if (ctx->plans.size() >= 8) ctx->plans.clear();  // bounded cache
    auto pc = std::make_unique<PlanCache>();
    pc->key = key;
    pc->rows.resize(desc->n_seg);
    it = ctx->plans.emplace(key, std::move(pc)).first;
  }
  auto &slot = it->second->rows[s];
  const DedispShape want = shape_for_row(ctx, desc, s);
  const DedispShape had = slot ? slot->req : want;
  if (slot && (had.groups != want.groups || had.tpw != want.tpw || had.waves != want.waves || had.kind != want.kind ||
               had.chunk != want.chunk))
    slot.reset();  // the tuned shape changed since the tables were built
  if (!slot) {
    auto rt = std::make_unique<RowTables>();
    try {
      build_row_tables(ctx, desc, freqs, s, want, *rt);
    } catch (const Error &e) {
      // the byte-quad default does not suit every row (delay spreads wider
      // than its LDS copies): such rows split their band between the two
      // tiles where the quads that do not fit lie at one end of it, else
      // keep the 16-bit tile
      const bool tuned = ctx->tuned.count(row_signature(desc, s)) > 0;
      if (e.status != GSP_EINVAL || want.kind != 2 || tuned) throw;
      std::vector<int32_t> delays = std::move(rt->delays_host);
      rt = std::make_unique<RowTables>();
      rt->delays_host = delays;
      DedispShape split = want;
      split.kind = 3;
      try {
        build_row_tables(ctx, desc, freqs, s, split, *rt);
      } catch (const Error &e2) {
        if (e2.status != GSP_EINVAL) throw;
        DedispShape pair;  // the 16-bit tile's default (4, 4, 8, 32)
        pair.kind = 0;
        pair.groups = 4;
        pair.tpw = 4;
        pair.waves = 8;
        pair.chunk = 32;
        rt = std::make_unique<RowTables>();
        rt->delays_host = std::move(delays);
        build_row_tables(ctx, desc, freqs, s, pair, *rt);
      }
    }
    rt->req = want;
    slot = std::move(rt);
  }
  return *slot;
}

}  // namespace gsp

using namespace gsp;


extern "C" {

const char *gsp_strerror(int status) {
  switch (status) {
    case GSP_OK: return "success";
    case GSP_EINVAL: return "invalid argument";
    case GSP_ETOOSHORT: return "input shorter than a plan row's maximum delay";
    case GSP_EOVERFLOW: return "sum or size overflow";
    case GSP_ECAPACITY: return "output capacity too small";
    case GSP_ENOMEM: return "out of memory";
    case GSP_EDEVICE: return "device error";
    case GSP_EAGAIN: return "not admitted now; retry later";
    default: return "unknown status";
  }
}

const char *gsp_last_error(const gsp_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int gsp_create(int device, gsp_ctx **out) {
  if (!out) return GSP_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return GSP_EDEVICE;
  if (device < 0 || device >= n) return GSP_EINVAL;
  try {
    auto *c = new gsp_ctx();
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) {
      delete c;
      return GSP_EDEVICE;
    }
    try {
      gsp::noalloc_init(device);  // once per device: address of the static search scratch
    } catch (const gsp::Error &e) {
      delete c;
      return e.status;
    }
    *out = c;
    return GSP_OK;
  } catch (...) {
    return GSP_ENOMEM;
  }
}

void gsp_destroy(gsp_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto &r : ctx->prof_recs) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
  delete ctx;
}

int gsp_profile_enable(gsp_ctx *ctx, int enable) {
  if (!ctx) return GSP_EINVAL;
  ctx->prof = enable != 0;
  return GSP_OK;
}

int gsp_profile_read(gsp_ctx *ctx, gsp_kernel_stat *out, int32_t cap, int32_t *n, int reset) {
  if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return GSP_EINVAL;
  return guarded(ctx, [&] {
    std::vector<gsp_kernel_stat> agg;
    for (auto &r : ctx->prof_recs) {
      check_hip(hipEventSynchronize(r.stop), "wait for event");
      float ms = 0.f;
      check_hip(hipEventElapsedTime(&ms, r.start, r.stop), "event time");
      auto it = std::find_if(agg.begin(), agg.end(), [&](const gsp_kernel_stat &k) { return r.name == k.name; });
      if (it == agg.end()) {
        gsp_kernel_stat k;
        std::memset(&k, 0, sizeof(k));
        std::strncpy(k.name, r.name.c_str(), sizeof(k.name) - 1);
        agg.push_back(k);
        it = agg.end() - 1;
      }
      it->launches += 1;
      it->total_ms += ms;
      it->work += r.work;
    }
    *n = (int32_t)agg.size();
    for (int32_t k = 0; k < std::min<int32_t>(cap, (int32_t)agg.size()); ++k) out[k] = agg[k];
    if (reset) {
      for (auto &r : ctx->prof_recs) {
        ctx->prof_pool.push_back(r.start);
        ctx->prof_pool.push_back(r.stop);
      }
      ctx->prof_recs.clear();
    }
  });
}

int gsp_plan_shape(int64_t nsamp, int32_t nchan, const double *freqs, double tsamp, const gsp_segment *segs,
                   int32_t n_seg, gsp_dmt_desc *desc) {
  return guarded(nullptr, [&] { plan_shape_impl(nsamp, nchan, freqs, tsamp, segs, n_seg, desc); });
}

int gsp_delay_table(const gsp_dmt_desc *desc, const double *freqs, int32_t seg, int32_t *out) {
  return guarded(nullptr, [&] {
    validate_desc(desc);
    if (!freqs || !out) fail(GSP_EINVAL, "null pointer argument");
    if (seg < 0 || seg >= desc->n_seg) fail(GSP_EINVAL, "row index out of range");
    compute_delays(desc, freqs, seg, out);
  });
}

int gsp_dedisperse(gsp_ctx *ctx, const uint8_t *fb, const double *freqs, const gsp_dmt_desc *desc, int32_t *dmt,
                   void *stream) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    validate_desc(desc);
    if (!fb || !freqs || !dmt) fail(GSP_EINVAL, "null pointer argument");
    if (desc->kind != 0) fail(GSP_EINVAL, "sub-band descriptor: use gsp_dedisperse_subband");
    if (fref_of(freqs, desc->nchan) != desc->fref_mhz)
      fail(GSP_EINVAL, "frequencies differ from those the plan was shaped with");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // rows without downsampling last: their staged rows are the channel-major
    // copy of fb that batch cutouts of this output can read afterwards
    for (int pass = 0; pass < 2; ++pass)
      for (int32_t s = 0; s < desc->n_seg; ++s) {
        if ((desc->seg[s].downsamp == 1) != (pass == 1)) continue;
        RowTables &rt = row_tables(ctx, desc, freqs, s);
        stage_row(ctx, fb, desc, rt, st);
        launch_dedisp(ctx, rt, dmt + desc->offset[s], st);
      }
    if (ctx->staged_tag.fb == fb && ctx->staged_tag.D == 1) ctx->staged_tag.dmt = dmt;
  });
}

int gsp_trial_stats(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, double *mu, double *sigma,
                    void *stream) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    validate_desc(desc);
    if (!dmt || !mu || !sigma) fail(GSP_EINVAL, "null pointer argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_stats(ctx, dmt, desc, st);
    std::vector<double> ms((size_t)desc->n_trials * 2);
    check_hip(hipMemcpyAsync(ms.data(), ctx->stats.ptr, ms.size() * sizeof(double), hipMemcpyDeviceToHost, st),
              "copy statistics");
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    for (int32_t g = 0; g < desc->n_trials; ++g) {
      mu[g] = ms[2 * (size_t)g];
      sigma[g] = ms[2 * (size_t)g + 1];
    }
  });
}

int gsp_single_pulse_search(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, const int32_t *widths,
                            int32_t n_widths, float threshold, gsp_candidate *cands, int64_t capacity,
                            int64_t *n_found, void *stream) {
  if (!ctx) return GSP_EINVAL;
  int status = GSP_OK;
  int rc = guarded(ctx, [&] {
    validate_desc(desc);
    if (!dmt || !widths || !n_found || (capacity > 0 && !cands) || capacity < 0)
      fail(GSP_EINVAL, "null pointer or negative capacity");
    if (n_widths < 1 || n_widths > 64) fail(GSP_EINVAL, "n_widths must be in [1, 64]");
    if (!std::isfinite(threshold)) fail(GSP_EINVAL, "threshold must be finite");
    std::vector<int32_t> w(widths, widths + n_widths);
    for (int32_t v : w)
      if (v < 1 || v > 4096) fail(GSP_EINVAL, "widths must be in [1, 4096]");
    std::sort(w.begin(), w.end());
    w.erase(std::unique(w.begin(), w.end()), w.end());
    hipStream_t st = static_cast<hipStream_t>(stream);
    ctx->widths.device = ctx->device;
    ctx->widths.reserve(w.size() * sizeof(int32_t));
    check_hip(hipMemcpyAsync(ctx->widths.ptr, w.data(), w.size() * sizeof(int32_t), hipMemcpyHostToDevice, st),
              "copy widths");
    ctx->counter.device = ctx->device;
    ctx->counter.reserve(sizeof(unsigned long long));
    ctx->frags.device = ctx->device;
    int64_t cap = std::max<int64_t>(1 << 16, (int64_t)(ctx->frags.bytes / sizeof(Frag)));
    launch_stats(ctx, dmt, desc, st);
    unsigned long long count = 0;
    for (int pass = 0; pass < 2; ++pass) {
      ctx->frags.reserve((size_t)cap * sizeof(Frag));
      launch_search(ctx, dmt, desc, ctx->widths.as<int32_t>(), (int32_t)w.size(), w.back(), threshold,
                    ctx->frags.as<Frag>(), cap, ctx->counter.as<unsigned long long>(), st);
      check_hip(hipMemcpyAsync(&count, ctx->counter.ptr, sizeof(count), hipMemcpyDeviceToHost, st), "copy count");
      check_hip(hipStreamSynchronize(st), "synchronise stream");
      if ((int64_t)count <= cap) break;
      cap = (int64_t)count + 1024;  // rerun once with room for every fragment
    }
    std::vector<Frag> fr(count);
    if (count)
      check_hip(hipMemcpy(fr.data(), ctx->frags.ptr, count * sizeof(Frag), hipMemcpyDeviceToHost), "copy fragments");
    // join fragments split at tile edges: order them by (trial, first box
    // end) with a counting pass over the trials and a sort of each trial's
    // few fragments (a trial's runs are disjoint, so the order is unique)
    {
      std::vector<int64_t> start((size_t)desc->n_trials + 1, 0);
      for (const Frag &f : fr) {
        if (f.trial < 0 || f.trial >= desc->n_trials) fail(GSP_EDEVICE, "search fragment of an unknown trial");
        ++start[(size_t)f.trial + 1];
      }
      for (int32_t g = 0; g < desc->n_trials; ++g) start[(size_t)g + 1] += start[(size_t)g];
      std::vector<Frag> by_trial(fr.size());
      std::vector<int64_t> fill(start.begin(), start.end() - 1);
      for (const Frag &f : fr) by_trial[(size_t)fill[(size_t)f.trial]++] = f;
      for (int32_t g = 0; g < desc->n_trials; ++g)
        if (start[(size_t)g + 1] - start[(size_t)g] > 1)
          std::sort(by_trial.begin() + start[(size_t)g], by_trial.begin() + start[(size_t)g + 1],
                    [](const Frag &a, const Frag &b) { return a.t_first < b.t_first; });
      fr.swap(by_trial);
    }
    std::vector<Frag> runs;
    runs.reserve(fr.size());
    for (const Frag &f : fr) {
      if (!runs.empty()) {
        Frag &p = runs.back();
        if (p.trial == f.trial && p.open_right && f.open_left && p.t_last + 1 == f.t_first) {
          if (f.snr > p.snr) {
            p.snr = f.snr;
            p.width = f.width;
            p.e_peak = f.e_peak;
          }
          p.t_last = f.t_last;
          p.open_right = f.open_right;
          continue;
        }
      }
      runs.push_back(f);
    }
    std::vector<gsp_candidate> out(runs.size());
    for (size_t k = 0; k < runs.size(); ++k) {
      const Frag &f = runs[k];
      int s = 0;
      for (int q = 1; q < desc->n_seg; ++q)
        if (f.trial >= desc->trial0[q]) s = q;
      gsp_candidate &c = out[k];
      std::memset(&c, 0, sizeof(c));
      c.seg = s;
      c.dm_index = f.trial - desc->trial0[s];
      c.dm = desc->seg[s].dm_lo + (double)c.dm_index * desc->seg[s].dm_step;
      c.width = f.width;
      c.t_peak = f.e_peak - f.width + 1;
      c.t_first = f.t_first;
      c.t_last = f.t_last;
      c.snr = (float)f.snr;
      c.time_s = ((double)c.t_peak + 0.5 * (double)c.width) * (double)desc->seg[s].downsamp * desc->tsamp;
    }
    // (seg, dm_index) is the trial order the runs already follow: sort each
    // trial's candidates by (t_peak, t_first)
    for (size_t b = 0; b < out.size();) {
      size_t e = b + 1;
      while (e < out.size() && out[e].seg == out[b].seg && out[e].dm_index == out[b].dm_index) ++e;
      if (e - b > 1)
        std::sort(out.begin() + (int64_t)b, out.begin() + (int64_t)e, [](const gsp_candidate &x, const gsp_candidate &y) {
          return x.t_peak != y.t_peak ? x.t_peak < y.t_peak : x.t_first < y.t_first;
        });
      b = e;
    }
    *n_found = (int64_t)out.size();
    const int64_t nw = std::min<int64_t>(capacity, (int64_t)out.size());
    if (nw > 0) std::memcpy(cands, out.data(), (size_t)nw * sizeof(gsp_candidate));
    if ((int64_t)out.size() > capacity) status = GSP_ECAPACITY;
  });
  if (rc == GSP_OK && status != GSP_OK) {
    ctx->last_error = "candidate capacity too small; *n_found holds the required count";
    return status;
  }
  return rc;
}

int gsp_group_candidates(const gsp_candidate *c, int64_t n, int64_t *rep, int64_t *n_groups) {
  return guarded(nullptr, [&] {
    if (n < 0 || (n > 0 && (!c || !rep)) || !n_groups) fail(GSP_EINVAL, "null pointer or negative count");
    // union-find over links between neighbouring trials of a row with
    // overlapping run extents; candidates sorted per (seg, trial, t_first)
    std::vector<int64_t> parent(n), order(n);
    std::iota(parent.begin(), parent.end(), 0);
    std::iota(order.begin(), order.end(), 0);
    // a search's output already runs in (seg, dm_index) order: then only each
    // trial's few candidates need ordering by t_first
    bool trial_order = true;
    for (int64_t k = 1; k < n && trial_order; ++k)
      trial_order = c[k - 1].seg < c[k].seg || (c[k - 1].seg == c[k].seg && c[k - 1].dm_index <= c[k].dm_index);
    if (trial_order) {
      for (int64_t b = 0; b < n;) {
        int64_t e = b + 1;
        while (e < n && c[e].seg == c[b].seg && c[e].dm_index == c[b].dm_index) ++e;
        if (e - b > 1)
          std::sort(order.begin() + b, order.begin() + e,
                    [&](int64_t x, int64_t y) { return c[x].t_first < c[y].t_first; });
        b = e;
      }
    } else {
      std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        if (c[a].seg != c[b].seg) return c[a].seg < c[b].seg;
        if (c[a].dm_index != c[b].dm_index) return c[a].dm_index < c[b].dm_index;
        return c[a].t_first < c[b].t_first;
      });
    }
    auto find = [&](int64_t v) {
      while (parent[v] != v) v = parent[v] = parent[parent[v]];
      return v;
    };
    auto unite = [&](int64_t a, int64_t b) {
      a = find(a);
      b = find(b);
      if (a != b) parent[std::max(a, b)] = std::min(a, b);
    };
    // runs of one trial are disjoint and sorted, so for each candidate only a
    // window of the next trial's list can overlap it: two-pointer sweep
    int64_t i = 0;
    while (i < n) {
      int64_t j = i;
      while (j < n && c[order[j]].seg == c[order[i]].seg && c[order[j]].dm_index == c[order[i]].dm_index) ++j;
      // [i, j) = one trial; find the next trial's block if it is dm_index + 1
      int64_t k = j, l = j;
      if (k < n && c[order[k]].seg == c[order[i]].seg && c[order[k]].dm_index == c[order[i]].dm_index + 1) {
        while (l < n && c[order[l]].seg == c[order[k]].seg && c[order[l]].dm_index == c[order[k]].dm_index) ++l;
        int64_t p = k;
        for (int64_t a = i; a < j; ++a) {
          const gsp_candidate &A = c[order[a]];
          while (p < l && c[order[p]].t_last < A.t_first) ++p;
          for (int64_t q = p; q < l && c[order[q]].t_first <= A.t_last; ++q) unite(order[a], order[q]);
        }
      }
      i = j;
    }
    std::vector<int64_t> best(n, -1);
    for (int64_t k = 0; k < n; ++k) {
      const int64_t r = find(k);
      const int64_t b = best[r];
      const bool better = b < 0 || c[k].snr > c[b].snr ||
                          (c[k].snr == c[b].snr && (c[k].dm_index < c[b].dm_index ||
                                                    (c[k].dm_index == c[b].dm_index && c[k].t_peak < c[b].t_peak)));
      if (better) best[r] = k;
    }
    int64_t groups = 0;
    for (int64_t k = 0; k < n; ++k) {
      rep[k] = best[find(k)];
      if (find(k) == k) ++groups;
    }
    *n_groups = groups;
  });
}

}  // extern "C"
