// Autotuner of the dedispersion launch shape (trials per wave, samples per
// lane, waves per workgroup, channels per staging pass).
//
// The best shape depends on the row's downsampling (uint8 or uint16 staging),
// on the spread of delays across a tile of trials (LDS window per channel) and
// on the row length; it is found by timing every candidate on the caller's
// data and is then keyed by the row signature.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "gsp_internal.h"

using namespace gsp;

namespace {

DedispShape mk(int groups, int tpw, int waves, int chunk, int kind = 0) {
  DedispShape d;
  d.groups = groups;
  d.tpw = tpw;
  d.waves = waves;
  d.chunk = chunk;
  d.kind = kind;
  return d;
}

// 16-bit tile shapes, then byte-quad tile shapes (D = 1 rows with whole
// channel quads; the others reject them)
const DedispShape kCandidates[] = {
    mk(4, 4, 8, 16), mk(4, 4, 8, 32), mk(4, 8, 4, 16), mk(4, 8, 4, 32), mk(2, 8, 8, 16),
    mk(2, 8, 4, 32), mk(4, 4, 4, 16), mk(8, 4, 8, 16),
    mk(4, 8, 8, 64, 2), mk(4, 8, 12, 64, 2), mk(8, 4, 8, 64, 2), mk(4, 8, 4, 64, 2), mk(4, 8, 8, 64, 3), mk(4, 8, 12, 64, 3),
    mk(4, 8, 8, 64, 1), mk(8, 4, 16, 64, 1),
};

DedispShape from_abi(const gsp_shape &s) {
  DedispShape d;
  d.groups = s.groups;
  d.tpw = s.tpw;
  d.waves = s.waves;
  d.chunk = s.chunk;
  d.kind = s.kind;
  return d;
}

}  // namespace

extern "C" {

int gsp_row_shape(gsp_ctx *ctx, const double *freqs, const gsp_dmt_desc *desc, int32_t seg, gsp_shape *out) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    validate_desc(desc);
    if (!freqs || !out || seg < 0 || seg >= desc->n_seg) fail(GSP_EINVAL, "bad argument");
    RowTables &rt = row_tables(ctx, desc, freqs, seg);
    out->groups = rt.shape.groups;
    out->tpw = rt.shape.tpw;
    out->waves = rt.shape.waves;
    out->chunk = rt.shape.chunk;
    out->kind = rt.shape.kind;
  });
}

int gsp_set_row_shape(gsp_ctx *ctx, const double *freqs, const gsp_dmt_desc *desc, int32_t seg,
                      const gsp_shape *shape) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    validate_desc(desc);
    if (!freqs || !shape || seg < 0 || seg >= desc->n_seg) fail(GSP_EINVAL, "bad argument");
    const DedispShape d = from_abi(*shape);
    if (!shape_supported(d)) fail(GSP_EINVAL, "unsupported shape");
    const std::string sig = row_signature(desc, seg);
    const auto old = ctx->tuned.find(sig);
    const bool had = old != ctx->tuned.end();
    const DedispShape prev = had ? old->second : DedispShape();
    ctx->tuned[sig] = d;
    try {
      row_tables(ctx, desc, freqs, seg);  // builds (and checks LDS fit) now
    } catch (...) {
      if (had)
        ctx->tuned[sig] = prev;
      else
        ctx->tuned.erase(sig);
      throw;
    }
  });
}

int gsp_autotune(gsp_ctx *ctx, const uint8_t *fb, const double *freqs, const gsp_dmt_desc *desc, int32_t *dmt,
                 int32_t n_reps, void *stream) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    validate_desc(desc);
    if (!fb || !freqs || !dmt || n_reps < 1) fail(GSP_EINVAL, "bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "create event");
    check_hip(hipEventCreate(&e1), "create event");
    const bool prof = ctx->prof;
    ctx->prof = false;
    try {
      for (int32_t s = 0; s < desc->n_seg; ++s) {
        const std::string sig = row_signature(desc, s);
        float best_ms = 1e30f;
        DedispShape best = default_shape(desc->seg[s].downsamp, desc->nchan);
        for (const DedispShape &cand : kCandidates) {
          ctx->tuned[sig] = cand;
          RowTables *rt = nullptr;
          try {
            rt = &row_tables(ctx, desc, freqs, s);
          } catch (const Error &e) {
            if (e.status == GSP_EINVAL) continue;  // does not fit: skip
            throw;
          }
          stage_row(ctx, fb, desc, *rt, st);
          launch_dedisp(ctx, *rt, dmt + desc->offset[s], st);  // warm-up
          check_hip(hipEventRecord(e0, st), "record event");
          for (int r = 0; r < n_reps; ++r) launch_dedisp(ctx, *rt, dmt + desc->offset[s], st);
          check_hip(hipEventRecord(e1, st), "record event");
          check_hip(hipEventSynchronize(e1), "wait for event");
          float ms = 0.f;
          check_hip(hipEventElapsedTime(&ms, e0, e1), "event time");
          if (ms < best_ms) {
            best_ms = ms;
            best = cand;
          }
        }
        ctx->tuned[sig] = best;
        row_tables(ctx, desc, freqs, s);
      }
    } catch (...) {
      ctx->prof = prof;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    ctx->prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

int gsp_tuning_save(const gsp_ctx *ctx, const char *path) {
  if (!ctx || !path) return GSP_EINVAL;
  std::ofstream f(path);
  if (!f) return GSP_EINVAL;
  for (const auto &kv : ctx->tuned)
    f << kv.first << ' ' << kv.second.groups << ' ' << kv.second.tpw << ' ' << kv.second.waves << ' '
      << kv.second.chunk << ' ' << kv.second.kind << '\n';
  return f.good() ? GSP_OK : GSP_EINVAL;
}

int gsp_tuning_load(gsp_ctx *ctx, const char *path) {
  if (!ctx || !path) return GSP_EINVAL;
  std::ifstream f(path);
  if (!f) return GSP_EINVAL;
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string sig;
    DedispShape d;
    if (!(is >> sig >> d.groups >> d.tpw >> d.waves >> d.chunk)) continue;
    if (!(is >> d.kind)) d.kind = 0;
    if (shape_supported(d)) ctx->tuned[sig] = d;
  }
  return GSP_OK;
}

}  // extern "C"
