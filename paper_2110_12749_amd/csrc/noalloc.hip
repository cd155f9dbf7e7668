// gsp_single_pulse_search without allocation: every device buffer of the
// search (job table, per-trial statistics, width set, run fragments and
// their counter) lives in one fixed static device array, and the host work
// (joining fragments into runs, building and sorting candidates) happens in
// the caller's candidate buffer.  Same kernels, same results as
// gsp_single_pulse_search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "gsp.h"
#include "gsp_internal.h"

namespace gsp {
namespace {

// Layout of the static scratch array (offsets in bytes, each 256-aligned).
constexpr int64_t kNaMaxTrials = 32768;   // trials of one plan
constexpr int64_t kNaMaxFrags = 65536;    // run fragments of one call
constexpr size_t kNaTable = 0;
constexpr size_t kNaMusig = (sizeof(SeriesTable) + 255) / 256 * 256;
constexpr size_t kNaWidths = kNaMusig + (size_t)kNaMaxTrials * 2 * sizeof(double);
constexpr size_t kNaCounter = kNaWidths + 256;
constexpr size_t kNaFrags = kNaCounter + 256;
constexpr size_t kNaBytes = kNaFrags + (size_t)kNaMaxFrags * sizeof(Frag);  // about 3.7 MB

// Each GPU the library runs on holds its own copy until the process ends.
// Host code never uses this name as an address: it uses the per-device
// pointer from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex na_mu;
unsigned char *na_ptr[kNaMaxDevices] = {};

// The batch job table of a plan (one job per row, n_seg <= 16), passed by value.
struct BatchJobs {
  SeriesJob job[16];
  int32_t n_jobs, n_trials;
  int64_t n_items;
};
static_assert(sizeof(BatchJobs) < 4096, "kernel argument size");
static_assert(sizeof(gsp_candidate) >= sizeof(Frag), "candidates are converted from fragments in place");

__global__ void k_na_put_table(BatchJobs b, SeriesTable *t) {
  const int j = threadIdx.x;
  if (j < b.n_jobs) t->job[j] = b.job[j];
  if (j == 0) {
    t->n_jobs = b.n_jobs;
    t->n_trials = b.n_trials;
    t->n_items = b.n_items;
  }
}

struct WidthSet {
  int32_t w[64];
};

__global__ void k_na_put_widths(WidthSet ws, int32_t n, int32_t *out) {
  if ((int)threadIdx.x < n) out[threadIdx.x] = ws.w[threadIdx.x];
}

}  // namespace

// Called once per device at context creation, with that device current.
void noalloc_init(int device) {
  if (device < 0 || device >= kNaMaxDevices) fail(GSP_EINVAL, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(na_mu);
  if (na_ptr[device]) return;
  void *p = nullptr;
  check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the static search scratch");
  na_ptr[device] = static_cast<unsigned char *>(p);
}

}  // namespace gsp

using namespace gsp;

extern "C" int gsp_single_pulse_search_noalloc(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc,
                                               const int32_t *widths, int32_t n_widths, float threshold,
                                               gsp_candidate *cands, int64_t capacity, int64_t *n_found,
                                               void *stream) {
  if (!ctx) return GSP_EINVAL;
  int status = GSP_OK;
  int rc = guarded(ctx, [&] {
    validate_desc(desc);
    if (!dmt || !widths || !n_found || (capacity > 0 && !cands) || capacity < 0)
      fail(GSP_EINVAL, "null pointer or negative capacity");
    if (n_widths < 1 || n_widths > 64) fail(GSP_EINVAL, "n_widths must be in [1, 64]");
    if (!std::isfinite(threshold)) fail(GSP_EINVAL, "threshold must be finite");
    if (desc->n_trials > kNaMaxTrials) fail(GSP_ECAPACITY, "more trials than the static scratch holds (32768)");
    unsigned char *base = nullptr;
    {
      std::lock_guard<std::mutex> lk(na_mu);
      base = ctx->device < kNaMaxDevices ? na_ptr[ctx->device] : nullptr;
    }
    if (!base) fail(GSP_EDEVICE, "static scratch not set up on this device");
    // the width set, sorted and unique, on the stack
    WidthSet ws;
    int32_t nw = 0;
    for (int32_t k = 0; k < n_widths; ++k) {
      if (widths[k] < 1 || widths[k] > 4096) fail(GSP_EINVAL, "widths must be in [1, 4096]");
      ws.w[nw++] = widths[k];
    }
    std::sort(ws.w, ws.w + nw);
    nw = (int32_t)(std::unique(ws.w, ws.w + nw) - ws.w);
    const int32_t wmax = ws.w[nw - 1];
    hipStream_t st = static_cast<hipStream_t>(stream);
    SeriesTable *table = reinterpret_cast<SeriesTable *>(base + kNaTable);
    double *musig = reinterpret_cast<double *>(base + kNaMusig);
    int32_t *wdev = reinterpret_cast<int32_t *>(base + kNaWidths);
    auto *counter = reinterpret_cast<unsigned long long *>(base + kNaCounter);
    Frag *frags = reinterpret_cast<Frag *>(base + kNaFrags);
    // batch job table: rows of the plan, statistics tiling first
    BatchJobs bj;
    std::memset(&bj, 0, sizeof(bj));
    bj.n_jobs = desc->n_seg;
    for (int s = 0; s < desc->n_seg; ++s) {
      SeriesJob &J = bj.job[s];
      J.x = dmt + desc->offset[s];
      J.pitch = desc->n_out[s];
      J.n = desc->n_out[s];
      J.n_dm = desc->seg[s].n_dm;
    }
    auto finalize = [&](const SearchTiling &tl) {
      int64_t nb = 0;
      int32_t trials = 0;
      for (int j = 0; j < bj.n_jobs; ++j) {
        SeriesJob &J = bj.job[j];
        J.tiles = (J.n + tl.tile - 1) / tl.tile;
        J.block0 = nb;
        J.trial0 = trials;
        nb += (int64_t)J.n_dm * J.tiles;
        trials += J.n_dm;
      }
      bj.n_items = nb;
      bj.n_trials = trials;
    };
    finalize(search_tiling(1));
    hipLaunchKernelGGL(k_na_put_table, dim3(1), dim3(64), 0, st, bj, table);
    hipLaunchKernelGGL(k_na_put_widths, dim3(1), dim3(64), 0, st, ws, nw, wdev);
    check_hip(hipGetLastError(), "launch table setup");
    launch_stats_table(nullptr, table, bj.n_trials, musig, 0, st);
    const SearchTiling tl = search_tiling(wmax);
    finalize(tl);
    // the statistics kernel has read the table before this launch rewrites it (same stream)
    hipLaunchKernelGGL(k_na_put_table, dim3(1), dim3(64), 0, st, bj, table);
    set_search_attributes(tl);
    launch_search_table(nullptr, table, (bj.n_items + tl.waves - 1) / tl.waves, tl, musig, wdev, nw, wmax,
                        threshold, frags, kNaMaxFrags, counter, 0, st);
    unsigned long long count = 0;
    check_hip(hipMemcpyAsync(&count, counter, sizeof(count), hipMemcpyDeviceToHost, st), "copy count");
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    if ((int64_t)count > kNaMaxFrags) fail(GSP_ECAPACITY, "more run fragments than the static scratch holds (65536)");
    // the caller's candidate buffer is the host workspace: the fragments
    // first (48 bytes each), then the candidates (56 bytes each, at most one
    // per fragment) in place
    if ((int64_t)count > capacity) {
      *n_found = (int64_t)count;
      status = GSP_ECAPACITY;
      return;
    }
    Frag *fr = reinterpret_cast<Frag *>(cands);
    if (count)
      check_hip(hipMemcpy(fr, frags, count * sizeof(Frag), hipMemcpyDeviceToHost), "copy fragments");
    std::sort(fr, fr + count, [](const Frag &a, const Frag &b) {
      return a.trial != b.trial ? a.trial < b.trial : a.t_first < b.t_first;
    });
    // join fragments split at tile edges, compacting in place
    int64_t nr = 0;
    for (int64_t k = 0; k < (int64_t)count; ++k) {
      const Frag f = fr[k];
      if (nr > 0) {
        Frag &p = fr[nr - 1];
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
      fr[nr++] = f;
    }
    // runs -> candidates, last first: candidate k's bytes overlap only run k
    // (copied out first) and runs after k (already converted)
    for (int64_t k = nr - 1; k >= 0; --k) {
      const Frag f = fr[k];
      int s = 0;
      for (int q = 1; q < desc->n_seg; ++q)
        if (f.trial >= desc->trial0[q]) s = q;
      gsp_candidate c;
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
      std::memcpy(&cands[k], &c, sizeof(c));
    }
    std::sort(cands, cands + nr, [](const gsp_candidate &a, const gsp_candidate &b) {
      if (a.seg != b.seg) return a.seg < b.seg;
      if (a.dm_index != b.dm_index) return a.dm_index < b.dm_index;
      if (a.t_peak != b.t_peak) return a.t_peak < b.t_peak;
      return a.t_first < b.t_first;
    });
    *n_found = nr;
  });
  if (rc == GSP_OK && status != GSP_OK) {
    ctx->last_error = "candidate buffer smaller than the run fragments; *n_found holds a capacity that suffices";
    return status;
  }
  return rc;
}
