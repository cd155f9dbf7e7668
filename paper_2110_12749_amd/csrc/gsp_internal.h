// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/gsp.h"

namespace gsp {

// Error carried from deep inside the runtime to the ABI boundary.
struct Error {
  int status;
  std::string msg;
};

[[noreturn]] void fail(int status, const std::string &msg);
void check_hip(hipError_t e, const char *what);

// Device buffer owned by the library (grow-only).
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  int device = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf();
  void reserve(size_t n);  // grow to at least n bytes; contents not preserved
  template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Launch shape of the dedispersion kernel for one plan row.
struct DedispShape {
  int tpw = 4;       // trials per wave
  int waves = 8;     // waves per block
  int groups = 8;    // dword groups per lane (samples per block = 128 * groups)
  int chunk = 32;    // channels staged per pass (kind 1: channel quads per pass)
  int kind = 0;      // 0: 16-bit pair tile (any row); 1: byte-quad tile (D = 1, nchan % 4 == 0);
                     // 2: byte-quad tile with 4 staging waves besides `waves` summing waves;
                     // 3: kind 2 over the channels whose copies fit, the 16-bit tile (default
                     //    shape) over a run of channels at one end of the band whose copies do not
  int trials_per_block() const { return tpw * waves; }
  // kind 0: a lane sums `groups` dwords of two samples; kinds 1, 2: `groups` dwords of one sample
  int samples_per_block() const { return (kind != 0 ? 64 : 128) * groups; }
};

// Per-row device tables for one plan (cached by plan key).
struct RowTables {
  int32_t n_dm = 0, D = 1, nchan = 0;
  int64_t N = 0;         // downsampled length
  int64_t n_out = 0;
  int64_t max_delay = 0;
  DedispShape shape;
  DedispShape req;           // shape requested (before LDS limits, or the byte-quad default that did not fit)
  int64_t lds_bytes = 0;     // dynamic LDS per block
  int32_t row_dwords = 0;    // LDS dwords per staged copy of the widest channel
  DevBuf passes;             // int32 pairs (first channel, dwords per staged copy) per staging pass + end
  int32_t n_passes = 0, max_chunk = 0, data_dw = 0;
  DevBuf addr;               // uint32 [n_dm_pad][nchan]: LDS dword offset per (trial, channel)
  DevBuf dmin;               // int32 [n_tiles][nchan]: aligned first delay per DM tile
  DevBuf delays_dev;         // int32 [n_dm][nchan] (cutouts)
  std::vector<int32_t> delays_host;  // int32 [n_dm][nchan]
  // byte-quad tile (shape.kind 1; addr then holds [nchan / 4][n_dm_pad])
  DevBuf q_tile_pass;        // int32 [n_tiles + 1]: first pass record of each DM tile
  DevBuf q_passes;           // int4 per pass {first quad, first copy, chunks per copy, magic} + a sentinel per tile
  DevBuf q_copies;           // int4 per staged copy: source byte offset of each of its 4 channels
  int64_t q_pitch = 0;       // staged pitch the quad tile needs
  int32_t y_ch0 = 0;         // first staged channel row the tables read (the row's own channels from here)
  int64_t pitch_override = 0;  // staged pitch shared with the other part of a split row (0: own)
  std::unique_ptr<RowTables> low;  // kind 3: the 16-bit tile's part of the row
  int32_t q_rec_dw = 0;      // LDS dwords of one buffer of copy records (data_dw: of copies)
  double q_staged_dw = 0;    // LDS dwords staged per time tile, summed over DM tiles (profile)
};

// One timed kernel launch (profiling enabled).
struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
  double work;
};

struct PlanCache {
  std::string key;
  std::vector<std::unique_ptr<RowTables>> rows;
};

struct Frag {  // one run of flagged box ends inside a search tile
  int32_t trial;    // global trial index
  int32_t width;    // peak width
  int64_t t_first;  // first box end
  int64_t t_last;   // last box end
  int64_t e_peak;   // box end of the peak
  double snr;
  int32_t open_left;   // run starts at the tile's first box end (tile > 0)
  int32_t open_right;  // run ends at the tile's last box end (not the series end)
};
static_assert(sizeof(Frag) == 48, "fragment layout");

// A series job: the n_dm trials of one plan row, each a row of `pitch` int32
// samples.  Box ends and statistics cover [e_begin, e_begin + n); boxes may
// start up to `look` samples before e_begin.  Reported times are
// abs0 + (index - e_begin).
struct SeriesJob {
  const int32_t *x;
  int64_t pitch;
  int64_t e_begin;
  int64_t n;
  int64_t look;
  int64_t abs0;
  int64_t tiles;   // search items (segments of box ends) per trial (finalize_table)
  int64_t block0;  // first search item of the job (finalize_table)
  int32_t n_dm;
  int32_t trial0;  // global trial index of the job's first trial (finalize_table)
};
static constexpr int kMaxJobs = 1024;
struct SeriesTable {
  SeriesJob job[kMaxJobs];
  int32_t n_jobs = 0;
  int32_t n_trials = 0;
  int64_t n_items = 0;
};
struct SearchTiling {
  int ring = 1024;  // prefix sums kept per wave (power of two >= w_max + 512)
  int waves = 4;    // waves per workgroup, one search item each
  int tile = 0;     // box ends per search item
  size_t lds = 0;   // dynamic LDS of the search kernel
};
}  // namespace gsp

struct gsp_ctx;

namespace gsp {
struct SubbandPlan;  // cached tables of a sub-band plan (subband.hip)
// Run f at the ABI boundary: select the context's device, turn every error
// into a status code and keep its message on the context.
template <class F>
int guarded(gsp_ctx *ctx, F &&f);
}  // namespace gsp

struct gsp_ctx {
  int device = 0;
  std::string last_error;
  std::map<std::string, std::unique_ptr<gsp::PlanCache>> plans;
  gsp::DevBuf staged;      // channel-major downsampled input of the current row
  struct {                 // what `staged` holds: rows of fb summed over D, `pitch` apart
    const uint8_t *fb = nullptr;
    int64_t nsamp = 0, pitch = 0;
    int32_t nchan = 0, D = 0;
    const int32_t *dmt = nullptr;  // set when a gsp_dedisperse into dmt staged them last
  } staged_tag;
  gsp::DevBuf stats;       // per-trial moments / mu / sigma
  gsp::DevBuf frags;       // search run fragments
  gsp::DevBuf counter;     // fragment counter
  gsp::DevBuf widths;      // device copy of the width set
  gsp::DevBuf jobs;        // device copy of the series-job table
  gsp::DevBuf ftsums;      // frequency-time band sums of batch cutouts
  gsp::DevBuf need;        // per trial: whether batch cutouts read its mean
  gsp::DevBuf rfi;         // RFI mitigation: spectrum sums, flags, block means
  gsp::DevBuf zbuf;        // sub-band series of sub-band dedispersion
  std::map<std::string, std::shared_ptr<gsp::SubbandPlan>> subband;
  std::unique_ptr<gsp::SeriesTable> jobs_host = std::make_unique<gsp::SeriesTable>();
  std::vector<uint8_t> host_scratch;
  // tuned shapes keyed by row signature
  std::map<std::string, gsp::DedispShape> tuned;
  // profiling
  bool prof = false;
  std::vector<gsp::ProfRec> prof_recs;
  std::vector<hipEvent_t> prof_pool;
};

namespace gsp {

// Profiling brackets around a kernel launch (no-ops when disabled).
struct ProfScope {
  gsp_ctx *ctx;
  hipStream_t st;
  size_t idx;
  ProfScope(gsp_ctx *c, const char *name, hipStream_t s, double work);
  ~ProfScope();
};

// Cached device tables of row s of a plan, built for the row's current shape (api.cpp)
RowTables &row_tables(gsp_ctx *ctx, const gsp_dmt_desc *desc, const double *freqs, int32_t s);

// Plan helpers (plan.cpp)
double fref_of(const double *freqs, int32_t nchan);
int64_t delay_of(double dm, double f, double fref, double tsamp, int32_t D);
void validate_desc(const gsp_dmt_desc *desc);
void plan_shape_impl(int64_t nsamp, int32_t nchan, const double *freqs, double tsamp, const gsp_segment *segs,
                     int32_t n_seg, gsp_dmt_desc *desc);
void compute_delays(const gsp_dmt_desc *desc, const double *freqs, int32_t s, int32_t *out);
std::string plan_key(const gsp_dmt_desc *desc, const double *freqs);

// Dedispersion (dedisp.hip)
// default: the byte-quad tile where it applies (D = 1, nchan % 4 == 0), else the 16-bit tile
DedispShape default_shape(int32_t D, int32_t nchan);
bool shape_supported(const DedispShape &s);
std::string row_signature(const gsp_dmt_desc *desc, int32_t s);
DedispShape shape_for_row(gsp_ctx *ctx, const gsp_dmt_desc *desc, int32_t s);
// units_per_thread: staging units each thread holds (the kernel's
// unit_max for its source type); 0 = the batch kernel's for the row's D
void build_row_tables(gsp_ctx *ctx, const gsp_dmt_desc *desc, const double *freqs, int32_t s,
                      const DedispShape &shape, RowTables &rt, int units_per_thread = 0);
// The same tables from an explicit delay table rt.delays_host [n_dm][nchan]
// (delays of D*tsamp samples, max_delay their largest; n_out outputs).
// lds_budget > 0: LDS bytes per workgroup the staging passes may use (default
// 80 KB: two workgroups per CU)
// pass_break > 0: no staging pass straddles a multiple of pass_break channels
// (segmented outputs, DedispArgs::seg_ch)
void build_tables_from_delays(gsp_ctx *ctx, int32_t n_dm, int32_t nchan, int32_t D, int64_t N, int64_t n_out,
                              int64_t max_delay, const DedispShape &shape, RowTables &rt, int units_per_thread = 0,
                              int64_t lds_budget = 0, int32_t pass_break = 0);
// pitch_override > 0: stage with that pitch (elements per channel row, a
// multiple of 256 covering every read of the kernels that use the copy)
void stage_row(gsp_ctx *ctx, const uint8_t *fb, const gsp_dmt_desc *desc, const RowTables &rt, hipStream_t st,
               int64_t pitch_override = 0);
void launch_dedisp(gsp_ctx *ctx, const RowTables &rt, int32_t *out_row, hipStream_t st);
int64_t staged_pitch(const RowTables &rt);
// Channel-major uint8 copy of the whole filterbank into ctx->staged, rows of
// `pitch` bytes (a multiple of 256, >= nsamp; bytes past nsamp are zero)
void stage_raw(gsp_ctx *ctx, const uint8_t *fb, int64_t nsamp, int32_t nchan, int64_t pitch, hipStream_t st);
// Byte-quad tile (dedisp_quad.hip): tables from rt.delays_host for rt.shape
// (kind 1); GSP_EINVAL when the row does not suit it (D > 1, nchan % 4, a
// quad's copies wider than the LDS or the staging registers)
bool quad_shape_supported(const DedispShape &s);
struct QuadHost {                  // the byte-quad tile's tables on the host
  std::vector<int32_t> tile_pass;  // first pass record of each DM tile (+ end)
  std::vector<int32_t> passes;     // 4 ints per record: first quad, first copy, chunks per copy, division magic
  std::vector<int32_t> copies;     // 4 ints per copy: source byte offset of each channel from the pass's first row
  std::vector<uint32_t> addr;      // [nchan / 4][n_dm_pad / 2] LDS dword offsets, two trials per dword
  int64_t pitch = 0, lds_dw = 0;   // staged pitch needed, LDS dwords of the largest pass's copies
  int rec_max = 0;                 // most copies in a pass
  double staged = 0;               // LDS dwords staged per time tile, all DM tiles
  int max_q = 0;
};
void quad_tables_host(const RowTables &rt, QuadHost &H, int64_t min_pitch = 0);
// kind 3: the channel range [*c0, *c1) the byte-quad tile takes (a multiple of
// 4 channels whose copies fit one pass each); the rest of the band, at one
// end of it, goes to the 16-bit tile.  Fails (GSP_EINVAL) where every quad
// fits (kind 2 applies) or where the quads that do not fit are not all at
// one end of the band.
void quad_split(const RowTables &rt, int32_t *c0, int32_t *c1);
void build_quad_tables(gsp_ctx *ctx, RowTables &rt);
void launch_dedisp_quad(gsp_ctx *ctx, const RowTables &rt, int32_t *out_row, hipStream_t st);

// Search (search.hip)
SearchTiling search_tiling(int32_t max_width);
void set_search_attributes(const SearchTiling &tl);
void finalize_table(SeriesTable &t, const SearchTiling &tl);
// Per-trial mean and sigma of every series of the table; with `need`, only
// of the trials g with need[g] != 0 (the others keep their old values).
void launch_stats_table(gsp_ctx *ctx, const SeriesTable *tb_dev, int64_t grid, double *musig, double bytes,
                        hipStream_t st, const uint32_t *need = nullptr);
void launch_search_table(gsp_ctx *ctx, const SeriesTable *tb_dev, int64_t grid, const SearchTiling &tl,
                         const double *musig, const int32_t *widths_dev, int32_t n_widths, int32_t max_width,
                         float thr, Frag *frags, int64_t cap, unsigned long long *counter, double bytes,
                         hipStream_t st);

void launch_stats(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, hipStream_t st,
                  const uint32_t *need = nullptr);
// Sub-band dedispersion (subband.hip)
void subband_plan_shape(int64_t nsamp, int32_t nchan, const double *freqs, double tsamp, const gsp_segment *segs,
                        int32_t n_seg, const int32_t *n_sub, const int32_t *group, gsp_dmt_desc *desc);
// Static search scratch of gsp_single_pulse_search_noalloc: per-device address (noalloc.hip)
void noalloc_init(int device);
// One streamed candidate's cutout sources (device state of its beam and row).
struct StreamCut {
  const int32_t *win;     // window buffer [n_dm][win_pitch]: column look + (t - a) holds time t
  int64_t win_pitch;
  int64_t a;              // absolute time of the window's first output
  const double *mu;       // mu[2 * trial]: the window's mean of each trial of the row
  const uint16_t *ring;   // downsampled samples [nchan][ring_pitch], time t at column t mod R
  int64_t ring_pitch, R;
  const int32_t *delays;  // [n_dm][nchan]
  int64_t t_peak;
  int32_t look, n_dm, nchan, dm_index, width;
};
void launch_cutouts_stream(const StreamCut *cuts_dev, int64_t n, uint16_t *out_dev, hipStream_t st);

// Device pointer of per-trial mu/sigma (double[2*n_trials]) after launch_stats.
const double *stats_musig(gsp_ctx *ctx, const gsp_dmt_desc *desc);
void launch_search(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, const int32_t *widths_dev,
                   int32_t n_widths, int32_t max_width, float thr, Frag *frags, int64_t cap,
                   unsigned long long *counter, hipStream_t st);

}  // namespace gsp

namespace gsp {
template <class F>
int guarded(gsp_ctx *ctx, F &&f) {
  try {
    if (ctx) check_hip(hipSetDevice(ctx->device), "select device");
    f();
    if (ctx) ctx->last_error.clear();
    return GSP_OK;
  } catch (const Error &e) {
    if (ctx) ctx->last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->last_error = "host allocation failed";
    return GSP_ENOMEM;
  } catch (...) {
    if (ctx) ctx->last_error = "unexpected internal error";
    return GSP_EDEVICE;
  }
}
}  // namespace gsp
