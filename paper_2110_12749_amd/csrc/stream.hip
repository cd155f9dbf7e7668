// Streaming engine: continuous batching of beams that arrive in blocks.
//
// The paper's prepsubband loop dedisperses a block using the previous one as
// overlap (Algorithm 2's lastdata/data; Algorithm 3 merges the two into one
// 2*numpts buffer).  Here the overlap is kept on the device as a per-(beam,
// plan row) ring of the channel-major downsampled samples, long enough for the
// row's maximum delay plus one block, so a block of B samples yields the B/D
// outputs whose inputs have all arrived:
//     window k of a row = [max(0, N_k - M), max(0, N_{k+1} - M)),
// with N_k the downsampled samples received before block k and M the row's
// maximum delay.  Statistics are taken per (window, trial); boxes end inside
// the window and may reach back up to (max width - 1) samples into earlier
// windows, which a look-back region in front of the window buffer retains.
// Runs of flagged box ends are split at window edges.  Nothing waits for a
// later block.
//
// One step processes one pending block of every active beam.  Its device
// work is a fixed sequence of five kernels (stage, dedisperse, stats, search,
// look-back shift) that read their work from device job tables; the sequence
// is captured once into a hipGraph and replayed, the host rewriting the job
// tables between replays.  While a step's kernels run, each beam's next
// pending block is copied to the device on a second stream, into the other of
// the beam's two input buffers.  Beams are admitted against a device-memory budget;
// a beam that does not fit waits in a queue (its blocks stay on the host) and
// is admitted when finished beams release their memory.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "dedisp_tile.h"
#include "gsp_internal.h"

namespace gsp {

static constexpr int kGuard = 32;          // mirrored samples past the ring end
static constexpr int kCutoutReach = 512;   // samples a cutout reaches back from the box end
static constexpr int kStreamGroups = 4;    // dedispersion shape used by streams
static constexpr int kStreamTpw = 4;
static constexpr int kStreamWaves = 8;
static constexpr int kStageTile = 128;     // outputs x channels per staging item

// ---------------------------------------------------------------------------
// device job tables
// ---------------------------------------------------------------------------
struct StageJob {
  const uint8_t *X;   // block, time-major uint8 [rows][nchan]
  uint16_t *Y;        // ring, uint16 [nchan][ring + kGuard]
  int64_t pitch;      // ring + kGuard
  int64_t ring;
  int64_t phys0;      // ring position of the block's first output
  int64_t n_new;      // downsampled outputs of the block
  int64_t item0;      // first work item of the job
  int32_t nchan, D;
  int32_t t_tiles, c_tiles;
};
struct StageTable {
  StageJob job[kMaxJobs];
  int32_t n_jobs;
  int64_t n_items;
};

struct DedispJob {
  DedispArgs a;
  int64_t item0;
};
struct DedispTable {
  DedispJob job[kMaxJobs];
  int32_t n_jobs;
  int64_t n_items;
};

struct TailJob {
  int32_t *x;      // window buffer, [n_dm][pitch]
  int64_t pitch;   // look + window capacity
  int64_t look;    // look-back samples kept in front of the window
  int64_t w;       // samples in the window just searched
  int32_t n_dm;
  int32_t trial0;
};
struct TailTable {
  TailJob job[kMaxJobs];
  int32_t n_jobs;
  int32_t n_trials;
};

template <class Tab>
__device__ __forceinline__ int find_by_item0(const Tab *t, int64_t b) {
  int lo = 0, hi = t->n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t->job[mid].item0 <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Staging into rings: item = (job, output tile, channel tile); the D raw
// spectra of each output are summed in registers, transposed through LDS and
// written as uint16 pairs; positions inside the guard band are written twice.
__global__ __launch_bounds__(256) void k_stage_ring(const StageTable *__restrict__ tb) {
  __shared__ uint16_t tile[kStageTile * (kStageTile + 1)];
  constexpr int TP = kStageTile + 1;
  const int tid = threadIdx.x;
  const int64_t n_items = tb->n_items;
  for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
    const StageJob J = tb->job[find_by_item0(tb, b)];
    const int64_t local = b - J.item0;
    const int ct = (int)(local % J.c_tiles);
    const int64_t tt = local / J.c_tiles;
    const int64_t j0 = tt * kStageTile;
    const int c0 = ct * kStageTile;
    if ((J.nchan & 15) == 0) {
      // 16 channels of 4 outputs per thread: one 16-byte load per raw
      // spectrum, the D spectra summed as 16-bit pairs (even bytes and odd
      // bytes of each dword apart; D * 255 stays below 2^16)
      static_assert(kStageTile == 128, "8 threads x 16 channels per output, 32 outputs per pass");
      const int cl = 16 * (tid & 7);
      const int c = c0 + cl;
      const int jl = tid >> 3;
      uint32_t ev[4][4], od[4][4];
      bool ok[4];
      const uint8_t *p[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t j = j0 + jl + 32 * i;
        ok[i] = c < J.nchan && j < J.n_new;
        p[i] = J.X + (j * J.D) * (int64_t)J.nchan + c;
#pragma unroll
        for (int d = 0; d < 4; ++d) ev[i][d] = od[i][d] = 0;
      }
      for (int m = 0; m < J.D; ++m) {
        uint4 w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          w[i] = ok[i] ? *reinterpret_cast<const uint4 *>(p[i] + (int64_t)m * J.nchan) : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t v[4] = {w[i].x, w[i].y, w[i].z, w[i].w};
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            ev[i][d] += v[d] & 0x00FF00FFu;         // channels 4d, 4d+2
            od[i][d] += (v[d] >> 8) & 0x00FF00FFu;  // channels 4d+1, 4d+3
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uint16_t *t = tile + cl * TP + jl + 32 * i;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          t[(4 * d + 0) * TP] = (uint16_t)ev[i][d];
          t[(4 * d + 1) * TP] = (uint16_t)od[i][d];
          t[(4 * d + 2) * TP] = (uint16_t)(ev[i][d] >> 16);
          t[(4 * d + 3) * TP] = (uint16_t)(od[i][d] >> 16);
        }
      }
    } else {
      for (int u = tid; u < kStageTile * kStageTile; u += 256) {
        const int cl = u % kStageTile, jl = u / kStageTile;
        const int c = c0 + cl;
        const int64_t j = j0 + jl;
        uint32_t acc = 0;
        if (c < J.nchan && j < J.n_new) {
          const uint8_t *p = J.X + (j * J.D) * (int64_t)J.nchan + c;
          for (int m = 0; m < J.D; ++m) acc += p[(int64_t)m * J.nchan];
        }
        tile[cl * TP + jl] = (uint16_t)acc;
      }
    }
    __syncthreads();
    // ring position of output j0 (even: phys0, j0 and ring are even); the
    // ring holds more than kStageTile samples, so j0 + 2q wraps at most once
    const int64_t pos0 = (J.phys0 + j0) % J.ring;
    for (int idx = tid; idx < kStageTile * (kStageTile / 2); idx += 256) {
      const int cl = idx / (kStageTile / 2);
      const int q = idx % (kStageTile / 2);
      const int c = c0 + cl;
      const int64_t j = j0 + 2 * q;
      if (c >= J.nchan || j >= J.n_new) continue;
      int64_t pos = pos0 + 2 * q;
      if (pos >= J.ring) pos -= J.ring;
      const uint16_t *t = tile + cl * TP + 2 * q;
      uint16_t *row = J.Y + (int64_t)c * J.pitch;
      if (j + 1 < J.n_new) {
        const uint32_t v = (uint32_t)t[0] | ((uint32_t)t[1] << 16);
        *reinterpret_cast<uint32_t *>(row + pos) = v;
        if (pos < kGuard) *reinterpret_cast<uint32_t *>(row + pos + J.ring) = v;
      } else {
        row[pos] = t[0];
        if (pos < kGuard) row[pos + J.ring] = t[0];
      }
    }
    __syncthreads();
  }
}

// Dedispersion of every active (beam, row) window: grid-stride over tiles.
// Workgroup x runs on XCD x % 8.  The tiles are cut into 8 contiguous
// ranges, one per XCD, and each XCD's workgroups stride through their own
// range, so the tiles in flight on one XCD are neighbouring DM tiles of the
// same samples, whose staged windows overlap in that XCD's L2.
// (at most 128 VGPRs, as the batch kernel: two workgroups of 8 waves per CU)
template <int K, int TPW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_dedisp_jobs(
    const DedispTable *__restrict__ tb) {
  extern __shared__ uint32_t lds[];
  const int64_t n_items = tb->n_items;
  int64_t first = blockIdx.x, end = n_items, stride = gridDim.x;
  if ((gridDim.x & 7) == 0) {
    const int x = blockIdx.x & 7;
    end = n_items * (x + 1) / 8;
    first = n_items * x / 8 + (blockIdx.x >> 3);
    stride = gridDim.x >> 3;
  }
  for (int64_t b = first; b < end; b += stride) {
    const int j = __builtin_amdgcn_readfirstlane(find_by_item0(tb, b));
    const DedispArgs a = tb->job[j].a;
    const int64_t local = b - tb->job[j].item0;
    __syncthreads();  // LDS of the previous tile is free
    dedisp_tile<K, TPW, uint16_t>(a, (int)(local % a.n_dm_tiles), (int)(local / a.n_dm_tiles), lds);
  }
}

// Look-back shift: the last `look` samples of [look-back | window] move to
// the front of each trial's buffer (through LDS: the ranges may overlap).
__global__ __launch_bounds__(256) void k_tail(const TailTable *__restrict__ tb) {
  extern __shared__ int32_t keep[];
  const int n_trials = tb->n_trials;
  for (int g = blockIdx.x; g < n_trials; g += gridDim.x) {
    int lo = 0, hi = tb->n_jobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tb->job[mid].trial0 <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    const TailJob J = tb->job[lo];
    int32_t *row = J.x + (int64_t)(g - J.trial0) * J.pitch;
    for (int64_t k = threadIdx.x; k < J.look; k += 256) keep[k] = row[J.w + k];
    __syncthreads();
    for (int64_t k = threadIdx.x; k < J.look; k += 256) row[k] = keep[k];
    __syncthreads();
  }
}

}  // namespace gsp

// ---------------------------------------------------------------------------
// host engine
// ---------------------------------------------------------------------------
using namespace gsp;
using Clock = std::chrono::steady_clock;

namespace {

struct PinnedBlock {
  uint8_t *p = nullptr;
  size_t bytes = 0;
};

struct PendingBlock {
  PinnedBlock buf;
  int64_t nsamp;
  Clock::time_point arrival;
};

struct StreamRow {
  int32_t D = 1, n_dm = 0;
  int64_t M = 0;          // maximum delay (row samples)
  RowTables tables;       // LDS offsets and staging bases for the stream shape
  DevBuf ring;            // uint16 [nchan][R + kGuard]
  int64_t R = 0;
  DevBuf win;             // int32 [n_dm][look + Wcap]
  int64_t Wcap = 0;
  int64_t N = 0;          // downsampled samples received
  int64_t emitted = 0;    // end of the last window
  int64_t last_w = 0;     // length of the window in the buffer (shifted out by the next step)
  // window of the last step (for read-back)
  int64_t last_a = 0, last_b = 0;
};

struct Beam {
  int32_t id = 0;
  int32_t nchan = 0;
  std::vector<double> freqs;
  double tsamp = 0;
  std::vector<gsp_segment> segs;
  gsp_dmt_desc desc;  // shaped with a nominal length: delays and maximum delays
  std::vector<std::unique_ptr<StreamRow>> rows;
  // uint8 [B][nchan] x 2: the current block, and the next one copied on the
  // copy stream while the current step's kernels run
  DevBuf in[2];
  int cur = 0;                     // buffer holding the block being processed
  const void *pf_src = nullptr;    // pinned host block copied into in[pf_buf] (null: none)
  int pf_buf = 0;
  std::deque<PendingBlock> pending;
  int64_t blocks_done = 0;
  int64_t samples_in = 0;
  bool admitted = false;
  bool inflight = false;  // a step is processing one of its blocks
  bool closing = false;  // no more blocks will be pushed
  bool ended = false;    // a short block was pushed
  int64_t mem = 0;
};

}  // namespace

struct gsp_stream {
  gsp_ctx *ctx = nullptr;
  hipStream_t st = nullptr;
  hipStream_t cst = nullptr;  // copies of the next step's blocks
  int32_t B = 0;
  int64_t budget = 0, used = 0;
  std::vector<int32_t> widths;
  int32_t wmax = 1;
  float thr = 6.f;
  SearchTiling tiling;
  int32_t look = 0;
  int32_t max_beams = 0;
  std::map<int32_t, std::unique_ptr<Beam>> beams;
  std::deque<int32_t> queue;  // waiting for admission
  int32_t next_id = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::vector<PinnedBlock> pool;
  // device tables and scratch
  DevBuf d_stage, d_dedisp, d_series, d_tail, d_widths, musig, frags, counter;
  std::unique_ptr<StageTable> h_stage = std::make_unique<StageTable>();
  std::unique_ptr<DedispTable> h_dedisp = std::make_unique<DedispTable>();
  std::unique_ptr<SeriesTable> h_series = std::make_unique<SeriesTable>();
  std::unique_ptr<TailTable> h_tail = std::make_unique<TailTable>();
  int64_t frag_cap = 1 << 16;
  int64_t regrown = 0;  // steps whose search ran again with a grown fragment buffer
  int64_t musig_cap = 0;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t graph_lds = -1;  // dedispersion LDS the graph was captured with
  bool use_graph = true;
  // learned triage (optional): cutouts of each step's candidates scored by a network
  gsp_cnn *cnn = nullptr;
  float triage_thr = 0.f;
  DevBuf d_cuts, d_cutimg, d_logits;
  int64_t scored = 0, rejected = 0;
  double triage_s = 0;
  // results
  std::vector<gsp_stream_candidate> out;
  std::vector<double> lat;
  int64_t steps = 0, blocks = 0;
  double busy_s = 0;
  // worker
  std::thread worker;
  bool running = false, stop = false;
  std::string last_error;
};

namespace {

int64_t grid_of(int per_cu) { return 256LL * per_cu; }

PinnedBlock take_pinned(gsp_stream *s, size_t bytes) {
  for (size_t k = 0; k < s->pool.size(); ++k)
    if (s->pool[k].bytes >= bytes) {
      PinnedBlock b = s->pool[k];
      s->pool.erase(s->pool.begin() + (long)k);
      return b;
    }
  PinnedBlock b;
  check_hip(hipHostMalloc((void **)&b.p, bytes, hipHostMallocDefault), "allocate pinned block");
  b.bytes = bytes;
  return b;
}

void give_pinned(gsp_stream *s, PinnedBlock b) {
  if (s->pool.size() < 64)
    s->pool.push_back(b);
  else
    (void)hipHostFree(b.p);
}

int64_t beam_bytes(const gsp_stream *s, const Beam &b) {
  int64_t m = 2 * (int64_t)s->B * b.nchan;
  for (const auto &r : b.rows) {
    m += (int64_t)b.nchan * (r->R + kGuard) * 2;
    m += (int64_t)r->n_dm * (s->look + r->Wcap) * 4;
    m += (int64_t)r->tables.addr.bytes + (int64_t)r->tables.dmin.bytes + (int64_t)r->tables.delays_host.size() * 4;
  }
  return m;
}

// Build the per-row state of a beam (host tables; device memory allocated at admission).
void plan_beam(gsp_stream *s, Beam &b) {
  gsp_dmt_desc d;
  plan_shape_impl(int64_t(1) << 40, b.nchan, b.freqs.data(), b.tsamp, b.segs.data(), (int32_t)b.segs.size(), &d);
  b.desc = d;
  DedispShape sh;
  sh.groups = kStreamGroups;
  sh.tpw = kStreamTpw;
  sh.waves = kStreamWaves;
  sh.chunk = 32;
  for (int32_t r = 0; r < d.n_seg; ++r) {
    if (s->B % (4 * d.seg[r].downsamp))
      fail(GSP_EINVAL, "block length must be a multiple of 4 x every downsampling factor");
    auto row = std::make_unique<StreamRow>();
    row->D = d.seg[r].downsamp;
    row->n_dm = d.seg[r].n_dm;
    row->M = d.max_delay[r];
    row->Wcap = s->B / row->D;
    // ring: the block, the maximum delay and kCutoutReach samples of history
    // for the frequency-time cutouts of candidates
    row->R = (row->Wcap + row->M + 8 + kCutoutReach + 3) / 4 * 4;
    row->tables.addr.device = s->ctx->device;
    row->tables.dmin.device = s->ctx->device;
    // the staged rows are uint16 for every D in a stream (one kernel instance)
    build_row_tables(s->ctx, &d, b.freqs.data(), r, sh, row->tables, unit_max<uint16_t>());  // rings are uint16
    b.rows.push_back(std::move(row));
  }
}

void admit(gsp_stream *s, Beam &b) {
  for (auto &in : b.in) {
    in.device = s->ctx->device;
    in.reserve((size_t)s->B * b.nchan);
  }
  b.pf_src = nullptr;
  for (auto &r : b.rows) {
    r->ring.device = s->ctx->device;
    r->ring.reserve((size_t)b.nchan * (r->R + kGuard) * 2);
    r->win.device = s->ctx->device;
    r->win.reserve((size_t)r->n_dm * (s->look + r->Wcap) * 4);
    r->tables.delays_dev.device = s->ctx->device;
    r->tables.delays_dev.reserve(r->tables.delays_host.size() * 4);
    check_hip(hipMemcpy(r->tables.delays_dev.ptr, r->tables.delays_host.data(), r->tables.delays_host.size() * 4,
                        hipMemcpyHostToDevice),
              "copy delays");
  }
  b.admitted = true;
  s->used += b.mem;
}

void release(gsp_stream *s, Beam &b) {
  if (!b.admitted) return;
  check_hip(hipStreamSynchronize(s->cst), "synchronise copy stream");  // no copy still writes b.in
  b.pf_src = nullptr;
  for (auto &in : b.in) in.reserve(0);
  s->used -= b.mem;
  b.admitted = false;
}

void admit_queued(gsp_stream *s) {
  while (!s->queue.empty()) {
    auto it = s->beams.find(s->queue.front());
    if (it == s->beams.end()) {
      s->queue.pop_front();
      continue;
    }
    Beam &b = *it->second;
    if (s->used + b.mem > s->budget) break;  // FIFO: later beams wait too
    admit(s, b);
    s->queue.pop_front();
  }
}

void set_attributes(gsp_stream *s, int64_t dd_lds) {
  set_search_attributes(s->tiling);
  check_hip(hipFuncSetAttribute((const void *)k_dedisp_jobs<kStreamGroups, kStreamTpw>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)dd_lds),
            "set LDS size");
}

// The fixed kernel sequence of a step (captured into the step graph).
// Kernel timing is not recorded inside it (no events in the graph).
void launch_sequence(gsp_stream *s, int64_t dd_lds) {
  gsp_ctx *ctx = nullptr;
  hipStream_t st = s->st;
  // the previous window's look-back shift first: after a step the window
  // buffer still holds [look-back | window], which the cutouts read
  hipLaunchKernelGGL(k_tail, dim3((unsigned)grid_of(4)), dim3(256), (size_t)s->look * 4, st,
                     s->d_tail.as<TailTable>());
  hipLaunchKernelGGL(k_stage_ring, dim3((unsigned)grid_of(4)), dim3(256), 0, st, s->d_stage.as<StageTable>());
  auto kd = k_dedisp_jobs<kStreamGroups, kStreamTpw>;
  hipLaunchKernelGGL(kd, dim3((unsigned)grid_of(2)), dim3(64 * kStreamWaves), (size_t)dd_lds, st,
                     s->d_dedisp.as<DedispTable>());
  launch_stats_table(ctx, s->d_series.as<SeriesTable>(), grid_of(8), s->musig.as<double>(), 0, st);
  launch_search_table(ctx, s->d_series.as<SeriesTable>(), grid_of(4), s->tiling, s->musig.as<double>(),
                      s->d_widths.as<int32_t>(), (int32_t)s->widths.size(), s->wmax, s->thr, s->frags.as<Frag>(),
                      s->frag_cap, s->counter.as<unsigned long long>(), 0, st);
  check_hip(hipGetLastError(), "launch streaming kernels");
}

// One step: one pending block of every admitted beam.  Returns blocks processed.
int64_t step_once(gsp_stream *s) {
  struct Work {
    Beam *b;
    PendingBlock blk;
  };
  std::vector<Work> work;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t rows = 0;  // one staging, dedispersion, series and shift job per (beam, row) at most
    for (auto &kv : s->beams) {
      Beam &b = *kv.second;
      if (b.admitted && !b.pending.empty()) {
        if (rows + (int64_t)b.rows.size() > kMaxJobs) break;  // the rest wait for the next step
        rows += (int64_t)b.rows.size();
        work.push_back({&b, b.pending.front()});
        b.pending.pop_front();
        b.inflight = true;
      }
    }
  }
  if (work.empty()) return 0;
  const auto t_start = Clock::now();
  hipStream_t st = s->st;
  // blocks copied ahead during the previous step have arrived; from here on
  // neither input buffer of any beam is being written or read
  check_hip(hipStreamSynchronize(s->cst), "synchronise copy stream");
  StageTable &ts = *s->h_stage;
  DedispTable &td = *s->h_dedisp;
  SeriesTable &tr = *s->h_series;
  TailTable &tt = *s->h_tail;
  ts.n_jobs = 0;
  ts.n_items = 0;
  td.n_jobs = 0;
  td.n_items = 0;
  tr.n_jobs = 0;
  tt.n_jobs = 0;
  tt.n_trials = 0;
  int64_t dd_lds = 0;
  struct JobRef {
    Beam *b;
    int32_t row;
    int64_t a;
  };
  std::vector<JobRef> series_refs;
  for (auto &w : work) {
    Beam &b = *w.b;
    if (b.pf_src != nullptr && b.pf_src == w.blk.buf.p) {
      b.cur = b.pf_buf;  // copied during the previous step
    } else {
      b.cur = 0;  // both buffers are idle here
      check_hip(hipMemcpyAsync(b.in[0].ptr, w.blk.buf.p, (size_t)w.blk.nsamp * b.nchan, hipMemcpyHostToDevice, st),
                "copy block");
    }
    b.pf_src = nullptr;
    for (int32_t r = 0; r < (int32_t)b.rows.size(); ++r) {
      StreamRow &R = *b.rows[r];
      const int64_t n_new = w.blk.nsamp / R.D;
      // staging job
      if (n_new > 0) {
        if (ts.n_jobs >= kMaxJobs) fail(GSP_ECAPACITY, "too many streaming jobs");
        StageJob &J = ts.job[ts.n_jobs++];
        J.X = b.in[b.cur].as<uint8_t>();
        J.Y = R.ring.as<uint16_t>();
        J.pitch = R.R + kGuard;
        J.ring = R.R;
        J.phys0 = R.N % R.R;
        J.n_new = n_new;
        J.nchan = b.nchan;
        J.D = R.D;
        J.t_tiles = (int32_t)((n_new + kStageTile - 1) / kStageTile);
        J.c_tiles = (b.nchan + kStageTile - 1) / kStageTile;
        J.item0 = ts.n_items;
        ts.n_items += (int64_t)J.t_tiles * J.c_tiles;
      }
      const int64_t N1 = R.N + n_new;
      const int64_t a = std::max<int64_t>(0, R.N - R.M);
      const int64_t e = std::max<int64_t>(0, N1 - R.M);
      R.last_a = a;
      R.last_b = e;
      R.N = N1;
      if (e <= a) continue;
      R.emitted = e;
      // dedispersion job over outputs [a, e)
      if (td.n_jobs >= kMaxJobs || tr.n_jobs >= kMaxJobs) fail(GSP_ECAPACITY, "too many streaming jobs");
      DedispJob &D = td.job[td.n_jobs++];
      const RowTables &rt = R.tables;
      DedispArgs &A = D.a;
      A.seg_ch = 0;  // one output for all channels
      A.seg_stride = 0;
      const int64_t origin = a & ~int64_t(3);
      A.Y = R.ring.ptr;
      A.pitch = R.R + kGuard;
      A.addr = rt.addr.as<uint32_t>();
      A.base = rt.dmin.as<int32_t>();
      A.out = R.win.as<int32_t>() + s->look;
      A.out_pitch = s->look + R.Wcap;
      A.t_origin = origin;
      A.t_lo = a;
      A.t_hi = e;
      A.ring = R.R;
      A.phys0 = origin % R.R;
      A.n_dm = R.n_dm;
      const int MT = rt.shape.trials_per_block();
      A.n_dm_tiles = (R.n_dm + MT - 1) / MT;
      A.n_dm_pad = A.n_dm_tiles * MT;
      A.nchan = b.nchan;
      A.chunks = rt.passes.as<int32_t>();
      A.n_chunks = rt.n_passes;
      A.max_chunk = rt.max_chunk;
      A.data_dw = rt.data_dw;
      A.flush = std::max(1, std::min(65535 / (255 * R.D), 256));
      const int64_t T = rt.shape.samples_per_block();
      A.n_t_tiles = (int32_t)((e - origin + T - 1) / T);
      D.item0 = td.n_items;
      td.n_items += (int64_t)A.n_dm_tiles * A.n_t_tiles;
      dd_lds = std::max<int64_t>(dd_lds, rt.lds_bytes);
      // search job over the window, boxes reaching back into the look-back
      SeriesJob &S = tr.job[tr.n_jobs++];
      S.x = R.win.as<int32_t>();
      S.pitch = s->look + R.Wcap;
      S.e_begin = s->look;
      S.n = e - a;
      S.look = std::min<int64_t>(s->look, a);
      S.abs0 = a;
      S.n_dm = R.n_dm;
      series_refs.push_back({&b, r, a});
      // look-back shift job
      TailJob &L = tt.job[tt.n_jobs++];
      L.x = R.win.as<int32_t>();
      L.pitch = s->look + R.Wcap;
      L.look = s->look;
      L.w = R.last_w;  // shift out the previous window (0 for the first)
      R.last_w = e - a;
      L.n_dm = R.n_dm;
      L.trial0 = tt.n_trials;
      tt.n_trials += R.n_dm;
    }
  }
  finalize_table(tr, s->tiling);
  // scratch sizes
  if (tr.n_trials * 2 > s->musig_cap) {
    s->musig_cap = std::max<int64_t>(tr.n_trials * 2, 4096);
    s->musig.reserve((size_t)s->musig_cap * sizeof(double));
    if (s->exec) {  // pointers captured in the graph changed
      (void)hipGraphExecDestroy(s->exec);
      s->exec = nullptr;
    }
  }
  if (dd_lds == 0) dd_lds = 16;
  // upload the tables (pageable copies are staged, the host tables may be
  // rewritten after the calls return)
  check_hip(hipMemcpyAsync(s->d_stage.ptr, &ts, sizeof(StageTable), hipMemcpyHostToDevice, st), "copy tables");
  check_hip(hipMemcpyAsync(s->d_dedisp.ptr, &td, sizeof(DedispTable), hipMemcpyHostToDevice, st), "copy tables");
  check_hip(hipMemcpyAsync(s->d_series.ptr, &tr, sizeof(SeriesTable), hipMemcpyHostToDevice, st), "copy tables");
  check_hip(hipMemcpyAsync(s->d_tail.ptr, &tt, sizeof(TailTable), hipMemcpyHostToDevice, st), "copy tables");
  // kernels: replay the captured graph (re-captured if the LDS need grew)
  const int64_t lds_need = std::max<int64_t>(dd_lds, 64 * 1024);
  if (s->use_graph) {
    if (!s->exec || lds_need > s->graph_lds) {
      if (s->exec) (void)hipGraphExecDestroy(s->exec);
      if (s->graph) (void)hipGraphDestroy(s->graph);
      s->exec = nullptr;
      s->graph = nullptr;
      set_attributes(s, lds_need);
      check_hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
      try {
        launch_sequence(s, lds_need);
      } catch (...) {
        hipGraph_t g;
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      check_hip(hipStreamEndCapture(st, &s->graph), "end capture");
      check_hip(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0), "instantiate graph");
      s->graph_lds = lds_need;
    }
    check_hip(hipGraphLaunch(s->exec, st), "launch graph");
  } else {
    set_attributes(s, lds_need);
    launch_sequence(s, lds_need);
  }
  // while the kernels run, copy each beam's next pending block into its other
  // input buffer (the front of a beam's queue only leaves it through a step,
  // so that block is the one the next step takes)
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &w : work) {
      Beam &b = *w.b;
      if (b.pending.empty()) continue;
      const PendingBlock &nx = b.pending.front();
      const int v = b.cur ^ 1;
      check_hip(hipMemcpyAsync(b.in[v].ptr, nx.buf.p, (size_t)nx.nsamp * b.nchan, hipMemcpyHostToDevice, s->cst),
                "copy next block");
      b.pf_src = nx.buf.p;
      b.pf_buf = v;
    }
  }
  // results
  unsigned long long count = 0;
  check_hip(hipMemcpyAsync(&count, s->counter.ptr, sizeof(count), hipMemcpyDeviceToHost, st), "copy count");
  check_hip(hipStreamSynchronize(st), "synchronise stream");
  if ((int64_t)count > s->frag_cap) {
    // Until the next step's look-back shift the window buffers and the
    // statistics of this step stay as they are: grow the fragment buffer and
    // search the same windows again, outside the graph (whose captured
    // buffer pointer is now stale, so the next step captures anew).
    s->frag_cap = ((int64_t)count + (int64_t)count / 4 + 4095) / 4096 * 4096;
    s->frags.reserve((size_t)s->frag_cap * sizeof(Frag));
    if (s->exec) {
      (void)hipGraphExecDestroy(s->exec);
      s->exec = nullptr;
    }
    set_search_attributes(s->tiling);
    launch_search_table(nullptr, s->d_series.as<SeriesTable>(), grid_of(4), s->tiling, s->musig.as<double>(),
                        s->d_widths.as<int32_t>(), (int32_t)s->widths.size(), s->wmax, s->thr, s->frags.as<Frag>(),
                        s->frag_cap, s->counter.as<unsigned long long>(), 0, st);
    check_hip(hipMemcpyAsync(&count, s->counter.ptr, sizeof(count), hipMemcpyDeviceToHost, st), "copy count");
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    s->regrown += 1;
    if ((int64_t)count > s->frag_cap) fail(GSP_EDEVICE, "the repeated search found more fragments");
  }
  std::vector<Frag> fr(count);
  if (count)
    check_hip(hipMemcpy(fr.data(), s->frags.ptr, count * sizeof(Frag), hipMemcpyDeviceToHost), "copy fragments");
  std::sort(fr.begin(), fr.end(), [](const Frag &x, const Frag &y) {
    return x.trial != y.trial ? x.trial < y.trial : x.t_first < y.t_first;
  });
  std::vector<Frag> runs;
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
  // learned triage: cutouts from the device state of this step, network logits
  std::vector<float> score(runs.size(), NAN);
  if (s->cnn && !runs.empty()) {
    const auto t_tri = Clock::now();
    const int64_t n = (int64_t)runs.size();
    std::vector<StreamCut> cuts((size_t)n);
    for (int64_t k = 0; k < n; ++k) {
      const Frag &f = runs[(size_t)k];
      int j = 0;
      while (j + 1 < tr.n_jobs && tr.job[j + 1].trial0 <= f.trial) ++j;
      const JobRef &ref = series_refs[j];
      StreamRow &R = *ref.b->rows[ref.row];
      StreamCut &C = cuts[(size_t)k];
      C.win = R.win.as<int32_t>();
      C.win_pitch = s->look + R.Wcap;
      C.a = ref.a;
      C.mu = s->musig.as<double>() + 2 * (int64_t)tr.job[j].trial0;
      C.ring = R.ring.as<uint16_t>();
      C.ring_pitch = R.R + kGuard;
      C.R = R.R;
      C.delays = R.tables.delays_dev.as<int32_t>();
      C.t_peak = f.e_peak - f.width + 1;
      C.look = s->look;
      C.n_dm = R.n_dm;
      C.nchan = ref.b->nchan;
      C.dm_index = f.trial - tr.job[j].trial0;
      C.width = f.width;
    }
    s->d_cuts.reserve((size_t)n * sizeof(StreamCut));
    s->d_cutimg.reserve((size_t)n * 2 * 4096 * 2);
    s->d_logits.reserve((size_t)n * 4);
    check_hip(hipMemcpyAsync(s->d_cuts.ptr, cuts.data(), (size_t)n * sizeof(StreamCut), hipMemcpyHostToDevice, st),
              "copy cutout sources");
    launch_cutouts_stream(s->d_cuts.as<StreamCut>(), n, s->d_cutimg.as<uint16_t>(), st);
    const int rc = gsp_cnn_forward(s->cnn, s->d_cutimg.as<uint16_t>(), n, s->d_logits.as<float>(), st);
    if (rc != GSP_OK) fail(rc, "triage network");
    check_hip(hipMemcpyAsync(score.data(), s->d_logits.ptr, (size_t)n * 4, hipMemcpyDeviceToHost, st), "copy scores");
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    s->scored += n;
    s->triage_s += std::chrono::duration<double>(Clock::now() - t_tri).count();
  }
  const auto t_done = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t k = 0; k < runs.size(); ++k) {
    const Frag &f = runs[k];
    if (s->cnn && !(score[k] > s->triage_thr)) {  // rejected by the network
      ++s->rejected;
      continue;
    }
    int j = 0;
    while (j + 1 < tr.n_jobs && tr.job[j + 1].trial0 <= f.trial) ++j;
    const JobRef &ref = series_refs[j];
    const gsp_segment &g = ref.b->segs[ref.row];
    gsp_stream_candidate sc;
    std::memset(&sc, 0, sizeof(sc));
    sc.beam = ref.b->id;
    sc.block = (int32_t)ref.b->blocks_done;
    gsp_candidate &c = sc.c;
    c.seg = ref.row;
    c.dm_index = f.trial - tr.job[j].trial0;
    c.dm = g.dm_lo + (double)c.dm_index * g.dm_step;
    c.width = f.width;
    c.t_peak = f.e_peak - f.width + 1;
    c.t_first = f.t_first;
    c.t_last = f.t_last;
    c.snr = (float)f.snr;
    c.time_s = ((double)c.t_peak + 0.5 * (double)c.width) * (double)g.downsamp * ref.b->tsamp;
    sc.score = score[k];
    s->out.push_back(sc);
  }
  for (auto &w : work) {
    Beam &b = *w.b;
    b.inflight = false;
    b.blocks_done += 1;
    b.samples_in += w.blk.nsamp;
    s->lat.push_back(std::chrono::duration<double>(t_done - w.blk.arrival).count());
    give_pinned(s, w.blk.buf);
  }
  s->steps += 1;
  s->blocks += (int64_t)work.size();
  s->busy_s += std::chrono::duration<double>(t_done - t_start).count();
  // finished beams release their memory; queued beams may now fit
  for (auto it = s->beams.begin(); it != s->beams.end();) {
    Beam &b = *it->second;
    if ((b.closing || b.ended) && b.pending.empty() && b.admitted) {
      release(s, b);
      it = s->beams.erase(it);
    } else {
      ++it;
    }
  }
  admit_queued(s);
  s->cv.notify_all();
  return (int64_t)work.size();
}

template <class F>
int sguard(gsp_stream *s, F &&f) {
  if (!s) return GSP_EINVAL;
  try {
    check_hip(hipSetDevice(s->ctx->device), "select device");
    f();
    return GSP_OK;
  } catch (const Error &e) {
    s->last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    s->last_error = "host allocation failed";
    return GSP_ENOMEM;
  } catch (...) {
    s->last_error = "unexpected internal error";
    return GSP_EDEVICE;
  }
}

}  // namespace

extern "C" {

int gsp_stream_create(gsp_ctx *ctx, int64_t mem_budget_bytes, int32_t block_nsamp, const int32_t *widths,
                      int32_t n_widths, float threshold, gsp_stream **out) {
  if (!ctx || !out || !widths) return GSP_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&] {
    if (mem_budget_bytes <= 0 || block_nsamp < 1) fail(GSP_EINVAL, "budget and block length must be positive");
    if (n_widths < 1 || n_widths > 64 || !std::isfinite(threshold)) fail(GSP_EINVAL, "bad width set or threshold");
    auto s = std::make_unique<gsp_stream>();
    s->ctx = ctx;
    s->budget = mem_budget_bytes;
    s->B = block_nsamp;
    s->widths.assign(widths, widths + n_widths);
    for (int32_t v : s->widths)
      if (v < 1 || v > 4096) fail(GSP_EINVAL, "widths must be in [1, 4096]");
    std::sort(s->widths.begin(), s->widths.end());
    s->widths.erase(std::unique(s->widths.begin(), s->widths.end()), s->widths.end());
    s->wmax = s->widths.back();
    s->look = std::max(s->wmax - 1, kCutoutReach - 1);  // boxes, and the cutouts' 64 bins of <= 8 samples
    s->thr = threshold;
    s->tiling = search_tiling(s->wmax);
    if ((int64_t)s->look * 4 > 64 * 1024) fail(GSP_EINVAL, "widths too large for the look-back shift");
    check_hip(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking), "create stream");
    check_hip(hipStreamCreateWithFlags(&s->cst, hipStreamNonBlocking), "create copy stream");
    for (DevBuf *d : {&s->d_stage, &s->d_dedisp, &s->d_series, &s->d_tail, &s->d_widths, &s->musig, &s->frags,
                      &s->counter, &s->d_cuts, &s->d_cutimg, &s->d_logits})
      d->device = ctx->device;
    s->d_stage.reserve(sizeof(StageTable));
    s->d_dedisp.reserve(sizeof(DedispTable));
    s->d_series.reserve(sizeof(SeriesTable));
    s->d_tail.reserve(sizeof(TailTable));
    s->d_widths.reserve(s->widths.size() * 4);
    check_hip(hipMemcpy(s->d_widths.ptr, s->widths.data(), s->widths.size() * 4, hipMemcpyHostToDevice),
              "copy widths");
    s->musig_cap = 4096;
    s->musig.reserve((size_t)s->musig_cap * sizeof(double));
    s->frags.reserve((size_t)s->frag_cap * sizeof(Frag));
    s->counter.reserve(sizeof(unsigned long long));
    *out = s.release();
  });
}

void gsp_stream_destroy(gsp_stream *s) {
  if (!s) return;
  gsp_stream_stop(s);
  (void)hipSetDevice(s->ctx->device);
  (void)hipStreamSynchronize(s->st);
  (void)hipStreamSynchronize(s->cst);
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  for (auto &kv : s->beams)
    for (auto &p : kv.second->pending) (void)hipHostFree(p.buf.p);
  for (auto &p : s->pool) (void)hipHostFree(p.p);
  s->beams.clear();
  (void)hipStreamDestroy(s->st);
  (void)hipStreamDestroy(s->cst);
  delete s;
}

const char *gsp_stream_last_error(const gsp_stream *s) { return s ? s->last_error.c_str() : ""; }

int gsp_stream_open_beam(gsp_stream *s, int32_t nchan, const double *freqs, double tsamp, const gsp_segment *segs,
                         int32_t n_seg, int32_t *beam_id) {
  int status = GSP_OK;
  int rc = sguard(s, [&] {
    if (!freqs || !segs || !beam_id || nchan < 1) fail(GSP_EINVAL, "bad beam arguments");
    auto b = std::make_unique<Beam>();
    b->nchan = nchan;
    b->freqs.assign(freqs, freqs + nchan);
    b->tsamp = tsamp;
    b->segs.assign(segs, segs + n_seg);
    plan_beam(s, *b);
    b->mem = beam_bytes(s, *b);
    if (b->mem > s->budget) fail(GSP_ENOMEM, "beam larger than the stream's memory budget");
    std::lock_guard<std::mutex> lk(s->mu);
    b->id = s->next_id++;
    *beam_id = b->id;
    const int32_t id = b->id;
    const bool fits = s->queue.empty() && s->used + b->mem <= s->budget;
    Beam &ref = *b;
    s->beams.emplace(id, std::move(b));
    if (fits)
      admit(s, ref);
    else {
      s->queue.push_back(id);
      status = GSP_EAGAIN;
    }
  });
  return rc == GSP_OK ? status : rc;
}

int gsp_stream_push(gsp_stream *s, int32_t beam_id, const uint8_t *block, int64_t nsamp) {
  return sguard(s, [&] {
    if (!block || nsamp < 0 || nsamp > s->B) fail(GSP_EINVAL, "block must hold 0 .. block_nsamp samples");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) fail(GSP_EINVAL, "unknown beam");
    if (it->second->ended || it->second->closing) fail(GSP_EINVAL, "beam already ended");
    const int32_t nchan = it->second->nchan;
    const size_t bytes = (size_t)s->B * nchan;
    PendingBlock p;
    p.buf = take_pinned(s, bytes);
    lk.unlock();  // the copy runs unlocked; the beam may be closed meanwhile
    std::memcpy(p.buf.p, block, (size_t)nsamp * nchan);
    lk.lock();
    it = s->beams.find(beam_id);
    if (it == s->beams.end() || it->second->ended || it->second->closing) {
      give_pinned(s, p.buf);
      fail(GSP_EINVAL, "beam closed while its block was being copied");
    }
    Beam &b = *it->second;
    p.nsamp = nsamp;
    p.arrival = Clock::now();
    if (nsamp < s->B) b.ended = true;
    b.pending.push_back(p);
    s->cv.notify_all();
  });
}

int gsp_stream_close_beam(gsp_stream *s, int32_t beam_id) {
  return sguard(s, [&] {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) fail(GSP_EINVAL, "unknown beam");
    Beam &b = *it->second;
    b.closing = true;
    if (b.pending.empty() && !b.inflight) {
      release(s, b);
      s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), beam_id), s->queue.end());
      s->beams.erase(it);
      admit_queued(s);
    }
  });
}

int gsp_stream_step(gsp_stream *s, int64_t *n_blocks) {
  return sguard(s, [&] {
    if (s->running) fail(GSP_EINVAL, "the stream's worker thread is running");
    const int64_t n = step_once(s);
    if (n_blocks) *n_blocks = n;
  });
}

int gsp_stream_start(gsp_stream *s) {
  return sguard(s, [&] {
    if (s->running) return;
    s->stop = false;
    s->running = true;
    s->worker = std::thread([s] {
      (void)hipSetDevice(s->ctx->device);
      for (;;) {
        {
          std::unique_lock<std::mutex> lk(s->mu);
          s->cv.wait(lk, [s] {
            if (s->stop) return true;
            for (auto &kv : s->beams)
              if (kv.second->admitted && !kv.second->pending.empty()) return true;
            return false;
          });
          if (s->stop) break;
        }
        std::string err;
        try {
          step_once(s);
        } catch (const Error &e) {
          err = e.msg;
        } catch (const std::bad_alloc &) {
          err = "host allocation failed";
        } catch (...) {
          err = "unexpected internal error";
        }
        if (!err.empty()) {
          std::lock_guard<std::mutex> lk(s->mu);
          s->last_error = err;
          s->stop = true;
          s->cv.notify_all();
          break;
        }
      }
    });
  });
}

int gsp_stream_stop(gsp_stream *s) {
  if (!s) return GSP_EINVAL;
  if (!s->running) return GSP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->running = false;
  return s->last_error.empty() ? GSP_OK : GSP_EDEVICE;
}

int gsp_stream_flush(gsp_stream *s) {
  return sguard(s, [&] {
    if (s->running) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [s] {
        if (s->stop) return true;
        for (auto &kv : s->beams)
          if ((kv.second->admitted && !kv.second->pending.empty()) || kv.second->inflight) return false;
        return true;
      });
      if (!s->last_error.empty()) fail(GSP_EDEVICE, s->last_error);
    } else {
      while (step_once(s) > 0) {
      }
    }
  });
}

int gsp_stream_poll(gsp_stream *s, gsp_stream_candidate *out, int64_t cap, int64_t *n) {
  return sguard(s, [&] {
    if (!n || cap < 0 || (cap > 0 && !out)) fail(GSP_EINVAL, "bad output buffer");
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t k = std::min<int64_t>(cap, (int64_t)s->out.size());
    if (k) std::memcpy(out, s->out.data(), (size_t)k * sizeof(gsp_stream_candidate));
    s->out.erase(s->out.begin(), s->out.begin() + k);
    *n = k;
  });
}

int gsp_stream_set_triage(gsp_stream *s, gsp_cnn *cnn, float threshold) {
  return sguard(s, [&] {
    if (s->running) fail(GSP_EINVAL, "the stream's worker thread is running");
    if (cnn && !std::isfinite(threshold)) fail(GSP_EINVAL, "bad triage threshold");
    std::lock_guard<std::mutex> lk(s->mu);
    s->cnn = cnn;
    s->triage_thr = threshold;
  });
}

int gsp_stream_report(gsp_stream *s, gsp_stream_stats *r) {
  return sguard(s, [&] {
    if (!r) fail(GSP_EINVAL, "null report");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(r, 0, sizeof(*r));
    std::vector<double> l = s->lat;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {  // nearest rank
      if (l.empty()) return 0.0;
      size_t k = (size_t)std::ceil(q * (double)l.size());
      k = k == 0 ? 0 : k - 1;
      return l[std::min(k, l.size() - 1)];
    };
    r->lat_p50_s = pct(0.5);
    r->lat_p99_s = pct(0.99);
    r->lat_max_s = l.empty() ? 0.0 : l.back();
    r->blocks = s->blocks;
    r->steps = s->steps;
    r->busy_s = s->busy_s;
    r->mem_used = s->used;
    r->mem_budget = s->budget;
    r->triage_scored = s->scored;
    r->triage_rejected = s->rejected;
    r->triage_s = s->triage_s;
    r->search_repeats = s->regrown;
    for (auto &kv : s->beams) {
      if (kv.second->admitted)
        r->beams_active += 1;
      else
        r->beams_queued += 1;
      r->blocks_pending += (int64_t)kv.second->pending.size();
    }
  });
}

int gsp_stream_window(gsp_stream *s, int32_t beam_id, int32_t seg, int32_t *host_out, int64_t cap, int64_t *t_first,
                      int64_t *n_t) {
  return sguard(s, [&] {
    if (s->running) fail(GSP_EINVAL, "the stream's worker thread is running");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) fail(GSP_EINVAL, "unknown beam");
    Beam &b = *it->second;
    if (seg < 0 || seg >= (int32_t)b.rows.size() || !t_first || !n_t) fail(GSP_EINVAL, "bad row");
    StreamRow &R = *b.rows[seg];
    const int64_t w = R.last_b - R.last_a;
    *t_first = R.last_a;
    *n_t = w;
    if (w <= 0) return;
    if (cap < (int64_t)R.n_dm * w || !host_out) fail(GSP_ECAPACITY, "window buffer too small");
    check_hip(hipMemcpy2D(host_out, (size_t)w * 4, R.win.as<int32_t>() + s->look, (size_t)(s->look + R.Wcap) * 4,
                          (size_t)w * 4, (size_t)R.n_dm, hipMemcpyDeviceToHost),
              "copy window");
  });
}

int gsp_stream_snapshot(gsp_stream *s, int32_t beam_id, void *host_buf, int64_t cap, int64_t *bytes) {
  return sguard(s, [&] {
    if (s->running) fail(GSP_EINVAL, "the stream's worker thread is running");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end() || !bytes) fail(GSP_EINVAL, "unknown beam");
    Beam &b = *it->second;
    if (!b.admitted || !b.pending.empty()) fail(GSP_EINVAL, "snapshot needs an admitted beam with no pending block");
    int64_t need = 3 * 8;
    for (auto &r : b.rows) need += 2 * 8 + (int64_t)b.nchan * (r->R + kGuard) * 2 + (int64_t)r->n_dm * s->look * 4;
    *bytes = need;
    if (!host_buf || cap < need) fail(GSP_ECAPACITY, "snapshot buffer too small");
    char *p = static_cast<char *>(host_buf);
    auto put = [&](int64_t v) {
      std::memcpy(p, &v, 8);
      p += 8;
    };
    put(b.blocks_done);
    put(b.samples_in);
    put((int64_t)b.rows.size());
    for (auto &r : b.rows) {
      put(r->N);
      put(r->emitted);
      const size_t rb = (size_t)b.nchan * (r->R + kGuard) * 2;
      check_hip(hipMemcpy(p, r->ring.ptr, rb, hipMemcpyDeviceToHost), "copy ring");
      p += rb;
      if (s->look) {  // the samples before the next window: the last `look` of [look-back | last window]
        check_hip(hipMemcpy2D(p, (size_t)s->look * 4, r->win.as<int32_t>() + r->last_w, (size_t)(s->look + r->Wcap) * 4,
                              (size_t)s->look * 4, (size_t)r->n_dm, hipMemcpyDeviceToHost),
                  "copy look-back");
        p += (size_t)r->n_dm * s->look * 4;
      }
    }
  });
}

int gsp_stream_restore(gsp_stream *s, int32_t beam_id, const void *host_buf, int64_t bytes) {
  return sguard(s, [&] {
    if (s->running) fail(GSP_EINVAL, "the stream's worker thread is running");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end() || !host_buf) fail(GSP_EINVAL, "unknown beam");
    Beam &b = *it->second;
    if (!b.admitted || !b.pending.empty() || b.blocks_done != 0)
      fail(GSP_EINVAL, "restore needs a freshly opened, admitted beam");
    const char *p = static_cast<const char *>(host_buf);
    const char *end = p + bytes;
    auto get = [&]() {
      if (p + 8 > end) fail(GSP_EINVAL, "snapshot truncated");
      int64_t v;
      std::memcpy(&v, p, 8);
      p += 8;
      return v;
    };
    const int64_t blocks_done = get(), samples_in = get(), nrows = get();
    if (nrows != (int64_t)b.rows.size()) fail(GSP_EINVAL, "snapshot of a different plan");
    for (auto &r : b.rows) {
      r->N = get();
      r->emitted = get();
      r->last_w = 0;  // the snapshot holds the look-back already shifted
      const size_t rb = (size_t)b.nchan * (r->R + kGuard) * 2;
      if (p + rb > end) fail(GSP_EINVAL, "snapshot truncated");
      check_hip(hipMemcpy(r->ring.ptr, p, rb, hipMemcpyHostToDevice), "copy ring");
      p += rb;
      if (s->look) {
        const size_t lb = (size_t)r->n_dm * s->look * 4;
        if (p + lb > end) fail(GSP_EINVAL, "snapshot truncated");
        check_hip(hipMemcpy2D(r->win.ptr, (size_t)(s->look + r->Wcap) * 4, p, (size_t)s->look * 4, (size_t)s->look * 4,
                              (size_t)r->n_dm, hipMemcpyHostToDevice),
                  "copy look-back");
        p += lb;
      }
    }
    b.blocks_done = blocks_done;
    b.samples_in = samples_in;
  });
}

int gsp_stream_set_graph(gsp_stream *s, int enable) {
  return sguard(s, [&] { s->use_graph = enable != 0; });
}

int gsp_stream_set_fragment_capacity(gsp_stream *s, int64_t cap) {
  return sguard(s, [&] {
    if (s->running) fail(GSP_EINVAL, "the stream's worker thread is running");
    if (cap < 1 || cap > (int64_t(1) << 30)) fail(GSP_EINVAL, "capacity must be in [1, 2^30]");
    check_hip(hipStreamSynchronize(s->st), "synchronise stream");
    s->frag_cap = cap;
    s->frags.reserve((size_t)cap * sizeof(Frag));
    if (s->exec) {  // the captured buffer pointer may have changed
      (void)hipGraphExecDestroy(s->exec);
      s->exec = nullptr;
    }
  });
}

}  // extern "C"
