// Sub-band (two-stage) dedispersion on gfx950.
//
// What is computed (paper Section 2.3: GSP runs the sub-band algorithm of
// PRESTO's prepsubband; Tables 2-3 are its survey plans).  Per plan row with
// downsampling D, the channels form n_sub bands, band b = channels
// [b*nchan/n_sub, (b+1)*nchan/n_sub) with reference frequency f_b = its
// highest channel; the row's trials form groups of `group` consecutive
// trials, group g with nominal DM_g at its centre.
//   stage 1: Z[g][b][t] = sum_{c in b} Y[c][t + d1(g, c)], d1 = delay of DM_g at
//            f_c against f_b;
//   stage 2: out[i][t] = sum_b Z[g(i)][b][t + d2(i, b)], d2 = delay of DM_i at
//            f_b against fref;
// delays rounded as in gsp_delay_table (the reference frequency replaced).
// The output is exact integer arithmetic on the composite delays d2 + d1,
// which differ from the brute-force ones by the smearing of |DM_i - DM_g|
// inside a band.  Adds per output: nchan / group (stage 1) + n_sub (stage 2)
// instead of nchan.
//
// How: both stages are the brute-force tile (dedisp_tile.h) run over job
// tables on a persistent grid.  Stage 1's jobs are the bands (trials = the
// groups, channels = the band's channels of the staged row, output the
// uint16 sub-band series: 255 * D * channels per band stays below 2^16),
// stage 2's jobs are the groups (trials = the group's trials, channels = the
// bands, input those uint16 series).  Job tables are built once per plan and
// hold offsets from base pointers passed at launch, so a call uploads
// nothing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "dedisp_tile.h"
#include "gsp_internal.h"

namespace gsp {

namespace {

constexpr int kSubMaxJobs = 1024;
constexpr int64_t kZBudget = int64_t(16) << 30;  // bytes of sub-band series held at once

struct SubJob {
  DedispArgs a;  // a.Y, a.out: byte offsets from the launch's source and destination bases
  int64_t item0;
};
struct SubTable {
  SubJob job[kSubMaxJobs];
  int32_t n_jobs;
  int64_t n_items;
};

__device__ __forceinline__ int sub_find(const SubTable *t, int64_t b) {
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

// Persistent grid over the tiles of every job; with a multiple of 8
// workgroups each XCD takes a contiguous eighth of the tiles (neighbouring
// tiles share their input windows in that XCD's L2).
template <int K, int TPW, typename SrcT, typename OutT, bool SEG>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_dedisp_sub(
    const SubTable *__restrict__ tb, const char *src_base, char *dst_base) {
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
    const int j = __builtin_amdgcn_readfirstlane(sub_find(tb, b));
    DedispArgs a = tb->job[j].a;
    a.Y = src_base + reinterpret_cast<intptr_t>(a.Y);
    a.out = dst_base + reinterpret_cast<intptr_t>(a.out);
    const int64_t local = b - tb->job[j].item0;
    __syncthreads();  // LDS of the previous tile is free
    dedisp_tile<K, TPW, SrcT, OutT, SEG>(a, (int)(local % a.n_dm_tiles), (int)(local / a.n_dm_tiles), lds);
  }
}

constexpr int kSubK = 4, kSubTpw = 4;

struct SubChunk {
  int32_t g0, g1;                                 // groups [g0, g1)
  std::vector<std::unique_ptr<RowTables>> s1;     // per band
  DevBuf t1, t2;                                  // job tables of the two stages
  int64_t lds1 = 0, lds2 = 0;
  double adds1 = 0, adds2 = 0;
  bool seg = false;  // stage 1 is one job with band segments
};

struct SubRow {
  int32_t n_sub = 0, group = 0, n_groups = 0, D = 1, n_dm = 0, cpb_max = 0;
  int64_t N = 0, n_out = 0, Zn = 0, Zpitch = 0, pitch = 0;
  std::vector<int32_t> c0;                       // band boundaries, n_sub + 1
  std::vector<std::unique_ptr<RowTables>> s2;    // per group
  std::vector<std::unique_ptr<SubChunk>> chunks;
  int32_t waves2 = 4;
};

}  // namespace

struct SubbandPlan {
  std::vector<std::unique_ptr<SubRow>> rows;
  int64_t z_bytes = 0;  // largest chunk's sub-band series
};

namespace {

double group_dm(const gsp_segment &s, int32_t group, int32_t g) {
  const int32_t first = g * group;
  const int32_t n_g = s.n_dm - first < group ? s.n_dm - first : group;
  return s.dm_lo + ((double)first + (double)(n_g - 1) / 2.0) * s.dm_step;
}

double band_ref(const double *freqs, int32_t c0, int32_t c1) {
  double f = freqs[c0];
  for (int32_t c = c0 + 1; c < c1; ++c) f = freqs[c] > f ? freqs[c] : f;
  return f;
}

void check_subband_args(const gsp_dmt_desc *d, const int32_t *n_sub, const int32_t *group) {
  if (!n_sub || !group) fail(GSP_EINVAL, "null n_sub or group");
  for (int32_t s = 0; s < d->n_seg; ++s) {
    if (n_sub[s] < 1 || n_sub[s] > d->nchan) fail(GSP_EINVAL, "n_sub must be in [1, nchan]");
    if (group[s] < 1 || group[s] > 64) fail(GSP_EINVAL, "group must be in [1, 64]");
    const int64_t cpb = (d->nchan + n_sub[s] - 1) / n_sub[s];
    if (255 * (int64_t)d->seg[s].downsamp * cpb > 65535)
      fail(GSP_EINVAL, "255 * downsamp * (channels per band) must not exceed 65535 (16-bit sub-band series)");
  }
}

// Composite-delay extent of a row: the largest d2(i, b) + max_{c in b} d1(g(i), c).
int64_t composite_max(const gsp_segment &g, int32_t nchan, const double *freqs, double fref, double tsamp,
                      int32_t n_sub, int32_t group, std::vector<int32_t> *d1_out, std::vector<int32_t> *d2_out,
                      int64_t *max_d2) {
  const int32_t n_groups = (g.n_dm + group - 1) / group;
  std::vector<int32_t> c0(n_sub + 1);
  for (int32_t b = 0; b <= n_sub; ++b) c0[b] = (int32_t)((int64_t)b * nchan / n_sub);
  std::vector<double> fb(n_sub);
  for (int32_t b = 0; b < n_sub; ++b) fb[b] = band_ref(freqs, c0[b], c0[b + 1]);
  // d1 [n_groups][nchan], m1 [n_groups][n_sub]
  std::vector<int32_t> d1((size_t)n_groups * nchan);
  std::vector<int64_t> m1((size_t)n_groups * n_sub, 0);
  for (int32_t q = 0; q < n_groups; ++q) {
    const double dmg = group_dm(g, group, q);
    for (int32_t b = 0; b < n_sub; ++b)
      for (int32_t c = c0[b]; c < c0[b + 1]; ++c) {
        const int64_t v = delay_of(dmg, freqs[c], fb[b], tsamp, g.downsamp);
        if (v > std::numeric_limits<int32_t>::max()) fail(GSP_EOVERFLOW, "delay exceeds int32");
        d1[(size_t)q * nchan + c] = (int32_t)v;
        m1[(size_t)q * n_sub + b] = std::max<int64_t>(m1[(size_t)q * n_sub + b], v);
      }
  }
  std::vector<int32_t> d2((size_t)g.n_dm * n_sub);
  int64_t m = 0, md2 = 0;
  for (int32_t i = 0; i < g.n_dm; ++i) {
    const double dm = g.dm_lo + (double)i * g.dm_step;
    for (int32_t b = 0; b < n_sub; ++b) {
      const int64_t v = delay_of(dm, fb[b], fref, tsamp, g.downsamp);
      if (v > std::numeric_limits<int32_t>::max()) fail(GSP_EOVERFLOW, "delay exceeds int32");
      d2[(size_t)i * n_sub + b] = (int32_t)v;
      m = std::max<int64_t>(m, v + m1[(size_t)(i / group) * n_sub + b]);
      md2 = std::max<int64_t>(md2, v);
    }
  }
  if (d1_out) *d1_out = std::move(d1);
  if (d2_out) *d2_out = std::move(d2);
  if (max_d2) *max_d2 = md2;
  return m;
}

std::string sub_key(const gsp_dmt_desc *desc, const double *freqs, const int32_t *n_sub, const int32_t *group) {
  std::string k = plan_key(desc, freqs);
  k.append(reinterpret_cast<const char *>(n_sub), sizeof(int32_t) * (size_t)desc->n_seg);
  k.append(reinterpret_cast<const char *>(group), sizeof(int32_t) * (size_t)desc->n_seg);
  return k;
}

void upload_jobs(gsp_ctx *ctx, DevBuf &dst, const std::vector<SubJob> &jobs) {
  if ((int)jobs.size() > kSubMaxJobs) fail(GSP_ECAPACITY, "too many sub-band jobs in one launch");
  auto t = std::make_unique<SubTable>();
  std::memset(t.get(), 0, sizeof(SubTable));
  int64_t items = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    t->job[j] = jobs[j];
    t->job[j].item0 = items;
    items += (int64_t)jobs[j].a.n_dm_tiles * jobs[j].a.n_t_tiles;
  }
  t->n_jobs = (int32_t)jobs.size();
  t->n_items = items;
  dst.device = ctx->device;
  dst.reserve(sizeof(SubTable));
  check_hip(hipMemcpy(dst.ptr, t.get(), sizeof(SubTable), hipMemcpyHostToDevice), "copy sub-band jobs");
}

// Arguments of one tile job; Y and out are byte offsets from the launch's bases.
DedispArgs job_args(const RowTables &rt, int64_t src_off, int64_t pitch, int64_t dst_off, int64_t out_pitch,
                    int64_t n_out, int32_t flush) {
  DedispArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Y = reinterpret_cast<const void *>(static_cast<intptr_t>(src_off));
  a.pitch = pitch;
  a.addr = rt.addr.as<uint32_t>();
  a.base = rt.dmin.as<int32_t>();
  a.out = reinterpret_cast<void *>(static_cast<intptr_t>(dst_off));
  a.out_pitch = out_pitch;
  a.t_origin = 0;
  a.t_lo = 0;
  a.t_hi = n_out;
  a.ring = 0;
  a.phys0 = 0;
  a.n_dm = rt.n_dm;
  const int MT = rt.shape.trials_per_block();
  a.n_dm_tiles = (rt.n_dm + MT - 1) / MT;
  a.n_dm_pad = a.n_dm_tiles * MT;
  a.nchan = rt.nchan;
  a.chunks = rt.passes.as<int32_t>();
  a.n_chunks = rt.n_passes;
  a.max_chunk = rt.max_chunk;
  a.data_dw = rt.data_dw;
  a.flush = flush;
  const int64_t T = rt.shape.samples_per_block();
  a.n_t_tiles = (int32_t)((n_out + T - 1) / T);
  return a;
}

SubbandPlan &subband_plan(gsp_ctx *ctx, const gsp_dmt_desc *desc, const double *freqs, const int32_t *n_sub,
                          const int32_t *group) {
  const std::string key = sub_key(desc, freqs, n_sub, group);
  auto it = ctx->subband.find(key);
  if (it != ctx->subband.end()) return *it->second;
  auto P = std::make_shared<SubbandPlan>();
  const int32_t nchan = desc->nchan;
  for (int32_t s = 0; s < desc->n_seg; ++s) {
    const gsp_segment &g = desc->seg[s];
    auto R = std::make_unique<SubRow>();
    R->n_sub = n_sub[s];
    R->group = group[s];
    R->n_groups = (g.n_dm + group[s] - 1) / group[s];
    R->D = g.downsamp;
    R->n_dm = g.n_dm;
    R->N = desc->nsamp / g.downsamp;
    R->n_out = desc->n_out[s];
    R->c0.resize(R->n_sub + 1);
    for (int32_t b = 0; b <= R->n_sub; ++b) R->c0[b] = (int32_t)((int64_t)b * nchan / R->n_sub);
    for (int32_t b = 0; b < R->n_sub; ++b) R->cpb_max = std::max(R->cpb_max, R->c0[b + 1] - R->c0[b]);
    std::vector<int32_t> d1, d2;
    int64_t md2 = 0;
    const int64_t m = composite_max(g, nchan, freqs, desc->fref_mhz, desc->tsamp, R->n_sub, R->group, &d1, &d2, &md2);
    if (m != desc->max_delay[s]) fail(GSP_EINVAL, "descriptor was not shaped for this sub-band plan");
    // sub-band series needed by the valid outputs: t + d2 < n_out + max d2
    R->Zn = R->n_out + md2;
    // stage 2 tables (one per group): trials = the group's, channels = bands
    R->waves2 = std::min(8, std::max(1, (R->group + kSubTpw - 1) / kSubTpw));
    DedispShape sh2;
    sh2.groups = kSubK;
    sh2.tpw = kSubTpw;
    sh2.waves = R->waves2;
    sh2.chunk = 32;
    int64_t zp = R->Zn;
    for (int32_t q = 0; q < R->n_groups; ++q) {
      const int32_t i0 = q * R->group, i1 = std::min(g.n_dm, i0 + R->group);
      auto rt = std::make_unique<RowTables>();
      rt->delays_host.resize((size_t)(i1 - i0) * R->n_sub);
      int64_t mx = 0;
      for (int32_t i = i0; i < i1; ++i)
        for (int32_t b = 0; b < R->n_sub; ++b) {
          const int32_t v = d2[(size_t)i * R->n_sub + b];
          rt->delays_host[(size_t)(i - i0) * R->n_sub + b] = v;
          mx = std::max<int64_t>(mx, v);
        }
      // LDS for as many workgroups of waves2 waves as fill a CU's 16 wave slots
      build_tables_from_delays(ctx, i1 - i0, R->n_sub, g.downsamp, R->Zn, R->n_out, mx, sh2, *rt,
                               unit_max<uint16_t>(), (int64_t)160 * 1024 * R->waves2 / 16);
      zp = std::max(zp, staged_pitch(*rt));
      R->s2.push_back(std::move(rt));
    }
    R->Zpitch = (zp + 255) / 256 * 256;
    // stage 1 tables per (chunk of groups, band): trials = the chunk's groups
    DedispShape sh1;
    sh1.groups = kSubK;
    sh1.tpw = kSubTpw;
    sh1.waves = 8;
    sh1.chunk = 32;
    const int MT1 = sh1.trials_per_block();
    const int64_t per_group = (int64_t)R->n_sub * R->Zpitch * 2;
    int32_t gc = (int32_t)std::max<int64_t>(1, kZBudget / per_group);
    gc = std::max(MT1, std::min(gc, kSubMaxJobs) / MT1 * MT1);  // stage 2 has one job per group
    gc = std::min(gc, R->n_groups);
    int64_t pitch = R->N;
    for (int32_t ga = 0; ga < R->n_groups; ga += gc) {
      auto C = std::make_unique<SubChunk>();
      C->g0 = ga;
      C->g1 = std::min(R->n_groups, ga + gc);
      const int32_t ng = C->g1 - C->g0;
      if (nchan % R->n_sub == 0) {
        // equal bands: one job over every channel of the row, the sums of
        // each band stored as an output segment of its own
        const int32_t cpb = nchan / R->n_sub;
        auto rt = std::make_unique<RowTables>();
        rt->delays_host.resize((size_t)ng * nchan);
        int64_t mx = 0;
        for (int32_t q = 0; q < ng; ++q)
          for (int32_t c = 0; c < nchan; ++c) {
            const int32_t v = d1[(size_t)(C->g0 + q) * nchan + c];
            rt->delays_host[(size_t)q * nchan + c] = v;
            mx = std::max<int64_t>(mx, v);
          }
        build_tables_from_delays(ctx, ng, nchan, g.downsamp, R->N, R->Zn, mx, sh1, *rt, 0, 0, cpb);
        pitch = std::max(pitch, staged_pitch(*rt));
        C->s1.push_back(std::move(rt));
        R->chunks.push_back(std::move(C));
        continue;
      }
      for (int32_t b = 0; b < R->n_sub; ++b) {
        const int32_t cb = R->c0[b], ce = R->c0[b + 1];
        auto rt = std::make_unique<RowTables>();
        rt->delays_host.resize((size_t)ng * (ce - cb));
        int64_t mx = 0;
        for (int32_t q = 0; q < ng; ++q)
          for (int32_t c = cb; c < ce; ++c) {
            const int32_t v = d1[(size_t)(C->g0 + q) * nchan + c];
            rt->delays_host[(size_t)q * (ce - cb) + (c - cb)] = v;
            mx = std::max<int64_t>(mx, v);
          }
        build_tables_from_delays(ctx, ng, ce - cb, g.downsamp, R->N, R->Zn, mx, sh1, *rt, 0);
        pitch = std::max(pitch, staged_pitch(*rt));
        C->s1.push_back(std::move(rt));
      }
      R->chunks.push_back(std::move(C));
    }
    R->pitch = (pitch + 255) / 256 * 256;
    const size_t elem = g.downsamp == 1 ? 1 : 2;
    // job tables (offsets: source = staged row or sub-band series, destination = series or DM-time output)
    for (auto &Cp : R->chunks) {
      SubChunk &C = *Cp;
      std::vector<SubJob> j1, j2;
      if (C.s1.size() == 1 && R->n_sub > 1) {  // one segmented job over the row
        const RowTables &rt = *C.s1[0];
        SubJob J;
        J.a = job_args(rt, 0, R->pitch, 0, (int64_t)R->n_sub * R->Zpitch, R->Zn,
                       std::max(1, std::min(65535 / (255 * R->D), 256)));
        J.a.seg_ch = nchan / R->n_sub;
        J.a.seg_stride = R->Zpitch;
        C.seg = true;
        J.item0 = 0;
        j1.push_back(J);
        C.lds1 = std::max(C.lds1, rt.lds_bytes);
        C.adds1 += (double)rt.n_dm * (double)R->Zn * (double)rt.nchan;
      }
      for (int32_t b = 0; b < R->n_sub && !(C.s1.size() == 1 && R->n_sub > 1); ++b) {
        const RowTables &rt = *C.s1[b];
        SubJob J;
        J.a = job_args(rt, (int64_t)R->c0[b] * R->pitch * (int64_t)elem, R->pitch,
                       (int64_t)b * R->Zpitch * 2, (int64_t)R->n_sub * R->Zpitch, R->Zn,
                       std::max(1, std::min(65535 / (255 * R->D), 256)));
        J.item0 = 0;
        j1.push_back(J);
        C.lds1 = std::max(C.lds1, rt.lds_bytes);
        C.adds1 += (double)rt.n_dm * (double)R->Zn * (double)rt.nchan;
      }
      for (int32_t q = C.g0; q < C.g1; ++q) {
        const RowTables &rt = *R->s2[q];
        SubJob J;
        J.a = job_args(rt, (int64_t)(q - C.g0) * R->n_sub * R->Zpitch * 2, R->Zpitch,
                       (int64_t)((int64_t)q * R->group * R->n_out) * 4, R->n_out, R->n_out,
                       std::max(1, std::min(65535 / (255 * R->D * R->cpb_max), 256)));
        J.item0 = 0;
        j2.push_back(J);
        C.lds2 = std::max(C.lds2, rt.lds_bytes);
        C.adds2 += (double)rt.n_dm * (double)R->n_out * (double)rt.nchan;
      }
      upload_jobs(ctx, C.t1, j1);
      upload_jobs(ctx, C.t2, j2);
      P->z_bytes = std::max<int64_t>(P->z_bytes, (int64_t)(C.g1 - C.g0) * R->n_sub * R->Zpitch * 2);
    }
    P->rows.push_back(std::move(R));
  }
  auto &slot = ctx->subband[key];
  slot = P;
  return *slot;
}

template <typename SrcT, typename OutT, bool SEG = false>
void launch_sub(const DevBuf &table, int waves, int64_t lds, const void *src, void *dst, hipStream_t st) {
  auto kern = k_dedisp_sub<kSubK, kSubTpw, SrcT, OutT, SEG>;
  check_hip(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
            "set LDS size");
  hipLaunchKernelGGL(kern, dim3(256 * 2), dim3(64 * waves), (size_t)lds, st, table.as<SubTable>(),
                     static_cast<const char *>(src), static_cast<char *>(dst));
}

}  // namespace

void subband_plan_shape(int64_t nsamp, int32_t nchan, const double *freqs, double tsamp, const gsp_segment *segs,
                        int32_t n_seg, const int32_t *n_sub, const int32_t *group, gsp_dmt_desc *desc) {
  gsp_dmt_desc d;
  plan_shape_impl(nsamp, nchan, freqs, tsamp, segs, n_seg, &d);  // validation and the row fields
  check_subband_args(&d, n_sub, group);
  int64_t off = 0;
  for (int32_t s = 0; s < n_seg; ++s) {
    const int64_t m = composite_max(d.seg[s], nchan, freqs, d.fref_mhz, tsamp, n_sub[s], group[s], nullptr, nullptr,
                                    nullptr);
    d.max_delay[s] = m;
    d.n_out[s] = nsamp / d.seg[s].downsamp - m;
    if (d.n_out[s] < 1) fail(GSP_ETOOSHORT, "input shorter than a row's largest composite delay");
    d.offset[s] = off;
    off += (int64_t)d.seg[s].n_dm * d.n_out[s];
  }
  d.total = off;
  d.kind = 1;
  *desc = d;
}

void dedisperse_subband(gsp_ctx *ctx, const uint8_t *fb, const double *freqs, const gsp_dmt_desc *desc,
                        const int32_t *n_sub, const int32_t *group, int32_t *dmt, hipStream_t st) {
  check_subband_args(desc, n_sub, group);
  if (desc->kind != 1) fail(GSP_EINVAL, "descriptor is not a sub-band plan (gsp_subband_plan_shape)");
  SubbandPlan &P = subband_plan(ctx, desc, freqs, n_sub, group);
  ctx->zbuf.device = ctx->device;
  ctx->zbuf.reserve((size_t)P.z_bytes + 256);
  for (int32_t s = 0; s < desc->n_seg; ++s) {
    SubRow &R = *P.rows[s];
    RowTables stage;  // shape of the staged copy only
    stage.N = R.N;
    stage.D = R.D;
    stage.nchan = desc->nchan;
    stage_row(ctx, fb, desc, stage, st, R.pitch);
    char *out_row = reinterpret_cast<char *>(dmt + desc->offset[s]);
    for (auto &Cp : R.chunks) {
      SubChunk &C = *Cp;
      {
        ProfScope prof(ctx, "subband1", st, C.adds1);
        const bool seg = C.seg;  // one job over the row with band segments
        if (R.D == 1 && seg)
          launch_sub<uint8_t, uint16_t, true>(C.t1, 8, C.lds1, ctx->staged.ptr, ctx->zbuf.ptr, st);
        else if (R.D == 1)
          launch_sub<uint8_t, uint16_t>(C.t1, 8, C.lds1, ctx->staged.ptr, ctx->zbuf.ptr, st);
        else if (seg)
          launch_sub<uint16_t, uint16_t, true>(C.t1, 8, C.lds1, ctx->staged.ptr, ctx->zbuf.ptr, st);
        else
          launch_sub<uint16_t, uint16_t>(C.t1, 8, C.lds1, ctx->staged.ptr, ctx->zbuf.ptr, st);
      }
      {
        ProfScope prof(ctx, "subband2", st, C.adds2);
        launch_sub<uint16_t, int32_t>(C.t2, R.waves2, C.lds2, ctx->zbuf.ptr, out_row, st);
      }
      check_hip(hipGetLastError(), "launch sub-band kernels");
    }
  }
}

}  // namespace gsp

using namespace gsp;

extern "C" {

int gsp_subband_plan_shape(int64_t nsamp, int32_t nchan, const double *freqs_mhz, double tsamp_s,
                           const gsp_segment *segs, int32_t n_seg, const int32_t *n_sub, const int32_t *group,
                           gsp_dmt_desc *desc) {
  return guarded(nullptr,
                 [&] { subband_plan_shape(nsamp, nchan, freqs_mhz, tsamp_s, segs, n_seg, n_sub, group, desc); });
}

int gsp_dedisperse_subband(gsp_ctx *ctx, const uint8_t *fb_dev, const double *freqs_mhz, const gsp_dmt_desc *desc,
                           const int32_t *n_sub, const int32_t *group, int32_t *dmt_dev, void *stream) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    validate_desc(desc);
    if (!fb_dev || !freqs_mhz || !dmt_dev) fail(GSP_EINVAL, "null pointer argument");
    dedisperse_subband(ctx, fb_dev, freqs_mhz, desc, n_sub, group, dmt_dev, static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
