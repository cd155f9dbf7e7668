// Candidate sifting and the candidate store (host side).
//
// The paper sifts single-pulse events with RRATtrap (Section 2.2: events of
// nearby DMs and times grouped, groups ranked and scored by rules; Section
// 3.2: ranks 3 to 6 with 6 the best, and a class of RFI or noise) and
// archives the results in a database of six tables (Section 2.2:
// T_FITS_INFO, T_SINGLEPULSE_GROUPS, T_SINGLEPULSE_CANDIDATES, T_PULSAR,
// T_FILE_PULSAR, T_SINGLEPULSE_PIC).  Neither the rules nor the schema's
// columns are printed; the ranking rules are the reading documented in
// gsp.h, and the store keeps the named tables with the columns the text
// lists, in memory, saved to and loaded from one CSV file per table.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <set>
#include <sstream>

#include "gsp_internal.h"

namespace gsp {
namespace {

constexpr double kRfiDm = 1.0;
constexpr double kFall[3] = {0.1, 0.2, 0.35};

}  // namespace
}  // namespace gsp

struct gsp_store {
  struct File {
    int64_t id;
    std::string name;
    int32_t beam, nchan;
    int64_t nsamp;
    double tsamp, f_lo, f_hi;
  };
  struct Summary {  // T_SINGLEPULSE_GROUPS: one row per file
    int64_t file_id, n_candidates, n_groups;
    int64_t per_rank[7];
  };
  struct Pulsar {
    int64_t id;
    std::string name;
    double dm;
  };
  struct Match {
    int64_t file_id, pulsar_id, n_groups;
    double best_snr;
  };
  struct Pic {
    int64_t cand_id;
    std::string path;
  };
  std::vector<File> files;
  std::vector<Summary> summaries;
  std::vector<gsp_store_candidate> cands;
  std::vector<Pulsar> pulsars;
  std::vector<Match> matches;
  std::vector<Pic> pics;
  std::string last_error;
};

using namespace gsp;

namespace {

template <class F>
int stguard(gsp_store *s, F &&f) {
  try {
    f();
    if (s) s->last_error.clear();
    return GSP_OK;
  } catch (const Error &e) {
    if (s) s->last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    if (s) s->last_error = "host allocation failed";
    return GSP_ENOMEM;
  } catch (...) {
    if (s) s->last_error = "unexpected internal error";
    return GSP_EDEVICE;
  }
}

bool plain_name(const char *p) {
  if (!p) return false;
  for (const char *q = p; *q; ++q)
    if (*q == ',' || *q == '\n' || *q == '\r' || *q == '"') return false;
  return true;
}

std::string path_join(const char *dir, const char *file) {
  std::string d(dir);
  if (!d.empty() && d.back() != '/') d += '/';
  return d + file;
}

std::vector<std::vector<std::string>> read_csv(const std::string &path) {
  std::ifstream f(path);
  if (!f) fail(GSP_EINVAL, "cannot read " + path);
  std::vector<std::vector<std::string>> rows;
  std::string line;
  bool header = true;
  while (std::getline(f, line)) {
    if (header) {
      header = false;
      continue;
    }
    if (line.empty()) continue;
    std::vector<std::string> cols;
    std::stringstream ss(line);
    std::string c;
    while (std::getline(ss, c, ',')) cols.push_back(c);
    if (!line.empty() && line.back() == ',') cols.push_back("");
    rows.push_back(cols);
  }
  return rows;
}

}  // namespace

extern "C" {

int gsp_rank_groups(const gsp_candidate *c, int64_t n, const int64_t *rep, const gsp_dmt_desc *desc,
                    gsp_group_record *out, int64_t cap, int64_t *n_groups) {
  return guarded(nullptr, [&] {
    if (n < 0 || (n > 0 && (!c || !rep)) || !n_groups || cap < 0 || (cap > 0 && !out))
      fail(GSP_EINVAL, "null pointer or negative count");
    validate_desc(desc);
    // members of each group, groups in order of their representative
    std::map<int64_t, std::vector<int64_t>> groups;
    for (int64_t k = 0; k < n; ++k) {
      if (rep[k] < 0 || rep[k] >= n || rep[rep[k]] != rep[k]) fail(GSP_EINVAL, "rep is not a grouping");
      groups[rep[k]].push_back(k);
    }
    int64_t g = 0;
    for (const auto &kv : groups) {
      const gsp_candidate &p = c[kv.first];
      if (p.seg < 0 || p.seg >= desc->n_seg) fail(GSP_EINVAL, "candidate row outside the plan");
      const double Dt = (double)desc->seg[p.seg].downsamp * desc->tsamp;
      gsp_group_record r;
      std::memset(&r, 0, sizeof(r));
      r.rep = kv.first;
      r.seg = p.seg;
      std::set<std::pair<int32_t, int32_t>> trials;
      double dmin = INFINITY, dmax = -INFINITY, start = INFINITY, end = -INFINITY;
      for (int64_t k : kv.second) {
        const gsp_candidate &m = c[k];
        trials.insert({m.seg, m.dm_index});
        dmin = std::min(dmin, m.dm);
        dmax = std::max(dmax, m.dm);
        start = std::min(start, (double)(m.t_first - m.width + 1) * Dt);
        end = std::max(end, (double)(m.t_last + 1) * Dt);
      }
      float lo = -INFINITY, hi = -INFINITY;
      for (int64_t k : kv.second) {
        if (c[k].dm == dmin) lo = std::max(lo, c[k].snr);
        if (c[k].dm == dmax) hi = std::max(hi, c[k].snr);
      }
      r.n_events = (int32_t)kv.second.size();
      r.n_trials = (int32_t)trials.size();
      r.dm_min = dmin;
      r.dm_max = dmax;
      r.dm_peak = p.dm;
      r.snr_max = p.snr;
      r.snr_lo = lo;
      r.snr_hi = hi;
      r.time_s = p.time_s;
      r.width_s = (double)p.width * Dt;
      r.start_s = start;
      r.duration_s = end - start;
      if (p.dm < kRfiDm) {
        r.rank = 2;
      } else if (r.n_trials < 3) {
        r.rank = 1;
      } else {
        const double f = std::min(1.0 - (double)lo / (double)p.snr, 1.0 - (double)hi / (double)p.snr);
        r.rank = f < kFall[0] ? 3 : (f < kFall[1] ? 4 : (f < kFall[2] ? 5 : 6));
      }
      if (g < cap) out[g] = r;
      ++g;
    }
    *n_groups = g;
    if (g > cap) fail(GSP_ECAPACITY, "group capacity too small; *n_groups holds the count");
  });
}

int gsp_store_create(gsp_store **out) {
  if (!out) return GSP_EINVAL;
  *out = nullptr;
  try {
    *out = new gsp_store();
    return GSP_OK;
  } catch (...) {
    return GSP_ENOMEM;
  }
}

void gsp_store_destroy(gsp_store *s) { delete s; }

const char *gsp_store_last_error(const gsp_store *s) { return s ? s->last_error.c_str() : ""; }

int gsp_store_add_file(gsp_store *s, const char *name, int32_t beam, int32_t nchan, int64_t nsamp, double tsamp,
                       double f_lo, double f_hi, int64_t *file_id) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (!plain_name(name) || !file_id || nchan < 1 || nsamp < 1 || !(tsamp > 0))
      fail(GSP_EINVAL, "bad file record (names must not hold commas, quotes or line breaks)");
    const int64_t id = (int64_t)s->files.size() + 1;
    s->files.push_back({id, name, beam, nchan, nsamp, tsamp, f_lo, f_hi});
    *file_id = id;
  });
}

int gsp_store_add_groups(gsp_store *s, int64_t file_id, int64_t n_candidates, const gsp_group_record *g, int64_t n,
                         int64_t *first_id) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (file_id < 1 || file_id > (int64_t)s->files.size()) fail(GSP_EINVAL, "unknown file");
    if (n < 0 || (n > 0 && !g) || n_candidates < 0) fail(GSP_EINVAL, "bad group records");
    for (const auto &m : s->summaries)
      if (m.file_id == file_id) fail(GSP_EINVAL, "the file's groups are already stored");
    gsp_store::Summary m;
    std::memset(&m, 0, sizeof(m));
    m.file_id = file_id;
    m.n_candidates = n_candidates;
    m.n_groups = n;
    const int64_t first = (int64_t)s->cands.size() + 1;
    for (int64_t k = 0; k < n; ++k) {
      if (g[k].rank < 1 || g[k].rank > 6) fail(GSP_EINVAL, "rank outside 1..6");
      gsp_store_candidate c;
      std::memset(&c, 0, sizeof(c));
      c.id = first + k;
      c.file_id = file_id;
      c.g = g[k];
      s->cands.push_back(c);
      m.per_rank[g[k].rank] += 1;
    }
    s->summaries.push_back(m);
    if (first_id) *first_id = first;
  });
}

int gsp_store_add_pulsar(gsp_store *s, const char *name, double dm, int64_t *pulsar_id) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (!plain_name(name) || !pulsar_id || !(dm >= 0) || !std::isfinite(dm)) fail(GSP_EINVAL, "bad pulsar record");
    const int64_t id = (int64_t)s->pulsars.size() + 1;
    s->pulsars.push_back({id, name, dm});
    *pulsar_id = id;
  });
}

int gsp_store_match_pulsars(gsp_store *s, int64_t file_id, double dm_tol, int32_t min_rank, int64_t *n_matches) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (file_id < 1 || file_id > (int64_t)s->files.size()) fail(GSP_EINVAL, "unknown file");
    if (!(dm_tol >= 0) || !n_matches) fail(GSP_EINVAL, "bad tolerance");
    s->matches.erase(std::remove_if(s->matches.begin(), s->matches.end(),
                                    [&](const gsp_store::Match &m) { return m.file_id == file_id; }),
                     s->matches.end());
    int64_t k = 0;
    for (const auto &p : s->pulsars) {
      gsp_store::Match m{file_id, p.id, 0, 0.0};
      for (const auto &c : s->cands)
        if (c.file_id == file_id && c.g.rank >= min_rank && std::fabs(c.g.dm_peak - p.dm) <= dm_tol) {
          m.n_groups += 1;
          m.best_snr = std::max(m.best_snr, (double)c.g.snr_max);
        }
      if (m.n_groups) {
        s->matches.push_back(m);
        ++k;
      }
    }
    *n_matches = k;
  });
}

int gsp_store_add_picture(gsp_store *s, int64_t cand_id, const char *path) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (cand_id < 1 || cand_id > (int64_t)s->cands.size()) fail(GSP_EINVAL, "unknown candidate");
    if (!plain_name(path)) fail(GSP_EINVAL, "bad picture path");
    s->pics.push_back({cand_id, path});
  });
}

int gsp_store_query(gsp_store *s, int32_t min_rank, double dm_lo, double dm_hi, gsp_store_candidate *out,
                    int64_t cap, int64_t *n) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (!n || cap < 0 || (cap > 0 && !out)) fail(GSP_EINVAL, "bad output buffer");
    int64_t k = 0;
    for (const auto &c : s->cands)
      if (c.g.rank >= min_rank && c.g.dm_peak >= dm_lo && c.g.dm_peak <= dm_hi) {
        if (k < cap) out[k] = c;
        ++k;
      }
    *n = k;
    if (k > cap) fail(GSP_ECAPACITY, "capacity too small; *n holds the count");
  });
}

int gsp_store_count(const gsp_store *s, int32_t table, int64_t *n) {
  if (!s || !n) return GSP_EINVAL;
  switch (table) {
    case GSP_T_FITS_INFO: *n = (int64_t)s->files.size(); break;
    case GSP_T_SINGLEPULSE_GROUPS: *n = (int64_t)s->summaries.size(); break;
    case GSP_T_SINGLEPULSE_CANDIDATES: *n = (int64_t)s->cands.size(); break;
    case GSP_T_PULSAR: *n = (int64_t)s->pulsars.size(); break;
    case GSP_T_FILE_PULSAR: *n = (int64_t)s->matches.size(); break;
    case GSP_T_SINGLEPULSE_PIC: *n = (int64_t)s->pics.size(); break;
    default: return GSP_EINVAL;
  }
  return GSP_OK;
}

int gsp_store_save(gsp_store *s, const char *dir) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (!dir) fail(GSP_EINVAL, "null directory");
    auto open = [&](const char *name) {
      std::ofstream f(path_join(dir, name));
      if (!f) fail(GSP_EINVAL, std::string("cannot write ") + name);
      f.precision(17);
      return f;
    };
    {
      auto f = open("T_FITS_INFO.csv");
      f << "id,name,beam,nchan,nsamp,tsamp_s,f_lo_mhz,f_hi_mhz\n";
      for (const auto &r : s->files)
        f << r.id << ',' << r.name << ',' << r.beam << ',' << r.nchan << ',' << r.nsamp << ',' << r.tsamp << ','
          << r.f_lo << ',' << r.f_hi << '\n';
    }
    {
      auto f = open("T_SINGLEPULSE_GROUPS.csv");
      f << "file_id,n_candidates,n_groups,rank1,rank2,rank3,rank4,rank5,rank6\n";
      for (const auto &m : s->summaries) {
        f << m.file_id << ',' << m.n_candidates << ',' << m.n_groups;
        for (int r = 1; r <= 6; ++r) f << ',' << m.per_rank[r];
        f << '\n';
      }
    }
    {
      auto f = open("T_SINGLEPULSE_CANDIDATES.csv");
      f << "id,file_id,rep,seg,rank,n_events,n_trials,dm_min,dm_max,dm_peak,snr_max,snr_lo,snr_hi,time_s,width_s,"
           "start_s,duration_s\n";
      for (const auto &c : s->cands) {
        const gsp_group_record &g = c.g;
        f << c.id << ',' << c.file_id << ',' << g.rep << ',' << g.seg << ',' << g.rank << ',' << g.n_events << ','
          << g.n_trials << ',' << g.dm_min << ',' << g.dm_max << ',' << g.dm_peak << ',' << g.snr_max << ','
          << g.snr_lo << ',' << g.snr_hi << ',' << g.time_s << ',' << g.width_s << ',' << g.start_s << ','
          << g.duration_s << '\n';
      }
    }
    {
      auto f = open("T_PULSAR.csv");
      f << "id,name,dm\n";
      for (const auto &p : s->pulsars) f << p.id << ',' << p.name << ',' << p.dm << '\n';
    }
    {
      auto f = open("T_FILE_PULSAR.csv");
      f << "file_id,pulsar_id,n_groups,best_snr\n";
      for (const auto &m : s->matches) f << m.file_id << ',' << m.pulsar_id << ',' << m.n_groups << ',' << m.best_snr << '\n';
    }
    {
      auto f = open("T_SINGLEPULSE_PIC.csv");
      f << "cand_id,path\n";
      for (const auto &p : s->pics) f << p.cand_id << ',' << p.path << '\n';
    }
  });
}

int gsp_store_load(gsp_store *s, const char *dir) {
  if (!s) return GSP_EINVAL;
  return stguard(s, [&] {
    if (!dir) fail(GSP_EINVAL, "null directory");
    gsp_store t;
    auto need = [&](const std::vector<std::string> &r, size_t k) {
      if (r.size() != k) fail(GSP_EINVAL, "malformed store table");
    };
    for (auto &r : read_csv(path_join(dir, "T_FITS_INFO.csv"))) {
      need(r, 8);
      t.files.push_back({std::stoll(r[0]), r[1], std::stoi(r[2]), std::stoi(r[3]), std::stoll(r[4]), std::stod(r[5]),
                         std::stod(r[6]), std::stod(r[7])});
    }
    for (auto &r : read_csv(path_join(dir, "T_SINGLEPULSE_GROUPS.csv"))) {
      need(r, 9);
      gsp_store::Summary m;
      std::memset(&m, 0, sizeof(m));
      m.file_id = std::stoll(r[0]);
      m.n_candidates = std::stoll(r[1]);
      m.n_groups = std::stoll(r[2]);
      for (int k = 1; k <= 6; ++k) m.per_rank[k] = std::stoll(r[2 + k]);
      t.summaries.push_back(m);
    }
    for (auto &r : read_csv(path_join(dir, "T_SINGLEPULSE_CANDIDATES.csv"))) {
      need(r, 17);
      gsp_store_candidate c;
      std::memset(&c, 0, sizeof(c));
      c.id = std::stoll(r[0]);
      c.file_id = std::stoll(r[1]);
      gsp_group_record &g = c.g;
      g.rep = std::stoll(r[2]);
      g.seg = std::stoi(r[3]);
      g.rank = std::stoi(r[4]);
      g.n_events = std::stoi(r[5]);
      g.n_trials = std::stoi(r[6]);
      g.dm_min = std::stod(r[7]);
      g.dm_max = std::stod(r[8]);
      g.dm_peak = std::stod(r[9]);
      g.snr_max = std::stof(r[10]);
      g.snr_lo = std::stof(r[11]);
      g.snr_hi = std::stof(r[12]);
      g.time_s = std::stod(r[13]);
      g.width_s = std::stod(r[14]);
      g.start_s = std::stod(r[15]);
      g.duration_s = std::stod(r[16]);
      t.cands.push_back(c);
    }
    for (auto &r : read_csv(path_join(dir, "T_PULSAR.csv"))) {
      need(r, 3);
      t.pulsars.push_back({std::stoll(r[0]), r[1], std::stod(r[2])});
    }
    for (auto &r : read_csv(path_join(dir, "T_FILE_PULSAR.csv"))) {
      need(r, 4);
      t.matches.push_back({std::stoll(r[0]), std::stoll(r[1]), std::stoll(r[2]), std::stod(r[3])});
    }
    for (auto &r : read_csv(path_join(dir, "T_SINGLEPULSE_PIC.csv"))) {
      need(r, 2);
      t.pics.push_back({std::stoll(r[0]), r[1]});
    }
    s->files = std::move(t.files);
    s->summaries = std::move(t.summaries);
    s->cands = std::move(t.cands);
    s->pulsars = std::move(t.pulsars);
    s->matches = std::move(t.matches);
    s->pics = std::move(t.pics);
  });
}

}  // extern "C"
