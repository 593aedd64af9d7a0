// Autotuner of the self-join: picks the compiled tile variant (queries per
// tile x corpus rows per accumulator block), the width of the corpus ranges
// and the number of ranges that one of the persistent kernel's work items
// visits, by timing the join kernel on the index itself, and remembers the
// choice in a small JSON file keyed by device architecture and workload class.
//
// Cache file: one JSON object with one entry per line,
//   "gfx950|join|n=2^20|m=2^20|nnz=2^7|t=0.70": {"variant": 1, "range_rows": 8192, "range_group": 1, "ms": 3741.5},
// written whole (temporary file + rename) after each tuning; entries without
// "range_group" mean 1.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <map>
#include <string>

#include "join.h"
#include "lib.h"

using namespace apss;

namespace {

struct Choice {
  int variant = 1;
  long long range_rows = 8192;
  int range_group = 1;
  double ms = 0.0;
};

std::string arch_name(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

int log2_bucket(double x) { return x < 1.0 ? 0 : (int)lround(log2(x)); }

std::string tune_key(const apss_index* ix, float t) {
  char buf[256];
  const double per_row = ix->n > 0 ? (double)ix->nnz / (double)ix->n : 0.0;
  snprintf(buf, sizeof(buf), "%s|%s|n=2^%d|m=2^%d|nnz=2^%d|t=%.2f", arch_name(ix->device).c_str(),
           ix->screen ? "screened" : "join", log2_bucket((double)ix->n), log2_bucket((double)ix->m),
           log2_bucket(per_row), (double)t);
  if (ix->screen) {
    const size_t l = strlen(buf);
    snprintf(buf + l, sizeof(buf) - l, "|head=%d", ix->screen->head_cut);
  }
  // the variants of the algorithm are tuned apart from the default join
  if (ix->opts.index_all) strncat(buf, "|index_all", sizeof(buf) - strlen(buf) - 1);
  if (ix->opts.local_parts > 1) {
    const size_t l = strlen(buf);
    snprintf(buf + l, sizeof(buf) - l, "|local=%d", ix->opts.local_parts);
  }
  if (ix->opts.remscore) strncat(buf, "|remscore", sizeof(buf) - strlen(buf) - 1);
  return buf;
}

std::map<std::string, Choice> read_cache(const char* path) {
  std::map<std::string, Choice> m;
  FILE* f = fopen(path, "r");
  if (!f) return m;
  char line[1024];
  while (fgets(line, sizeof(line), f)) {
    char key[512];
    Choice c;
    if (sscanf(line, " \"%511[^\"]\": {\"variant\": %d, \"range_rows\": %lld, \"range_group\": %d, \"ms\": %lf}",
               key, &c.variant, &c.range_rows, &c.range_group, &c.ms) == 5 ||
        sscanf(line, " \"%511[^\"]\": {\"variant\": %d, \"range_rows\": %lld, \"ms\": %lf}", key, &c.variant,
               &c.range_rows, &c.ms) == 4)
      m[key] = c;
  }
  fclose(f);
  return m;
}

bool write_cache(const char* path, const std::map<std::string, Choice>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : m) {
    fprintf(f, " \"%s\": {\"variant\": %d, \"range_rows\": %lld, \"range_group\": %d, \"ms\": %.3f}%s\n",
            kv.first.c_str(), kv.second.variant, kv.second.range_rows, kv.second.range_group, kv.second.ms,
            ++k < m.size() ? "," : "");
  }
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path) == 0;
}

// Kernel time of one self-join under (variant, range rows, ranges per item)
// on the index that the join kernel runs on (the head-cut index for the
// screened join).
int time_config(apss_index* ix, apss_index* target, float t, int variant, long long rr, int rg, double* ms) {
  target->variant = variant;
  target->range_rows = rr;
  target->range_group = rg;
  int64_t cnt = 0;
  int rc = ix->screen ? run_screen_join(ix, ix->ws, t, 16 * ix->n, &cnt)
                      : run_join(ix, ix->ws,
                                 QuerySet{ix->rows.rp.p, ix->rows.rc.p, ix->rows.mw.p, ix->n, ix->nnz,
                                          ix->rows.rp_host.data()},
                                 1, t, nullptr, 16 * ix->n, &cnt);
  if (rc) return rc;
  *ms = ix->ws.last.ms_candidates;
  return APSS_OK;
}

}  // namespace

extern "C" int apss_autotune(apss_index* ix, float t, double budget_ms, const char* cache_path, apss_tune_result* out) {
  if (!ix || !out) {
    set_error("NULL argument");
    return APSS_EINVAL;
  }
  memset(out, 0, sizeof(*out));
  int rc = check_t(ix, t);
  if (rc) return rc;
  apss_index* target = ix->screen ? ix->screen : ix;
  const std::string key = tune_key(ix, t);
  std::map<std::string, Choice> cache;
  if (cache_path && *cache_path) {
    cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end() && it->second.variant >= 0 && it->second.variant < join_num_variants() &&
        variant_available(it->second.variant) && it->second.range_rows > 0 && it->second.range_group >= 1 &&
        it->second.range_group <= kMaxRangeGroup) {
      target->variant = it->second.variant;
      target->range_rows = it->second.range_rows;
      target->range_group = it->second.range_group;
      // the chosen geometry's tables exist before the next join, which then
      // allocates none of them
      if ((rc = prepare(target, ix->ws.stream, target->variant, target->range_rows))) return rc;
      out->variant = it->second.variant;
      out->range_rows = (int32_t)it->second.range_rows;
      out->range_group = it->second.range_group;
      out->ms = it->second.ms;
      out->from_cache = 1;
      return APSS_OK;
    }
  }
  const int v0 = target->variant;
  const long long r0 = target->range_rows;
  const int g0 = target->range_group;
  auto restore = [&]() {
    target->variant = v0;
    target->range_rows = r0;
    target->range_group = g0;
  };
  Choice best;
  best.variant = v0;
  best.range_rows = r0;
  best.range_group = g0;
  best.ms = INFINITY;
  const auto start = std::chrono::steady_clock::now();
  // the current configuration first, so that a small budget still gives a valid choice
  const long long ranges[] = {8192, 16384, 4096, 2048};
  int tried = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int v = 0; v < join_num_variants(); ++v) {
      for (long long rr : ranges) {
        const bool current = v == v0 && rr == r0;
        if ((pass == 0) != current) continue;
        int qt = 0, cb = 0;
        (void)join_variant_geometry(v, &qt, &cb);
        if (rr < cb) continue;
        if (!variant_available(v)) continue;
        const double spent =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - start).count();
        if (tried > 0 && budget_ms > 0.0 && spent >= budget_ms) continue;
        double ms = 0.0;
        // the current configuration with its own ranges per item, the others with one
        const int rg = current ? g0 : 1;
        if ((rc = time_config(ix, target, t, v, rr, rg, &ms))) {
          restore();
          return rc;
        }
        ++tried;
        if (ms < best.ms) {
          best.variant = v;
          best.range_rows = rr;
          best.range_group = rg;
          best.ms = ms;
        }
      }
    }
  }
  // then the ranges per item of the best geometry (an item stages its tile
  // once for all of them)
  const Choice geo = best;
  for (int rg : {1, 2, 4, 8}) {
    if (rg == geo.range_group) continue;
    const double spent = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - start).count();
    if (budget_ms > 0.0 && spent >= budget_ms) break;
    double ms = 0.0;
    if ((rc = time_config(ix, target, t, geo.variant, geo.range_rows, rg, &ms))) {
      restore();
      return rc;
    }
    ++tried;
    if (ms < best.ms) {
      best = geo;
      best.range_group = rg;
      best.ms = ms;
    }
  }
  target->variant = best.variant;
  target->range_rows = best.range_rows;
  target->range_group = best.range_group;
  if ((rc = prepare(target, ix->ws.stream, target->variant, target->range_rows))) return rc;
  out->variant = best.variant;
  out->range_rows = (int32_t)best.range_rows;
  out->range_group = best.range_group;
  out->ms = best.ms;
  out->tried = tried;
  if (cache_path && *cache_path) {
    cache[key] = best;
    if (!write_cache(cache_path, cache)) out->cache_write_failed = 1;
  }
  return APSS_OK;
}
