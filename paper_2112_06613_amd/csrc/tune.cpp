// Autotuner of the pair-kernel schedule (texts per work item, resident waves,
// pattern masks in VGPRs or LDS, one or two patterns per lane) for plain and
// batched launches, and its persisted table.
//
// Every candidate gives the same edges and degrees; only speed differs.  A
// candidate's time is the device time of the whole launch sequence (events
// around all device work), the fastest of two runs.  Choices are kept per
// context under (form, size class = bits of the sequence count, k) and can be
// saved to / loaded from a JSON file whose entries also carry the device's
// arch name and CU count (entries of another device are ignored on load).
#define TCRNET_BUILDING 1
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace tcr;

namespace {

const uint32_t kTs[] = {256, 512, 1024, 2048, 4096, 8192, 16384};
const uint32_t kWs[] = {4, 6, 8};

struct Candidate {
  Sched s;
  double ms = 1e30;
};

std::vector<Candidate> candidates(const tcrnet_opts& o) {
  std::vector<Candidate> out;
  for (uint32_t T : kTs)
    for (uint32_t W : kWs)
      for (int lds = 0; lds < 2; ++lds)
        for (int pack = 1; pack >= 0; --pack) {
          if ((o.flags & TCRNET_F_NO_PACK) && pack) continue;
          Candidate c;
          c.s.texts_per_item = T;
          c.s.waves_per_simd = W;
          c.s.peq_lds = lds != 0;
          c.s.pack = pack != 0;
          out.push_back(c);
        }
  return out;
}

// Options that force exactly schedule s on a run_pipeline call.
tcrnet_opts forcing(const tcrnet_opts& base, const Sched& s) {
  tcrnet_opts o = base;
  o.flags = (base.flags | TCRNET_F_NO_AUTOTUNE) & ~(TCRNET_F_PEQ_LDS | TCRNET_F_PEQ_VGPR | TCRNET_F_NO_PACK);
  o.flags |= s.peq_lds ? TCRNET_F_PEQ_LDS : TCRNET_F_PEQ_VGPR;
  if (!s.pack) o.flags |= TCRNET_F_NO_PACK;
  o.texts_per_item = s.texts_per_item;
  o.waves_per_simd = s.waves_per_simd;
  return o;
}

void remember(tcrnet_ctx* ctx, int form, uint64_t n, int k, const Candidate& best) {
  TuneKey key;
  key.form = form;
  key.size_class = (int)bits_for(n ? n : 1);
  key.k = k;
  TuneEntry e;
  e.sched = best.s;
  e.sched.tuned = false;
  e.ms = best.ms;
  ctx->tuned[key] = e;
}

const char* form_name(int form) { return form == kFormBatch ? "batch" : "plain"; }

// Minimal reader of the flat JSON this file writes: the objects of the
// "entries" array, each with string or number values.
struct Obj {
  std::vector<std::pair<std::string, std::string>> kv;
  const std::string* get(const char* k) const {
    for (auto& p : kv)
      if (p.first == k) return &p.second;
    return nullptr;
  }
};

bool parse_entries(const std::string& txt, std::vector<Obj>* out) {
  size_t i = txt.find("\"entries\"");
  if (i == std::string::npos) return false;
  i = txt.find('[', i);
  if (i == std::string::npos) return false;
  ++i;
  auto skip = [&]() {
    while (i < txt.size() && (txt[i] == ' ' || txt[i] == '\n' || txt[i] == '\t' || txt[i] == '\r' || txt[i] == ','))
      ++i;
  };
  for (;;) {
    skip();
    if (i >= txt.size()) return false;
    if (txt[i] == ']') return true;
    if (txt[i] != '{') return false;
    ++i;
    Obj o;
    for (;;) {
      skip();
      if (i >= txt.size()) return false;
      if (txt[i] == '}') {
        ++i;
        break;
      }
      if (txt[i] != '"') return false;
      const size_t ke = txt.find('"', i + 1);
      if (ke == std::string::npos) return false;
      std::string key = txt.substr(i + 1, ke - i - 1);
      i = txt.find(':', ke);
      if (i == std::string::npos) return false;
      ++i;
      skip();
      std::string val;
      if (i < txt.size() && txt[i] == '"') {
        const size_t ve = txt.find('"', i + 1);
        if (ve == std::string::npos) return false;
        val = txt.substr(i + 1, ve - i - 1);
        i = ve + 1;
      } else {
        const size_t b = i;
        while (i < txt.size() && txt[i] != ',' && txt[i] != '}' && txt[i] != '\n') ++i;
        val = txt.substr(b, i - b);
        while (!val.empty() && val.back() == ' ') val.pop_back();
      }
      o.kv.emplace_back(key, val);
    }
    out->push_back(o);
  }
}

bool to_u32(const std::string* s, uint32_t* v) {
  if (!s || s->empty()) return false;
  char* end = nullptr;
  errno = 0;
  const unsigned long long x = strtoull(s->c_str(), &end, 10);
  if (errno || *end || x > 0xFFFFFFFFull) return false;
  *v = (uint32_t)x;
  return true;
}

}  // namespace

extern "C" {

int32_t tcrnet_autotune(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k) {
  if (!ctx) return set_error(TCRNET_EINVAL, "NULL context");
  int32_t rc;
  if ((rc = check_k(k)) || (rc = check_host_seqs(seqs, "tcrnet_autotune"))) return rc;
  if (seqs->n < 2) return TCRNET_OK;
  (void)hipSetDevice(ctx->device);
  const uint32_t n = seqs->n;
  const uint64_t base = seqs->offsets[0];
  const uint64_t bytes = seqs->offsets[n] - base;
  std::vector<uint64_t> off(n + 1);
  for (uint32_t i = 0; i <= n; ++i) off[i] = seqs->offsets[i] - base;
  hipError_t e;
  if ((e = ctx->in_data.ensure(bytes ? bytes : 1)) != hipSuccess) return hip_error(e, "input allocation");
  if ((e = ctx->in_off.ensure((uint64_t)(n + 1) * 8)) != hipSuccess) return hip_error(e, "input allocation");
  if ((e = ctx->out_deg.ensure((uint64_t)n * 4)) != hipSuccess) return hip_error(e, "output allocation");
  if (bytes && (e = hipMemcpyAsync(ctx->in_data.p, seqs->data + base, bytes, hipMemcpyHostToDevice, ctx->stream)) !=
                   hipSuccess)
    return hip_error(e, "input copy");
  if ((e = hipMemcpyAsync(ctx->in_off.p, off.data(), (uint64_t)(n + 1) * 8, hipMemcpyHostToDevice, ctx->stream)) !=
      hipSuccess)
    return hip_error(e, "input copy");
  const tcrnet_opts saved = ctx->opts;
  std::vector<Candidate> cands = candidates(saved);
  Candidate best;
  uint64_t E_ref = ~0ull;
  for (Candidate& c : cands) {
    ctx->opts = forcing(saved, c.s);
    for (int rep = 0; rep < 2; ++rep) {
      PipeParams pp;
      pp.d_data = ctx->in_data.as<char>();
      pp.d_off = ctx->in_off.as<uint64_t>();
      pp.n = n;
      pp.k = k;
      pp.capacity = saved.edge_capacity ? saved.edge_capacity : std::max<uint64_t>(65536, 4ull * n);
      pp.d_deg = ctx->out_deg.as<int32_t>();
      uint64_t E = 0;
      tcrnet_build_info info{};
      rc = run_pipeline(ctx, ctx->pipe, pp, ctx->stream, true, &ctx->out_pairs, &E, &info);
      if (rc) {
        ctx->opts = saved;
        return rc;
      }
      if (E_ref == ~0ull) E_ref = E;
      if (E != E_ref) {
        ctx->opts = saved;
        return set_error(TCRNET_EDEVICE, "autotune: schedules gave different edge counts (internal)");
      }
      const double t = info.build_ms / (info.pair_launches ? info.pair_launches : 1);
      if (t < c.ms) c.ms = t;
    }
    if (c.ms < best.ms) best = c;
  }
  ctx->opts = saved;
  remember(ctx, kFormPlain, n, k, best);
  return TCRNET_OK;
}

int32_t tcrnet_autotune_batch(tcrnet_ctx* ctx, const tcrnet_seqs* reps, uint32_t n_reps, int32_t k) {
  if (!ctx || (n_reps && !reps)) return set_error(TCRNET_EINVAL, "NULL argument");
  int32_t rc;
  if ((rc = check_k(k))) return rc;
  (void)hipSetDevice(ctx->device);
  BatchInput bi;
  if ((rc = batch_upload(ctx, reps, n_reps, &bi))) return rc;
  if (bi.n < 2) return TCRNET_OK;
  std::vector<Candidate> cands = candidates(ctx->opts);
  Candidate best;
  uint64_t E_ref = ~0ull;
  for (Candidate& c : cands) {
    // the first run captures the candidate's graph; the next two replay it
    for (int rep = 0; rep < 3; ++rep) {
      uint64_t E = 0;
      tcrnet_build_info info{};
      if ((rc = batch_launch(ctx, bi, k, c.s, &E, &info))) return rc;
      if (E_ref == ~0ull) E_ref = E;
      if (E != E_ref) return set_error(TCRNET_EDEVICE, "autotune: schedules gave different edge counts (internal)");
      if (rep > 0 && info.build_ms < c.ms) c.ms = info.build_ms;
    }
    if (c.ms < best.ms) best = c;
  }
  remember(ctx, kFormBatch, bi.n, k, best);
  return TCRNET_OK;
}

int32_t tcrnet_autotune_get(const tcrnet_ctx* ctx, int32_t batch, uint64_t n, int32_t k, tcrnet_tune_entry* out) {
  if (!ctx || !out) return set_error(TCRNET_EINVAL, "NULL argument");
  TuneKey key;
  key.form = batch ? kFormBatch : kFormPlain;
  key.size_class = (int)bits_for(n ? n : 1);
  key.k = k;
  auto it = ctx->tuned.find(key);
  if (it == ctx->tuned.end()) return set_error(TCRNET_ESTATE, "no tuned schedule for this form, size class and k");
  const Sched& s = it->second.sched;
  out->texts_per_item = s.texts_per_item;
  out->waves_per_simd = s.waves_per_simd;
  out->peq_lds = s.peq_lds ? 1 : 0;
  out->pack = s.pack ? 1 : 0;
  out->ms = it->second.ms;
  return TCRNET_OK;
}

int32_t tcrnet_autotune_save(const tcrnet_ctx* ctx, const char* path) {
  if (!ctx || !path) return set_error(TCRNET_EINVAL, "NULL argument");
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return set_error(TCRNET_EINVAL, "cannot write %s: %s", tmp.c_str(), strerror(errno));
  fprintf(f, "{\n  \"format\": \"tcrnet-autotune\",\n  \"version\": 1,\n  \"entries\": [");
  bool first = true;
  for (const auto& kv : ctx->tuned) {
    const Sched& s = kv.second.sched;
    fprintf(f,
            "%s\n    {\"arch\": \"%s\", \"cus\": %d, \"form\": \"%s\", \"size_class\": %d, \"k\": %d, "
            "\"texts_per_item\": %u, \"waves_per_simd\": %u, \"peq_lds\": %d, \"pack\": %d, \"ms\": %.17g}",
            first ? "" : ",", ctx->arch, ctx->cus, form_name(kv.first.form), kv.first.size_class, kv.first.k,
            s.texts_per_item, s.waves_per_simd, s.peq_lds ? 1 : 0, s.pack ? 1 : 0, kv.second.ms);
    first = false;
  }
  fprintf(f, "\n  ]\n}\n");
  const bool ok = fflush(f) == 0 && ferror(f) == 0;
  if (fclose(f) != 0 || !ok) return set_error(TCRNET_EINVAL, "cannot write %s", tmp.c_str());
  if (rename(tmp.c_str(), path) != 0) return set_error(TCRNET_EINVAL, "cannot rename to %s: %s", path, strerror(errno));
  return TCRNET_OK;
}

int32_t tcrnet_autotune_load(tcrnet_ctx* ctx, const char* path, uint32_t* n_loaded) {
  if (!ctx || !path) return set_error(TCRNET_EINVAL, "NULL argument");
  if (n_loaded) *n_loaded = 0;
  FILE* f = fopen(path, "r");
  if (!f) return set_error(TCRNET_EINVAL, "cannot read %s: %s", path, strerror(errno));
  std::string txt;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
  fclose(f);
  std::vector<Obj> objs;
  if (txt.find("\"tcrnet-autotune\"") == std::string::npos || !parse_entries(txt, &objs))
    return set_error(TCRNET_EINVAL, "%s is not an autotune table", path);
  std::vector<std::pair<TuneKey, TuneEntry>> take;
  for (const Obj& o : objs) {
    const std::string* arch = o.get("arch");
    const std::string* form = o.get("form");
    uint32_t cus, sc, k, T, W, lds, pack;
    if (!arch || !form || !to_u32(o.get("cus"), &cus) || !to_u32(o.get("size_class"), &sc) ||
        !to_u32(o.get("k"), &k) || !to_u32(o.get("texts_per_item"), &T) || !to_u32(o.get("waves_per_simd"), &W) ||
        !to_u32(o.get("peq_lds"), &lds) || !to_u32(o.get("pack"), &pack) || (*form != "plain" && *form != "batch") ||
        k > TCRNET_MAX_K || sc > 64 || T == 0 || T > (1u << 20) || W == 0 || W > 8 || lds > 1 || pack > 1)
      return set_error(TCRNET_EINVAL, "%s: malformed autotune entry", path);
    if (*arch != ctx->arch || (int)cus != ctx->cus) continue;  // another device's choice
    TuneKey key;
    key.form = *form == "batch" ? kFormBatch : kFormPlain;
    key.size_class = (int)sc;
    key.k = (int)k;
    TuneEntry e;
    e.sched.texts_per_item = T;
    e.sched.waves_per_simd = W;
    e.sched.peq_lds = lds != 0;
    e.sched.pack = pack != 0;
    const std::string* ms = o.get("ms");
    e.ms = ms ? strtod(ms->c_str(), nullptr) : 0.0;
    take.emplace_back(key, e);
  }
  for (auto& kv : take) ctx->tuned[kv.first] = kv.second;
  if (n_loaded) *n_loaded = (uint32_t)take.size();
  return TCRNET_OK;
}

}  // extern "C"
