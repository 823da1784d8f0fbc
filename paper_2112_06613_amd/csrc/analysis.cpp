// C-ABI of the network analysis: connected components / LCC and site
// percolation on an edge list.
#define TCRNET_BUILDING 1
#include <algorithm>
#include <vector>

#include "api_internal.h"
#include "graph.h"

using namespace tcr;

namespace {

int32_t check_pairs(const uint32_t* pairs, uint64_t E, uint32_t n) {
  if (E && !pairs) return set_error(TCRNET_EINVAL, "NULL edge list");
  for (uint64_t e = 0; e < 2 * E; ++e)
    if (pairs[e] >= n) return set_error(TCRNET_EINVAL, "edge %llu names node %u of %u", (unsigned long long)(e / 2),
                                        pairs[e], n);
  return TCRNET_OK;
}

// Upload the edge list into the context's edge buffer.
int32_t upload_pairs(tcrnet_ctx* ctx, const uint32_t* pairs, uint64_t E) {
  hipError_t e;
  if ((e = ctx->out_pairs.ensure((E ? E : 1) * 8)) != hipSuccess) return hip_error(e, "edge buffer");
  if (E && (e = hipMemcpyAsync(ctx->out_pairs.p, pairs, E * 8, hipMemcpyHostToDevice, ctx->stream)) != hipSuccess)
    return hip_error(e, "edge copy");
  return TCRNET_OK;
}

}  // namespace

extern "C" {

int32_t tcrnet_components(tcrnet_ctx* ctx, const uint32_t* pairs, uint64_t n_edges, uint32_t n, uint32_t* labels,
                          uint32_t* sizes, tcrnet_cc_info* info) {
  if (!ctx || !info) return set_error(TCRNET_EINVAL, "NULL context or info");
  int32_t rc;
  if ((rc = check_pairs(pairs, n_edges, n))) return rc;
  *info = tcrnet_cc_info{};
  if (n == 0) return TCRNET_OK;
  (void)hipSetDevice(ctx->device);
  if ((rc = upload_pairs(ctx, pairs, n_edges))) return rc;
  hipError_t e;
  if ((e = ctx->ana_ws.ensure(cc_workspace_bytes(n, 1))) != hipSuccess) return hip_error(e, "workspace");
  if ((e = ctx->ana_out.ensure((uint64_t)n * 8 + 64)) != hipSuccess) return hip_error(e, "workspace");
  uint32_t* d_labels = ctx->ana_out.as<uint32_t>();
  uint32_t* d_sizes = d_labels + n;
  uint32_t* d_small = static_cast<uint32_t*>(ctx->ana_ws.p) + (cc_workspace_bytes(n, 1) - 256) / 4;
  launch_components(ctx->out_pairs.as<uint32_t>(), n_edges, n, nullptr, nullptr, 1, ctx->ana_ws.p, d_labels,
                    d_sizes, d_small, d_small + 1, ctx->stream);
  uint32_t small[2];
  (void)hipMemcpyAsync(small, d_small, 8, hipMemcpyDeviceToHost, ctx->stream);
  if (labels) (void)hipMemcpyAsync(labels, d_labels, (uint64_t)n * 4, hipMemcpyDeviceToHost, ctx->stream);
  if (sizes) (void)hipMemcpyAsync(sizes, d_sizes, (uint64_t)n * 4, hipMemcpyDeviceToHost, ctx->stream);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_error(e, "components");
  info->lcc_size = small[0];
  info->n_components = small[1];
  return TCRNET_OK;
}

int32_t tcrnet_robustness(tcrnet_ctx* ctx, const uint32_t* pairs, uint64_t n_edges, uint32_t n,
                          const uint32_t* order, const uint32_t* removed, uint32_t n_runs, uint32_t* lcc) {
  if (!ctx || (n_runs && (!removed || !lcc))) return set_error(TCRNET_EINVAL, "NULL argument");
  if (n && !order) return set_error(TCRNET_EINVAL, "NULL removal order");
  int32_t rc;
  if ((rc = check_pairs(pairs, n_edges, n))) return rc;
  {
    std::vector<uint8_t> seen(n, 0);
    for (uint32_t t = 0; t < n; ++t) {
      if (order[t] >= n || seen[order[t]]) return set_error(TCRNET_EINVAL, "removal order is not a permutation");
      seen[order[t]] = 1;
    }
  }
  for (uint32_t q = 0; q < n_runs; ++q)
    if (removed[q] > n) return set_error(TCRNET_EINVAL, "removal count %u exceeds n = %u", removed[q], n);
  if (n == 0) {
    for (uint32_t q = 0; q < n_runs; ++q) lcc[q] = 0;
    return TCRNET_OK;
  }
  (void)hipSetDevice(ctx->device);
  if ((rc = upload_pairs(ctx, pairs, n_edges))) return rc;
  // runs in chunks of at most ~1 GiB of parent/size arrays
  const uint32_t chunk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(n_runs, (1ull << 30) / ((uint64_t)n * 8)));
  hipError_t e;
  if ((e = ctx->ana_ws.ensure(cc_workspace_bytes(n, chunk))) != hipSuccess) return hip_error(e, "workspace");
  if ((e = ctx->ana_out.ensure((uint64_t)n * 4 + (uint64_t)n_runs * 12 + 64)) != hipSuccess)
    return hip_error(e, "workspace");
  uint32_t* d_order = ctx->ana_out.as<uint32_t>();
  uint32_t* d_removed = d_order + n;
  uint32_t* d_lcc = d_removed + n_runs;
  uint32_t* d_comps = d_lcc + n_runs;
  (void)hipMemcpyAsync(d_order, order, (uint64_t)n * 4, hipMemcpyHostToDevice, ctx->stream);
  (void)hipMemcpyAsync(d_removed, removed, (uint64_t)n_runs * 4, hipMemcpyHostToDevice, ctx->stream);
  for (uint32_t q0 = 0; q0 < n_runs; q0 += chunk) {
    const uint32_t P = std::min(chunk, n_runs - q0);
    launch_components(ctx->out_pairs.as<uint32_t>(), n_edges, n, d_order, d_removed + q0, P, ctx->ana_ws.p, nullptr,
                      nullptr, d_lcc + q0, d_comps + q0, ctx->stream);
  }
  (void)hipMemcpyAsync(lcc, d_lcc, (uint64_t)n_runs * 4, hipMemcpyDeviceToHost, ctx->stream);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_error(e, "robustness");
  return TCRNET_OK;
}

int32_t tcrnet_graph_stats(tcrnet_ctx* ctx, const uint32_t* pairs, uint64_t n_edges, uint32_t n, int32_t* degree,
                           uint64_t* deg_count, uint64_t* nbr_deg_sum, uint32_t hist_len, double* clustering,
                           tcrnet_stats* out) {
  if (!ctx || !out || (hist_len && (!deg_count || !nbr_deg_sum)))
    return set_error(TCRNET_EINVAL, "NULL argument");
  int32_t rc;
  if ((rc = check_pairs(pairs, n_edges, n))) return rc;
  for (uint64_t e = 0; e < n_edges; ++e) {
    const bool ordered = pairs[2 * e] < pairs[2 * e + 1];
    const bool sorted = e == 0 || pairs[2 * e - 2] < pairs[2 * e] ||
                        (pairs[2 * e - 2] == pairs[2 * e] && pairs[2 * e - 1] < pairs[2 * e + 1]);
    if (!ordered || !sorted)
      return set_error(TCRNET_EINVAL, "edge list must be canonical (i < j, sorted, distinct) at edge %llu",
                       (unsigned long long)e);
  }
  *out = tcrnet_stats{};
  if (n == 0) return TCRNET_OK;
  (void)hipSetDevice(ctx->device);
  if ((rc = upload_pairs(ctx, pairs, n_edges))) return rc;
  hipError_t e;
  const uint32_t hl = hist_len ? hist_len : 1;
  const uint64_t out_bytes = (uint64_t)hl * 16 + (uint64_t)n * 12 + sizeof(GraphStatsDev) + 64;
  if ((e = ctx->ana_ws.ensure(stats_workspace_bytes(n))) != hipSuccess) return hip_error(e, "workspace");
  if ((e = ctx->ana_out.ensure(out_bytes)) != hipSuccess) return hip_error(e, "workspace");
  char* base = ctx->ana_out.as<char>();
  GraphStatsDev* d_out = reinterpret_cast<GraphStatsDev*>(base);
  unsigned long long* d_count = reinterpret_cast<unsigned long long*>(base + 64);
  unsigned long long* d_nbr = d_count + hl;
  double* d_clu = reinterpret_cast<double*>(d_nbr + hl);
  uint32_t* d_deg = reinterpret_cast<uint32_t*>(d_clu + n);
  launch_graph_stats(ctx->out_pairs.as<uint32_t>(), n_edges, n, ctx->ana_ws.p, hl, d_count, d_nbr,
                     clustering ? d_clu : nullptr, d_deg, d_out, ctx->stream);
  GraphStatsDev h;
  (void)hipMemcpyAsync(&h, d_out, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
  if (hist_len) {
    (void)hipMemcpyAsync(deg_count, d_count, (uint64_t)hist_len * 8, hipMemcpyDeviceToHost, ctx->stream);
    (void)hipMemcpyAsync(nbr_deg_sum, d_nbr, (uint64_t)hist_len * 8, hipMemcpyDeviceToHost, ctx->stream);
  }
  if (clustering) (void)hipMemcpyAsync(clustering, d_clu, (uint64_t)n * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (degree) (void)hipMemcpyAsync(degree, d_deg, (uint64_t)n * 4, hipMemcpyDeviceToHost, ctx->stream);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_error(e, "graph stats");
  out->max_degree = h.max_degree;
  out->triangles = h.triangles;
  out->assortativity = h.real[0];
  out->avg_clustering = h.real[1];
  out->sum_jk = h.sums[0];
  out->sum_j_plus_k = h.sums[1];
  out->sum_j2_plus_k2 = h.sums[2];
  if (h.max_degree >= hist_len)
    return set_error(TCRNET_ETRUNC, "hist_len %u too small: the maximum degree is %u", hist_len, h.max_degree);
  return TCRNET_OK;
}

int32_t tcrnet_lcc_norm(const uint32_t* lcc, const uint32_t* removed, uint32_t n_runs, uint32_t n, double* norm1,
                        double* norm2) {
  if (n_runs && (!lcc || !removed)) return set_error(TCRNET_EINVAL, "NULL argument");
  for (uint32_t q = 0; q < n_runs; ++q)
    if (removed[q] > n || lcc[q] > n - removed[q])
      return set_error(TCRNET_EINVAL, "run %u: removed or LCC size exceeds the nodes", q);
  if (norm2 && n_runs && removed[0] != 0)
    return set_error(TCRNET_EINVAL, "LCC_norm,2 needs removed[0] = 0 (the intact network)");
  // LCC_norm,1(p) = LCC(p) / ((1 - p) N) with p = removed / N: the largest
  // component as a fraction of the nodes left; 0 once none is left
  auto n1 = [&](uint32_t q) -> double {
    const uint32_t left = n - removed[q];
    return left ? (double)lcc[q] / (double)left : 0.0;
  };
  const double base = n_runs ? n1(0) : 0.0;
  for (uint32_t q = 0; q < n_runs; ++q) {
    const double v = n1(q);
    if (norm1) norm1[q] = v;
    // LCC_norm,2(p) = LCC_norm,1(p) / LCC_norm,1(0)
    if (norm2) norm2[q] = base > 0.0 ? v / base : v;
  }
  return TCRNET_OK;
}

}  // extern "C"
