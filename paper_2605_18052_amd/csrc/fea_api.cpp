// C ABI of libfastea: context lifetime, input validation, the IRLS round
// loop of FastMap's epipolar adjustment (Method > Epipolar Adjustment:
// re-weighting rounds, outlier filtering with a decreasing threshold, focal
// lengths folded into the essential matrix) and the host-side bookkeeping of
// the O(pairs + cameras) metadata.  All O(matches) work runs in the HIP
// kernels of fea_segment.hip, fea_resgrad.hip and fea_camera.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "fea_ctx.h"
#include "fea_focal.h"
#include "fea_rotation.h"
#include "fea_trans.h"

using fea::DBuf;

namespace {

fea_status fail(fea_ctx* c, fea_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_OR_FAIL(c, expr)                                                                    \
  do {                                                                                          \
    hipError_t _e = (expr);                                                                     \
    if (_e != hipSuccess) return fail((c), FEA_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int now = -1;
    if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
  }
};

// Bumped whenever a device buffer is freed or replaced: a captured step
// graph holds raw device pointers in its kernel arguments, so one captured
// before the bump is captured again before its next launch.
std::atomic<uint64_t> g_buffer_gen{0};

hipError_t dalloc(DBuf& b, size_t bytes) {
  bytes = std::max<size_t>(bytes, 16);
  if (b.p && b.bytes >= bytes) return hipSuccess;
  g_buffer_gen.fetch_add(1);
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e == hipSuccess) b.bytes = bytes;
  return e;
}

void dfree(DBuf& b) {
  if (b.p) g_buffer_gen.fetch_add(1);
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

// Small host-to-device copies (per-round tables, counters) go through a
// pinned staging ring so that they are queued without blocking the host;
// when the ring is full the stream is drained and the ring reused.
constexpr size_t kStageBytes = 16u << 20;

hipError_t stage_copy(fea_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  if (bytes > kStageBytes) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
  hipError_t e = hipSuccess;
  if (!c->stage) {
    if ((e = hipHostMalloc(&c->stage, kStageBytes, hipHostMallocDefault)) != hipSuccess) {
      c->stage = nullptr;
      return e;
    }
    c->stage_used = 0;
  }
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (c->stage_used + need > kStageBytes) {
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
    c->stage_used = 0;
  }
  uint8_t* p = static_cast<uint8_t*>(c->stage) + c->stage_used;
  c->stage_used += need;
  std::memcpy(p, src, bytes);
  return hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, c->stream);
}

template <class T>
hipError_t upload(fea_ctx* c, DBuf& b, const T* src, size_t n) {
  hipError_t e = dalloc(b, n * sizeof(T));
  if (e != hipSuccess || n == 0) return e;
  return stage_copy(c, b.p, src, n * sizeof(T));
}

template <class T>
hipError_t download(fea_ctx* c, std::vector<T>& dst, const DBuf& b, size_t n) {
  dst.resize(n);
  if (n == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(dst.data(), b.p, n * sizeof(T), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

std::vector<DBuf*> all_bufs(fea_ctx* c) {
  std::vector<DBuf*> v;
  for (int b = 0; b < 3; ++b) {
    for (int a = 0; a < 4; ++a) v.push_back(&c->lay[b][a]);
    v.push_back(&c->lpos[b]);
  }
  DBuf* one[] = {&c->perm, &c->swp, &c->item_rec, &c->d_scene_item_off, &c->scene_loss, &c->pair_item_off,
                 &c->item_keep, &c->item_base, &c->part, &c->d_pair_i, &c->d_pair_j, &c->d_cam_off,
                 &c->d_cam_ent, &c->d_group, &c->d_grp_off, &c->d_grp_cams, &c->d_cx, &c->d_cy, &c->a6,
                 &c->tp, &c->logf, &c->m_a6, &c->v_a6, &c->m_t, &c->v_t, &c->m_f, &c->v_f, &c->R[0],
                 &c->R[1], &c->T[0], &c->T[1], &c->Fc[0], &c->Fc[1], &c->Rh, &c->Th, &c->Fh, &c->gR,
                 &c->gt, &c->gf, &c->loss_cam, &c->loss, &c->logR, &c->errflag, &c->wait_state, &c->Re, &c->Te, &c->Fe, &c->d_pair_scene, &c->d_inv_z, &c->d_tau, &c->ptab, &c->qpart, &c->qW, &c->qmask, &c->stab, &c->counters,
                 &c->Rh1, &c->Th1, &c->Fh1, &c->Rh2, &c->Th2, &c->Fh2, &c->d_fbar, &c->mlp, &c->wlay,
                 &c->item_wsum, &c->d_inv_zw, &c->d_scene_mode, &c->d_fbar_hist, &c->d_scene_cam_off, &c->d_scene_cams, &c->d_scene_z, &c->a6h, &c->tph, &c->logfh, &c->d_learned_ok, &c->d_fallbacks, &c->d_judge_l0, &c->d_judge_l1};
  for (DBuf* b : one) v.push_back(b);
  return v;
}

bool options_valid(const fea_options* o, std::string* why) {
  auto bad = [&](const char* s) {
    *why = s;
    return false;
  };
  if (o->rounds < 0 || o->rounds > 100000) return bad("rounds must be in [0, 100000]");
  if (o->iters_per_round < 0) return bad("iters_per_round must be >= 0");
  if (!(o->tau_px_init > 0) || !(o->tau_px_min > 0)) return bad("tau_px_init and tau_px_min must be > 0");
  if (!(o->tau_decay > 0 && o->tau_decay <= 1)) return bad("tau_decay must be in (0, 1]");
  if (!(o->delta > 0) || !std::isfinite(o->delta)) return bad("delta must be finite and > 0");
  if (!(o->lr_rot >= 0) || !(o->lr_t >= 0) || !(o->lr_logf >= 0)) return bad("learning rates must be >= 0");
  if (!(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1)) return bad("betas must be in [0,1)");
  if (!(o->adam_eps >= 0)) return bad("adam_eps must be >= 0");
  if (o->log_every < 0 || o->max_log < 0) return bad("log_every and max_log must be >= 0");
  if (!(o->lr_decay > 0) || !std::isfinite(o->lr_decay)) return bad("lr_decay must be finite and > 0");
  if (o->reset_moments != 0 && o->reset_moments != 1) return bad("reset_moments must be 0 or 1");
  if (o->tile_matches != 0 && o->tile_matches != 1024 && o->tile_matches != 2048 && o->tile_matches != 4096 &&
      o->tile_matches != 8192)
    return bad("tile_matches must be 0, 1024, 2048, 4096 or 8192");
  if (o->use_graphs != 0 && o->use_graphs != 1) return bad("use_graphs must be 0 or 1");
  if (o->weight_mode != 0 && o->weight_mode != 1) return bad("weight_mode must be 0 or 1");
  if (o->inner_loop != 0 && o->inner_loop != 1) return bad("inner_loop must be 0 or 1");
  // A profiled solve with learned weights, the quadratic form and
  // 1024-match work items ended in a host-side fault inside the runtime's
  // graph launch whose cause has not been shown; until it is, that
  // combination is refused (the default items of the quadratic form are
  // 8192 matches).
  if (o->weight_mode == 1 && o->inner_loop == 1 && o->tile_matches != 0 && o->tile_matches != 8192)
    return bad("learned weights with the quadratic form support tile_matches 0 or 8192 only");
  if (o->tile_persistent != 0 && o->tile_persistent != 1) return bad("tile_persistent must be 0 or 1");
  if (o->tile_persistent == 1 && o->tile_matches != 1024 && o->tile_matches != 2048 && o->tile_matches != 4096)
    return bad("tile_persistent = 1 needs tile_matches 1024, 2048 or 4096");
  if (o->persistent_steps != 0 && o->persistent_steps != 1) return bad("persistent_steps must be 0 or 1");
  if (o->wait_limit_us < 0) return bad("wait_limit_us must be >= 0");
  if (!(o->converge_deg >= 0) || !std::isfinite(o->converge_deg)) return bad("converge_deg must be finite and >= 0");
  return true;
}

// Scenes the non-finite guard has stopped (waits for the stream): the counts
// of converged and stopped scenes, and FEA_ENONFINITE if more are stopped
// than at the previous check.
fea_status check_nonfinite(fea_ctx* c, int32_t* converged = nullptr, int32_t* stopped = nullptr) {
  std::vector<unsigned> ws;
  HIP_OR_FAIL(c, download(c, ws, c->wait_state, 2));
  if (ws[1] != 0) {
    // a persistent launch left early: its steps did not all run; the
    // context keeps to one launch per step from here on
    c->quad_steps_cap = 0;
    c->wait_base = 0;
    HIP_OR_FAIL(c, hipMemsetAsync(c->wait_state.p, 0, 2 * sizeof(unsigned), c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return fail(c, FEA_EDEVICE, "a device-wide wait between the steps of a persistent launch timed out");
  }
  std::vector<int32_t> done;
  HIP_OR_FAIL(c, download(c, done, c->d_scene_done, (size_t)c->S));
  int32_t nc = 0, nb = 0;
  std::string which;
  for (int s = 0; s < c->S; ++s) {
    nc += done[s] > 0 ? 1 : 0;
    if (done[s] < 0) {
      ++nb;
      if (which.size() < 120) which += " " + std::to_string(s);
    }
  }
  if (converged) *converged = nc;
  if (stopped) *stopped = nb;
  const int32_t before = c->n_nonfinite;
  c->n_nonfinite = nb;
  if (nb > before)
    return fail(c, FEA_ENONFINITE,
                "non-finite parameters, poses or loss in scene(s)" + which +
                    ": their poses are the last finite round snapshot and they take no further steps");
  return FEA_OK;
}

double median(std::vector<double> v) {
  if (v.empty()) return 1.0;
  std::sort(v.begin(), v.end());
  const size_t n = v.size();
  return (n % 2) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

// Work items of the current layout: runs of <= tile matches of one pair
// (pairs with no retained match get none), and each camera's int4 entries
// {2n+side, first item, end item, other camera} for the epilogue.
// No scene converged (start of a solve, new scenes).
hipError_t clear_convergence(fea_ctx* c) {
  c->n_done = 0;
  c->n_nonfinite = 0;
  c->prev_tau_px = -1.0;
  c->scene_done_h.assign(c->S, 0);
  hipError_t e = hipSuccess;
  if (c->d_scene_done.p && (e = hipMemsetAsync(c->d_scene_done.p, 0, c->d_scene_done.bytes, c->stream)) != hipSuccess)
    return e;
  if (c->d_scene_change.p) e = hipMemsetAsync(c->d_scene_change.p, 0, c->d_scene_change.bytes, c->stream);
  return e;
}

hipError_t build_items(fea_ctx* c) {
  const int64_t tile = fea::tile_matches_of(c->tile_cfg);
  c->h_item_pair.clear();
  c->h_item_start.clear();
  c->h_item_count.clear();
  c->h_pair_item_off.assign(c->P + 1, 0);
  for (int64_t n = 0; n < c->P; ++n) {
    c->h_pair_item_off[n] = (int32_t)c->h_item_pair.size();
    for (int64_t s = 0; s < c->cur_len[n]; s += tile) {
      c->h_item_pair.push_back((int32_t)n);
      c->h_item_start.push_back((int32_t)(c->phys_off[n] + s));
      c->h_item_count.push_back((int32_t)std::min<int64_t>(tile, c->cur_len[n] - s));
    }
  }
  c->h_pair_item_off[c->P] = (int32_t)c->h_item_pair.size();
  c->n_items = (int64_t)c->h_item_pair.size();
  c->h_item_rec.assign(4 * c->n_items, 0);
  const bool flags = c->n_done > 0 && (int)c->scene_done_h.size() == c->S;
  for (int64_t it = 0; it < c->n_items; ++it) {
    c->h_item_rec[4 * it] = c->h_item_pair[it];
    c->h_item_rec[4 * it + 1] = c->h_item_start[it];
    c->h_item_rec[4 * it + 2] = c->h_item_count[it];
    // items of converged scenes are skipped by the steps
    c->h_item_rec[4 * it + 3] = flags && c->scene_done_h[c->pair_scene[c->h_item_pair[it]]] != 0 ? 1 : 0;
  }
  c->h_cam_ent4.assign(4 * 2 * c->P, 0);
  for (size_t e = 0; e < c->cam_ent.size(); ++e) {
    const int32_t code = c->cam_ent[e];
    const int64_t n = code >> 1;
    const int side = code & 1;
    c->h_cam_ent4[4 * e] = code;
    c->h_cam_ent4[4 * e + 1] = c->h_pair_item_off[n];
    c->h_cam_ent4[4 * e + 2] = c->h_pair_item_off[n + 1];
    c->h_cam_ent4[4 * e + 3] = side ? c->pair_i[n] : c->pair_j[n];
  }
  hipError_t e;
  if ((e = upload(c, c->item_rec, c->h_item_rec.data(), c->h_item_rec.size())) != hipSuccess) return e;
  // items of each scene: pairs are sorted by their first camera, so when a
  // scene's cameras have contiguous ids its items are a contiguous range
  c->scene_items_contiguous = true;
  for (int64_t it = 1; it < c->n_items; ++it)
    if (c->pair_scene[c->h_item_pair[it]] < c->pair_scene[c->h_item_pair[it - 1]]) c->scene_items_contiguous = false;
  std::vector<int32_t> soff(c->S + 1, (int32_t)c->n_items);
  for (int64_t it = c->n_items - 1; it >= 0; --it) soff[c->pair_scene[c->h_item_pair[it]]] = (int32_t)it;
  for (int sc = c->S - 1; sc >= 0; --sc) soff[sc] = std::min(soff[sc], soff[sc + 1]);
  if ((e = upload(c, c->d_scene_item_off, soff.data(), soff.size())) != hipSuccess) return e;
  if ((e = dalloc(c->scene_loss, (size_t)std::max(c->S, 1) * sizeof(double))) != hipSuccess) return e;
  if ((e = upload(c, c->pair_item_off, c->h_pair_item_off.data(), c->P + 1)) != hipSuccess) return e;
  if ((e = upload(c, c->d_cam_ent, c->h_cam_ent4.data(), c->h_cam_ent4.size())) != hipSuccess) return e;
  if ((e = dalloc(c->qpart, std::max<int64_t>(c->n_items, 1) * 36 * sizeof(double))) != hipSuccess) return e;
  if ((e = dalloc(c->part, std::max<int64_t>(c->n_items, 1) * fea::kPartStride * sizeof(double))) != hipSuccess)
    return e;
  if ((e = dalloc(c->item_keep, std::max<int64_t>(c->n_items, 1) * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = dalloc(c->item_wsum, std::max<int64_t>(c->n_items, 1) * sizeof(double))) != hipSuccess) return e;
  return dalloc(c->item_base, std::max<int64_t>(c->n_items, 1) * 2 * sizeof(int32_t));
}

// Every scene may use learned weights again, no rejection counted.
hipError_t reset_judge(fea_ctx* c) {
  c->scene_learned_ok.assign(c->S, 1);
  c->fallbacks = 0;
  c->fallbacks_base = 0;
  c->judge_pending = false;
  hipError_t e = upload(c, c->d_learned_ok, c->scene_learned_ok.data(), c->S);
  if (e != hipSuccess || c->S == 0) return e;
  return hipMemsetAsync(c->d_fallbacks.p, 0, (size_t)c->S * sizeof(int32_t), c->stream);
}

// The judge's per-scene verdicts and weighting modes as the device holds
// them, into the host's records (waits for the stream).
hipError_t refresh_learned_host(fea_ctx* c) {
  if (c->S == 0) return hipSuccess;
  std::vector<int32_t> fb;
  hipError_t e;
  if ((e = download(c, c->scene_learned_ok, c->d_learned_ok, c->S)) != hipSuccess) return e;
  if ((e = download(c, c->scene_mode, c->d_scene_mode, c->S)) != hipSuccess) return e;
  if ((e = download(c, fb, c->d_fallbacks, c->S)) != hipSuccess) return e;
  c->fallbacks = c->fallbacks_base;
  for (int32_t v : fb) c->fallbacks += v;
  c->judge_pending = false;
  return hipSuccess;
}

// Per-scene device arrays sized by the number of scenes.
hipError_t alloc_scene_arrays(fea_ctx* c) {
  hipError_t e;
  if ((e = dalloc(c->d_inv_z, (size_t)c->S * sizeof(float))) != hipSuccess) return e;
  if ((e = dalloc(c->d_inv_zw, (size_t)c->S * sizeof(float))) != hipSuccess) return e;
  if ((e = dalloc(c->d_scene_mode, (size_t)c->S * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = dalloc(c->d_fbar, 3 * (size_t)c->S * sizeof(float))) != hipSuccess) return e;
  if ((e = dalloc(c->d_fbar_hist, 3 * (size_t)c->S * sizeof(double))) != hipSuccess) return e;
  if ((e = dalloc(c->d_tau, (size_t)c->S * sizeof(double))) != hipSuccess) return e;
  if ((e = dalloc(c->d_scene_z, ((size_t)c->S + 1) * sizeof(int64_t))) != hipSuccess) return e;
  if ((e = dalloc(c->d_scene_done, (size_t)c->S * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = dalloc(c->d_scene_change, (size_t)c->S * sizeof(double))) != hipSuccess) return e;
  if ((e = dalloc(c->d_learned_ok, (size_t)c->S * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = dalloc(c->d_fallbacks, (size_t)c->S * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = dalloc(c->d_judge_l0, (size_t)c->S * sizeof(double))) != hipSuccess) return e;
  if ((e = dalloc(c->d_judge_l1, (size_t)c->S * sizeof(double))) != hipSuccess) return e;
  c->judge_written = false;
  if ((e = upload(c, c->d_cam_scene, c->cam_scene.data(), c->cam_scene.size())) != hipSuccess) return e;
  // cameras of each scene, for the device round start
  std::vector<int32_t> off(c->S + 1, 0), cams(c->N, 0);
  for (int i = 0; i < c->N; ++i) off[c->cam_scene[i] + 1] += 1;
  for (int s = 0; s < c->S; ++s) off[s + 1] += off[s];
  c->max_scene_cams = 0;
  for (int s = 0; s < c->S; ++s) c->max_scene_cams = std::max(c->max_scene_cams, off[s + 1] - off[s]);
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int i = 0; i < c->N; ++i) cams[fill[c->cam_scene[i]]++] = i;
  }
  if ((e = upload(c, c->d_scene_cam_off, off.data(), off.size())) != hipSuccess) return e;
  if ((e = upload(c, c->d_scene_cams, cams.data(), cams.size())) != hipSuccess) return e;
  c->host_tau_stale = c->host_z_stale = false;
  if ((e = hipMemsetAsync(c->d_inv_zw.p, 0, c->d_inv_zw.bytes, c->stream)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(c->d_scene_mode.p, 0, c->d_scene_mode.bytes, c->stream)) != hipSuccess) return e;
  if ((e = clear_convergence(c)) != hipSuccess) return e;
  c->scene_mode.assign(c->S, 0);
  return reset_judge(c);
}

// The round values computed on the device (thresholds and focal-length
// medians at the round start; quadratic form: survivors per scene and the
// learned normalisers) copied into the host's records when they are read.
hipError_t refresh_round_host(fea_ctx* c) {
  hipError_t e = hipSuccess;
  if (c->host_tau_stale) {
    if ((e = download(c, c->taus, c->d_tau, c->S)) != hipSuccess) return e;
    if ((e = download(c, c->fbar_hist, c->d_fbar_hist, 3 * (size_t)c->S)) != hipSuccess) return e;
    c->tau = c->taus.empty() ? 0.0 : c->taus[0];
    c->host_tau_stale = false;
  }
  if (c->host_z_stale) {
    std::vector<int64_t> z;
    if ((e = download(c, z, c->d_scene_z, (size_t)c->S + 1)) != hipSuccess) return e;
    c->Zs.assign(z.begin(), z.begin() + c->S);
    c->Z = z[c->S];
    if (c->learned_any && (e = download(c, c->inv_zw_h, c->d_inv_zw, c->S)) != hipSuccess) return e;
    c->host_z_stale = false;
  }
  return e;
}

// The host's focal-length medians to both device copies.
hipError_t upload_fbar(fea_ctx* c) {
  std::vector<float> fb(c->fbar_hist.begin(), c->fbar_hist.end());
  hipError_t e = upload(c, c->d_fbar, fb.data(), fb.size());
  if (e != hipSuccess) return e;
  return upload(c, c->d_fbar_hist, c->fbar_hist.data(), c->fbar_hist.size());
}

int tile_cfg_for(int32_t tile_matches, bool persistent = false) {
  for (int k = 0; k < fea::kNumTiles; ++k)
    if (fea::tile_matches_of(k) == tile_matches && fea::kTiles[k].persistent == persistent) return k;
  return -1;
}

// Autotuner results of this process, keyed by device and by the layout's
// size class (retained matches and pairs, each to a factor of 2^(1/4)): a
// later context with a problem of the same class reuses the choice, so the
// choice is deterministic within a process.
struct TileKey {
  int device, z_class, p_class;
  bool operator<(const TileKey& o) const {
    return device != o.device ? device < o.device : (z_class != o.z_class ? z_class < o.z_class : p_class < o.p_class);
  }
};
std::mutex g_tile_mu;
std::map<TileKey, int> g_tile_cache;

int size_class(int64_t n) { return n > 0 ? (int)std::lround(4.0 * std::log2((double)n)) : -1; }

// Picks the work-item shape of the per-match kernel for the current layout:
// the requested size, the shape chosen earlier in this process for a problem
// of the same size class, or the fastest of the candidate shapes timed on
// this layout with HIP events (three launches each after one warm-up).
hipError_t choose_tile_impl(fea_ctx* c);

hipError_t choose_tile(fea_ctx* c) {
  const hipError_t e = choose_tile_impl(c);
  if (e == hipSuccess) fea::prepare_resgrad(c->tile_cfg);
  return e;
}

hipError_t choose_tile_impl(fea_ctx* c) {
  if (c->tile_tuned) return hipSuccess;
  if (c->opt.tile_matches > 0) {
    c->tile_cfg = tile_cfg_for(c->opt.tile_matches, c->opt.tile_persistent == 1);
    c->tile_tuned = true;
    return hipSuccess;
  }
  if (c->opt.inner_loop == 1) {
    // steps do not stream the matches; the once-per-round passes (form
    // build, filter) amortise their per-item reductions best over the
    // largest items
    c->tile_cfg = tile_cfg_for(8192);
    c->tile_tuned = true;
    return hipSuccess;
  }
  const TileKey key{c->device, size_class(c->Z), size_class(c->P)};
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tile_cache.find(key);
    if (it != g_tile_cache.end()) {
      c->tile_cfg = it->second;
      c->tile_tuned = true;
      return hipSuccess;
    }
  }
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  std::vector<float> times(fea::kNumTiles, 0.f);
  for (int k = 0; k < fea::kNumTiles && e == hipSuccess; ++k) {
    c->tile_cfg = k;
    if ((e = build_items(c)) != hipSuccess) break;
    if ((e = fea::launch_resgrad_cfg(c, k)) != hipSuccess) break;
    if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = fea::launch_resgrad_cfg(c, k);
    if (e != hipSuccess) break;
    if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    times[k] = ms / 3.f;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  // the first shape, in the table's order, within 3% of the fastest: shapes
  // whose times differ by less than the run-to-run noise would otherwise
  // trade places between runs
  const float best = *std::min_element(times.begin(), times.end());
  int best_cfg = 0;
  while (times[best_cfg] > 1.03f * best) ++best_cfg;
  c->tune_ms = times;
  c->tile_cfg = best_cfg;
  c->tile_tuned = true;
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile_cache.emplace(key, best_cfg);
  return hipSuccess;
}

// Per-scene retained counts -> Z and 1/Z on the device.
hipError_t upload_scene_z(fea_ctx* c) {
  c->Zs.assign(c->S, 0);
  for (int64_t n = 0; n < c->P; ++n) c->Zs[c->pair_scene[n]] += c->cur_len[n];
  c->Z = 0;
  std::vector<float> inv(c->S, 0.f);
  for (int s = 0; s < c->S; ++s) {
    c->Z += c->Zs[s];
    inv[s] = c->Zs[s] > 0 ? (float)(1.0 / (double)c->Zs[s]) : 0.f;
  }
  c->host_z_stale = false;
  return upload(c, c->d_inv_z, inv.data(), c->S);
}

// Back to the full (unfiltered) layout.
hipError_t reset_layout(fea_ctx* c) {
  c->cur = 0;
  int64_t off = 0;
  for (int64_t n = 0; n < c->P; ++n) {
    c->cur_len[n] = c->seg_off[n + 1] - c->seg_off[n];
    c->phys_off[n] = off;
    off += (c->cur_len[n] + fea::kAlign - 1) / fea::kAlign * fea::kAlign;
  }
  c->layout_len = off;
  hipError_t e = upload_scene_z(c);
  if (e != hipSuccess) return e;
  return build_items(c);
}

void reset_round_state(fea_ctx* c) {
  c->round = -1;
  c->step = 0;
  c->global_step = 0;
  c->n_logged = 0;
  c->tau = std::numeric_limits<double>::infinity();
  c->host_tau_stale = c->host_z_stale = false;
}

fea_status load_matches_common(fea_ctx* c, int64_t n, const float* x1, const float* y1, const float* x2,
                               const float* y2, const int32_t* cam1, const int32_t* cam2) {
  c->have_matches = false;
  c->have_poses = false;
  c->M = n;
  int bad = 0;
  hipError_t e = fea::segment_matches(c, x1, y1, x2, y2, cam1, cam2, &bad);
  if (e != hipSuccess) return fail(c, FEA_EDEVICE, std::string("segmenting: ") + hipGetErrorString(e));
  if (bad & fea::kErrRange) return fail(c, FEA_EINVAL, "a camera id is outside [0, n_cams)");
  if (bad & fea::kErrSameCam) return fail(c, FEA_EINVAL, "a match has cam1 == cam2");
  if (bad & fea::kErrNonFinite) return fail(c, FEA_ENONFINITE, "a keypoint coordinate is not finite");
  if (c->layout_len >= (int64_t)1 << 31) return fail(c, FEA_EINVAL, "too many matches for 32-bit offsets");
  // pristine full layout lives in buffer 0; buffers 1 and 2 take the
  // filtered layouts of successive rounds
  for (int b = 1; b < 3; ++b) {
    for (int a = 0; a < 4; ++a)
      HIP_OR_FAIL(c, dalloc(c->lay[b][a], std::max<int64_t>(c->layout_len, 1) * sizeof(float)));
    HIP_OR_FAIL(c, dalloc(c->lpos[b], std::max<int64_t>(c->layout_len, 1) * sizeof(int32_t)));
  }
  // every pair must lie inside one scene
  c->pair_scene.assign(c->P, 0);
  for (int64_t k = 0; k < c->P; ++k) {
    if (c->cam_scene[c->pair_i[k]] != c->cam_scene[c->pair_j[k]])
      return fail(c, FEA_EINVAL, "a match links cameras of different scenes");
    c->pair_scene[k] = c->cam_scene[c->pair_i[k]];
  }
  HIP_OR_FAIL(c, upload(c, c->d_pair_scene, c->pair_scene.data(), c->P));
  HIP_OR_FAIL(c, dalloc(c->d_tau, (size_t)c->S * sizeof(double)));
  HIP_OR_FAIL(c, dalloc(c->ptab, (size_t)std::max<int64_t>(c->P, 1) * fea::kPairRow * sizeof(double)));
  HIP_OR_FAIL(c, dalloc(c->qW, (size_t)std::max<int64_t>(c->P, 1) * 45 * sizeof(double)));
  HIP_OR_FAIL(c, dalloc(c->qmask, (size_t)std::max<int64_t>(c->layout_len, 4)));
  c->ptab_current = false;
  HIP_OR_FAIL(c, dalloc(c->stab, (size_t)std::max<int64_t>(c->P, 1) * 40 * sizeof(double)));
  HIP_OR_FAIL(c, dalloc(c->wlay, std::max<int64_t>(c->layout_len, 4) * sizeof(uint16_t)));
  // padding slots never get a weight from the network: keep them zero
  HIP_OR_FAIL(c, hipMemsetAsync(c->wlay.p, 0, c->wlay.bytes, c->stream));
  // camera -> incident (pair, side) entries, in pair order
  const int N = c->N;
  c->cam_off.assign(N + 1, 0);
  for (int64_t k = 0; k < c->P; ++k) {
    c->cam_off[c->pair_i[k] + 1]++;
    c->cam_off[c->pair_j[k] + 1]++;
  }
  for (int i = 0; i < N; ++i) c->cam_off[i + 1] += c->cam_off[i];
  c->cam_ent.assign(2 * c->P, 0);
  std::vector<int32_t> fill(c->cam_off.begin(), c->cam_off.end() - 1);
  for (int64_t k = 0; k < c->P; ++k) {
    c->cam_ent[fill[c->pair_i[k]]++] = (int32_t)(2 * k);
    c->cam_ent[fill[c->pair_j[k]]++] = (int32_t)(2 * k + 1);
  }
  HIP_OR_FAIL(c, upload(c, c->d_pair_i, c->pair_i.data(), c->P));
  HIP_OR_FAIL(c, upload(c, c->d_pair_j, c->pair_j.data(), c->P));
  HIP_OR_FAIL(c, upload(c, c->d_cam_off, c->cam_off.data(), N + 1));
  c->tile_tuned = false;
  c->tile_cfg = (c->opt.tile_matches > 0) ? tile_cfg_for(c->opt.tile_matches, c->opt.tile_persistent == 1) : 0;
  HIP_OR_FAIL(c, reset_layout(c));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  reset_round_state(c);
  c->have_matches = true;
  return FEA_OK;
}

void rot6d_to_R_host(const double a[6], double R[9]) {
  const double n1 = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  const double b1[3] = {a[0] / n1, a[1] / n1, a[2] / n1};
  const double d = b1[0] * a[3] + b1[1] * a[4] + b1[2] * a[5];
  const double v[3] = {a[3] - d * b1[0], a[4] - d * b1[1], a[5] - d * b1[2]};
  const double n2 = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double b2[3] = {v[0] / n2, v[1] / n2, v[2] / n2};
  R[0] = b1[0]; R[3] = b1[1]; R[6] = b1[2];
  R[1] = b2[0]; R[4] = b2[1]; R[7] = b2[2];
  R[2] = b1[1] * b2[2] - b1[2] * b2[1];
  R[5] = b1[2] * b2[0] - b1[0] * b2[2];
  R[8] = b1[0] * b2[1] - b1[1] * b2[0];
}

// Marks the captured steps out of date (their kernel arguments changed); the
// executable graph is kept and updated in place by the next capture.
void drop_graph(fea_ctx* c) { c->graph_pcur = -1; }

void destroy_graph(fea_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_pcur = -1;
}

// Issues one step (per-match kernel, per-camera chain + Adam, shared-focal
// update); all step bookkeeping the kernels need lives on the device.
hipError_t issue_step(fea_ctx* c) {
  // quadratic form: the camera kernel evaluates each pair's form itself.
  // Per match: the pose table holds F at the current poses; after the
  // update it is rebuilt at the new ones for the next step.
  const bool quad = c->opt.inner_loop == 1;
  hipError_t e = quad ? hipSuccess : fea::launch_resgrad(c, true);
  if (e == hipSuccess) e = fea::launch_camgrad(c, 1, quad);
  if (e == hipSuccess && !c->all_single) e = fea::launch_focal_update(c);
  const int nx = c->pcur ^ 1;
  if (e == hipSuccess && !quad)
    e = fea::launch_pair_pose(c, c->R[nx].as<double>(), c->T[nx].as<double>(), c->Fc[nx].as<double>(), false);
  c->pcur = nx;
  c->ptab_current = !quad;
  return e;
}

// Captures kGraphSteps steps starting at the current pose parity; an existing
// executable graph of the same shape is updated with the new arguments
// (cheaper than instantiating again each round).
hipError_t capture_graph(fea_ctx* c) {
  const int p0 = c->pcur;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int k = 0; k < fea::kGraphSteps && le == hipSuccess; ++k) le = issue_step(c);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->stream, &g);
  c->pcur = p0;
  if (le != hipSuccess) e = le;
  bool updated = false;
  if (e == hipSuccess && c->graph) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(c->graph, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      updated = true;
    } else {
      (void)hipGetLastError();  // a refused update is not an error of the next call
      destroy_graph(c);
    }
  }
  if (e == hipSuccess && !updated) e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    destroy_graph(c);
    return e;
  }
  c->graph_pcur = p0;
  c->graph_gen = g_buffer_gen.load();
  return hipSuccess;
}

fea_status run_steps(fea_ctx* c, int32_t n_steps) {
  // the quadratic form's steps in one cooperative launch, where every step
  // is the camera kernel alone (no shared intrinsics group)
  if (n_steps >= 2 && c->opt.inner_loop == 1 && c->opt.persistent_steps && c->all_single && !c->timing &&
      c->stream != nullptr && c->n_items > 0) {
    const int blocks = fea::quad_steps_blocks(c);
    if (blocks > 0) {
      HIP_OR_FAIL(c, fea::launch_quad_steps(c, n_steps, blocks));
      c->last_quad_blocks = blocks;
      c->pcur ^= (n_steps & 1);
      c->ptab_current = false;
      c->step += n_steps;
      c->adam_t += n_steps;
      c->global_step += n_steps;
      if (c->opt.log_every > 0)
        c->n_logged = (int32_t)std::min<int64_t>(c->opt.max_log, c->global_step / c->opt.log_every);
      return FEA_OK;
    }
  }
  const bool graphs = c->opt.use_graphs && !c->timing && c->stream != nullptr && c->n_items > 0;
  if (n_steps > 0 && c->opt.inner_loop != 1 && !c->ptab_current)
    HIP_OR_FAIL(c, fea::launch_pair_pose(c, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                                         c->Fc[c->pcur].as<double>(), false));
  while (n_steps > 0) {
    if (graphs && n_steps >= fea::kGraphSteps) {
      if (!c->graph || c->graph_pcur != c->pcur || c->graph_gen != g_buffer_gen.load())
        HIP_OR_FAIL(c, capture_graph(c));
      HIP_OR_FAIL(c, hipGraphLaunch(c->graph, c->stream));
      c->ptab_current = c->opt.inner_loop != 1;
      n_steps -= fea::kGraphSteps;
      c->step += fea::kGraphSteps;
      c->adam_t += fea::kGraphSteps;
      c->global_step += fea::kGraphSteps;
    } else {
      HIP_OR_FAIL(c, issue_step(c));
      n_steps -= 1;
      c->step += 1;
      c->adam_t += 1;
      c->global_step += 1;
    }
  }
  if (c->opt.log_every > 0)
    c->n_logged = (int32_t)std::min<int64_t>(c->opt.max_log, c->global_step / c->opt.log_every);
  return FEA_OK;
}

// Host -> device copy of the step counters: Adam count `t` and global count
// `g` into the slots of the current parity, and the round's learning-rate
// factor.
hipError_t set_counters(fea_ctx* c, int64_t t, int64_t g) {
  fea::StepCounters h;
  std::memset(&h, 0, sizeof(h));
  h.adam_t[c->pcur] = t;
  h.global_t[c->pcur] = g;
  h.b1t[c->pcur] = std::pow(c->opt.beta1, (double)t);
  h.b2t[c->pcur] = std::pow(c->opt.beta2, (double)t);
  h.lr_scale = c->lr_scale;
  return stage_copy(c, c->counters.p, &h, sizeof(h));
}

// Stable compaction of the live layout into the other filtered buffer: the
// matches that pass the snapshot threshold (mask == nullptr; the pose table
// must hold this round's F_hat and tau) or whose sorted position is set in the
// device bit mask.  Leaves the new layout live with its per-pair lengths.
hipError_t compact_layout(fea_ctx* c, const uint32_t* mask) {
  hipError_t e = fea::launch_filter_count(c, mask);
  if (e != hipSuccess) return e;
  std::vector<int32_t> keep;
  if ((e = download(c, keep, c->item_keep, c->n_items)) != hipSuccess) return e;
  // new per-pair lengths, aligned offsets and per-item destinations; the
  // last item of each pair also gets the aligned end of the pair's run, up
  // to which it clears the padding
  std::vector<int64_t> new_len(c->P, 0), new_off(c->P, 0);
  std::vector<int32_t> base(2 * c->n_items, -1);
  for (int64_t n = 0; n < c->P; ++n)
    for (int32_t it = c->h_pair_item_off[n]; it < c->h_pair_item_off[n + 1]; ++it) new_len[n] += keep[it];
  int64_t off = 0;
  for (int64_t n = 0; n < c->P; ++n) {
    new_off[n] = off;
    int64_t run = off;
    for (int32_t it = c->h_pair_item_off[n]; it < c->h_pair_item_off[n + 1]; ++it) {
      base[2 * it] = (int32_t)run;
      run += keep[it];
    }
    off += (new_len[n] + fea::kAlign - 1) / fea::kAlign * fea::kAlign;
    if (c->h_pair_item_off[n + 1] > c->h_pair_item_off[n]) base[2 * (c->h_pair_item_off[n + 1] - 1) + 1] = (int32_t)off;
  }
  const int dst = (c->cur == 1) ? 2 : 1;
  if ((e = upload(c, c->item_base, base.data(), base.size())) != hipSuccess) return e;
  if ((e = fea::launch_filter_scatter(c, dst, mask)) != hipSuccess) return e;
  // no wait: later work on the stream sees the new layout in order, and the
  // host builds the work items meanwhile
  c->cur = dst;
  c->cur_len = new_len;
  c->phys_off = new_off;
  c->layout_len = off;
  return hipSuccess;
}

// The quadratic form's round: one pass over the whole layout tests the
// threshold on the matches the retained mask still holds, updates the mask,
// counts the survivors and sums their weighted outer products; the per-scene
// normalisers follow from the counts and W_n from the item sums.  The layout
// itself is never compacted (steps do not stream it).  The learned weights
// (if any) were computed on the layout before the pass.
hipError_t quad_round(fea_ctx* c) {
  hipError_t e = fea::launch_quad_build(c);
  if (e != hipSuccess) return e;
  if (c->scene_items_contiguous) {
    // per-scene counts and normalisers on the device: no host round trip
    if ((e = fea::launch_scene_z(c)) != hipSuccess) return e;
    c->host_z_stale = true;
    return fea::launch_quad_reduce(c, c->pair_item_off.as<int32_t>());
  }
  std::vector<int32_t> keep;
  if ((e = download(c, keep, c->item_keep, c->n_items)) != hipSuccess) return e;
  // a converged scene keeps its count (its items were not passed over)
  const bool frozen = c->opt.converge_deg > 0 && c->n_done > 0 && (int)c->Zs.size() == c->S &&
                      (int)c->scene_done_h.size() == c->S;
  std::vector<int64_t> zs(c->S, 0);
  for (int64_t it = 0; it < c->n_items; ++it) zs[c->pair_scene[c->h_item_pair[it]]] += keep[it];
  if ((int)c->Zs.size() != c->S) c->Zs.assign(c->S, 0);
  for (int sc = 0; sc < c->S; ++sc)
    if (!(frozen && c->scene_done_h[sc] != 0)) c->Zs[sc] = zs[sc];
  c->Z = 0;
  std::vector<float> inv(c->S, 0.f);
  for (int sc = 0; sc < c->S; ++sc) {
    c->Z += c->Zs[sc];
    inv[sc] = c->Zs[sc] > 0 ? (float)(1.0 / (double)c->Zs[sc]) : 0.f;
  }
  if ((e = upload(c, c->d_inv_z, inv.data(), c->S)) != hipSuccess) return e;
  if (c->learned_any) {
    std::vector<double> ws;
    if ((e = download(c, ws, c->item_wsum, c->n_items)) != hipSuccess) return e;
    std::vector<double> zw(c->S, 0.0);
    for (int64_t it = 0; it < c->n_items; ++it) zw[c->pair_scene[c->h_item_pair[it]]] += ws[it];
    if ((int)c->inv_zw_h.size() != c->S) c->inv_zw_h.assign(c->S, 0.f);
    for (int sc = 0; sc < c->S; ++sc)
      if (!(frozen && c->scene_done_h[sc] != 0)) c->inv_zw_h[sc] = zw[sc] > 0 ? (float)(1.0 / zw[sc]) : 0.f;
    if ((e = upload(c, c->d_inv_zw, c->inv_zw_h.data(), c->S)) != hipSuccess) return e;
  }
  c->host_z_stale = false;
  return fea::launch_quad_reduce(c, c->pair_item_off.as<int32_t>());
}

// Per-scene weighting mode of the round (chosen now, or kept as restored
// from a checkpoint) and, for scenes on learned weights, the network's weight
// of every retained match and 1 / (sum of weights).
hipError_t round_weights(fea_ctx* c, bool choose_mode) {
  hipError_t e = hipSuccess;
  if (choose_mode) {
    // the device holds the judge's verdicts; the host reads its copy of
    // them only once the copy has landed (no wait), so it may run the
    // network one round longer than needed -- the modes themselves come
    // from the device's flags
    if (c->judge_pending && hipEventQuery(c->judge_ev) == hipSuccess) {
      c->scene_learned_ok.assign(c->judge_ok_h, c->judge_ok_h + c->S);
      c->judge_pending = false;
    }
    const bool enabled = c->opt.weight_mode == 1 && c->have_mlp;
    c->learned_any = false;
    for (int sc = 0; sc < c->S; ++sc) {
      c->scene_mode[sc] = (enabled && c->scene_learned_ok[sc]) ? 1 : 0;
      c->learned_any = c->learned_any || c->scene_mode[sc];
    }
    e = fea::launch_choose_mode(c, enabled);
  } else {
    c->learned_any = false;
    for (int sc = 0; sc < c->S; ++sc) c->learned_any = c->learned_any || c->scene_mode[sc];
    e = upload(c, c->d_scene_mode, c->scene_mode.data(), c->S);
  }
  if (e != hipSuccess || !c->learned_any) return e;
  // the feature table reads the medians the round start left on the device
  if ((e = fea::launch_mlp_weights(c, c->mlp.as<float>(), c->wlay.as<unsigned short>(),
                                   c->item_wsum.as<double>(), nullptr)) != hipSuccess)
    return e;
  // quadratic form: the round's pass sums the survivors' weights itself
  if (c->opt.inner_loop == 1) return hipSuccess;
  std::vector<double> ws;
  if ((e = download(c, ws, c->item_wsum, c->n_items)) != hipSuccess) return e;
  std::vector<double> zw(c->S, 0.0);
  for (int64_t it = 0; it < c->n_items; ++it) zw[c->pair_scene[c->h_item_pair[it]]] += ws[it];
  c->inv_zw_h.assign(c->S, 0.f);
  for (int sc = 0; sc < c->S; ++sc) c->inv_zw_h[sc] = zw[sc] > 0 ? (float)(1.0 / zw[sc]) : 0.f;
  return upload(c, c->d_inv_zw, c->inv_zw_h.data(), c->S);
}

// sync: wait for the round's set-up work before returning (the solver's own
// rounds do not, so that graph capture and the host's item building overlap
// the device's compaction).
fea_status begin_round(fea_ctx* c, double tau_px, bool sync) {
  const size_t N = c->N;
  // a scene whose parameters, poses or loss went non-finite in the round
  // that just ended gets its snapshot back and stops
  if (c->round >= 0) HIP_OR_FAIL(c, fea::launch_guard(c, c->round + 1));
  if (c->opt.converge_deg > 0 && c->round >= 0) {
    // per-scene convergence over the round that just ended (before its
    // snapshot is replaced); a scene can converge only while the threshold
    // schedule stays put
    HIP_OR_FAIL(c, fea::launch_scene_converge(c, tau_px == c->prev_tau_px, c->round + 1));
    HIP_OR_FAIL(c, download(c, c->scene_done_h, c->d_scene_done, (size_t)c->S));
    c->n_done = 0;
    for (int sc = 0; sc < c->S; ++sc) c->n_done += c->scene_done_h[sc] != 0 ? 1 : 0;
  }
  c->prev_tau_px = tau_px;
  // snapshot and its history (learned features), round parameters for the
  // judge's restore, and (new objective) fresh Adam moments -- one kernel
  const bool zero = c->opt.reset_moments || c->round < 0;
  HIP_OR_FAIL(c, fea::launch_round_start(c, c->round >= 0, c->round < 0, zero));
  if (zero) c->adam_t = 0;
  if (c->max_scene_cams <= fea::kMaxSceneCams) {
    // thresholds and focal-length medians on the device: no host round trip
    HIP_OR_FAIL(c, fea::launch_scene_tau(c, tau_px, c->round < 0));
    c->host_tau_stale = true;
  } else {
    HIP_OR_FAIL(c, refresh_round_host(c));
    std::vector<double> fnow;
    HIP_OR_FAIL(c, download(c, fnow, c->Fc[c->pcur], N));
    // threshold per scene: tau_px over the scene's median focal length
    std::vector<std::vector<double>> fs(c->S);
    for (size_t i = 0; i < N; ++i) fs[c->cam_scene[i]].push_back(fnow[i]);
    if (c->round < 0) {
      c->fbar_hist.assign(3 * c->S, 0.0);
      for (int sc = 0; sc < c->S; ++sc)
        for (int k = 0; k < 3; ++k) c->fbar_hist[k * c->S + sc] = fs[sc].empty() ? 1.0 : median(fs[sc]);
    } else {
      for (int sc = 0; sc < c->S; ++sc) {
        c->fbar_hist[2 * c->S + sc] = c->fbar_hist[c->S + sc];
        c->fbar_hist[c->S + sc] = c->fbar_hist[sc];
        c->fbar_hist[sc] = fs[sc].empty() ? 1.0 : median(fs[sc]);
      }
    }
    c->taus.assign(c->S, std::numeric_limits<double>::infinity());
    if (!std::isinf(tau_px))
      for (int sc = 0; sc < c->S; ++sc) c->taus[sc] = tau_px / (fs[sc].empty() ? 1.0 : median(fs[sc]));
    HIP_OR_FAIL(c, upload(c, c->d_tau, c->taus.data(), c->S));
    HIP_OR_FAIL(c, upload_fbar(c));
    c->tau = c->taus.empty() ? 0.0 : c->taus[0];
  }
  const bool quad = c->opt.inner_loop == 1;
  if (quad) {
    // the full layout stays; a mask marks the retained matches.  The
    // round's weighting modes and learned weights come first, as the fused
    // pass applies them.
    if (!c->tile_tuned) {
      HIP_OR_FAIL(c, choose_tile(c));
      HIP_OR_FAIL(c, build_items(c));
      drop_graph(c);
    }
    if (c->round < 0) HIP_OR_FAIL(c, fea::launch_mask_init(c));
    HIP_OR_FAIL(c, round_weights(c, true));
    HIP_OR_FAIL(c, fea::launch_pair_pose(c, c->Rh.as<double>(), c->Th.as<double>(), c->Fh.as<double>(), true));
    HIP_OR_FAIL(c, quad_round(c));
  } else {
    // pose table at the snapshot (F_hat, principal points, tau), then the
    // survivors compacted into the other buffer
    HIP_OR_FAIL(c, fea::launch_pair_pose(c, c->Rh.as<double>(), c->Th.as<double>(), c->Fh.as<double>(), true));
    HIP_OR_FAIL(c, compact_layout(c, nullptr));
    HIP_OR_FAIL(c, upload_scene_z(c));
    HIP_OR_FAIL(c, choose_tile(c));
    HIP_OR_FAIL(c, build_items(c));
  }
  c->lr_scale = std::pow(c->opt.lr_decay, (double)(c->round + 1));
  HIP_OR_FAIL(c, set_counters(c, c->adam_t, c->global_step));
  // per match, the layout changed: recapture on the next run of steps.  The
  // quadratic form's steps read only per-pair forms and device counters, so
  // its captured graph stays valid across rounds.
  if (!quad) drop_graph(c);
  if (!quad) {
    // learned weights of this round's retained matches, then the pose
    // table at the current poses with this round's normalisers
    HIP_OR_FAIL(c, round_weights(c, true));
    HIP_OR_FAIL(c, fea::launch_pair_pose(c, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                                         c->Fc[c->pcur].as<double>(), false));
  }
  if (sync) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->round += 1;
  c->step = 0;
  return FEA_OK;
}


constexpr char kStateMagic[8] = {'F', 'E', 'A', 'S', 'T', 'A', 'T', 'E'};
constexpr int32_t kStateVersion = 2;

// Fixed header of a checkpoint; the sections listed in state_sections and
// the retained-match bit mask follow it.
struct StateHdr {
  char magic[8];
  int32_t version, N, G, S;
  int64_t P, M;
  uint64_t structure;  // hash of the loaded problem's structure
  fea_options opt;
  int32_t round, step, n_logged, fallbacks, tile_cfg, pcur, learned_any, have_mlp;
  int64_t adam_t, global_step;
  double tau, lr_scale;
  double prev_tau_px;  // threshold of the last round begun (early exit)
};

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  for (size_t k = 0; k < n; ++k) {
    h ^= b[k];
    h *= 1099511628211ull;
  }
  return h;
}

// Pair table, segment ranges, scene partition, intrinsics groups and the
// sorted order of the matches: a checkpoint only fits a context that loaded
// the same problem.
hipError_t structure_hash(fea_ctx* c, uint64_t* out) {
  std::vector<int32_t> perm;
  hipError_t e = download(c, perm, c->perm, (size_t)c->M);
  if (e != hipSuccess) return e;
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, c->pair_i.data(), c->pair_i.size() * sizeof(int32_t));
  h = fnv1a(h, c->pair_j.data(), c->pair_j.size() * sizeof(int32_t));
  h = fnv1a(h, c->seg_off.data(), c->seg_off.size() * sizeof(int64_t));
  h = fnv1a(h, c->cam_scene.data(), c->cam_scene.size() * sizeof(int32_t));
  h = fnv1a(h, c->group.data(), c->group.size() * sizeof(int32_t));
  h = fnv1a(h, perm.data(), perm.size() * sizeof(int32_t));
  *out = h;
  return hipSuccess;
}

// Device arrays of the solver state, in checkpoint order, with their sizes.
std::vector<std::pair<DBuf*, size_t>> state_sections(fea_ctx* c) {
  const size_t N = c->N, G = c->G, d = sizeof(double);
  const int p = c->pcur;
  return {{&c->a6, 6 * N * d},  {&c->tp, 3 * N * d},   {&c->logf, G * d},   {&c->m_a6, 6 * N * d},
          {&c->v_a6, 6 * N * d}, {&c->m_t, 3 * N * d},  {&c->v_t, 3 * N * d}, {&c->m_f, G * d},
          {&c->v_f, G * d},      {&c->R[p], 9 * N * d}, {&c->T[p], 3 * N * d}, {&c->Fc[p], N * d},
          {&c->Rh, 9 * N * d},   {&c->Th, 3 * N * d},   {&c->Fh, N * d},      {&c->Rh1, 9 * N * d},
          {&c->Th1, 3 * N * d},  {&c->Fh1, N * d},      {&c->Rh2, 9 * N * d}, {&c->Th2, 3 * N * d},
          {&c->Fh2, N * d},      {&c->a6h, 6 * N * d},  {&c->tph, 3 * N * d}, {&c->logfh, G * d},
          {&c->counters, sizeof(fea::StepCounters)}, {&c->qW, (size_t)c->P * 45 * d},
          {&c->d_scene_done, (size_t)c->S * sizeof(int32_t)}};
}

size_t state_bytes(fea_ctx* c) {
  size_t n = sizeof(StateHdr);
  for (auto& sec : state_sections(c)) n += sec.second;
  const size_t S = c->S;
  n += S * sizeof(double) + 3 * S * sizeof(double) + 2 * S * sizeof(int32_t) + 4 * S * sizeof(double);
  n += (size_t)((c->M + 31) / 32) * sizeof(uint32_t);
  n += S * sizeof(float);  // 1 / sum of learned weights per scene
  return n;
}

template <class T>
void put(uint8_t*& w, const T* src, size_t n) {
  std::memcpy(w, src, n * sizeof(T));
  w += n * sizeof(T);
}

template <class T>
void take(const uint8_t*& r, T* dst, size_t n) {
  std::memcpy(dst, r, n * sizeof(T));
  r += n * sizeof(T);
}

}  // namespace

extern "C" {

int32_t fea_version(void) { return FEA_VERSION; }

const char* fea_status_string(fea_status s) {
  switch (s) {
    case FEA_OK: return "ok";
    case FEA_EINVAL: return "invalid argument";
    case FEA_ENOMEM: return "out of memory";
    case FEA_EDEVICE: return "HIP device error";
    case FEA_ESTATE: return "call out of order";
    case FEA_EDEGENERATE: return "degenerate camera pair (coincident centres)";
    case FEA_ENONFINITE: return "non-finite input";
  }
  return "unknown status";
}

fea_status fea_check_options(const fea_options* opt, char* why, size_t why_len) {
  std::string msg;
  const bool ok = opt != nullptr && options_valid(opt, &msg);
  if (!opt) msg = "null options";
  if (why && why_len > 0) {
    const size_t n = ok ? 0 : std::min(msg.size(), why_len - 1);
    std::memcpy(why, msg.data(), n);
    why[n] = '\0';
  }
  return ok ? FEA_OK : FEA_EINVAL;
}

fea_status fea_default_options(fea_options* o) {
  if (!o) return FEA_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->rounds = 20;
  o->iters_per_round = 50;
  o->tau_px_init = 128.0;
  o->tau_px_min = 4.0;
  o->tau_decay = 0.5;
  o->delta = 1e-4;
  o->lr_rot = 3e-3;
  o->lr_t = 4e-2;
  o->lr_logf = 1e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->adam_eps = 1e-12;
  o->optimize_focal = 1;
  o->gauge_normalize = 1;
  o->log_every = 0;
  o->max_log = 0;
  o->lr_decay = 0.9;
  o->reset_moments = 1;
  o->tile_matches = 0;
  o->use_graphs = 1;
  o->weight_mode = 0;
  o->inner_loop = 0;
  o->persistent_steps = 0;
  return FEA_OK;
}

fea_status fea_create(fea_ctx** out, int32_t device, const fea_options* opt, void* hip_stream) {
  if (!out) return FEA_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FEA_EDEVICE;
  if (device < 0 || device >= ndev) return FEA_EINVAL;
  fea_options o;
  if (opt) {
    o = *opt;
    std::string why;
    if (!options_valid(&o, &why)) return FEA_EINVAL;
  } else {
    fea_default_options(&o);
  }
  fea_ctx* c = new (std::nothrow) fea_ctx();
  if (!c) return FEA_ENOMEM;
  c->device = device;
  c->opt = o;
  DeviceGuard g(device);
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n_cu < 1)
    n_cu = 256;
  c->n_cu = n_cu;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return FEA_EDEVICE;
    }
    c->own_stream = true;
  }
  if (dalloc(c->errflag, sizeof(int)) != hipSuccess || dalloc(c->loss, sizeof(double)) != hipSuccess ||
      dalloc(c->wait_state, 2 * sizeof(unsigned)) != hipSuccess) {
    fea_destroy(c);
    return FEA_ENOMEM;
  }
  if (hipMemsetAsync(c->wait_state.p, 0, 2 * sizeof(unsigned), c->stream) != hipSuccess) {
    fea_destroy(c);
    return FEA_EDEVICE;
  }
  // a device-wide wait between two steps gives up after half a second
  int clock_khz = 0;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || clock_khz < 1)
    clock_khz = 100000;
  c->wall_clock_khz = clock_khz;
  *out = c;
  return FEA_OK;
}

void fea_destroy(fea_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (DBuf* b : all_bufs(c)) dfree(*b);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  destroy_graph(c);
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->loss_log) (void)hipHostFree(c->loss_log);
  if (c->inl_log) (void)hipHostFree(c->inl_log);
  if (c->judge_ok_h) (void)hipHostFree(c->judge_ok_h);
  if (c->judge_ev) (void)hipEventDestroy(c->judge_ev);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* fea_last_error(const fea_ctx* c) { return c ? c->err.c_str() : "null context"; }

fea_status fea_set_options(fea_ctx* c, const fea_options* opt) {
  if (!c || !opt) return fail(c, FEA_EINVAL, "null argument");
  std::string why;
  if (!options_valid(opt, &why)) return fail(c, FEA_EINVAL, why);
  if (opt->inner_loop != c->opt.inner_loop && c->round >= 0)
    return fail(c, FEA_ESTATE, "inner_loop can change only before the first round (or after fea_init_poses)");
  if (opt->tile_matches != c->opt.tile_matches || opt->inner_loop != c->opt.inner_loop) c->tile_tuned = false;
  if (opt->log_every > 0 && opt->max_log > 0 && c->have_intr) {
    DeviceGuard g(c->device);
    HIP_OR_FAIL(c, dalloc(c->logR, (size_t)opt->max_log * 9 * c->N * sizeof(double)));
  }
  c->opt = *opt;
  drop_graph(c);
  return FEA_OK;
}

fea_status fea_load_intrinsics(fea_ctx* c, int32_t n_cams, const double* f, const double* cx, const double* cy,
                               const int32_t* intr_group) {
  if (!c) return FEA_EINVAL;
  if (n_cams < 2 || n_cams > 65535) return fail(c, FEA_EINVAL, "n_cams must be in [2, 65535]");
  if (!f || !cx || !cy) return fail(c, FEA_EINVAL, "f, cx and cy are required");
  DeviceGuard g(c->device);
  for (int i = 0; i < n_cams; ++i) {
    if (!std::isfinite(f[i]) || !std::isfinite(cx[i]) || !std::isfinite(cy[i]))
      return fail(c, FEA_ENONFINITE, "non-finite intrinsics");
    if (!(f[i] > 0)) return fail(c, FEA_EINVAL, "focal lengths must be > 0");
    if (intr_group && (intr_group[i] < 0 || intr_group[i] >= n_cams))
      return fail(c, FEA_EINVAL, "intrinsics group id outside [0, n_cams)");
  }
  c->have_intr = c->have_matches = c->have_poses = false;
  c->N = n_cams;
  c->S = 1;
  c->cam_scene.assign(n_cams, 0);
  c->gauge_c.assign(3, 0.0);
  c->gauge_s.assign(1, 1.0);
  c->f_in.assign(f, f + n_cams);
  c->cx.assign(cx, cx + n_cams);
  c->cy.assign(cy, cy + n_cams);
  c->group.resize(n_cams);
  int G = 0;
  for (int i = 0; i < n_cams; ++i) {
    c->group[i] = intr_group ? intr_group[i] : i;
    G = std::max(G, c->group[i] + 1);
  }
  c->G = G;
  c->grp_off.assign(G + 1, 0);
  for (int i = 0; i < n_cams; ++i) c->grp_off[c->group[i] + 1]++;
  for (int k = 0; k < G; ++k) c->grp_off[k + 1] += c->grp_off[k];
  c->all_single = true;
  for (int k = 0; k < G; ++k)
    if (c->grp_off[k + 1] - c->grp_off[k] > 1) c->all_single = false;
  c->grp_cams.assign(n_cams, 0);
  std::vector<int32_t> fill(c->grp_off.begin(), c->grp_off.end() - 1);
  for (int i = 0; i < n_cams; ++i) c->grp_cams[fill[c->group[i]]++] = i;
  HIP_OR_FAIL(c, alloc_scene_arrays(c));
  HIP_OR_FAIL(c, dalloc(c->counters, sizeof(fea::StepCounters)));
  HIP_OR_FAIL(c, dalloc(c->mlp, fea::kMlpParams * sizeof(float)));
  HIP_OR_FAIL(c, hipMemsetAsync(c->mlp.p, 0, c->mlp.bytes, c->stream));
  HIP_OR_FAIL(c, upload(c, c->d_cx, c->cx.data(), n_cams));
  HIP_OR_FAIL(c, upload(c, c->d_cy, c->cy.data(), n_cams));
  HIP_OR_FAIL(c, upload(c, c->d_group, c->group.data(), n_cams));
  HIP_OR_FAIL(c, upload(c, c->d_grp_off, c->grp_off.data(), G + 1));
  HIP_OR_FAIL(c, upload(c, c->d_grp_cams, c->grp_cams.data(), n_cams));
  const size_t N = n_cams;
  DBuf* per_cam[] = {&c->a6, &c->m_a6, &c->v_a6, &c->a6h};
  for (DBuf* b : per_cam) HIP_OR_FAIL(c, dalloc(*b, 6 * N * sizeof(double)));
  DBuf* per_cam3[] = {&c->tp, &c->m_t, &c->v_t, &c->T[0], &c->T[1], &c->Th, &c->gt, &c->Te, &c->Th1, &c->Th2,
                      &c->tph};
  for (DBuf* b : per_cam3) HIP_OR_FAIL(c, dalloc(*b, 3 * N * sizeof(double)));
  DBuf* per_cam9[] = {&c->R[0], &c->R[1], &c->Rh, &c->gR, &c->Re, &c->Rh1, &c->Rh2};
  for (DBuf* b : per_cam9) HIP_OR_FAIL(c, dalloc(*b, 9 * N * sizeof(double)));
  DBuf* per_cam1[] = {&c->Fc[0], &c->Fc[1], &c->Fh, &c->gf, &c->loss_cam, &c->Fe, &c->Fh1, &c->Fh2};
  for (DBuf* b : per_cam1) HIP_OR_FAIL(c, dalloc(*b, N * sizeof(double)));
  DBuf* per_grp[] = {&c->logf, &c->m_f, &c->v_f, &c->logfh};
  for (DBuf* b : per_grp) HIP_OR_FAIL(c, dalloc(*b, (size_t)G * sizeof(double)));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->have_intr = true;
  return FEA_OK;
}

fea_status fea_set_scenes(fea_ctx* c, int32_t n_scenes, const int32_t* cam_scene) {
  if (!c) return FEA_EINVAL;
  if (!c->have_intr) return fail(c, FEA_ESTATE, "load intrinsics first");
  if (n_scenes < 1 || n_scenes > c->N) return fail(c, FEA_EINVAL, "n_scenes must be in [1, n_cams]");
  if (n_scenes > 1 && !cam_scene) return fail(c, FEA_EINVAL, "cam_scene is required");
  std::vector<int32_t> cs(c->N, 0);
  for (int i = 0; i < c->N && cam_scene; ++i) {
    if (cam_scene[i] < 0 || cam_scene[i] >= n_scenes) return fail(c, FEA_EINVAL, "scene id outside [0, n_scenes)");
    cs[i] = cam_scene[i];
  }
  for (int g = 0; g < c->G; ++g)
    for (int k = c->grp_off[g] + 1; k < c->grp_off[g + 1]; ++k)
      if (cs[c->grp_cams[k]] != cs[c->grp_cams[c->grp_off[g]]])
        return fail(c, FEA_EINVAL, "an intrinsics group spans several scenes");
  c->have_matches = c->have_poses = false;
  c->S = n_scenes;
  c->cam_scene = cs;
  c->gauge_c.assign(3 * n_scenes, 0.0);
  c->gauge_s.assign(n_scenes, 1.0);
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, alloc_scene_arrays(c));
  return FEA_OK;
}

fea_status fea_get_scene_stats(fea_ctx* c, double* loss, int64_t* retained, double* gauge_center,
                               double* gauge_scale, int32_t* learned) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, refresh_round_host(c));
  HIP_OR_FAIL(c, refresh_learned_host(c));
  if (loss) {
    std::vector<double> lc;
    HIP_OR_FAIL(c, download(c, lc, c->loss_cam, c->N));
    for (int s = 0; s < c->S; ++s) loss[s] = 0.0;
    for (int i = 0; i < c->N; ++i) loss[c->cam_scene[i]] += lc[i];
  }
  for (int s = 0; s < c->S; ++s) {
    if (retained) retained[s] = c->Zs.empty() ? 0 : c->Zs[s];
    if (gauge_center)
      for (int k = 0; k < 3; ++k) gauge_center[3 * s + k] = c->gauge_c[3 * s + k];
    if (gauge_scale) gauge_scale[s] = c->gauge_s[s];
    if (learned) learned[s] = c->scene_mode.empty() ? 0 : (c->scene_mode[s] && c->scene_learned_ok[s]);
  }
  return FEA_OK;
}

fea_status fea_get_judge_losses(fea_ctx* c, double* loss_snapshot, double* loss_end) {
  if (!c) return FEA_EINVAL;
  DeviceGuard g(c->device);
  for (int k = 0; k < 2; ++k) {
    double* out = k == 0 ? loss_snapshot : loss_end;
    const DBuf& src = k == 0 ? c->d_judge_l0 : c->d_judge_l1;
    if (!out) continue;
    std::vector<double> h;
    if (c->judge_written) HIP_OR_FAIL(c, download(c, h, src, (size_t)c->S));
    for (int s = 0; s < c->S; ++s) out[s] = h.empty() ? 0.0 : h[s];
  }
  return FEA_OK;
}

fea_status fea_load_matches(fea_ctx* c, int64_t n, const float* x1, const float* y1, const float* x2,
                            const float* y2, const int32_t* cam1, const int32_t* cam2) {
  if (!c) return FEA_EINVAL;
  if (!c->have_intr) return fail(c, FEA_ESTATE, "load intrinsics first");
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, FEA_EINVAL, "n must be in [0, 2^31)");
  if (n > 0 && (!x1 || !y1 || !x2 || !y2 || !cam1 || !cam2)) return fail(c, FEA_EINVAL, "null match array");
  DeviceGuard g(c->device);
  DBuf t[6];
  struct Free {
    DBuf* t;
    ~Free() {
      for (int k = 0; k < 6; ++k) dfree(t[k]);
    }
  } fr{t};
  const void* src[6] = {x1, y1, x2, y2, cam1, cam2};
  for (int k = 0; k < 6; ++k) {
    HIP_OR_FAIL(c, dalloc(t[k], std::max<int64_t>(n, 1) * 4));
    if (n > 0) HIP_OR_FAIL(c, hipMemcpyAsync(t[k].p, src[k], n * 4, hipMemcpyHostToDevice, c->stream));
  }
  fea_status s = load_matches_common(c, n, t[0].as<float>(), t[1].as<float>(), t[2].as<float>(),
                                     t[3].as<float>(), t[4].as<int32_t>(), t[5].as<int32_t>());
  (void)hipStreamSynchronize(c->stream);
  return s;
}

fea_status fea_load_matches_device(fea_ctx* c, int64_t n, const float* x1, const float* y1, const float* x2,
                                   const float* y2, const int32_t* cam1, const int32_t* cam2) {
  if (!c) return FEA_EINVAL;
  if (!c->have_intr) return fail(c, FEA_ESTATE, "load intrinsics first");
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, FEA_EINVAL, "n must be in [0, 2^31)");
  if (n > 0 && (!x1 || !y1 || !x2 || !y2 || !cam1 || !cam2)) return fail(c, FEA_EINVAL, "null match array");
  DeviceGuard g(c->device);
  return load_matches_common(c, n, x1, y1, x2, y2, cam1, cam2);
}

namespace {

// Validates caller-frame poses, writes the 6D parameters, the derived R/t
// (internal gauge) and, if f is given, log f per group and f per camera.
// With set_gauge the gauge (centre, scale) is recomputed from these poses.
fea_status put_poses(fea_ctx* c, const double* R, const double* t, const double* f, bool set_gauge) {
  const int N = c->N;
  c->ptab_current = false;
  std::vector<double> tt(t, t + 3 * N);
  for (int i = 0; i < 9 * N; ++i)
    if (!std::isfinite(R[i])) return fail(c, FEA_ENONFINITE, "non-finite rotation");
  for (int i = 0; i < 3 * N; ++i)
    if (!std::isfinite(t[i])) return fail(c, FEA_ENONFINITE, "non-finite translation");
  if (f)
    for (int i = 0; i < N; ++i)
      if (!std::isfinite(f[i]) || !(f[i] > 0)) return fail(c, FEA_EINVAL, "focal lengths must be finite and > 0");
  std::vector<double> a6(6 * N), Rc(9 * N);
  for (int i = 0; i < N; ++i) {
    const double* r = R + 9 * i;
    const double det = r[0] * (r[4] * r[8] - r[5] * r[7]) - r[1] * (r[3] * r[8] - r[5] * r[6]) +
                       r[2] * (r[3] * r[7] - r[4] * r[6]);
    if (!(det > 0)) return fail(c, FEA_EINVAL, "rotations must have det > 0");
    for (int k = 0; k < 3; ++k) {
      a6[6 * i + k] = r[3 * k];
      a6[6 * i + 3 + k] = r[3 * k + 1];
    }
    rot6d_to_R_host(&a6[6 * i], &Rc[9 * i]);
  }
  // camera centres o = -R^T t
  std::vector<double> o(3 * N);
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k)
      o[3 * i + k] = -(Rc[9 * i + k] * tt[3 * i] + Rc[9 * i + 3 + k] * tt[3 * i + 1] + Rc[9 * i + 6 + k] * tt[3 * i + 2]);
  std::vector<double> base(c->P);
  double maxd = 0.0;
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) maxd = std::max(maxd, std::fabs(o[3 * i + k]));
  for (int64_t n = 0; n < c->P; ++n) {
    const double* oi = &o[3 * c->pair_i[n]];
    const double* oj = &o[3 * c->pair_j[n]];
    const double d = std::sqrt((oi[0] - oj[0]) * (oi[0] - oj[0]) + (oi[1] - oj[1]) * (oi[1] - oj[1]) +
                               (oi[2] - oj[2]) * (oi[2] - oj[2]));
    if (!(d > 1e-12 * std::max(1.0, maxd))) return fail(c, FEA_EDEGENERATE, "two matched cameras share a centre");
    base[n] = d;
  }
  if (set_gauge) {
    // per scene: centres to mean 0, median matched-pair baseline to 1
    c->gauge_c.assign(3 * c->S, 0.0);
    c->gauge_s.assign(c->S, 1.0);
    if (c->opt.gauge_normalize) {
      std::vector<int64_t> cnt(c->S, 0);
      for (int i = 0; i < N; ++i) {
        const int sc = c->cam_scene[i];
        cnt[sc] += 1;
        for (int k = 0; k < 3; ++k) c->gauge_c[3 * sc + k] += o[3 * i + k];
      }
      for (int sc = 0; sc < c->S; ++sc)
        for (int k = 0; k < 3; ++k) c->gauge_c[3 * sc + k] /= std::max<int64_t>(cnt[sc], 1);
      std::vector<std::vector<double>> bs(c->S);
      for (int64_t n = 0; n < c->P; ++n) bs[c->pair_scene[n]].push_back(base[n]);
      for (int sc = 0; sc < c->S; ++sc) {
        const double m = bs[sc].empty() ? 1.0 : median(bs[sc]);
        c->gauge_s[sc] = (m > 0) ? m : 1.0;
      }
    }
  }
  for (int i = 0; i < N; ++i) {
    const int sc = c->cam_scene[i];
    double on[3];
    for (int k = 0; k < 3; ++k) on[k] = (o[3 * i + k] - c->gauge_c[3 * sc + k]) / c->gauge_s[sc];
    for (int k = 0; k < 3; ++k)
      tt[3 * i + k] = -(Rc[9 * i + 3 * k] * on[0] + Rc[9 * i + 3 * k + 1] * on[1] + Rc[9 * i + 3 * k + 2] * on[2]);
  }
  HIP_OR_FAIL(c, upload(c, c->a6, a6.data(), 6 * N));
  HIP_OR_FAIL(c, upload(c, c->tp, tt.data(), 3 * N));
  HIP_OR_FAIL(c, upload(c, c->R[c->pcur], Rc.data(), 9 * N));
  HIP_OR_FAIL(c, upload(c, c->T[c->pcur], tt.data(), 3 * N));
  if (f) {
    // one focal length per group: geometric mean of its cameras' values
    std::vector<double> logf(c->G, 0.0), fc(N);
    for (int gi = 0; gi < c->G; ++gi) {
      const int b = c->grp_off[gi], e = c->grp_off[gi + 1];
      for (int k = b; k < e; ++k) logf[gi] += std::log(f[c->grp_cams[k]]);
      if (e > b) logf[gi] /= (e - b);
    }
    for (int i = 0; i < N; ++i) fc[i] = std::exp(logf[c->group[i]]);
    HIP_OR_FAIL(c, upload(c, c->Fc[c->pcur], fc.data(), N));
    HIP_OR_FAIL(c, upload(c, c->logf, logf.data(), c->G));
  }
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return FEA_OK;
}

}  // namespace

fea_status fea_init_poses(fea_ctx* c, const double* R, const double* t) {
  if (!c) return FEA_EINVAL;
  if (!c->have_matches) return fail(c, FEA_ESTATE, "load matches first");
  if (!R || !t) return fail(c, FEA_EINVAL, "R and t are required");
  DeviceGuard g(c->device);
  c->have_poses = false;
  c->pcur = 0;
  fea_status s = put_poses(c, R, t, c->f_in.data(), true);
  if (s != FEA_OK) return s;
  HIP_OR_FAIL(c, reset_layout(c));
  // the per-camera loss shares are read by the non-finite guard before any
  // step may have written them
  HIP_OR_FAIL(c, hipMemsetAsync(c->loss_cam.p, 0, c->loss_cam.bytes, c->stream));
  if (c->opt.log_every > 0 && c->opt.max_log > 0)
    HIP_OR_FAIL(c, dalloc(c->logR, (size_t)c->opt.max_log * 9 * c->N * sizeof(double)));
  drop_graph(c);
  reset_round_state(c);
  HIP_OR_FAIL(c, clear_convergence(c));
  c->adam_t = 0;
  HIP_OR_FAIL(c, set_counters(c, 0, 0));
  c->scene_mode.assign(c->S, 0);
  c->learned_any = false;
  HIP_OR_FAIL(c, reset_judge(c));
  c->have_poses = true;
  return FEA_OK;
}

fea_status fea_set_poses(fea_ctx* c, const double* R, const double* t, const double* f) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  if (!R || !t) return fail(c, FEA_EINVAL, "R and t are required");
  DeviceGuard g(c->device);
  return put_poses(c, R, t, f, false);
}

fea_status fea_begin_round(fea_ctx* c, double tau_px) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  if (std::isnan(tau_px) || !(tau_px > 0)) return fail(c, FEA_EINVAL, "tau_px must be > 0 (or INFINITY)");
  DeviceGuard g(c->device);
  fea_status s = begin_round(c, tau_px, true);
  if (s != FEA_OK) return s;
  return check_nonfinite(c);
}

fea_status fea_residual_grad(fea_ctx* c, double* loss_dev, double* gR_dev, double* gt_dev, double* gf_dev) {
  if (!c) return FEA_EINVAL;
  if (c->round < 0) return fail(c, FEA_ESTATE, "begin a round first");
  DeviceGuard g(c->device);
  const bool quad = c->opt.inner_loop == 1;
  if (!quad) {
    if (!c->ptab_current)
      HIP_OR_FAIL(c, fea::launch_pair_pose(c, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                                           c->Fc[c->pcur].as<double>(), false));
    HIP_OR_FAIL(c, fea::launch_resgrad(c));
  }
  HIP_OR_FAIL(c, fea::launch_camgrad(c, 0, quad));
  HIP_OR_FAIL(c, fea::launch_loss_sum(c));
  const size_t N = c->N;
  if (loss_dev)
    HIP_OR_FAIL(c, hipMemcpyAsync(loss_dev, c->loss.p, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (gR_dev)
    HIP_OR_FAIL(c, hipMemcpyAsync(gR_dev, c->gR.p, 9 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (gt_dev)
    HIP_OR_FAIL(c, hipMemcpyAsync(gt_dev, c->gt.p, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (gf_dev)
    HIP_OR_FAIL(c, hipMemcpyAsync(gf_dev, c->gf.p, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return FEA_OK;
}

fea_status fea_get_params_dev(fea_ctx* c, double* a6_dev, double* t_dev, double* logf_dev) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  DeviceGuard g(c->device);
  const size_t N = c->N;
  if (a6_dev)
    HIP_OR_FAIL(c, hipMemcpyAsync(a6_dev, c->a6.p, 6 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (t_dev)
    HIP_OR_FAIL(c, hipMemcpyAsync(t_dev, c->tp.p, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (logf_dev)
    HIP_OR_FAIL(c, hipMemcpyAsync(logf_dev, c->logf.p, (size_t)c->G * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream));
  return FEA_OK;
}

fea_status fea_set_params_dev(fea_ctx* c, const double* a6_dev, const double* t_dev, const double* logf_dev) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  if (!a6_dev || !t_dev || !logf_dev) return fail(c, FEA_EINVAL, "null device array");
  DeviceGuard g(c->device);
  const size_t N = c->N, d = sizeof(double);
  const int p = c->pcur;
  HIP_OR_FAIL(c, fea::launch_params_to_pose(c, a6_dev, t_dev, logf_dev));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->a6.p, a6_dev, 6 * N * d, hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->tp.p, t_dev, 3 * N * d, hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->logf.p, logf_dev, (size_t)c->G * d, hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->R[p].p, c->Re.p, 9 * N * d, hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->T[p].p, c->Te.p, 3 * N * d, hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->Fc[p].p, c->Fe.p, N * d, hipMemcpyDeviceToDevice, c->stream));
  c->ptab_current = false;
  return FEA_OK;
}

fea_status fea_loss_dev(fea_ctx* c, const double* a6_dev, const double* t_dev, const double* logf_dev,
                        double* loss_dev) {
  if (!c) return FEA_EINVAL;
  if (c->round < 0) return fail(c, FEA_ESTATE, "begin a round first");
  if (!a6_dev || !t_dev || !logf_dev || !loss_dev) return fail(c, FEA_EINVAL, "null device array");
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, fea::launch_params_to_pose(c, a6_dev, t_dev, logf_dev));
  HIP_OR_FAIL(c, fea::launch_resgrad_at(c, c->tile_cfg, c->Re.as<double>(), c->Te.as<double>(),
                                        c->Fe.as<double>(), true, false));
  HIP_OR_FAIL(c, fea::launch_item_loss(c, loss_dev));
  return FEA_OK;
}

fea_status fea_adjoint_dev(fea_ctx* c, const double* a6_dev, const double* t_dev, const double* logf_dev,
                           const double* gout_dev, double* ga6_dev, double* gt_dev, double* glogf_dev) {
  if (!c) return FEA_EINVAL;
  if (c->round < 0) return fail(c, FEA_ESTATE, "begin a round first");
  if (!a6_dev || !t_dev || !logf_dev) return fail(c, FEA_EINVAL, "null device array");
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, fea::launch_params_to_pose(c, a6_dev, t_dev, logf_dev));
  HIP_OR_FAIL(c, fea::launch_resgrad_at(c, c->tile_cfg, c->Re.as<double>(), c->Te.as<double>(),
                                        c->Fe.as<double>(), false, false));
  HIP_OR_FAIL(c, fea::launch_camgrad_at(c, c->Re.as<double>(), c->Te.as<double>(), c->Fe.as<double>()));
  HIP_OR_FAIL(c, fea::launch_param_grad(c, a6_dev, gout_dev, ga6_dev, gt_dev, glogf_dev));
  return FEA_OK;
}

fea_status fea_step(fea_ctx* c, int32_t n_steps) {
  if (!c) return FEA_EINVAL;
  if (c->round < 0) return fail(c, FEA_ESTATE, "begin a round first");
  if (n_steps < 0) return fail(c, FEA_EINVAL, "n_steps must be >= 0");
  DeviceGuard g(c->device);
  return run_steps(c, n_steps);
}

namespace {

// Plain IRLS objective per scene at poses (R, T, F) with this round's
// snapshot weights (loss-only pass, learned weights ignored) into the
// device array out [S], and the same objective at the round's snapshot
// into out_snap [S] (the pass's snapshot residuals); no host wait unless
// the scenes' items interleave.
fea_status plain_loss_per_scene(fea_ctx* c, const double* R, const double* T, const double* F, DBuf& out,
                                DBuf& out_snap) {
  HIP_OR_FAIL(c, fea::launch_resgrad_at(c, c->tile_cfg, R, T, F, true, true));
  if (c->scene_items_contiguous) {
    HIP_OR_FAIL(c, fea::launch_scene_loss(c, out.as<double>(), out_snap.as<double>()));
    return FEA_OK;
  }
  // scenes with interleaved camera ids: sum the item losses on the host
  std::vector<double> part, sum(c->S, 0.0), sum_snap(c->S, 0.0);
  HIP_OR_FAIL(c, download(c, part, c->part, (size_t)c->n_items * fea::kPartStride));
  for (int64_t it = 0; it < c->n_items; ++it) {
    const int sc = c->pair_scene[c->h_item_pair[it]];
    sum[sc] += part[it * fea::kPartStride + 9];
    sum_snap[sc] += part[it * fea::kPartStride + 8];
  }
  HIP_OR_FAIL(c, upload(c, out, sum.data(), (size_t)c->S));
  HIP_OR_FAIL(c, upload(c, out_snap, sum_snap.data(), (size_t)c->S));
  return FEA_OK;
}

// After a learned round: the judge on the device, then its verdicts copied
// to pinned memory for the host to pick up later without waiting.
fea_status judge_round(fea_ctx* c) {
  HIP_OR_FAIL(c, fea::launch_judge(c));
  if (c->judge_ok_cap < c->S) {
    if (c->judge_ok_h) HIP_OR_FAIL(c, hipHostFree(c->judge_ok_h));
    c->judge_ok_h = nullptr;
    c->judge_ok_cap = 0;
    HIP_OR_FAIL(c, hipHostMalloc(reinterpret_cast<void**>(&c->judge_ok_h), (size_t)c->S * sizeof(int32_t),
                                 hipHostMallocDefault));
    c->judge_ok_cap = c->S;
  }
  if (!c->judge_ev) HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->judge_ev, hipEventDisableTiming));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->judge_ok_h, c->d_learned_ok.p, (size_t)c->S * sizeof(int32_t),
                                hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipEventRecord(c->judge_ev, c->stream));
  c->judge_pending = true;
  return FEA_OK;
}

}  // namespace

fea_status fea_epipolar_adjust(fea_ctx* c, fea_report* out) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  DeviceGuard g(c->device);
  const auto t0 = std::chrono::steady_clock::now();
  fea_report rep;
  std::memset(&rep, 0, sizeof(rep));
  // per-scene logs of the rounds (loss, retained matches), kept on the device
  HIP_OR_FAIL(c, dalloc(c->d_scene_loss_log, 64 * (size_t)c->S * sizeof(double)));
  HIP_OR_FAIL(c, dalloc(c->d_scene_z_log, 64 * (size_t)c->S * sizeof(int64_t)));
  for (int r = 0; r < c->opt.rounds; ++r) {
    const double tau_px = std::max(c->opt.tau_px_init * std::pow(c->opt.tau_decay, (double)r), c->opt.tau_px_min);
    fea_status s = begin_round(c, tau_px, false);
    if (s != FEA_OK) return s;
    if (c->opt.converge_deg > 0 && c->n_done == c->S) break;  // every scene converged
    const bool judge = c->learned_any;
    s = run_steps(c, c->opt.iters_per_round);
    if (s != FEA_OK) return s;
    if (judge) {
      // judge: a learned round must lower the plain objective of its scene;
      // one pass gives that objective at the round's end and at its
      // snapshot (the residual the weights are taken from)
      s = plain_loss_per_scene(c, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                               c->Fc[c->pcur].as<double>(), c->d_judge_l1, c->d_judge_l0);
      if (s != FEA_OK) return s;
      c->judge_written = true;
      if ((s = judge_round(c)) != FEA_OK) return s;
    }
    if (r < 64) {
      // into pinned memory, so the copy is queued without waiting for the
      // round's steps
      if (!c->loss_log) HIP_OR_FAIL(c, hipHostMalloc(&c->loss_log, 64 * sizeof(double), hipHostMallocDefault));
      if (!c->inl_log) HIP_OR_FAIL(c, hipHostMalloc(&c->inl_log, 64 * sizeof(int64_t), hipHostMallocDefault));
      if (c->host_z_stale)
        HIP_OR_FAIL(c, hipMemcpyAsync(c->inl_log + r, c->d_scene_z.as<int64_t>() + c->S, sizeof(int64_t),
                                      hipMemcpyDeviceToHost, c->stream));
      else
        c->inl_log[r] = c->Z;
      HIP_OR_FAIL(c, fea::launch_loss_sum(c));
      HIP_OR_FAIL(c, hipMemcpyAsync(c->loss_log + r, c->loss.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIP_OR_FAIL(c, fea::launch_scene_loss_log(c, r));
      int64_t* zrow = c->d_scene_z_log.as<int64_t>() + (size_t)r * c->S;
      if (c->host_z_stale)
        HIP_OR_FAIL(c, hipMemcpyAsync(zrow, c->d_scene_z.p, (size_t)c->S * sizeof(int64_t), hipMemcpyDeviceToDevice,
                                      c->stream));
      else
        HIP_OR_FAIL(c, stage_copy(c, zrow, c->Zs.data(), (size_t)c->S * sizeof(int64_t)));
    }
    rep.rounds_run = r + 1;
    rep.iters_run += c->opt.iters_per_round;
  }
  // the last round's end is checked as every round's is
  if (rep.rounds_run > 0) HIP_OR_FAIL(c, fea::launch_guard(c, c->round + 1));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  for (int r = 0; r < std::min(rep.rounds_run, 64); ++r) {
    rep.loss_per_round[r] = c->loss_log[r];
    rep.inliers_per_round[r] = c->inl_log[r];
  }
  rep.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  rep.n_logged = c->n_logged;
  HIP_OR_FAIL(c, refresh_learned_host(c));
  rep.fallbacks = c->fallbacks;
  const fea_status guard = check_nonfinite(c, &rep.scenes_converged, &rep.scenes_nonfinite);
  if (out) *out = rep;
  return guard;
}

namespace {

// Frees the working context and the export buffers of fea_batch_solve.
struct BatchScratch {
  fea_ctx* work = nullptr;
  DBuf x1, y1, x2, y2, c1, c2, seg;
  ~BatchScratch() {
    DBuf* bs[] = {&x1, &y1, &x2, &y2, &c1, &c2, &seg};
    for (DBuf* b : bs) dfree(*b);
    fea_destroy(work);
  }
};

}  // namespace

fea_status fea_batch_solve(int32_t n_scenes, fea_ctx* const* scenes, const fea_options* opt, fea_report* out) {
  if (n_scenes < 1 || !scenes) return FEA_EINVAL;
  for (int k = 0; k < n_scenes; ++k)
    if (!scenes[k]) return FEA_EINVAL;
  fea_ctx* c0 = scenes[0];
  int64_t N = 0, M = 0;
  for (int k = 0; k < n_scenes; ++k) {
    fea_ctx* c = scenes[k];
    if (!c->have_poses) return fail(c, FEA_ESTATE, "fea_batch_solve: initialise poses first");
    if (c->S != 1) return fail(c, FEA_EINVAL, "fea_batch_solve: each context must hold one scene");
    if (c->device != c0->device) return fail(c, FEA_EINVAL, "fea_batch_solve: every context on one device");
    for (int j = 0; j < k; ++j)
      if (scenes[j] == c) return fail(c, FEA_EINVAL, "fea_batch_solve: a context is listed twice");
    N += c->N;
    M += c->M;
  }
  if (N > 65535) return fail(c0, FEA_EINVAL, "fea_batch_solve: more than 65535 cameras in all");
  if (M >= (int64_t(1) << 31)) return fail(c0, FEA_EINVAL, "fea_batch_solve: 2^31 matches or more in all");
  fea_options o = opt ? *opt : c0->opt;
  std::string why;
  if (!options_valid(&o, &why)) return fail(c0, FEA_EINVAL, "fea_batch_solve: " + why);
  if (o.weight_mode == 1 && !c0->have_mlp) return fail(c0, FEA_ESTATE, "fea_batch_solve: load the network first");
  DeviceGuard g(c0->device);
  // each scene's current poses (caller's frame) and intrinsics, one problem
  std::vector<double> R(9 * N), t(3 * N), f(N), cx(N), cy(N);
  std::vector<int32_t> grp(N), cam_scene(N);
  std::vector<int64_t> cam_off(n_scenes + 1, 0);
  for (int k = 0; k < n_scenes; ++k) {
    fea_ctx* c = scenes[k];
    const int64_t b = cam_off[k];
    cam_off[k + 1] = b + c->N;
    fea_status st = fea_get_poses(c, &R[9 * b], &t[3 * b], &f[b]);
    if (st != FEA_OK) return st;
    int32_t gbase = 0;
    for (int j = 0; j < k; ++j) gbase += scenes[j]->G;
    for (int i = 0; i < c->N; ++i) {
      cx[b + i] = c->cx[i];
      cy[b + i] = c->cy[i];
      grp[b + i] = gbase + c->group[i];
      cam_scene[b + i] = k;
    }
  }
  BatchScratch w;
  // the sorted matches of every scene, exported on the device
  if (dalloc(w.x1, M * sizeof(float)) != hipSuccess || dalloc(w.y1, M * sizeof(float)) != hipSuccess ||
      dalloc(w.x2, M * sizeof(float)) != hipSuccess || dalloc(w.y2, M * sizeof(float)) != hipSuccess ||
      dalloc(w.c1, M * sizeof(int32_t)) != hipSuccess || dalloc(w.c2, M * sizeof(int32_t)) != hipSuccess)
    return fail(c0, FEA_ENOMEM, "fea_batch_solve: no device memory for the exported matches");
  int64_t m0 = 0;
  for (int k = 0; k < n_scenes; ++k) {
    fea_ctx* c = scenes[k];
    HIP_OR_FAIL(c, upload(c, w.seg, c->seg_off.data(), c->seg_off.size()));
    HIP_OR_FAIL(c, fea::export_sorted(c, (int32_t)cam_off[k], w.seg.as<int64_t>(), w.x1.as<float>() + m0,
                                      w.y1.as<float>() + m0, w.x2.as<float>() + m0, w.y2.as<float>() + m0,
                                      w.c1.as<int32_t>() + m0, w.c2.as<int32_t>() + m0));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));  // w.seg is reused by the next scene
    m0 += c->M;
  }
  // the working context: every scene at once
  fea_status st = fea_create(&w.work, c0->device, &o, nullptr);
  if (st != FEA_OK) return fail(c0, st, "fea_batch_solve: could not create the working context");
  fea_ctx* b = w.work;
  auto pass = [&](fea_status s) -> fea_status {
    if (s != FEA_OK) c0->err = "fea_batch_solve: " + b->err;
    return s;
  };
  if ((st = pass(fea_load_intrinsics(b, (int32_t)N, f.data(), cx.data(), cy.data(), grp.data()))) != FEA_OK) return st;
  if ((st = pass(fea_set_scenes(b, n_scenes, cam_scene.data()))) != FEA_OK) return st;
  if (o.weight_mode == 1) {
    std::vector<float> params;
    HIP_OR_FAIL(c0, download(c0, params, c0->mlp, fea::kMlpParams));
    if ((st = pass(fea_set_mlp(b, params.data()))) != FEA_OK) return st;
  }
  if ((st = pass(fea_load_matches_device(b, M, w.x1.as<float>(), w.y1.as<float>(), w.x2.as<float>(),
                                         w.y2.as<float>(), w.c1.as<int32_t>(), w.c2.as<int32_t>()))) != FEA_OK)
    return st;
  if ((st = pass(fea_init_poses(b, R.data(), t.data()))) != FEA_OK) return st;
  // each scene's own parameters, poses and gauge, bit for bit: the
  // caller-frame poses above only set the working context up (their round
  // trip through the caller's frame is exact only to rounding)
  {
    const size_t d = sizeof(double);
    int32_t gbase = 0;
    for (int k = 0; k < n_scenes; ++k) {
      fea_ctx* c = scenes[k];
      const size_t q = (size_t)cam_off[k], n = (size_t)c->N;
      HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
      const std::pair<void*, const void*> cp[] = {
          {b->a6.as<double>() + 6 * q, c->a6.p},
          {b->tp.as<double>() + 3 * q, c->tp.p},
          {b->R[b->pcur].as<double>() + 9 * q, c->R[c->pcur].p},
          {b->T[b->pcur].as<double>() + 3 * q, c->T[c->pcur].p},
          {b->Fc[b->pcur].as<double>() + q, c->Fc[c->pcur].p}};
      const size_t len[] = {6 * n * d, 3 * n * d, 9 * n * d, 3 * n * d, n * d};
      for (int a = 0; a < 5; ++a)
        HIP_OR_FAIL(c0, hipMemcpyAsync(cp[a].first, cp[a].second, len[a], hipMemcpyDeviceToDevice, b->stream));
      HIP_OR_FAIL(c0, hipMemcpyAsync(b->logf.as<double>() + gbase, c->logf.p, (size_t)c->G * d,
                                     hipMemcpyDeviceToDevice, b->stream));
      for (int a = 0; a < 3; ++a) b->gauge_c[3 * k + a] = c->gauge_c[a];
      b->gauge_s[k] = c->gauge_s[0];
      gbase += c->G;
    }
    HIP_OR_FAIL(c0, hipStreamSynchronize(b->stream));
    b->ptab_current = false;
  }
  fea_report rep;
  const fea_status solved = pass(fea_epipolar_adjust(b, &rep));
  if (solved != FEA_OK && solved != FEA_ENONFINITE) return solved;
  // results back into each scene's context
  std::vector<double> Rb(9 * N), tb(3 * N), fb(N);
  if ((st = pass(fea_get_poses(b, Rb.data(), tb.data(), fb.data()))) != FEA_OK) return st;
  std::vector<int32_t> done;
  std::vector<double> slog;
  std::vector<int64_t> zlog;
  HIP_OR_FAIL(c0, download(b, done, b->d_scene_done, (size_t)n_scenes));
  HIP_OR_FAIL(c0, download(b, slog, b->d_scene_loss_log, 64 * (size_t)n_scenes));
  HIP_OR_FAIL(c0, download(b, zlog, b->d_scene_z_log, 64 * (size_t)n_scenes));
  for (int k = 0; k < n_scenes; ++k) {
    fea_ctx* c = scenes[k];
    const int64_t q = cam_off[k];
    if ((st = fea_init_poses(c, &Rb[9 * q], &tb[3 * q])) != FEA_OK) return st;
    if ((st = fea_set_poses(c, &Rb[9 * q], &tb[3 * q], &fb[q])) != FEA_OK) return st;
    if (!out) continue;
    fea_report& r = out[k];
    std::memset(&r, 0, sizeof(r));
    const int32_t ended = done[k] > 0 ? done[k] - 1 : (done[k] < 0 ? -done[k] - 1 : rep.rounds_run);
    r.rounds_run = std::min(ended, rep.rounds_run);
    r.iters_run = r.rounds_run * o.iters_per_round;
    for (int j = 0; j < std::min(r.rounds_run, 64); ++j) {
      r.loss_per_round[j] = slog[(size_t)j * n_scenes + k];
      r.inliers_per_round[j] = zlog[(size_t)j * n_scenes + k];
    }
    r.fallbacks = (o.weight_mode == 1 && !b->scene_learned_ok[k]) ? 1 : 0;
    r.scenes_converged = done[k] > 0 ? 1 : 0;
    r.scenes_nonfinite = done[k] < 0 ? 1 : 0;
    r.ms_total = rep.ms_total;
  }
  return solved;
}

fea_status fea_get_scene_convergence(fea_ctx* c, int32_t* converged_round, double* change_deg) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  DeviceGuard g(c->device);
  std::vector<int32_t> done;
  std::vector<double> ch;
  HIP_OR_FAIL(c, download(c, done, c->d_scene_done, (size_t)c->S));
  HIP_OR_FAIL(c, download(c, ch, c->d_scene_change, (size_t)c->S));
  for (int s = 0; s < c->S; ++s) {
    if (converged_round) converged_round[s] = done[s] > 0 ? done[s] - 1 : -1;
    if (change_deg) change_deg[s] = ch[s];
  }
  return FEA_OK;
}

fea_status fea_get_scene_nonfinite(fea_ctx* c, int32_t* stopped_round) {
  if (!c || !stopped_round) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  DeviceGuard g(c->device);
  std::vector<int32_t> done;
  HIP_OR_FAIL(c, download(c, done, c->d_scene_done, (size_t)c->S));
  for (int s = 0; s < c->S; ++s) stopped_round[s] = done[s] < 0 ? -done[s] - 1 : -1;
  return FEA_OK;
}

fea_status fea_get_poses(fea_ctx* c, double* R, double* t, double* f) {
  if (!c) return FEA_EINVAL;
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  DeviceGuard g(c->device);
  const int N = c->N;
  std::vector<double> Rh, th, fh;
  HIP_OR_FAIL(c, download(c, Rh, c->R[c->pcur], 9 * N));
  HIP_OR_FAIL(c, download(c, th, c->T[c->pcur], 3 * N));
  HIP_OR_FAIL(c, download(c, fh, c->Fc[c->pcur], N));
  for (int i = 0; i < N; ++i) {
    const double* r = &Rh[9 * i];
    double o[3], tw[3];
    const int sc = c->cam_scene[i];
    for (int k = 0; k < 3; ++k)
      o[k] = -(r[k] * th[3 * i] + r[3 + k] * th[3 * i + 1] + r[6 + k] * th[3 * i + 2]) * c->gauge_s[sc] +
             c->gauge_c[3 * sc + k];
    for (int k = 0; k < 3; ++k) tw[k] = -(r[3 * k] * o[0] + r[3 * k + 1] * o[1] + r[3 * k + 2] * o[2]);
    if (t)
      for (int k = 0; k < 3; ++k) t[3 * i + k] = tw[k];
  }
  if (R) std::memcpy(R, Rh.data(), sizeof(double) * 9 * N);
  if (f) std::memcpy(f, fh.data(), sizeof(double) * N);
  return FEA_OK;
}

fea_status fea_get_segments(fea_ctx* c, int32_t* perm, uint8_t* swapped, int32_t* pair_cams, int64_t* seg_off) {
  if (!c) return FEA_EINVAL;
  if (!c->have_matches) return fail(c, FEA_ESTATE, "load matches first");
  DeviceGuard g(c->device);
  if (perm && c->M > 0) {
    HIP_OR_FAIL(c, hipMemcpyAsync(perm, c->perm.p, c->M * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  }
  if (swapped && c->M > 0) {
    HIP_OR_FAIL(c, hipMemcpyAsync(swapped, c->swp.p, c->M, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (pair_cams)
    for (int64_t k = 0; k < c->P; ++k) {
      pair_cams[2 * k] = c->pair_i[k];
      pair_cams[2 * k + 1] = c->pair_j[k];
    }
  if (seg_off) std::memcpy(seg_off, c->seg_off.data(), sizeof(int64_t) * (c->P + 1));
  return FEA_OK;
}

namespace {

// Retained matches of the current round by sorted position: the live layout
// (compacted rounds) or the full layout and its retained mask (quadratic
// form; before the first round every match).
hipError_t retained_by_position(fea_ctx* c, std::vector<uint8_t>& keep) {
  keep.assign((size_t)c->M, 0);
  std::vector<int32_t> pos;
  hipError_t e = download(c, pos, c->lpos[c->cur], c->layout_len);
  if (e != hipSuccess) return e;
  std::vector<uint8_t> qm;
  const bool masked = c->opt.inner_loop == 1 && c->round >= 0;
  if (masked && (e = download(c, qm, c->qmask, c->layout_len)) != hipSuccess) return e;
  for (int64_t n = 0; n < c->P; ++n)
    for (int64_t k = 0; k < c->cur_len[n]; ++k) {
      const int64_t slot = c->phys_off[n] + k;
      const int32_t p = pos[slot];
      if (p >= 0 && p < c->M && (!masked || qm[slot])) keep[p] = 1;
    }
  return hipSuccess;
}

}  // namespace

fea_status fea_get_mask(fea_ctx* c, uint8_t* mask, int64_t* n_retained) {
  if (!c) return FEA_EINVAL;
  if (!c->have_matches) return fail(c, FEA_ESTATE, "load matches first");
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, refresh_round_host(c));
  if (n_retained) *n_retained = c->Z;
  if (!mask) return FEA_OK;
  std::vector<uint8_t> keep;
  std::vector<int32_t> perm;
  HIP_OR_FAIL(c, retained_by_position(c, keep));
  HIP_OR_FAIL(c, download(c, perm, c->perm, c->M));
  for (int64_t p = 0; p < c->M; ++p) mask[perm[p]] = keep[p];
  return FEA_OK;
}

fea_status fea_get_state(fea_ctx* c, void* buf, size_t* len) {
  if (!c || !len) return fail(c, FEA_EINVAL, "null argument");
  if (!c->have_poses) return fail(c, FEA_ESTATE, "initialise poses first");
  const size_t need = state_bytes(c);
  if (!buf) {
    *len = need;
    return FEA_OK;
  }
  if (*len < need) {
    *len = need;
    return fail(c, FEA_EINVAL, "buffer too small for the state (size written to *len)");
  }
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, refresh_round_host(c));
  HIP_OR_FAIL(c, refresh_learned_host(c));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  StateHdr h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kStateMagic, sizeof(kStateMagic));
  h.version = kStateVersion;
  h.N = c->N;
  h.G = c->G;
  h.S = c->S;
  h.P = c->P;
  h.M = c->M;
  HIP_OR_FAIL(c, structure_hash(c, &h.structure));
  h.opt = c->opt;
  h.round = c->round;
  h.step = c->step;
  h.n_logged = c->n_logged;
  h.fallbacks = c->fallbacks;
  h.tile_cfg = c->tile_cfg;
  h.pcur = c->pcur;
  h.learned_any = c->learned_any ? 1 : 0;
  h.have_mlp = c->have_mlp ? 1 : 0;
  h.adam_t = c->adam_t;
  h.global_step = c->global_step;
  h.tau = c->tau;
  h.lr_scale = c->lr_scale;
  h.prev_tau_px = c->prev_tau_px;
  uint8_t* w = static_cast<uint8_t*>(buf);
  put(w, &h, 1);
  for (auto& sec : state_sections(c)) {
    HIP_OR_FAIL(c, hipMemcpyAsync(w, sec.first->p, sec.second, hipMemcpyDeviceToHost, c->stream));
    w += sec.second;
  }
  const size_t S = c->S;
  std::vector<double> taus(c->taus), fb(c->fbar_hist), gc(c->gauge_c), gs(c->gauge_s);
  std::vector<int32_t> mode(c->scene_mode), ok(c->scene_learned_ok);
  taus.resize(S, std::numeric_limits<double>::infinity());
  fb.resize(3 * S, 1.0);
  gc.resize(3 * S, 0.0);
  gs.resize(S, 1.0);
  mode.resize(S, 0);
  ok.resize(S, 1);
  put(w, taus.data(), S);
  put(w, fb.data(), 3 * S);
  put(w, mode.data(), S);
  put(w, ok.data(), S);
  put(w, gc.data(), 3 * S);
  put(w, gs.data(), S);
  // retained matches of the live layout, one bit per sorted position
  std::vector<uint32_t> bits((size_t)((c->M + 31) / 32), 0u);
  if (c->round >= 0) {
    std::vector<uint8_t> keep;
    HIP_OR_FAIL(c, retained_by_position(c, keep));
    for (int64_t q = 0; q < c->M; ++q)
      if (keep[q]) bits[q >> 5] |= 1u << (q & 31);
  }
  put(w, bits.data(), bits.size());
  std::vector<float> izw(c->inv_zw_h);
  izw.resize(S, 0.f);
  put(w, izw.data(), S);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  *len = need;
  return FEA_OK;
}

fea_status fea_set_state(fea_ctx* c, const void* buf, size_t len) {
  if (!c || !buf) return fail(c, FEA_EINVAL, "null argument");
  if (!c->have_matches) return fail(c, FEA_ESTATE, "load intrinsics and matches first");
  if (len < sizeof(StateHdr)) return fail(c, FEA_EINVAL, "state too short");
  StateHdr h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kStateMagic, sizeof(kStateMagic)) != 0 || h.version != kStateVersion)
    return fail(c, FEA_EINVAL, "not a state of this library version");
  if (h.N != c->N || h.G != c->G || h.S != c->S || h.P != c->P || h.M != c->M)
    return fail(c, FEA_EINVAL, "state is of a problem with other sizes");
  if (len != state_bytes(c)) return fail(c, FEA_EINVAL, "state has the wrong length");
  std::string why;
  if (!options_valid(&h.opt, &why)) return fail(c, FEA_EINVAL, "state options: " + why);
  if (h.tile_cfg < 0 || h.tile_cfg >= fea::kNumTiles || (h.pcur != 0 && h.pcur != 1) || h.round < -1)
    return fail(c, FEA_EINVAL, "state header is corrupt");
  if (h.learned_any && !c->have_mlp) return fail(c, FEA_ESTATE, "load the network (fea_set_mlp) first");
  DeviceGuard g(c->device);
  uint64_t hs = 0;
  HIP_OR_FAIL(c, structure_hash(c, &hs));
  if (hs != h.structure) return fail(c, FEA_EINVAL, "state is of another set of matches");
  if (h.opt.log_every > 0 && h.opt.max_log > 0)
    HIP_OR_FAIL(c, dalloc(c->logR, (size_t)h.opt.max_log * 9 * c->N * sizeof(double)));
  c->opt = h.opt;
  c->pcur = h.pcur;
  const uint8_t* r = static_cast<const uint8_t*>(buf) + sizeof(StateHdr);
  for (auto& sec : state_sections(c)) {
    HIP_OR_FAIL(c, hipMemcpyAsync(sec.first->p, r, sec.second, hipMemcpyHostToDevice, c->stream));
    r += sec.second;
  }
  const size_t S = c->S;
  c->taus.resize(S);
  c->fbar_hist.resize(3 * S);
  c->scene_mode.resize(S);
  c->scene_learned_ok.resize(S);
  c->gauge_c.resize(3 * S);
  c->gauge_s.resize(S);
  take(r, c->taus.data(), S);
  take(r, c->fbar_hist.data(), 3 * S);
  take(r, c->scene_mode.data(), S);
  take(r, c->scene_learned_ok.data(), S);
  take(r, c->gauge_c.data(), 3 * S);
  take(r, c->gauge_s.data(), S);
  std::vector<uint32_t> bits((size_t)((c->M + 31) / 32));
  take(r, bits.data(), bits.size());
  c->inv_zw_h.assign(S, 0.f);
  take(r, c->inv_zw_h.data(), S);
  c->host_tau_stale = c->host_z_stale = false;
  c->round = h.round;
  c->step = h.step;
  c->n_logged = h.n_logged;
  // the judge's verdicts back onto the device; earlier rejections are
  // counted on the host
  c->fallbacks = h.fallbacks;
  c->fallbacks_base = h.fallbacks;
  c->judge_pending = false;
  HIP_OR_FAIL(c, upload(c, c->d_learned_ok, c->scene_learned_ok.data(), S));
  HIP_OR_FAIL(c, upload(c, c->d_scene_mode, c->scene_mode.data(), S));
  HIP_OR_FAIL(c, hipMemsetAsync(c->d_fallbacks.p, 0, S * sizeof(int32_t), c->stream));
  c->adam_t = h.adam_t;
  c->global_step = h.global_step;
  c->tau = h.tau;
  c->lr_scale = h.lr_scale;
  c->prev_tau_px = h.prev_tau_px;
  c->have_poses = true;
  drop_graph(c);
  // converged scenes (their flags came with the sections)
  HIP_OR_FAIL(c, download(c, c->scene_done_h, c->d_scene_done, S));
  c->n_done = 0;
  for (size_t sc = 0; sc < S; ++sc) c->n_done += c->scene_done_h[sc] != 0 ? 1 : 0;
  // rebuild the live layout: the full one, then the saved retained set
  c->tile_cfg = h.tile_cfg;
  c->tile_tuned = true;
  fea::prepare_resgrad(c->tile_cfg);
  HIP_OR_FAIL(c, reset_layout(c));
  if (c->round >= 0) {
    if (c->opt.inner_loop == 1) {
      // quadratic form: the full layout with the retained mask per slot
      std::vector<int32_t> pos;
      HIP_OR_FAIL(c, download(c, pos, c->lpos[0], c->layout_len));
      std::vector<uint8_t> qm((size_t)c->layout_len, 0);
      c->Zs.assign(S, 0);
      for (int64_t n = 0; n < c->P; ++n)
        for (int64_t k = 0; k < c->cur_len[n]; ++k) {
          const int64_t slot = c->phys_off[n] + k;
          const int32_t q = pos[slot];
          if (q >= 0 && ((bits[q >> 5] >> (q & 31)) & 1u)) {
            qm[slot] = 1;
            c->Zs[c->pair_scene[n]] += 1;
          }
        }
      HIP_OR_FAIL(c, upload(c, c->qmask, qm.data(), qm.size()));
      c->Z = 0;
      std::vector<float> inv(S, 0.f);
      for (size_t sc = 0; sc < S; ++sc) {
        c->Z += c->Zs[sc];
        inv[sc] = c->Zs[sc] > 0 ? (float)(1.0 / (double)c->Zs[sc]) : 0.f;
      }
      HIP_OR_FAIL(c, upload(c, c->d_inv_z, inv.data(), S));
      // the device's per-scene counts (converged scenes keep theirs)
      std::vector<int64_t> zd(c->Zs);
      zd.push_back(c->Z);
      HIP_OR_FAIL(c, upload(c, c->d_scene_z, zd.data(), zd.size()));
    } else {
      DBuf d_bits;
      hipError_t e = upload(c, d_bits, bits.data(), bits.size());
      if (e == hipSuccess) e = compact_layout(c, d_bits.as<uint32_t>());
      dfree(d_bits);
      HIP_OR_FAIL(c, e);
      HIP_OR_FAIL(c, upload_scene_z(c));
      HIP_OR_FAIL(c, build_items(c));
    }
    HIP_OR_FAIL(c, upload(c, c->d_tau, c->taus.data(), S));
    HIP_OR_FAIL(c, upload_fbar(c));
    const std::vector<float> izw_saved(c->inv_zw_h);
    HIP_OR_FAIL(c, round_weights(c, false));
    // the learned normalisers as they were (their sums ran over the
    // retained matches of the round's pass)
    c->inv_zw_h = izw_saved;
    HIP_OR_FAIL(c, upload(c, c->d_inv_zw, c->inv_zw_h.data(), S));
    HIP_OR_FAIL(c, fea::launch_pair_pose(c, c->Rh.as<double>(), c->Th.as<double>(), c->Fh.as<double>(), true));
  }
  // the step counters (with their running powers) came with the sections
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return FEA_OK;
}

fea_status fea_ablation(fea_ctx* c, int32_t variant, int32_t reps, double* ms_per_pass, float* pair_sums) {
  if (!c || !ms_per_pass) return fail(c, FEA_EINVAL, "null argument");
  if (c->round < 0) return fail(c, FEA_ESTATE, "begin a round first");
  if (variant < 0 || variant > 3 || reps < 1) return fail(c, FEA_EINVAL, "variant must be 0..3 and reps >= 1");
  if (c->opt.inner_loop != 0) return fail(c, FEA_EINVAL, "ablations are of the per-match inner loop (inner_loop = 0)");
  if (variant == 1 && !(fea::kTiles[c->tile_cfg].threads == 256 && fea::kTiles[c->tile_cfg].steps == 2))
    return fail(c, FEA_EINVAL, "variant 1 needs tile_matches = 2048");
  if (c->n_items == 0) return fail(c, FEA_EINVAL, "no retained matches");
  DeviceGuard g(c->device);
  DBuf sums;
  hipError_t e = dalloc(sums, (size_t)c->P * fea::kPartStride * sizeof(float));
  if (e == hipSuccess) e = fea::run_ablation(c, variant, reps, ms_per_pass, sums.as<float>());
  if (e == hipSuccess && pair_sums)
    e = hipMemcpy(pair_sums, sums.p, (size_t)c->P * fea::kPartStride * sizeof(float), hipMemcpyDeviceToHost);
  dfree(sums);
  HIP_OR_FAIL(c, e);
  return FEA_OK;
}

fea_status fea_get_info(fea_ctx* c, fea_info* out) {
  if (!c || !out) return fail(c, FEA_EINVAL, "null argument");
  if (c->host_tau_stale || c->host_z_stale) {
    DeviceGuard g(c->device);
    HIP_OR_FAIL(c, refresh_round_host(c));
  }
  std::memset(out, 0, sizeof(*out));
  out->n_cams = c->N;
  out->n_groups = c->G;
  out->n_matches = c->have_matches ? c->M : 0;
  out->n_pairs = c->have_matches ? c->P : 0;
  out->n_retained = c->have_matches ? c->Z : 0;
  out->n_items = c->have_matches ? c->n_items : 0;
  out->layout_matches = c->have_matches ? c->layout_len : 0;
  out->round = c->round;
  out->step = c->step;
  for (int k = 0; k < 3; ++k) out->gauge_center[k] = c->gauge_c.size() >= 3 ? c->gauge_c[k] : 0.0;
  out->gauge_scale = c->gauge_s.empty() ? 1.0 : c->gauge_s[0];
  out->n_scenes = c->S;
  out->tau = c->tau;
  out->tile_matches = fea::tile_matches_of(c->tile_cfg);
  out->tile_threads = fea::kTiles[c->tile_cfg].threads;
  out->tile_persistent = fea::kTiles[c->tile_cfg].persistent ? 1 : 0;
  out->quad_steps_blocks = c->last_quad_blocks;
  return FEA_OK;
}

fea_status fea_get_tile_timings(fea_ctx* c, float* ms, int32_t cap, int32_t* n) {
  if (!c || !n || (cap > 0 && !ms)) return FEA_EINVAL;
  *n = (int32_t)c->tune_ms.size();
  for (int32_t k = 0; k < std::min<int32_t>(cap, *n); ++k) ms[k] = c->tune_ms[k];
  return FEA_OK;
}

fea_status fea_synchronize(fea_ctx* c) {
  if (!c) return FEA_EINVAL;
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return FEA_OK;
}

fea_status fea_get_stream(fea_ctx* c, void** stream) {
  if (!c || !stream) return FEA_EINVAL;
  *stream = static_cast<void*>(c->stream);
  return FEA_OK;
}

fea_status fea_set_mlp(fea_ctx* c, const float* params) {
  if (!c || !params) return fail(c, FEA_EINVAL, "null argument");
  if (!c->have_intr) return fail(c, FEA_ESTATE, "load intrinsics first");
  for (int k = 0; k < fea::kMlpParams; ++k)
    if (!std::isfinite(params[k])) return fail(c, FEA_ENONFINITE, "non-finite network parameter");
  // inference converts W1, W2 and w3 to fp16 (the biases stay fp32): a weight
  // beyond fp16's largest finite value would become infinite there
  constexpr int kH = fea::kMlpHidden, kF = fea::kMlpFeat;
  constexpr int kW1 = 0, kW2 = kH * kF + kH, kW3 = kW2 + kH * kH + kH;
  constexpr float kHalfMax = 65504.f;
  for (const auto& r : {std::pair<int, int>{kW1, kH * kF}, {kW2, kH * kH}, {kW3, kH}})
    for (int k = r.first; k < r.first + r.second; ++k)
      if (std::fabs(params[k]) > kHalfMax)
        return fail(c, FEA_EINVAL, "network weight beyond the fp16 range (|w| > 65504)");
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, upload(c, c->mlp, params, fea::kMlpParams));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->have_mlp = true;
  return FEA_OK;
}

fea_status fea_mlp_features_dev(fea_ctx* c, float* feat_dev, int32_t* slot_pos_dev) {
  if (!c) return FEA_EINVAL;
  if (c->round < 0) return fail(c, FEA_ESTATE, "begin a round first");
  if (!feat_dev) return fail(c, FEA_EINVAL, "feat_dev is required");
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, hipMemsetAsync(feat_dev, 0, (size_t)c->layout_len * fea::kMlpFeat * sizeof(float), c->stream));
  HIP_OR_FAIL(c, fea::launch_mlp_weights(c, c->mlp.as<float>(), c->wlay.as<unsigned short>(),
                                         c->item_wsum.as<double>(), feat_dev));
  if (slot_pos_dev) {
    HIP_OR_FAIL(c, hipMemcpyAsync(slot_pos_dev, c->lpos[c->cur].p, (size_t)c->layout_len * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, c->stream));
    // quadratic form: the layout is whole; dropped matches are marked -1
    if (c->opt.inner_loop == 1) HIP_OR_FAIL(c, fea::launch_mask_slots(c, slot_pos_dev));
  }
  return FEA_OK;
}

namespace {

// IEEE binary16 bits to float (the learned weights are stored as fp16).
float half_to_float(uint16_t h) {
  const uint32_t sign = (uint32_t)(h >> 15) << 31, e = (h >> 10) & 31u, m = h & 1023u;
  float v;
  if (e == 0) {
    v = std::ldexp((float)m, -24);  // zero or subnormal
  } else if (e == 31) {
    v = m ? std::numeric_limits<float>::quiet_NaN() : std::numeric_limits<float>::infinity();
  } else {
    v = std::ldexp((float)(m | 1024u), (int)e - 25);
  }
  return sign ? -v : v;
}

}  // namespace

fea_status fea_get_learned_weights(fea_ctx* c, float* w) {
  if (!c || !w) return fail(c, FEA_EINVAL, "null argument");
  if (c->round < 0) return fail(c, FEA_ESTATE, "begin a round first");
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, refresh_learned_host(c));
  std::vector<int32_t> pos, perm;
  std::vector<uint16_t> wl;
  HIP_OR_FAIL(c, download(c, pos, c->lpos[c->cur], c->layout_len));
  HIP_OR_FAIL(c, download(c, perm, c->perm, c->M));
  HIP_OR_FAIL(c, download(c, wl, c->wlay, c->layout_len));
  std::vector<uint8_t> qm;
  const bool masked = c->opt.inner_loop == 1;
  if (masked) HIP_OR_FAIL(c, download(c, qm, c->qmask, c->layout_len));
  for (int64_t m = 0; m < c->M; ++m) w[m] = 0.f;
  for (int64_t n = 0; n < c->P; ++n) {
    const bool learned = c->scene_mode[c->pair_scene[n]] != 0;
    for (int64_t k = 0; k < c->cur_len[n]; ++k) {
      const int64_t slot = c->phys_off[n] + k;
      const int32_t p = pos[slot];
      if (p < 0 || p >= c->M || (masked && !qm[slot])) continue;
      w[perm[p]] = learned ? half_to_float(wl[slot]) : 1.f;
    }
  }
  return FEA_OK;
}

namespace {

struct MlpScratch {
  float *gpart = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  double *lpart = nullptr, *loss = nullptr;
  ~MlpScratch() {
    for (void* p : {(void*)gpart, (void*)grad, (void*)m, (void*)v, (void*)lpart, (void*)loss})
      if (p) (void)hipFree(p);
  }
  hipError_t alloc(int64_t parts) {
    hipError_t e;
    if ((e = hipMalloc(&gpart, std::max<int64_t>(parts, 1) * fea::kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&grad, fea::kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&m, fea::kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&v, fea::kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&lpart, std::max<int64_t>(parts, 1) * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&loss, sizeof(double))) != hipSuccess) return e;
    if ((e = hipMemset(m, 0, fea::kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMemset(v, 0, fea::kMlpParams * sizeof(float))) != hipSuccess) return e;
    return hipMemset(loss, 0, sizeof(double));
  }
};

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

fea_status fea_mlp_train(int32_t device, const float* feat_dev, const float* target_dev, int64_t n, int32_t epochs,
                         int32_t batch, double lr, uint64_t seed, float* params_dev, double* loss_per_epoch) {
  if (!feat_dev || !target_dev || !params_dev || n < 1 || n >= ((int64_t)1 << 31) || epochs < 0 || batch < 1 ||
      !(lr > 0))
    return FEA_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FEA_EINVAL;
  DeviceGuard g(device);
  const int64_t B = std::min<int64_t>(batch, n);
  const int64_t parts = (B + fea::mlp_train_threads() - 1) / fea::mlp_train_threads();
  MlpScratch sc;
  if (sc.alloc(parts) != hipSuccess) return FEA_ENOMEM;
  const int64_t nb = n / B;
  uint64_t st = seed * 0x9E3779B97F4A7C15ull + 1;
  int64_t t = 0;
  for (int32_t ep = 0; ep < epochs; ++ep) {
    // a stride coprime with n gives this epoch's visiting order
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    int64_t stride = (int64_t)((st >> 17) % (uint64_t)n);
    if (stride == 0) stride = 1;
    while (gcd64(stride, n) != 1) stride = (stride + 1) % n ? (stride + 1) % n : 1;
    if (hipMemset(sc.loss, 0, sizeof(double)) != hipSuccess) return FEA_EDEVICE;
    for (int64_t b = 0; b < nb; ++b) {
      ++t;
      if (fea::mlp_train_step(nullptr, feat_dev, target_dev, n, B, stride, b, params_dev, sc.m, sc.v, sc.gpart,
                              sc.lpart, sc.grad, sc.loss, (float)lr, t) != hipSuccess)
        return FEA_EDEVICE;
    }
    double L = 0.0;
    if (hipMemcpy(&L, sc.loss, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return FEA_EDEVICE;
    if (loss_per_epoch) loss_per_epoch[ep] = L / (double)(nb * B);
  }
  return hipDeviceSynchronize() == hipSuccess ? FEA_OK : FEA_EDEVICE;
}

fea_status fea_mlp_grad(int32_t device, const float* feat_dev, const float* target_dev, int64_t n,
                        const float* params_dev, float* grad_dev, double* loss) {
  if (!feat_dev || !target_dev || !params_dev || !grad_dev || n < 1 || n >= ((int64_t)1 << 31)) return FEA_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FEA_EINVAL;
  DeviceGuard g(device);
  const int64_t parts = (n + fea::mlp_train_threads() - 1) / fea::mlp_train_threads();
  MlpScratch sc;
  if (sc.alloc(parts) != hipSuccess) return FEA_ENOMEM;
  if (fea::mlp_grad_once(nullptr, feat_dev, target_dev, n, params_dev, sc.gpart, sc.lpart, grad_dev, sc.loss) !=
      hipSuccess)
    return FEA_EDEVICE;
  double L = 0.0;
  if (hipMemcpy(&L, sc.loss, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return FEA_EDEVICE;
  if (loss) *loss = L / (double)n;
  return hipDeviceSynchronize() == hipSuccess ? FEA_OK : FEA_EDEVICE;
}

fea_status fea_set_kernel_timing(fea_ctx* c, int32_t enable) {
  if (!c) return FEA_EINVAL;
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->timing = enable != 0;
  c->ev_used = 0;
  return FEA_OK;
}

fea_status fea_get_kernel_timing(fea_ctx* c, double* resgrad_ms, int64_t* resgrad_launches) {
  if (!c) return FEA_EINVAL;
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.f;
    HIP_OR_FAIL(c, hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
    total += ms;
  }
  if (resgrad_ms) *resgrad_ms = total;
  if (resgrad_launches) *resgrad_launches = (int64_t)(c->ev_used / 2);
  return FEA_OK;
}

fea_status fea_get_kernel_times(fea_ctx* c, float* ms, int64_t cap, int64_t* n) {
  if (!c || cap < 0 || (cap > 0 && !ms)) return FEA_EINVAL;
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  const int64_t launches = (int64_t)(c->ev_used / 2);
  for (int64_t k = 0; k < std::min(cap, launches); ++k)
    HIP_OR_FAIL(c, hipEventElapsedTime(&ms[k], c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
  if (n) *n = launches;
  return FEA_OK;
}

fea_status fea_get_rotation_log(fea_ctx* c, double* R_log, int32_t* n_logged) {
  if (!c) return FEA_EINVAL;
  if (n_logged) *n_logged = c->n_logged;
  if (!R_log || c->n_logged == 0) return FEA_OK;
  DeviceGuard g(c->device);
  HIP_OR_FAIL(c, hipMemcpyAsync(R_log, c->logR.p, sizeof(double) * 9 * c->N * c->n_logged,
                                hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return FEA_OK;
}

}  // extern "C"

// ---- Global Translation ---------------------------------------------------------

namespace {

// Device memory owned by one call: freed (after the stream has drained) when
// the call returns, on every path.
struct CallScratch {
  hipStream_t st;
  std::vector<void*> ptrs;
  explicit CallScratch(hipStream_t s) : st(s) {}
  ~CallScratch() {
    (void)hipStreamSynchronize(st);
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t alloc(T*& p, size_t n) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n * sizeof(T), 16));
    if (e == hipSuccess) {
      ptrs.push_back(q);
      p = static_cast<T*>(q);
    }
    return e;
  }
  template <class T>
  hipError_t put(T*& p, const T* src, size_t n) {
    hipError_t e = alloc(p, n);
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyHostToDevice, st);
  }
};

template <class T>
hipError_t fetch(hipStream_t st, T* dst, const T* src, size_t n) {
  if (!dst || n == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, st);
}

bool all_finite(const double* a, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(a[k])) return false;
  return true;
}

// Camera -> (2 * pair + side) entries in pair order; side 1 = the pair's
// second camera.
void camera_entries(int32_t n_cams, int64_t n_pairs, const int32_t* pi, const int32_t* pj,
                    std::vector<int32_t>& off, std::vector<int32_t>& ent) {
  off.assign((size_t)n_cams + 1, 0);
  for (int64_t p = 0; p < n_pairs; ++p) {
    off[pi[p] + 1]++;
    off[pj[p] + 1]++;
  }
  for (int32_t i = 0; i < n_cams; ++i) off[i + 1] += off[i];
  ent.assign((size_t)2 * n_pairs, 0);
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (int64_t p = 0; p < n_pairs; ++p) {
    ent[fill[pi[p]]++] = (int32_t)(2 * p);
    ent[fill[pj[p]]++] = (int32_t)(2 * p + 1);
  }
}

}  // namespace

extern "C" {

fea_status fea_relative_translations(fea_ctx* c, const double* R, const double* f, double tau_px, int32_t n_cand,
                                     const double* cand, double* t_rel, int32_t* best, int32_t* vote,
                                     double* score_best, float* scores, float* score_ms) {
  if (!c) return FEA_EINVAL;
  if (!c->have_matches) return fail(c, FEA_ESTATE, "load matches first");
  if (!R || !cand || !t_rel) return fail(c, FEA_EINVAL, "R, cand and t_rel are required");
  if (n_cand < 1 || n_cand > (1 << 22)) return fail(c, FEA_EINVAL, "n_cand must be in [1, 2^22]");
  const int32_t N = c->N;
  if (!all_finite(R, (size_t)9 * N)) return fail(c, FEA_ENONFINITE, "non-finite rotation");
  std::vector<double> fv(f ? f : c->f_in.data(), (f ? f : c->f_in.data()) + N);
  for (double x : fv)
    if (!std::isfinite(x) || !(x > 0.0)) return fail(c, FEA_EINVAL, "focal lengths must be finite and > 0");
  if (std::isnan(tau_px) || !(tau_px > 0.0)) return fail(c, FEA_EINVAL, "tau_px must be > 0 (inf: no cap)");
  // the cap in normalised units: pixels over the median focal length
  double tau = tau_px;
  if (std::isfinite(tau_px)) {
    std::vector<double> fs(fv);
    std::sort(fs.begin(), fs.end());
    const size_t n = fs.size();
    tau = tau_px / ((n & 1) ? fs[n / 2] : 0.5 * (fs[n / 2 - 1] + fs[n / 2]));
  }
  for (int32_t k = 0; k < n_cand; ++k) {
    const double* u = cand + 3 * (size_t)k;
    if (!all_finite(u, 3)) return fail(c, FEA_ENONFINITE, "non-finite candidate");
    if (std::fabs(std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - 1.0) > 1e-6)
      return fail(c, FEA_EINVAL, "candidates must be unit vectors");
  }
  const int64_t P = c->P;
  if (P == 0) return FEA_OK;
  // work items over the full layout (each pair's run aligned as when loaded)
  std::vector<int4> items;
  std::vector<int32_t> pio((size_t)P + 1);
  int64_t off = 0;
  for (int64_t n = 0; n < P; ++n) {
    const int64_t cnt = c->seg_off[n + 1] - c->seg_off[n];
    pio[n] = (int32_t)items.size();
    for (int64_t s = 0; s < cnt; s += fea::kRtItem) {
      if (off + s > INT32_MAX) return fail(c, FEA_EINVAL, "layout too large for the candidate search");
      items.push_back(make_int4((int)n, (int)(off + s), (int)std::min<int64_t>(fea::kRtItem, cnt - s), 0));
    }
    off += (cnt + fea::kAlign - 1) / fea::kAlign * fea::kAlign;
  }
  pio[P] = (int32_t)items.size();
  const int64_t n_items = (int64_t)items.size();
  const int groups = (n_cand + fea::kRtGroup - 1) / fea::kRtGroup;
  const int kp = groups * fea::kRtGroup;
  std::vector<float> cs((size_t)3 * kp, 0.f);  // structure of arrays, zero-padded
  for (int32_t k = 0; k < n_cand; ++k)
    for (int a = 0; a < 3; ++a) cs[(size_t)a * kp + k] = (float)cand[3 * (size_t)k + a];

  DeviceGuard g(c->device);
  CallScratch sc(c->stream);
  double *dR, *df, *rowd, *dt, *dsb;
  float *dcand, *rowf, *part, *dscores = nullptr;
  int4* ditems;
  int32_t *dpio, *dbest, *dvote;
  HIP_OR_FAIL(c, sc.put(dR, R, (size_t)9 * N));
  HIP_OR_FAIL(c, sc.put(df, fv.data(), (size_t)N));
  HIP_OR_FAIL(c, sc.put(dcand, cs.data(), cs.size()));
  HIP_OR_FAIL(c, sc.put(ditems, items.data(), items.size()));
  HIP_OR_FAIL(c, sc.put(dpio, pio.data(), pio.size()));
  HIP_OR_FAIL(c, sc.alloc(rowf, (size_t)fea::kRtRow * P));
  HIP_OR_FAIL(c, sc.alloc(rowd, (size_t)fea::kRtRow * P));
  HIP_OR_FAIL(c, sc.alloc(part, (size_t)n_items * kp));
  HIP_OR_FAIL(c, sc.alloc(dbest, (size_t)P));
  HIP_OR_FAIL(c, sc.alloc(dvote, (size_t)P));
  HIP_OR_FAIL(c, sc.alloc(dt, (size_t)3 * P));
  HIP_OR_FAIL(c, sc.alloc(dsb, (size_t)P));
  if (scores) HIP_OR_FAIL(c, sc.alloc(dscores, (size_t)P * n_cand));
  const float *x1 = c->lay[0][0].as<float>(), *y1 = c->lay[0][1].as<float>(), *x2 = c->lay[0][2].as<float>(),
              *y2 = c->lay[0][3].as<float>();
  HIP_OR_FAIL(c, fea::launch_rt_pairs(c->stream, P, c->d_pair_i.as<int32_t>(), c->d_pair_j.as<int32_t>(), dR, df,
                                      c->d_cx.as<double>(), c->d_cy.as<double>(), rowf, rowd));
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (score_ms) {
    HIP_OR_FAIL(c, hipEventCreate(&ev[0]));
    HIP_OR_FAIL(c, hipEventCreate(&ev[1]));
  }
  hipError_t e = fea::launch_rt_score(c->stream, n_items, groups, ditems, rowf, x1, y1, x2, y2, dcand, kp, tau,
                                      part, ev[0], ev[1]);
  if (e == hipSuccess)
    e = fea::launch_rt_select(c->stream, P, n_cand, kp, tau, dpio, ditems, part, dcand, rowd, x1, y1, x2, y2,
                              dscores, dbest, dvote, dt, dsb);
  if (e == hipSuccess) e = fetch(c->stream, t_rel, dt, (size_t)3 * P);
  if (e == hipSuccess) e = fetch(c->stream, best, dbest, (size_t)P);
  if (e == hipSuccess) e = fetch(c->stream, vote, dvote, (size_t)P);
  if (e == hipSuccess) e = fetch(c->stream, score_best, dsb, (size_t)P);
  if (e == hipSuccess) e = fetch(c->stream, scores, dscores, (size_t)P * n_cand);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && score_ms) e = hipEventElapsedTime(score_ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  HIP_OR_FAIL(c, e);
  return FEA_OK;
}

fea_status fea_ta_default_options(fea_ta_options* o) {
  if (!o) return FEA_EINVAL;
  o->iters_run = 1500;
  o->iters_final = 500;
  o->lr = 2e-2;
  o->lr_final = 2e-3;
  o->lr_end_frac = 1e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->adam_eps = 1e-12;
  return FEA_OK;
}

}  // extern "C"

namespace {

// Steps of one alignment phase: a captured graph of an even number of steps
// (the parity, and so the buffer roles, are the same at its end as at its
// start) replayed, then the remainder launched directly.
struct TaPhase {
  fea_ctx* c;
  int runs, N;
  int64_t P;
  const int32_t *off, *ent, *oth;
  const double* tg;
  double* o[2];
  double *m, *v;
  fea::TaCounters* ctr;
  double b1, b2, eps, decay;
  int parity = 0;

  hipError_t step() {
    hipError_t e = fea::launch_ta_step(c->stream, runs, N, P, off, ent, oth, tg, o[parity], o[parity ^ 1], m, v,
                                       ctr, parity, b1, b2, eps, decay);
    parity ^= 1;
    return e;
  }
  hipError_t run(int iters) {
    constexpr int kChunk = 64;
    int done = 0;
    if (iters >= 2 * kChunk) {
      hipGraph_t g = nullptr;
      hipGraphExec_t x = nullptr;
      hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      hipError_t le = hipSuccess;
      const int p0 = parity;
      for (int k = 0; k < kChunk && le == hipSuccess; ++k) le = step();
      e = hipStreamEndCapture(c->stream, &g);
      parity = p0;
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      for (; e == hipSuccess && done + kChunk <= iters; done += kChunk) e = hipGraphLaunch(x, c->stream);
      if (x) (void)hipGraphExecDestroy(x);
      if (e != hipSuccess) return e;
    }
    for (; done < iters; ++done) {
      hipError_t e = step();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

}  // namespace

extern "C" {

fea_status fea_translation_align(fea_ctx* c, int32_t n_cams, int64_t n_pairs, const int32_t* pair_i,
                                 const int32_t* pair_j, const double* R, const double* t_rel, int32_t n_runs,
                                 const double* o_init, const fea_ta_options* opt, double* o_out,
                                 int32_t* run_of_cam, double* run_loss, double* final_loss, double* run_o,
                                 double* cam_loss, float* ms) {
  if (!c) return FEA_EINVAL;
  if (!pair_i || !pair_j || !R || !t_rel || !o_init || !o_out)
    return fail(c, FEA_EINVAL, "pair_i, pair_j, R, t_rel, o_init and o_out are required");
  if (n_cams < 2 || n_pairs < 1 || n_pairs > INT32_MAX / 2)
    return fail(c, FEA_EINVAL, "need n_cams >= 2 and 1 <= n_pairs < 2^30");
  if (n_runs < 1 || n_runs > 64) return fail(c, FEA_EINVAL, "n_runs must be in [1, 64]");
  fea_ta_options o;
  fea_ta_default_options(&o);
  if (opt) o = *opt;
  if (o.iters_run < 0 || o.iters_final < 0 || !(o.lr > 0) || !(o.lr_final > 0) || !(o.lr_end_frac > 0) ||
      !(o.lr_end_frac <= 1) || !(o.beta1 >= 0 && o.beta1 < 1) || !(o.beta2 >= 0 && o.beta2 < 1) ||
      !(o.adam_eps >= 0))
    return fail(c, FEA_EINVAL, "invalid alignment options");
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int32_t i = pair_i[p], j = pair_j[p];
    if (i < 0 || j < 0 || i >= n_cams || j >= n_cams || i == j) return fail(c, FEA_EINVAL, "invalid camera pair");
    const double* t = t_rel + 3 * p;
    if (!all_finite(t, 3)) return fail(c, FEA_ENONFINITE, "non-finite relative translation");
    if (!(t[0] * t[0] + t[1] * t[1] + t[2] * t[2] > 0.0))
      return fail(c, FEA_EDEGENERATE, "zero relative translation");
  }
  if (!all_finite(R, (size_t)9 * n_cams)) return fail(c, FEA_ENONFINITE, "non-finite rotation");
  const size_t n3 = (size_t)3 * n_cams, r3 = n3 * (size_t)n_runs;
  if (!all_finite(o_init, r3)) return fail(c, FEA_ENONFINITE, "non-finite initial centre");
  std::vector<int32_t> off, ent;
  camera_entries(n_cams, n_pairs, pair_i, pair_j, off, ent);
  // the other camera of each entry, so that a step reads it without the pair
  std::vector<int32_t> oth(ent.size());
  for (size_t e = 0; e < ent.size(); ++e) oth[e] = (ent[e] & 1) ? pair_i[ent[e] >> 1] : pair_j[ent[e] >> 1];

  DeviceGuard g(c->device);
  CallScratch sc(c->stream);
  int32_t *dpi, *dpj, *doff, *dent, *doth, *derr, *drun;
  double *dR, *dt, *tg, *o0, *o1, *m, *v, *pl, *cl, *rl, *om0, *om1, *fl;
  fea::TaCounters* ctr;
  HIP_OR_FAIL(c, sc.put(dpi, pair_i, (size_t)n_pairs));
  HIP_OR_FAIL(c, sc.put(dpj, pair_j, (size_t)n_pairs));
  HIP_OR_FAIL(c, sc.put(doff, off.data(), off.size()));
  HIP_OR_FAIL(c, sc.put(dent, ent.data(), ent.size()));
  HIP_OR_FAIL(c, sc.put(doth, oth.data(), oth.size()));
  HIP_OR_FAIL(c, sc.put(dR, R, (size_t)9 * n_cams));
  HIP_OR_FAIL(c, sc.put(dt, t_rel, (size_t)3 * n_pairs));
  HIP_OR_FAIL(c, sc.put(o0, o_init, r3));
  HIP_OR_FAIL(c, sc.alloc(tg, (size_t)3 * n_pairs));
  HIP_OR_FAIL(c, sc.alloc(o1, r3));
  HIP_OR_FAIL(c, sc.alloc(m, r3));
  HIP_OR_FAIL(c, sc.alloc(v, r3));
  HIP_OR_FAIL(c, sc.alloc(pl, (size_t)n_pairs * n_runs));
  HIP_OR_FAIL(c, sc.alloc(cl, (size_t)n_cams * n_runs));
  HIP_OR_FAIL(c, sc.alloc(rl, (size_t)n_runs));
  HIP_OR_FAIL(c, sc.alloc(om0, n3));
  HIP_OR_FAIL(c, sc.alloc(om1, n3));
  HIP_OR_FAIL(c, sc.alloc(fl, 1));
  HIP_OR_FAIL(c, sc.alloc(drun, (size_t)n_cams));
  HIP_OR_FAIL(c, sc.alloc(derr, 1));
  HIP_OR_FAIL(c, sc.alloc(ctr, 1));
  HIP_OR_FAIL(c, hipMemsetAsync(m, 0, r3 * sizeof(double), c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(v, 0, r3 * sizeof(double), c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(derr, 0, sizeof(int32_t), c->stream));
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (ms) {
    HIP_OR_FAIL(c, hipEventCreate(&ev[0]));
    HIP_OR_FAIL(c, hipEventCreate(&ev[1]));
  }
  hipError_t e = hipSuccess;
  if (ev[0]) e = hipEventRecord(ev[0], c->stream);
  if (e == hipSuccess) e = fea::launch_ta_targets(c->stream, n_pairs, dpj, dR, dt, tg);
  // the runs, side by side
  TaPhase ph{c, n_runs, n_cams, n_pairs, doff, dent, doth, tg, {o0, o1}, m, v, ctr,
             o.beta1, o.beta2, o.adam_eps, o.iters_run > 0 ? std::pow(o.lr_end_frac, 1.0 / o.iters_run) : 1.0};
  if (e == hipSuccess) e = fea::launch_ta_counters(c->stream, ctr, o.lr);
  if (e == hipSuccess) e = ph.run(o.iters_run);
  double* ro = ph.o[ph.parity];
  if (e == hipSuccess) e = fea::launch_ta_align(c->stream, n_runs, n_cams, ro, derr);
  if (e == hipSuccess) e = fea::launch_ta_losses(c->stream, n_runs, n_cams, n_pairs, doff, dent, dpi, dpj, tg, ro, pl, cl, rl);
  if (e == hipSuccess) e = fea::launch_ta_merge(c->stream, n_runs, n_cams, ro, cl, om0, drun);
  // the merged centres, one more loop
  if (e == hipSuccess) e = hipMemsetAsync(m, 0, n3 * sizeof(double), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(v, 0, n3 * sizeof(double), c->stream);
  TaPhase fin{c, 1, n_cams, n_pairs, doff, dent, doth, tg, {om0, om1}, m, v, ctr,
              o.beta1, o.beta2, o.adam_eps, o.iters_final > 0 ? std::pow(o.lr_end_frac, 1.0 / o.iters_final) : 1.0};
  if (e == hipSuccess) e = fea::launch_ta_counters(c->stream, ctr, o.lr_final);
  if (e == hipSuccess) e = fin.run(o.iters_final);
  double* fo = fin.o[fin.parity];
  if (e == hipSuccess) e = fea::launch_ta_align(c->stream, 1, n_cams, fo, derr);
  if (e == hipSuccess) e = fea::launch_ta_losses(c->stream, 1, n_cams, n_pairs, doff, dent, dpi, dpj, tg, fo, pl, nullptr, fl);
  if (e == hipSuccess && ev[1]) e = hipEventRecord(ev[1], c->stream);
  int32_t herr = 0;
  double hfl = 0.0;
  if (e == hipSuccess) e = fetch(c->stream, o_out, fo, n3);
  if (e == hipSuccess) e = fetch(c->stream, run_of_cam, drun, (size_t)n_cams);
  if (e == hipSuccess) e = fetch(c->stream, run_loss, rl, (size_t)n_runs);
  if (e == hipSuccess) e = fetch(c->stream, run_o, ro, r3);
  if (e == hipSuccess) e = fetch(c->stream, cam_loss, cl, (size_t)n_cams * n_runs);
  if (e == hipSuccess) e = fetch(c->stream, &hfl, fl, 1);
  if (e == hipSuccess) e = fetch(c->stream, &herr, derr, 1);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && ms) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  HIP_OR_FAIL(c, e);
  if (herr) return fail(c, FEA_EDEGENERATE, "all camera centres coincide");
  if (final_loss) *final_loss = hfl;
  return FEA_OK;
}

fea_status fea_focal_vote(fea_ctx* c, int32_t n_cams, int64_t n_pairs, const int32_t* pair_i,
                          const int32_t* pair_j, const double* F, const int32_t* group, const double* f_cur,
                          int32_t n_cand, const double* cand_f, double tau, double* f_best, int32_t* k_best,
                          double* votes, float* ms) {
  if (!c) return FEA_EINVAL;
  if (!pair_i || !pair_j || !F || !cand_f || !f_best)
    return fail(c, FEA_EINVAL, "pair_i, pair_j, F, cand_f and f_best are required");
  if (n_cams < 2 || n_pairs < 1 || n_pairs > INT32_MAX) return fail(c, FEA_EINVAL, "need n_cams >= 2 and n_pairs >= 1");
  if (n_cand < 1 || n_cand > (1 << 20)) return fail(c, FEA_EINVAL, "n_cand must be in [1, 2^20]");
  if (!std::isfinite(tau) || !(tau > 0.0)) return fail(c, FEA_EINVAL, "tau must be finite and > 0");
  std::vector<int32_t> grp(group ? group : nullptr, group ? group + n_cams : nullptr);
  if (!group) grp.assign((size_t)n_cams, 0);
  int32_t G = 0;
  for (int32_t g : grp) {
    if (g < 0 || g >= n_cams) return fail(c, FEA_EINVAL, "group ids must be in [0, n_cams)");
    G = std::max(G, g + 1);
  }
  std::vector<double> fc((size_t)G, 1.0);
  if (G > 1) {
    if (!f_cur) return fail(c, FEA_EINVAL, "f_cur is required with more than one group");
    for (int32_t g = 0; g < G; ++g) {
      if (!std::isfinite(f_cur[g]) || !(f_cur[g] > 0.0)) return fail(c, FEA_EINVAL, "f_cur must be finite and > 0");
      fc[g] = f_cur[g];
    }
  }
  for (int32_t k = 0; k < n_cand; ++k)
    if (!std::isfinite(cand_f[k]) || !(cand_f[k] > 0.0))
      return fail(c, FEA_EINVAL, "candidate focal lengths must be finite and > 0");
  if (!all_finite(F, (size_t)9 * n_pairs)) return fail(c, FEA_ENONFINITE, "non-finite fundamental matrix");
  // group -> its pairs, in pair order (a pair within one group is listed once)
  std::vector<int32_t> off((size_t)G + 1, 0), lst;
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int32_t i = pair_i[p], j = pair_j[p];
    if (i < 0 || j < 0 || i >= n_cams || j >= n_cams || i == j) return fail(c, FEA_EINVAL, "invalid camera pair");
    off[grp[i] + 1]++;
    if (grp[j] != grp[i]) off[grp[j] + 1]++;
  }
  for (int32_t g = 0; g < G; ++g) off[g + 1] += off[g];
  lst.assign((size_t)off[G], 0);
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int32_t gi = grp[pair_i[p]], gj = grp[pair_j[p]];
    lst[fill[gi]++] = (int32_t)p;
    if (gj != gi) lst[fill[gj]++] = (int32_t)p;
  }
  DeviceGuard dg(c->device);
  CallScratch sc(c->stream);
  int32_t *dpi, *dpj, *dgrp, *doff, *dlst, *dkb;
  double *dF, *dfc, *dcand, *dvotes, *dfb;
  HIP_OR_FAIL(c, sc.put(dpi, pair_i, (size_t)n_pairs));
  HIP_OR_FAIL(c, sc.put(dpj, pair_j, (size_t)n_pairs));
  HIP_OR_FAIL(c, sc.put(dgrp, grp.data(), grp.size()));
  HIP_OR_FAIL(c, sc.put(doff, off.data(), off.size()));
  HIP_OR_FAIL(c, sc.put(dlst, lst.data(), lst.size()));
  HIP_OR_FAIL(c, sc.put(dF, F, (size_t)9 * n_pairs));
  HIP_OR_FAIL(c, sc.put(dfc, fc.data(), fc.size()));
  HIP_OR_FAIL(c, sc.put(dcand, cand_f, (size_t)n_cand));
  HIP_OR_FAIL(c, sc.alloc(dvotes, (size_t)G * n_cand));
  HIP_OR_FAIL(c, sc.alloc(dfb, (size_t)G));
  HIP_OR_FAIL(c, sc.alloc(dkb, (size_t)G));
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (ms) {
    HIP_OR_FAIL(c, hipEventCreate(&ev[0]));
    HIP_OR_FAIL(c, hipEventCreate(&ev[1]));
  }
  hipError_t e = fea::launch_fv_vote(c->stream, G, n_cand, doff, dlst, dpi, dpj, dgrp, dF, dfc, dcand, tau, dvotes,
                                     ev[0], ev[1]);
  if (e == hipSuccess) e = fea::launch_fv_best(c->stream, G, n_cand, dvotes, dcand, dfb, dkb);
  if (e == hipSuccess) e = fetch(c->stream, f_best, dfb, (size_t)G);
  if (e == hipSuccess) e = fetch(c->stream, k_best, dkb, (size_t)G);
  if (e == hipSuccess) e = fetch(c->stream, votes, dvotes, (size_t)G * n_cand);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && ms) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  HIP_OR_FAIL(c, e);
  return FEA_OK;
}

fea_status fea_ra_default_options(fea_ra_options* o) {
  if (!o) return FEA_EINVAL;
  o->init_iters = 200000;
  o->iters = 1000;
  o->lr = 1e-2;
  o->lr_end_frac = 1e-2;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->adam_eps = 1e-12;
  return FEA_OK;
}

}  // extern "C"

namespace {

// Runs `iters` iterations of `step` (which flips `parity`), an even number
// at a time from a captured graph, the rest launched directly.
template <class Step>
hipError_t run_captured(hipStream_t st, int iters, int& parity, Step step) {
  constexpr int kChunk = 64;
  int done = 0;
  if (iters >= 2 * kChunk) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    const int p0 = parity;
    for (int k = 0; k < kChunk && le == hipSuccess; ++k) le = step();
    e = hipStreamEndCapture(st, &g);
    parity = p0;
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    for (; e == hipSuccess && done + kChunk <= iters; done += kChunk) e = hipGraphLaunch(x, st);
    if (x) (void)hipGraphExecDestroy(x);
    if (e != hipSuccess) return e;
  }
  for (; done < iters; ++done) {
    hipError_t e = step();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

namespace {

// Lanczos scratch (device arrays): basis V [(kmax+1) x n], the step's vector
// w [n], the apply kernel's per-camera side output sq [n], both passes'
// projections h1, h2, the tridiagonal alpha, beta, the Ritz coefficients s
// [kmax+1] and the norm partials.
struct LzScratch {
  int64_t n = 0;
  int kmax = 0;
  double *V = nullptr, *w = nullptr, *sq = nullptr, *h1 = nullptr, *h2 = nullptr, *alpha = nullptr,
         *beta = nullptr, *s = nullptr, *part = nullptr;
};

// A = wm M + wp diag(c1 c1^T) over the pair graph (device arrays).
struct LzOperator {
  int n_cams;
  const int32_t *cam_off, *cam_ent, *pair_i, *pair_j;
  const double* Rrel;
  const double* c1;
  double wm, wp;
};

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..m) and off-diagonal b[0..m-1) (the signs of the pivots of
// its LDL^T factorisation, Sylvester's law of inertia).
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, int m, double x) {
  int count = 0;
  double q = 1.0;
  for (int i = 0; i < m; ++i) {
    q = (a[i] - x) - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
    if (q == 0.0) q = -1e-300;  // a zero pivot: x is an eigenvalue; count it below
    if (q < 0.0) ++count;
  }
  return count;
}

// The smallest eigenvalue of that matrix by bisection between Gershgorin
// bounds, to the last bits.
double tridiag_smallest(const std::vector<double>& a, const std::vector<double>& b, int m) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_below(a, b, m, mid) >= 1)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// A unit eigenvector of that matrix for eigenvalue theta: two steps of
// inverse iteration, (T - theta I) x_new = x, by Gaussian elimination with
// partial pivoting on the dense m x m matrix (m <= a few hundred).
std::vector<double> tridiag_eigvec(const std::vector<double>& a, const std::vector<double>& b, int m, double theta) {
  std::vector<double> x(m, 1.0 / std::sqrt((double)m));
  const double scale = std::max(1e-300, std::fabs(theta) + std::fabs(a[0]));
  for (int rep = 0; rep < 2; ++rep) {
    std::vector<double> M((size_t)m * m, 0.0), r(x);
    for (int i = 0; i < m; ++i) {
      M[(size_t)i * m + i] = a[i] - theta;
      if (i + 1 < m) M[(size_t)i * m + i + 1] = M[(size_t)(i + 1) * m + i] = b[i];
    }
    for (int col = 0; col < m; ++col) {
      int piv = col;
      for (int i = col + 1; i < m; ++i)
        if (std::fabs(M[(size_t)i * m + col]) > std::fabs(M[(size_t)piv * m + col])) piv = i;
      if (piv != col) {
        for (int k = 0; k < m; ++k) std::swap(M[(size_t)col * m + k], M[(size_t)piv * m + k]);
        std::swap(r[col], r[piv]);
      }
      double d = M[(size_t)col * m + col];
      if (std::fabs(d) < 1e-15 * scale) d = M[(size_t)col * m + col] = (d < 0 ? -1e-15 : 1e-15) * scale;
      for (int i = col + 1; i < m; ++i) {
        const double l = M[(size_t)i * m + col] / d;
        if (l == 0.0) continue;
        for (int k = col; k < m; ++k) M[(size_t)i * m + k] -= l * M[(size_t)col * m + k];
        r[i] -= l * r[col];
      }
    }
    for (int i = m - 1; i >= 0; --i) {
      double t = r[i];
      for (int k = i + 1; k < m; ++k) t -= M[(size_t)i * m + k] * x[k];
      x[i] = t / M[(size_t)i * m + i];
    }
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return std::vector<double>(m, 0.0);
    for (double& v : x) v /= nrm;
  }
  return x;
}

// The Ritz vector of A's smallest eigenvalue into y (device [n]): Lanczos
// from the start vector v0 (host [n]), at most kmax steps between restarts
// (a restart starts again from the current Ritz vector), until the smallest
// Ritz value changes by at most 3e-5 of itself (or 1e-12 sigma) over 16
// steps, the Krylov space is exhausted, or max_apply products with A have
// run.  Inside the near-null cluster (split by noise) any vector is a valid
// column, so the test only has to see the bottom of the spectrum arrive.
hipError_t lanczos_bottom(hipStream_t st, const LzOperator& A, double sigma, const double* v0, int max_apply,
                          LzScratch& z, double* y) {
  const int64_t n = z.n;
  std::vector<double> v(v0, v0 + n);
  double nrm = 0.0;
  for (double t : v) nrm += t * t;
  nrm = std::sqrt(nrm);
  if (!(nrm > 0.0)) return hipErrorInvalidValue;
  for (double& t : v) t /= nrm;
  hipError_t e = hipMemcpyAsync(z.V, v.data(), n * sizeof(double), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  int applied = 0;
  double theta_prev = std::numeric_limits<double>::quiet_NaN();
  std::vector<double> a, b;
  for (;;) {
    int m = 0;
    bool done = false;
    double theta = 0.0;
    for (int j = 0; j < z.kmax; ++j) {
      e = fea::launch_lz_step(st, A.n_cams, A.cam_off, A.cam_ent, A.pair_i, A.pair_j, A.Rrel, A.c1, A.wm, A.wp, z.V,
                              j, z.w, z.sq, z.h1, z.h2, z.part, z.alpha, z.beta);
      if (e != hipSuccess) return e;
      ++applied;
      m = j + 1;
      if (m % 16 != 0 && m != z.kmax && applied < max_apply) continue;
      a.assign(m, 0.0);
      b.assign(m, 0.0);
      if ((e = hipMemcpyAsync(a.data(), z.alpha, m * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (e = hipMemcpyAsync(b.data(), z.beta, m * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (e = hipStreamSynchronize(st)) != hipSuccess)
        return e;
      theta = tridiag_smallest(a, b, m);
      const bool exhausted = !(b[m - 1] > 1e-14 * sigma);
      const bool settled = std::fabs(theta - theta_prev) <= 3e-5 * std::fabs(theta) + 1e-12 * sigma;
      theta_prev = theta;
      if (exhausted || settled || applied >= max_apply) {
        done = true;
        break;
      }
    }
    // the Ritz vector of the basis built so far
    const std::vector<double> sv = tridiag_eigvec(a, b, m, theta);
    if ((e = hipMemcpyAsync(z.s, sv.data(), m * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if ((e = fea::launch_lz_combine(st, n, m, z.V, z.s, done ? y : z.w)) != hipSuccess) return e;
    if (done) return hipStreamSynchronize(st);
    // restart from it (a unit vector: the basis is orthonormal)
    if ((e = hipMemcpyAsync(z.V, z.w, n * sizeof(double), hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
  }
}

}  // namespace

extern "C" {

fea_status fea_rotation_averaging(fea_ctx* c, int32_t n_cams, int64_t n_pairs, const int32_t* pair_i,
                                  const int32_t* pair_j, const double* R_rel, const double* v0,
                                  const double* a6_init, const fea_ra_options* opt, double* R_out, double* R_init,
                                  double* loss, float* ms) {
  if (!c) return FEA_EINVAL;
  if (!pair_i || !pair_j || !R_rel || !R_out || (!v0 && !a6_init))
    return fail(c, FEA_EINVAL, "pair_i, pair_j, R_rel, R_out and v0 (or a6_init) are required");
  if (n_cams < 2 || n_pairs < 1 || n_pairs > INT32_MAX / 2)
    return fail(c, FEA_EINVAL, "need n_cams >= 2 and 1 <= n_pairs < 2^30");
  fea_ra_options o;
  fea_ra_default_options(&o);
  if (opt) o = *opt;
  if (o.init_iters < 0 || o.iters < 0 || !(o.lr > 0) || !(o.lr_end_frac > 0) || !(o.lr_end_frac <= 1) ||
      !(o.beta1 >= 0 && o.beta1 < 1) || !(o.beta2 >= 0 && o.beta2 < 1) || !(o.adam_eps >= 0))
    return fail(c, FEA_EINVAL, "invalid rotation options");
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int32_t i = pair_i[p], j = pair_j[p];
    if (i < 0 || j < 0 || i >= n_cams || j >= n_cams || i == j) return fail(c, FEA_EINVAL, "invalid camera pair");
  }
  if (!all_finite(R_rel, (size_t)9 * n_pairs)) return fail(c, FEA_ENONFINITE, "non-finite relative rotation");
  if (v0 && !all_finite(v0, (size_t)6 * n_cams)) return fail(c, FEA_ENONFINITE, "non-finite start vector");
  if (a6_init && !all_finite(a6_init, (size_t)6 * n_cams)) return fail(c, FEA_ENONFINITE, "non-finite a6_init");
  std::vector<int32_t> off, ent;
  camera_entries(n_cams, n_pairs, pair_i, pair_j, off, ent);
  int32_t max_deg = 0;
  for (int32_t i = 0; i < n_cams; ++i) max_deg = std::max(max_deg, off[i + 1] - off[i]);
  const size_t N3 = (size_t)3 * n_cams, N6 = (size_t)6 * n_cams;

  DeviceGuard g(c->device);
  CallScratch sc(c->stream);
  int32_t *dpi, *dpj, *doff, *dent, *derr;
  double *dR, *col, *c1, *a6[2], *m, *v, *dloss;
  fea::TaCounters* ctr;
  HIP_OR_FAIL(c, sc.put(dpi, pair_i, (size_t)n_pairs));
  HIP_OR_FAIL(c, sc.put(dpj, pair_j, (size_t)n_pairs));
  HIP_OR_FAIL(c, sc.put(doff, off.data(), off.size()));
  HIP_OR_FAIL(c, sc.put(dent, ent.data(), ent.size()));
  HIP_OR_FAIL(c, sc.put(dR, R_rel, (size_t)9 * n_pairs));
  HIP_OR_FAIL(c, sc.alloc(col, N3));  // the column being solved for
  HIP_OR_FAIL(c, sc.alloc(c1, N3));
  HIP_OR_FAIL(c, sc.alloc(a6[0], N6));
  HIP_OR_FAIL(c, sc.alloc(a6[1], N6));
  HIP_OR_FAIL(c, sc.alloc(m, N6));
  HIP_OR_FAIL(c, sc.alloc(v, N6));
  HIP_OR_FAIL(c, sc.alloc(dloss, 2));
  HIP_OR_FAIL(c, sc.alloc(derr, 1));
  HIP_OR_FAIL(c, sc.alloc(ctr, 1));
  HIP_OR_FAIL(c, hipMemsetAsync(derr, 0, sizeof(int32_t), c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(m, 0, N6 * sizeof(double), c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(v, 0, N6 * sizeof(double), c->stream));
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (ms) {
    HIP_OR_FAIL(c, hipEventCreate(&ev[0]));
    HIP_OR_FAIL(c, hipEventCreate(&ev[1]));
  }
  hipError_t e = hipSuccess;
  if (ev[0]) e = hipEventRecord(ev[0], c->stream);
  if (a6_init) {
    if (e == hipSuccess)
      e = hipMemcpyAsync(a6[0], a6_init, N6 * sizeof(double), hipMemcpyHostToDevice, c->stream);
  } else {
    // column 1: smallest eigenvector of M; column 2: of M/|P| + B/|I|, each
    // by Lanczos from its start vector; the spectrum's scale (the Gershgorin
    // bound) sets the stopping test's absolute term
    const double sig1 = 2.0 * max_deg, sig2 = 2.0 * (max_deg / (double)n_pairs + 0.5 / n_cams);
    LzScratch z;
    z.n = (int64_t)N3;
    z.kmax = (int)std::min<int64_t>({256, z.n, std::max<int64_t>(o.init_iters, 1)});
    if (e == hipSuccess) e = sc.alloc(z.V, (size_t)(z.kmax + 1) * N3);
    if (e == hipSuccess) e = sc.alloc(z.w, N3);
    if (e == hipSuccess) e = sc.alloc(z.sq, N3);
    if (e == hipSuccess) e = sc.alloc(z.h1, (size_t)z.kmax + 1);
    if (e == hipSuccess) e = sc.alloc(z.h2, (size_t)z.kmax + 1);
    if (e == hipSuccess) e = sc.alloc(z.alpha, (size_t)z.kmax + 1);
    if (e == hipSuccess) e = sc.alloc(z.beta, (size_t)z.kmax + 1);
    if (e == hipSuccess) e = sc.alloc(z.s, (size_t)z.kmax + 1);
    if (e == hipSuccess) e = sc.alloc(z.part, (size_t)fea::lz_orth_blocks(z.n));
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
      const LzOperator A{n_cams, doff, dent, dpi, dpj, dR, k == 0 ? nullptr : c1, k == 0 ? 1.0 : 1.0 / n_pairs,
                         1.0 / n_cams};
      e = lanczos_bottom(c->stream, A, k == 0 ? sig1 : sig2, v0 + (size_t)k * N3, o.init_iters, z, col);
      if (e == hipSuccess)
        e = fea::launch_ra_columns(c->stream, n_cams, col, k == 0 ? nullptr : c1, k == 0 ? c1 : a6[0], derr);
    }
  }
  if (e == hipSuccess) e = fea::launch_ra_loss(c->stream, n_pairs, dpi, dpj, dR, a6[0], dloss);
  double* dRinit = nullptr;
  if (e == hipSuccess && R_init) {
    e = sc.alloc(dRinit, (size_t)9 * n_cams);
    if (e == hipSuccess) e = fea::launch_ra_to_R(c->stream, n_cams, a6[0], dRinit);
  }
  int par = 0;
  const double decay = o.iters > 0 ? std::pow(o.lr_end_frac, 1.0 / o.iters) : 1.0;
  if (e == hipSuccess) e = fea::launch_ta_counters(c->stream, ctr, o.lr);
  auto ostep = [&]() {
    hipError_t r = fea::launch_ra_step(c->stream, n_cams, n_pairs, doff, dent, dpi, dpj, dR, a6[par], a6[par ^ 1], m,
                                       v, ctr, par, o.beta1, o.beta2, o.adam_eps, decay);
    par ^= 1;
    return r;
  };
  if (e == hipSuccess) e = run_captured(c->stream, o.iters, par, ostep);
  if (e == hipSuccess) e = fea::launch_ra_loss(c->stream, n_pairs, dpi, dpj, dR, a6[par], dloss + 1);
  double* dRout = nullptr;
  if (e == hipSuccess) e = sc.alloc(dRout, (size_t)9 * n_cams);
  if (e == hipSuccess) e = fea::launch_ra_to_R(c->stream, n_cams, a6[par], dRout);
  if (e == hipSuccess && ev[1]) e = hipEventRecord(ev[1], c->stream);
  int32_t herr = 0;
  if (e == hipSuccess) e = fetch(c->stream, R_out, dRout, (size_t)9 * n_cams);
  if (e == hipSuccess && R_init) e = fetch(c->stream, R_init, dRinit, (size_t)9 * n_cams);
  if (e == hipSuccess) e = fetch(c->stream, loss, dloss, 2);
  if (e == hipSuccess) e = fetch(c->stream, &herr, derr, 1);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && ms) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  HIP_OR_FAIL(c, e);
  if (herr) return fail(c, FEA_EDEGENERATE, "a camera's column vanished in the initialisation (unconnected camera?)");
  return FEA_OK;
}

}  // extern "C"
