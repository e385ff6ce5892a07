// Uneven batches: many path instances (grid sizes, screen counts,
// wavelengths and distances of their own) propagated by one call.  Each
// instance has its own plan.  In the forward pass, instances that share the
// grid size, realization count and transfer-function form run as groups,
// one launch per pass and step for all members (group.cpp); the others run
// their own plan's call.  Groups and single instances are spread over a few
// internal streams (longest processing time first, cost R N^2 (M + 1)),
// forked from and joined back to the caller's stream with events, each
// stream with its own slice of the workspace.  The adjoint runs the same
// groups backwards.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <map>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "group.hpp"
#include "report.hpp"
#include "turpy.h"

namespace {

constexpr int kLanes = 4;  // internal streams (the device's hardware queues)
constexpr size_t kAlign = 256;
constexpr uint64_t kSeedStep = 0x9E3779B97F4A7C15ull;
constexpr size_t kDefaultGroupLimit = size_t(1) << 30;
std::atomic<size_t> g_group_limit{kDefaultGroupLimit};

// Bytes a member keeps in flight during a group's pass: its fields and its
// workspace slice.
size_t member_bytes(const turpy_plan* pl, const turpy_path& p) {
  size_t ws = 0;
  turpy_workspace_size(pl, TURPY_OP_PROPAGATE, &ws);
  return static_cast<size_t>(p.realizations) * p.n * p.n * 8 + ws;
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// A unit of work on one internal stream: a group's forward pass, or one
// instance's own call.
struct Unit {
  int group;     // index into turpy_batch::groups, or -1
  int instance;  // instance index when group < 0
};

}  // namespace

struct turpy_batch {
  int device = 0;
  std::vector<turpy_plan*> plans;
  std::vector<turpy_path> paths;
  std::vector<int64_t> offsets;      // field offsets (complex elements)
  std::vector<int64_t> ck_offsets;   // checkpoint offsets (complex elements)
  std::vector<turpy::Group*> groups;
  std::vector<std::vector<int>> group_members;  // instances of each group
  std::vector<std::vector<Unit>> lanes[2];  // work per internal stream: forward, backward
  std::vector<size_t> lane_ws[2];           // workspace bytes per lane: forward, backward
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
};

namespace {

turpy_status fail_hip(hipError_t e, const char* where) {
  return turpy::report(TURPY_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

size_t total_ws(const turpy_batch* b, int which) {
  size_t s = 0;
  for (size_t v : b->lane_ws[which]) s += align_up(v);
  return s;
}

// Fork the lanes from the caller's stream, run `fn(unit, lane stream, lane
// workspace)` for every unit of the pass (`which`: 0 forward, 1 adjoint),
// join the lanes back.
template <class Fn>
turpy_status run(turpy_batch* b, void* ws, int which, void* stream, Fn&& fn) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipEventRecord(b->fork, st);
  if (e != hipSuccess) return fail_hip(e, "batch: fork");
  char* base = static_cast<char*>(ws);
  turpy_status status = TURPY_OK;
  for (size_t l = 0; l < b->lanes[which].size(); ++l) {
    e = hipStreamWaitEvent(b->streams[l], b->fork, 0);
    if (e != hipSuccess) return fail_hip(e, "batch: fork");
    for (const Unit& u : b->lanes[which][l]) {
      status = fn(u, b->streams[l], base, b->lane_ws[which][l]);
      if (status != TURPY_OK) break;
    }
    e = hipEventRecord(b->done[l], b->streams[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->done[l], 0);
    if (e != hipSuccess) return fail_hip(e, "batch: join");
    if (status != TURPY_OK) return status;
    base += align_up(b->lane_ws[which][l]);
  }
  return TURPY_OK;
}

}  // namespace

extern "C" {

turpy_status turpy_batch_destroy(turpy_batch* b) {
  if (!b) return TURPY_OK;
  for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  for (turpy::Group* g : b->groups) turpy::group_destroy(g);
  for (turpy_plan* p : b->plans) turpy_plan_destroy(p);
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
  return TURPY_OK;
}

turpy_status turpy_batch_create(turpy_batch** out, const turpy_path* paths, const int64_t* field_offsets,
                                int32_t num_paths, uint32_t flags) {
  if (!out || !paths || !field_offsets || num_paths < 1)
    return turpy::report(TURPY_E_INVALID, "batch_create: NULL argument or num_paths < 1");
  *out = nullptr;
  if (flags & TURPY_SCREEN_CHECKPOINTS)
    return turpy::report(TURPY_E_INVALID, "batch_create: TURPY_SCREEN_CHECKPOINTS is not available for batches");
  turpy_batch* b = new turpy_batch;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return turpy::report(TURPY_E_HIP, "batch_create: no current device");
  }
  int64_t ck = 0;
  for (int32_t i = 0; i < num_paths; ++i) {
    if (field_offsets[i] < 0) {
      turpy_batch_destroy(b);
      return turpy::report(TURPY_E_INVALID, "batch_create: field_offsets[%d] < 0", i);
    }
    turpy_plan* p = nullptr;
    if (turpy_status s = turpy_plan_create(&p, &paths[i], flags)) {
      turpy_batch_destroy(b);
      return s;  // the message names the path's problem
    }
    b->plans.push_back(p);
    turpy_path q = paths[i];
    q.dz = nullptr;  // the caller's arrays are not kept
    q.cn2dz = nullptr;
    b->paths.push_back(q);
    b->offsets.push_back(field_offsets[i]);
    b->ck_offsets.push_back(ck);
    ck += paths[i].realizations * paths[i].num_screens * static_cast<int64_t>(paths[i].n) * paths[i].n;
  }
  // fields of different instances must not overlap
  std::vector<int> order(num_paths);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int c) { return b->offsets[a] < b->offsets[c]; });
  for (size_t k = 1; k < order.size(); ++k) {
    const turpy_path& p = b->paths[order[k - 1]];
    const int64_t end = b->offsets[order[k - 1]] + p.realizations * static_cast<int64_t>(p.n) * p.n;
    if (end > b->offsets[order[k]]) {
      turpy_batch_destroy(b);
      return turpy::report(TURPY_E_INVALID, "batch_create: fields of instances %d and %d overlap",
                           order[k - 1], order[k]);
    }
  }
  // forward groups: eligible instances with the same key, two or more
  std::map<std::string, std::vector<int>> by_key;
  for (int i = 0; i < num_paths; ++i)
    if (turpy::group_eligible(b->plans[i])) by_key[turpy::group_key(b->plans[i])].push_back(i);
  std::vector<char> grouped(num_paths, 0);
  std::vector<int> group_of(num_paths, -1);
  const size_t limit = g_group_limit.load();
  for (const auto& kv : by_key) {
    // cut the key's instances, in batch order, into groups within the limit
    std::vector<std::vector<int>> cuts(1);
    size_t used = 0;
    for (int i : kv.second) {
      const size_t m = member_bytes(b->plans[i], b->paths[i]);
      if (!cuts.back().empty() && used + m > limit) {
        cuts.emplace_back();
        used = 0;
      }
      cuts.back().push_back(i);
      used += m;
    }
    for (const std::vector<int>& cut : cuts) {
      if (cut.size() < 2) continue;
      std::vector<turpy::GroupMember> members;
      for (int i : cut) {
        members.push_back(turpy::GroupMember{b->plans[i], kSeedStep * static_cast<uint64_t>(i),
                                             static_cast<size_t>(b->offsets[i]) * 8,
                                             static_cast<size_t>(b->ck_offsets[i]) * 8});
        grouped[i] = 1;
        group_of[i] = static_cast<int>(b->groups.size());
      }
      turpy::Group* g = nullptr;
      if (turpy_status s = turpy::group_create(members, &g)) {
        turpy_batch_destroy(b);
        return s;
      }
      b->groups.push_back(g);
      b->group_members.push_back(cut);
    }
  }
  // longest processing time first over the lanes, for each pass
  auto cost_of = [&](int i) {
    return static_cast<double>(b->paths[i].realizations) * b->paths[i].n * b->paths[i].n *
           (b->paths[i].num_screens + 1);
  };
  std::vector<std::pair<Unit, double>> units[2];
  for (int w = 0; w < 2; ++w) {
    for (size_t gi = 0; gi < b->groups.size(); ++gi)
      units[w].push_back({Unit{static_cast<int>(gi), -1}, static_cast<double>(turpy::group_cost(b->groups[gi]))});
    for (int i = 0; i < num_paths; ++i)
      if (!grouped[i]) units[w].push_back({Unit{-1, i}, cost_of(i)});
  }
  int lanes_needed = 0;
  for (int w = 0; w < 2; ++w) {
    auto& us = units[w];
    std::stable_sort(us.begin(), us.end(), [](const auto& a, const auto& c) { return a.second > c.second; });
    const int lanes = std::min<int>(kLanes, static_cast<int>(us.size()));
    lanes_needed = std::max(lanes_needed, lanes);
    std::vector<double> load(lanes, 0.0);
    b->lanes[w].assign(lanes, {});
    b->lane_ws[w].assign(lanes, 0);
    for (const auto& u : us) {
      const int l = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      b->lanes[w][l].push_back(u.first);
      load[l] += u.second;
      const int op = w == 0 ? TURPY_OP_PROPAGATE : TURPY_OP_PROPAGATE_BACKWARD;
      size_t need = 0;
      if (u.first.group >= 0) {
        need = turpy::group_workspace(b->groups[u.first.group]);
        if (w == 1)  // without grad_u_in the members' own adjoints run one by one
          for (int i = 0; i < num_paths; ++i)
            if (group_of[i] == u.first.group) {
              size_t v = 0;
              turpy_workspace_size(b->plans[i], op, &v);
              need = std::max(need, v);
            }
      } else {
        turpy_workspace_size(b->plans[u.first.instance], op, &need);
      }
      b->lane_ws[w][l] = std::max(b->lane_ws[w][l], need);
    }
  }
  const int lanes = lanes_needed;
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int l = 0; e == hipSuccess && l < lanes; ++l) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) b->streams.push_back(s);
    hipEvent_t ev = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->done.push_back(ev);
  }
  if (e != hipSuccess) {
    turpy_batch_destroy(b);
    return fail_hip(e, "batch_create: streams and events");
  }
  *out = b;
  return TURPY_OK;
}

turpy_status turpy_batch_group_limit(size_t bytes) {
  g_group_limit.store(bytes ? bytes : kDefaultGroupLimit);
  return TURPY_OK;
}

turpy_status turpy_batch_bind_time(turpy_batch* b, const void* dev_t) {
  if (!b) return turpy::report(TURPY_E_INVALID, "batch_bind_time: NULL batch");
  for (turpy_plan* p : b->plans)
    if (turpy_status s = turpy_plan_bind_time(p, dev_t)) return s;
  return TURPY_OK;
}

turpy_status turpy_batch_workspace_size(const turpy_batch* b, int32_t op, size_t* bytes) {
  if (!b || !bytes) return turpy::report(TURPY_E_INVALID, "batch_workspace_size: NULL argument");
  if (op == TURPY_OP_PROPAGATE) {
    *bytes = total_ws(b, 0);
  } else if (op == TURPY_OP_PROPAGATE_BACKWARD) {
    *bytes = total_ws(b, 1);
  } else if (op == TURPY_OP_TUNE) {
    size_t m = 0;
    for (const turpy_plan* p : b->plans) {
      size_t v = 0;
      turpy_workspace_size(p, TURPY_OP_TUNE, &v);
      m = std::max(m, v);
    }
    *bytes = m;
  } else {
    return turpy::report(TURPY_E_INVALID, "batch_workspace_size: op %d is not available for batches", op);
  }
  return TURPY_OK;
}

turpy_status turpy_batch_tune(turpy_batch* b, uint32_t flags, void* ws, size_t ws_bytes, void* stream) {
  if (!b) return turpy::report(TURPY_E_INVALID, "batch_tune: NULL batch");
  std::set<std::string> done;  // keys measured by this call
  for (turpy_plan* p : b->plans) {
    const std::string key = turpy::tune_signature(p);
    const uint32_t f = done.count(key) ? (flags & ~TURPY_TUNE_FORCE) : flags;
    if (turpy_status s = turpy_plan_tune(p, f, ws, ws_bytes, stream, nullptr, nullptr)) return s;
    done.insert(key);
  }
  return TURPY_OK;
}

turpy_status turpy_batch_propagate(turpy_batch* b, uint64_t seed, int64_t t, const void* u_in, void* u_out,
                                   void* checkpoints, void* ws, size_t ws_bytes, void* stream) {
  if (!b || !u_in || !u_out) return turpy::report(TURPY_E_INVALID, "batch_propagate: NULL argument");
  if (t < 0 || t > 0xFFFFFFFFll) return turpy::report(TURPY_E_INVALID, "batch_propagate: t out of range");
  if (!ws || ws_bytes < total_ws(b, 0))
    return turpy::report(TURPY_E_WORKSPACE, "batch_propagate: workspace %zu < %zu bytes", ws_bytes,
                         total_ws(b, 0));
  const auto* in = static_cast<const char*>(u_in);
  auto* out = static_cast<char*>(u_out);
  auto* ck = static_cast<char*>(checkpoints);
  return run(b, ws, 0, stream, [&](const Unit& u, hipStream_t st, char* lws, size_t lbytes) {
    if (u.group >= 0)
      return turpy::group_propagate(b->groups[u.group], seed, static_cast<uint32_t>(t), u_in, u_out, checkpoints, lws,
                                    st);
    const int i = u.instance;
    const int64_t plane = static_cast<int64_t>(b->paths[i].n) * b->paths[i].n;
    const size_t off = static_cast<size_t>(b->offsets[i]) * 8;
    return turpy_propagate(b->plans[i], seed + kSeedStep * static_cast<uint64_t>(i), t, in + off, plane,
                           TURPY_SCREENS_SYNTH, nullptr, out + off,
                           ck ? ck + static_cast<size_t>(b->ck_offsets[i]) * 8 : nullptr, lws, lbytes, st);
  });
}

turpy_status turpy_batch_propagate_backward(turpy_batch* b, uint64_t seed, int64_t t, const void* grad_u_out,
                                            const void* checkpoints, void* grad_u_in, float* grad_screens,
                                            void* ws, size_t ws_bytes, void* stream) {
  if (!b || !grad_u_out) return turpy::report(TURPY_E_INVALID, "batch_propagate_backward: NULL argument");
  if (t < 0 || t > 0xFFFFFFFFll) return turpy::report(TURPY_E_INVALID, "batch_propagate_backward: t out of range");
  if (!ws || ws_bytes < total_ws(b, 1))
    return turpy::report(TURPY_E_WORKSPACE, "batch_propagate_backward: workspace %zu < %zu bytes", ws_bytes,
                         total_ws(b, 1));
  const auto* gout = static_cast<const char*>(grad_u_out);
  const auto* ck = static_cast<const char*>(checkpoints);
  auto* gin = static_cast<char*>(grad_u_in);
  auto own = [&](int i, hipStream_t st, char* lws, size_t lbytes) {
    const size_t off = static_cast<size_t>(b->offsets[i]) * 8;
    const size_t co = static_cast<size_t>(b->ck_offsets[i]);
    return turpy_propagate_backward(b->plans[i], seed + kSeedStep * static_cast<uint64_t>(i), t, gout + off,
                                    ck ? ck + co * 8 : nullptr, TURPY_SCREENS_SYNTH, nullptr,
                                    gin ? gin + off : nullptr, int64_t(b->paths[i].n) * b->paths[i].n,
                                    grad_screens ? grad_screens + co : nullptr, lws, lbytes, st);
  };
  return run(b, ws, 1, stream, [&](const Unit& u, hipStream_t st, char* lws, size_t lbytes) {
    if (u.group < 0) return own(u.instance, st, lws, lbytes);
    if (ck && gin)
      return turpy::group_propagate_backward(b->groups[u.group], seed, static_cast<uint32_t>(t), grad_u_out, ck, gin,
                                             grad_screens, lws, st);
    for (int i : b->group_members[u.group])
      if (turpy_status s = own(i, st, lws, lbytes)) return s;
    return TURPY_OK;
  });
}

}  // extern "C"
