// Grouped launches of uneven batches.  Many small path instances launched
// one by one leave most of the GPU idle between launches.  Here the members
// of a group (same N, same R, same transfer-function form) run each pass of
// the forward schedule of turpy_propagate as one launch for all of them: the
// subharmonics, the source row transform, column pass 0 and screen 0's
// synthesis, then per screen step s the row pass of screen s, column pass
// s + 1 and synthesis s + 1 for the members that still have them (members are
// sorted by screen count, so these are a prefix), and the final inverse row
// pass of every member at the end.  The adjoint runs the same way backwards
// (turpy_propagate_backward's schedule, screen steps counted from each
// member's last screen).  Each member's arithmetic, noise key and buffers are
// those of its own plan's call, so its results are the same bits.  A
// launch's blocks find their member's argument record by their z (or y)
// index; the records hold offsets into the call's buffers, uploaded once at
// creation, so a call uploads nothing and can be captured.
#include "group.hpp"

#include <algorithm>
#include <cstring>

#include "runtime.hpp"

namespace turpy {

namespace {

// K_ROW_SOURCE reads the call's input fields; K_ROW_SCREEN passes the
// checkpoints (and, in the adjoint, dL/dphi).
enum Kind { K_SH, K_ROW_SOURCE, K_COL, K_SYNTH, K_ROW_SCREEN, K_ROW };

// Grid limit of the instance index (y and z grid dimensions).
constexpr size_t kMaxMembers = 65535;
// Pixels per pass (R N^2) beyond which one instance's launches fill the GPU
// alone: grouping them gains nothing (measured at N = 2048, R = 1: 274 ms
// alone against 279-288 ms in groups for 252 instances of the serving mix).
constexpr int64_t kFillsAlone = int64_t(1) << 20;

struct Launch {
  Kind kind;
  uint32_t count;  // members in this launch: a prefix of the sorted members
  size_t offset;   // byte offset of its records in the table
};

template <class T>
T* off_ptr(size_t bytes) {
  return reinterpret_cast<T*>(static_cast<uintptr_t>(bytes));
}

}  // namespace

struct Group {
  std::vector<GroupMember> members;  // sorted: screen count descending
  std::vector<size_t> ws_off;        // byte offset of each member's workspace slice
  size_t ws_bytes = 0;
  int n = 0, max_m = 0;
  int64_t R = 0, P = 0;
  bool has_sh = false;
  std::vector<Launch> launches[2];  // forward, adjoint
  std::vector<unsigned char> host;  // the records, as uploaded
  void* dev = nullptr;
  int device = 0;
};

bool group_eligible(const turpy_plan* pl) {
  if (pl->M < 1 || pl->screen_ck || pl->d_nonfinite || pl->d_moments) return false;
  if (pl->R * int64_t(pl->n) * pl->n > kFillsAlone) return false;
  for (double d : pl->dz)
    if (!(d > 0)) return false;
  return true;
}

std::string group_key(const turpy_plan* pl) {
  const int mode = pl->tf_kind != TURPY_TF_ANGULAR_SPECTRUM ? 0 : (pl->d_as ? 2 : 1);
  return std::to_string(pl->n) + "/" + std::to_string(pl->R) + "/" + std::to_string(mode);
}

size_t group_workspace(const Group* g) { return g->ws_bytes; }

int64_t group_cost(const Group* g) {
  int64_t c = 0;
  for (const GroupMember& m : g->members) c += m.plan->R * int64_t(m.plan->n) * m.plan->n * (m.plan->M + 1);
  return c;
}

void group_destroy(Group* g) {
  if (!g) return;
  if (g->dev) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    (void)hipFree(g->dev);
    (void)hipSetDevice(cur);
  }
  delete g;
}

turpy_status group_create(std::vector<GroupMember> members, Group** out) {
  *out = nullptr;
  if (members.empty() || members.size() > kMaxMembers)
    return report(TURPY_E_INVALID, "batch: a group holds 1..%zu instances", kMaxMembers);
  std::stable_sort(members.begin(), members.end(),
                   [](const GroupMember& a, const GroupMember& b) { return a.plan->M > b.plan->M; });
  Group* g = new Group;
  g->members = members;
  const turpy_plan* p0 = members[0].plan;
  g->n = p0->n;
  g->R = p0->R;
  g->P = p0->P;
  g->max_m = p0->M;
  g->device = p0->device;
  for (const GroupMember& m : members) {
    g->ws_off.push_back(g->ws_bytes);
    g->ws_bytes += align_up(m.plan->ws_forward());
    g->has_sh = g->has_sh || m.plan->sh_levels > 0;
  }
  const size_t cnt = members.size();
  // members with more than s screens
  auto active = [&](int s) {
    size_t a = 0;
    while (a < cnt && members[a].plan->M > s) ++a;
    return static_cast<uint32_t>(a);
  };
  int pass = 0;  // the schedule being built: 0 forward, 1 adjoint
  auto add = [&](Kind kind, uint32_t count, auto&& record) {
    using Rec = decltype(record(size_t(0)));
    g->host.resize(align_up(g->host.size()));
    const size_t at = g->host.size();
    g->host.resize(at + count * sizeof(Rec));
    for (uint32_t k = 0; k < count; ++k) {
      const Rec r = record(size_t(k));
      std::memcpy(g->host.data() + at + k * sizeof(Rec), &r, sizeof(Rec));
    }
    g->launches[pass].push_back(Launch{kind, count, at});
  };
  // a member's workspace and buffers, as offsets
  auto ws_of = [&](size_t k) {
    const turpy_plan* pl = members[k].plan;
    const size_t b = g->ws_off[k];
    Ws w{off_ptr<float2>(b), off_ptr<float2>(b + pl->off_sh()), off_ptr<float2>(b + pl->off_src()),
         off_ptr<float2>(b + pl->off_gbuf())};
    return w;
  };
  auto field = [&](size_t k) { return off_ptr<float2>(members[k].field_bytes); };
  auto row_base = [&](size_t k) {
    const turpy_plan* pl = members[k].plan;
    RowArgs a = base_row(pl);
    a.in = field(k);
    a.in_stride = int64_t(pl->n) * pl->n;
    a.out = field(k);
    return a;
  };

  if (g->has_sh)
    add(K_SH, static_cast<uint32_t>(cnt), [&](size_t k) {
      return sh_args(members[k].plan, members[k].seed_offset, 0, ws_of(k).sh);
    });
  add(K_ROW_SOURCE, static_cast<uint32_t>(cnt), [&](size_t k) {
    RowArgs a = row_base(k);
    a.out_spectral = 1;
    a.post = members[k].plan->d_row;
    return a;
  });
  // column pass of distance `step(k)` and synthesis of screen `screen(k)`
  auto col = [&](uint32_t count, auto&& step) {
    add(K_COL, count, [&](size_t k) {
      const turpy_plan* pl = members[k].plan;
      return col_args(pl, step(k), field(k), int64_t(pl->n) * pl->n, field(k), pl->R, pass == 1);
    });
  };
  auto synth = [&](uint32_t count, auto&& screen) {
    add(K_SYNTH, count, [&](size_t k) {
      return synth_args(members[k].plan, members[k].seed_offset, 0, screen(k), nullptr, ws_of(k));
    });
  };
  auto M_of = [&](size_t k) { return members[k].plan->M; };
  col(static_cast<uint32_t>(cnt), [](size_t) { return 0; });
  synth(static_cast<uint32_t>(cnt), [](size_t) { return 0; });
  for (int s = 0; s < g->max_m; ++s) {
    const uint32_t a_s = active(s), a_next = active(s + 1);
    add(K_ROW_SCREEN, a_s, [&, s](size_t k) {
      const turpy_plan* pl = members[k].plan;
      RowArgs a = row_base(k);
      a.in_spectral = 1;
      a.out_spectral = 1;
      a.post = pl->d_row + static_cast<size_t>(s + 1) * pl->n;
      a.scale = 1.0f / pl->n;
      screen_fields(pl, TURPY_SCREENS_SYNTH, nullptr, ws_of(k), s, &a);
      a.ckpt_out = off_ptr<float2>(members[k].ck_bytes);
      return a;
    });
    col(a_s, [s](size_t) { return s + 1; });
    if (a_next > 0) synth(a_next, [s](size_t) { return s + 1; });
  }
  add(K_ROW, static_cast<uint32_t>(cnt), [&](size_t k) {
    RowArgs a = row_base(k);
    a.in_spectral = 1;
    a.scale = 1.0f / members[k].plan->n;
    return a;
  });

  // the adjoint: adjoint of the final inverse row pass (reading dL/du_out),
  // then, q steps after each member's last screen s = M - 1 - q, its screen
  // pass, the adjoint column pass of distance s and the synthesis of screen
  // s - 1; the adjoint of the source row transform of every member at the end
  pass = 1;
  if (g->has_sh)
    add(K_SH, static_cast<uint32_t>(cnt), [&](size_t k) {
      return sh_args(members[k].plan, members[k].seed_offset, 0, ws_of(k).sh);
    });
  add(K_ROW_SOURCE, static_cast<uint32_t>(cnt), [&](size_t k) {
    RowArgs a = row_base(k);
    a.out_spectral = 1;
    a.scale = 1.0f / members[k].plan->n;
    return a;
  });
  col(static_cast<uint32_t>(cnt), [&](size_t k) { return M_of(k); });
  synth(static_cast<uint32_t>(cnt), [&](size_t k) { return M_of(k) - 1; });
  for (int q = 0; q < g->max_m; ++q) {
    const uint32_t a_q = active(q), a_next = active(q + 1);
    add(K_ROW_SCREEN, a_q, [&, q](size_t k) {
      const turpy_plan* pl = members[k].plan;
      const int s = M_of(k) - 1 - q;
      RowArgs a = row_base(k);
      a.in_spectral = 1;
      a.pre = pl->d_row + static_cast<size_t>(s + 1) * pl->n;
      a.conj_tables = 1;
      a.out_spectral = 1;
      a.scale = 1.0f / pl->n;
      screen_fields(pl, TURPY_SCREENS_SYNTH, nullptr, ws_of(k), s, &a);
      a.backward = 1;
      a.ckpt_in = off_ptr<const float2>(members[k].ck_bytes);
      a.grad_screens = off_ptr<float>(members[k].ck_bytes / 2);  // floats where the checkpoints hold complex
      return a;
    });
    col(a_q, [&, q](size_t k) { return M_of(k) - 1 - q; });
    if (a_next > 0) synth(a_next, [&, q](size_t k) { return M_of(k) - 2 - q; });
  }
  add(K_ROW, static_cast<uint32_t>(cnt), [&](size_t k) {
    RowArgs a = row_base(k);
    a.in_spectral = 1;
    a.pre = members[k].plan->d_row;
    a.conj_tables = 1;
    return a;
  });
  hipError_t e = hipMalloc(&g->dev, std::max<size_t>(g->host.size(), 256));
  if (e == hipSuccess) e = hipMemcpy(g->dev, g->host.data(), g->host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    group_destroy(g);
    return hip_fail(e, "batch_create: group tables");
  }
  *out = g;
  return TURPY_OK;
}

namespace {

// Enqueue one schedule: `in` the fields the first row pass reads, `out` the
// fields every pass writes; `ck` / `gs` the checkpoints and dL/dphi of the
// screen passes.
turpy_status group_run(Group* g, int pass, uint64_t seed, uint32_t t, const void* in, void* out, const void* ck,
                       float* gs, void* ws, hipStream_t st) {
  const turpy_plan* p0 = g->members[0].plan;
  // launch choices that change the arithmetic come from the plans as they are
  // now (a batch may be tuned after creation); the members must agree
  for (const GroupMember& m : g->members)
    if (m.plan->col_radix != p0->col_radix || m.plan->synth_radix != p0->synth_radix)
      return report(TURPY_E_INVALID, "batch: the instances of a group have different radix plans");
  GroupCall call{};
  call.out = static_cast<char*>(out);
  call.ws = static_cast<char*>(ws);
  call.seed = seed;
  call.t = t;
  call.t_dev = p0->d_t;
  const char* dev = static_cast<const char*>(g->dev);
  for (const Launch& l : g->launches[pass]) {
    const unsigned char* rec = g->host.data() + l.offset;
    GroupCall c = call;
    c.in = static_cast<const char*>(l.kind == K_ROW_SOURCE ? in : out);
    switch (l.kind) {
      case K_SH:
        TURPY_HIP(timed("sh", st, [&] {
                    return launch_sh_group(reinterpret_cast<const ShArgs*>(dev + l.offset), l.count, g->P, g->max_m,
                                           c, st);
                  }),
                  "batch: subharmonics");
        break;
      case K_COL: {
        ColArgs proto;
        std::memcpy(&proto, rec, sizeof(proto));
        proto.radix = p0->col_radix;
        TURPY_HIP(timed("col", st, [&] {
                    return launch_col_group(g->n, proto, reinterpret_cast<const ColArgs*>(dev + l.offset), l.count, c,
                                            st);
                  }),
                  "batch: column pass");
        break;
      }
      case K_SYNTH: {
        SynthArgs proto;
        std::memcpy(&proto, rec, sizeof(proto));
        proto.radix = p0->synth_radix;
        TURPY_HIP(timed("synth", st, [&] {
                    return launch_synth_group(g->n, proto, reinterpret_cast<const SynthArgs*>(dev + l.offset), l.count,
                                              c, st);
                  }),
                  "batch: synthesis");
        break;
      }
      default: {
        RowArgs proto;
        std::memcpy(&proto, rec, sizeof(proto));
        if (l.kind == K_ROW_SCREEN) {
          c.ck = static_cast<char*>(const_cast<void*>(ck));
          c.gs = reinterpret_cast<char*>(gs);
        }
        TURPY_HIP(timed(row_family(proto), st, [&] {
                    return launch_row_group(g->n, proto, reinterpret_cast<const RowArgs*>(dev + l.offset), l.count,
                                            g->P, c, st);
                  }),
                  "batch: row pass");
        break;
      }
    }
  }
  return TURPY_OK;
}

}  // namespace

turpy_status group_propagate(Group* g, uint64_t seed, uint32_t t, const void* u_in, void* u_out, void* checkpoints,
                             void* ws, hipStream_t st) {
  return group_run(g, 0, seed, t, u_in, u_out, checkpoints, nullptr, ws, st);
}

turpy_status group_propagate_backward(Group* g, uint64_t seed, uint32_t t, const void* grad_u_out,
                                      const void* checkpoints, void* grad_u_in, float* grad_screens, void* ws,
                                      hipStream_t st) {
  if (!checkpoints || !grad_u_in)
    return report(TURPY_E_INVALID, "batch: a group's adjoint needs the checkpoints and grad_u_in");
  return group_run(g, 1, seed, t, grad_u_out, grad_u_in, checkpoints, grad_screens, ws, st);
}

}  // namespace turpy
