// Grouped launches of uneven batches: the forward pass, and its adjoint, of
// many path instances that share the grid size, the realization count and
// the transfer-function form, one launch per pass and step for all of them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "turpy.h"

namespace turpy {

struct Group;

// Instances that can join a group: every distance > 0, at least one screen,
// at most 2^20 pixels per pass (R N^2), no checkpointed screens, no output
// check, no bound moments.
bool group_eligible(const turpy_plan* pl);
// Instances with the same key may share a group.
std::string group_key(const turpy_plan* pl);

// One member: its plan, its index in the batch (noise key seed + index *
// step) and the byte offsets of its fields and checkpoints.
struct GroupMember {
  const turpy_plan* plan;
  uint64_t seed_offset;
  size_t field_bytes;
  size_t ck_bytes;
};

// Builds the schedule and uploads its argument records (synchronous).
turpy_status group_create(std::vector<GroupMember> members, Group** out);
void group_destroy(Group* g);
size_t group_workspace(const Group* g);
int64_t group_cost(const Group* g);
// The forward pass of every member, as turpy_propagate with synthesised
// screens and its own plan would compute it.
turpy_status group_propagate(Group* g, uint64_t seed, uint32_t t, const void* u_in, void* u_out, void* checkpoints,
                             void* ws, hipStream_t st);
// The adjoint of every member, as turpy_propagate_backward with its own plan
// (checkpoints and grad_u_in required; the gradient of each member's own
// source planes).
turpy_status group_propagate_backward(Group* g, uint64_t seed, uint32_t t, const void* grad_u_out,
                                      const void* checkpoints, void* grad_u_in, float* grad_screens, void* ws,
                                      hipStream_t st);

}  // namespace turpy
