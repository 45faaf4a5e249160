// flow_types.hpp — task types of the dataflow large-front launch, shared by
// the host task-list builder and the kernel.
#pragma once

namespace ncl {
enum { kFlowDiag = 0, kFlowPanel = 1, kFlowUpd = 2 };
}  // namespace ncl
