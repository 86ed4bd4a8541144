// Host-runtime declarations shared by wf_api.hip and wf_plan.hip (not part of the public ABI).
#pragma once

#include "wf_internal.h"

namespace wf {

// The workspace of (device 'dev', stream 's'), created on first use and grown to at least
// 'words' handoff words.  Sweeps enqueued on different streams use different workspaces
// (control block, handoff words, selections), so they may run concurrently on one device.
int ensure_ws_on(int dev, hipStream_t s, size_t words, DeviceWs** out);

// A control block of its own (zeroed, epoch 1, the device's injected fault mode), for a plan;
// wf_last_async_error reads its error word with the device's other control blocks.
int new_control(int dev, Control** out);
void free_control(Control* ctl);

}  // namespace wf
