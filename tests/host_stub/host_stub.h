// Work on a stand-in stream: run now, or record while the stream is captured.  Test support only.
#pragma once
#include <functional>

#include "hip/hip_runtime.h"

void stub_submit(hipStream_t s, std::function<void()> fn);
