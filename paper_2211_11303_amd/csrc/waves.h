// Launching the planned task waves of a factorisation (or of the Schulz
// inverse's products) on the device.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.h"

namespace hlu {

// which task kinds of a wave launch_wave launches
constexpr int kWaveAll = 0, kWaveNoTrunc = 1, kWaveTruncOnly = 2;
// second stream and fork/join events of run_waves
struct WaveStreams {
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  WaveStreams() = default;
  WaveStreams(const WaveStreams&) = delete;
  WaveStreams& operator=(const WaveStreams&) = delete;
  ~WaveStreams();
};
// One wave of a plan on stream s (the kinds `part` selects).  peak
// (optional, one int per rank slot): each truncation raises its slot's
// entry to the eps-rank it asked for, before any capacity cap.
template <class T>
hipError_t launch_wave(T* arena, const DevPlan& P, const Wave& w, int32_t* dims, int32_t* status, double eps,
                       double floor_rel, int32_t max_leaf, int32_t tile_base, bool compute64, hipStream_t s,
                       int32_t* peak = nullptr, int part = kWaveAll);
// All waves of a plan in order on stream s.  With ws, a wave holding both
// truncations and other tasks runs its truncations on ws's second stream
// (made on first use, default priority), forked from and joined back to s
// by two events: the tasks of one wave are independent, so the result is
// the same bit for bit.
template <class T>
hipError_t run_waves(T* arena, const DevPlan& P, const std::vector<Wave>& waves, int32_t* dims, int32_t* status,
                     double eps, double floor_rel, int32_t max_leaf, bool compute64, hipStream_t s, int32_t* peak,
                     WaveStreams* ws);

}  // namespace hlu
