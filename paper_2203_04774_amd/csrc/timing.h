// RAII HIP-event timer for one phase of a library call.
#pragma once
#include <hip/hip_runtime.h>

class PhaseTimer {
  public:
    PhaseTimer(int phase, hipStream_t s);
    ~PhaseTimer();
    void stop();
    PhaseTimer(const PhaseTimer &) = delete;
    PhaseTimer &operator=(const PhaseTimer &) = delete;

  private:
    int phase_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool armed_ = false, stopped_ = false;
};
