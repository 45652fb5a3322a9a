// Kernel timing with HIP events recorded on the launch stream (diagnostics).
#pragma once
#include "common.hpp"

namespace omss {

bool profile_enabled();

// Records a start event on construction and a stop event on destruction for
// kernel class `cls`, accounting `bytes` algorithmic bytes to the launch.
class ProfScope {
public:
    ProfScope(const char* cls, hipStream_t s, double bytes);
    ~ProfScope();
    // record the stop event now (the destructor then only books the launch)
    void stop();
    // algorithmic bytes known only after the launch
    void set_bytes(double b) { bytes_ = b; }
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

private:
    const char* cls_;
    hipStream_t s_;
    double bytes_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool stopped_ = false;
};

}  // namespace omss
