// Host build of the search's launch-side limits (k_nns.hip, vicp_internal.hpp)
// for the CPU test test_host_limits.py: the global search's 64-bit work count,
// its launcher's refusal of batches it cannot take (before any launch), and
// the coordinate limit that keeps float32 squared distances finite.
#include <cstdint>

#include "k_nns.hip"

// The launchers may take timing events from the runtime; this harness has no
// runtime scope open, so none is ever taken.
bool vicp::prof_take_ext_events(hipEvent_t*, hipEvent_t*) { return false; }

extern "C" int64_t vicp_test_fallback_items(int64_t F, int64_t n) { return vicp::fallback_items(F, n); }

// Only arguments the launcher refuses reach it here: nothing is launched.
extern "C" int vicp_test_launch_fallback_refuses(int npairs, int grid)
{
    if (npairs >= 1 && npairs <= vicp::kFbMaxPairs && grid >= 1) return -1;
    return vicp::launch_fallback(nullptr, npairs, grid, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr)
               ? 0
               : 1;
}

extern "C" int vicp_test_grid_box_fits(const float* lo, const float* hi) { return vicp::grid_box_fits(lo, hi) ? 1 : 0; }
