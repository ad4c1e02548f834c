// Host build of the device-side rigid-transform solve (k_solve.hip), for the
// CPU test test_solve_host.py.  Only the solve's host/device functions are used.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "k_solve.hip"

// The launchers in k_solve.hip may take timing events from the runtime; this
// harness has no runtime and never launches, so no scope is ever open.
bool vicp::prof_take_ext_events(hipEvent_t*, hipEvent_t*) { return false; }

extern "C" int vicp_test_kabsch(const double* mom, const double* c, double* Rt)
{
    return vicp::kabsch(mom, c, Rt, nullptr, false) ? 1 : 0;
}

// The same, with the polar factor refined from a given starting rotation.
extern "C" int vicp_test_kabsch_from(const double* mom, const double* c, const double* Rprev, double* Rt)
{
    return vicp::kabsch(mom, c, Rt, Rprev, false) ? 1 : 0;
}
