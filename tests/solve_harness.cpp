// Host build of the device-side rigid-transform solve (k_solve.hip), for the
// CPU test test_solve_host.py.  Only the solve's host/device functions are used.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "k_solve.hip"

extern "C" int vicp_test_kabsch(const double* mom, const double* c, double* Rt)
{
    return vicp::kabsch(mom, c, Rt) ? 1 : 0;
}
