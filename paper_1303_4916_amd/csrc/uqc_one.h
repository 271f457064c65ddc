// Device view of the shells of a basis for the one-electron integrals (uqc_one.hip).
#pragma once
#include "uqc_internal.h"

namespace uqc {

struct ShellsDev {
    const int* K;          // [nshell] contraction depth
    const int* off;        // [nshell] first basis function
    const int* pstart;     // [nshell] first primitive in alpha / c
    const double* A;       // [nshell][3] centre
    const double* alpha;   // [nprim] exponents
    const double* c;       // [nprim] coefficients with primitive and contraction normalisation of the axis components
    int nshell;
};

// Pair classes 0..5 = (s,s), (p,s), (p,p), (d,s), (d,p), (d,d); pairs (a, b) with l_a = la, l_b = lb and, for
// la == lb, a >= b.  Z [natom], R [natom][3] on the device; any of S, T, V may be null.
hipError_t launch_one_electron(int pair_class, const ShellsDev& sh, const int2* pairs, int npairs, int natom,
                               const double* Z, const double* R, const double* f, double* S, double* T, double* V,
                               int N, const double* boys64tab, hipStream_t s);

}  // namespace uqc
