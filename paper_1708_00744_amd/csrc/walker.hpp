// walker.hpp -- device state and kernel launchers of the host-driven single
// walker (look-ahead ratio, its gradient, accept with bordering).
#pragma once
#include "dsu_internal.hpp"

namespace dsu {

// Single-walker device state (one walker, precision T behind the void*).
struct WalkerDev {
    void *bt;          // np x np, T
    void *u;           // kp x np, T
    void *vg;          // kp x np, T
    double *a;         // np x np, FP64 Slater matrix
    void *phi;         // np, T: pending proposal row
    double *phi64;     // np, FP64 copy of the proposal row
    double *cinv;      // kp x (kp+1): C_k^{-1} in pending order
    double *dots;      // 1 + 2 kp: r0, p[0..k), q[0..k)
    double *t;         // kp: C_k^{-1} q
    double *ratio;     // device copy of R
    double *ratio_host;// pinned host memory (mapped): R, grad R (or the drift), then the call's completion tag
    void *dphi;        // 3 x np, T: gradient rows (x, y, z) of the proposal or of the present row
    double *gdots;     // 3 (kp + 1) + kp: gradient rows against BT[e] and Vg, then q of the drift call
    int *idx;          // kp pending electrons
    unsigned *counter; // blocks finished (last-block reduction)
    int ldc;           // kp + 1
};

// Multideterminant state of an FP64 walker (single-reference expansion).
struct MdDev {
    double *v;      // np x m: virtual orbitals, row i = electron i (zero rows past n)
    double *t;      // np x m: table T = A^{-1} V (row j = occupied orbital j)
    double *c;      // np: column e of the current inverse (look-ahead corrected)
    double *vphi;   // m: virtual row of the proposal
    double *x;      // m: (vphi - phi T) / R
    int *order;     // ndet: substitutions per determinant (0..4)
    int *occ;       // ndet x 4: occupied orbitals replaced
    int *virt;      // ndet x 4: virtual orbitals put in their place
    double *coef;   // ndet
    double *q;      // [0]: sum_I c_I det S_I of the pending proposal; [1]: of the present state
    int m, ndet;
};

// Single-walker look-ahead ratio and accept (bordering).
// grad_mode 0: ratio; 1: ratio and its gradient; 2: gradient of the present
// row only (m = pending slot held by e, or -1).  The results are written to
// ratio_host, then `tag` to ratio_host[4] (after a system-scope fence), so the
// host can wait for the call by watching that word.
template <typename T>
hipError_t launch_walker_propose(WalkerDev *wd, int n, int np, int k, int e, int grad_mode, int m, unsigned tag,
                                 hipStream_t s);
template <typename T>
hipError_t launch_walker_accept(WalkerDev *wd, int n, int np, int k, int kp, int e, hipStream_t s);
// Row copy into a padded device row: mode 0 FP64->FP64, 1 FP64->float, 2 float->FP64.
hipError_t launch_row_to(const double *src, void *dst, int mode, int n, int np, hipStream_t s);
// count FP64 values from mapped pinned host memory (device address) into
// dst64 and, if dst32 is not NULL, their float casts into dst32.
hipError_t launch_rows_from_host(const double *src_mapped, double *dst64, float *dst32, int count, hipStream_t s);
// Multideterminant steps (FP64).  table: T = BT^T V.  propose: after the
// look-ahead kernel (ratio R and t in *wd), c = BT[e] - sum_j t_j Vg[j], x =
// (vphi - phi T) / R, Q' = sum_I c_I det(S_I + c_J x_V) -> ratio_host[0..2] =
// (R Q' / Q, R, Q'), then `tag` to ratio_host[4].  init: Q = sum_I c_I det S_I
// of the present table -> q[1] and ratio_host[2], then the tag.  accept:
// T += c x, V[e] = vphi, Q = Q'.
hipError_t launch_md_table(const WalkerDev *wd, const MdDev *md, int n, int np, hipStream_t s);
hipError_t launch_md_propose(const WalkerDev *wd, const MdDev *md, int n, int np, int k, int e, unsigned tag,
                             hipStream_t s);
hipError_t launch_md_init(const WalkerDev *wd, const MdDev *md, unsigned tag, hipStream_t s);
hipError_t launch_md_accept(const MdDev *md, int n, int np, int e, hipStream_t s);

}  // namespace dsu
