// tables.h -- layout of the constant tables shared by host and device code.
#pragma once

namespace hank {

constexpr int J0_SERIES_TERMS = 14;     // sum_t (-1)^t (z^2/4)^t/(t!)^2 for z < 2
constexpr int J0_TAYLOR_INTERVALS = 36; // [2, 20) in steps of 1/2
constexpr int J0_TAYLOR0_PIECES = 4;    // [0, 2) in steps of 1/2 (the 8-term near-field step)
constexpr int J0_TAYLOR_DEG = 14;       // coefficients per interval (degree 13)
constexpr double J0_TAYLOR_Z0 = 2.0;
constexpr double J0_TAYLOR_H = 0.5;
constexpr double J0_ASY_Z = 20.0;       // Hankel branch from here on
constexpr int HANKEL_TERMS = 26;        // a_0 .. a_25 for nu = 0, 1
constexpr int TW_SMALL = 8192;          // twiddles inside one LDS-resident FFT
constexpr int TW_BIG = 1 << 23;         // largest four-step FFT length
constexpr int TW_LO = 4096;
constexpr int TW_HI = TW_BIG / TW_LO;   // 2048

struct DeviceTables {
    double ser[J0_SERIES_TERMS];
    double tay[J0_TAYLOR_INTERVALS][J0_TAYLOR_DEG];
    double tay0[J0_TAYLOR0_PIECES][J0_TAYLOR_DEG];
    double hank[2][HANKEL_TERMS];
    double tw_small[TW_SMALL][2];
    double tw_hi[TW_HI][2];
    double tw_lo[TW_LO][2];
};

void build_tables(DeviceTables& t);

// Per-order table of J_nu for the Schlomilch tasks of order nu = 1..8 (device
// memory of the plan), NU_TAB_SIZE doubles:
//   [NU_TAB_P + m]  (-1)^m a_2m(nu),   [NU_TAB_Q + m]  (-1)^m a_2m+1(nu),  m < 12
//       (Hankel expansion, Sec. 3.1: 12 pairs keep the remainder below 1e-17
//        for z >= 20 + nu/2, eq. (errorBound))
//   [NU_TAB_SER + t] (-1)^t / (t! (t+nu)!), t < 14  (series, z < 2)
//   [NU_TAB_TAY + 14 i + u]  Taylor coefficients of J_nu about 2.25 + i/2,
//       i < NU_TAYLOR_INTERVALS  (pieces on [2, 24), degree 13)
constexpr int NU_HANKEL_PAIRS = 12;
constexpr int NU_SERIES_TERMS = 14;
constexpr int NU_TAYLOR_INTERVALS = 44;
constexpr int NU_TAB_P = 0;
constexpr int NU_TAB_Q = NU_HANKEL_PAIRS;
constexpr int NU_TAB_SER = 2 * NU_HANKEL_PAIRS;
constexpr int NU_TAB_TAY = NU_TAB_SER + NU_SERIES_TERMS;
constexpr int NU_TAB_SIZE = NU_TAB_TAY + NU_TAYLOR_INTERVALS * J0_TAYLOR_DEG;
void build_nu_table(int nu, double* out);

} // namespace hank
