// driver.cpp -- entry points of the operation-counting build of the oracle.
//
// TEST AND MEASUREMENT INFRASTRUCTURE.  Each call copies plain double inputs
// into the counting type, runs the oracle's own step function (compiled from
// the unchanged oracle sources with counted_double.hpp force-included), copies
// the result back and returns the operation counts of that call.
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "counted_double.hpp"
#undef double
#undef malloc

namespace flopcount {
uint64_t ops[5];
}

// the oracle's functions as they are compiled in the counting build
int gamer_oracle_hydro_solve_lim(const cdouble *, int64_t, cdouble, cdouble, cdouble, cdouble, int,
                                 cdouble *, cdouble *, long long *);
void gamer_oracle_group_prim(const cdouble *, cdouble, cdouble *);
void gamer_oracle_group_slopes(const cdouble *, cdouble, cdouble *);
long long gamer_oracle_group_predict(const cdouble *, const cdouble *, const cdouble *, cdouble, cdouble,
                                     cdouble, cdouble *);
long long gamer_oracle_group_fluxes(const cdouble *, cdouble, cdouble *);
void gamer_oracle_group_update(const cdouble *, const cdouble *, cdouble, cdouble, cdouble *, cdouble *);
cdouble gamer_oracle_max_speed(const cdouble *, int64_t, cdouble);
void gamer_oracle_conserved_sums(const cdouble *, int64_t, cdouble, cdouble *);
int gamer_oracle_ctu_solve(const cdouble *, int64_t, cdouble, cdouble, cdouble, cdouble, cdouble *,
                           cdouble *, long long *);
int gamer_oracle_rtvd_solve(const cdouble *, int64_t, cdouble, cdouble, cdouble, int, cdouble *, long long *);

static std::vector<cdouble> in_copy(const double *p, size_t n) {
    std::vector<cdouble> v(n);
    for (size_t i = 0; i < n; ++i) v[i].v = p[i];
    return v;
}

static void out_copy(const std::vector<cdouble> &v, double *p) {
    for (size_t i = 0; i < v.size(); ++i) p[i] = v[i].v;
}

static void take(uint64_t *counts) {
    for (int k = 0; k < 5; ++k) counts[k] = flopcount::ops[k];
}

extern "C" {

// MUSCL-Hancock + Roe step (char_limiting 0: primitive limiting)
int fc_hydro_solve(const double *in, int64_t n, double dt, double dh, double g, double theta,
                   int char_limiting, double *out, long long *fallbacks, uint64_t *counts) {
    auto a = in_copy(in, size_t(n) * 5 * 20 * 20 * 20);
    std::vector<cdouble> b(size_t(n) * 5 * 16 * 16 * 16);
    memset(flopcount::ops, 0, sizeof flopcount::ops);
    int rc = gamer_oracle_hydro_solve_lim(a.data(), n, {dt}, {dh}, {g}, {theta}, char_limiting, nullptr,
                                          b.data(), fallbacks);
    take(counts);
    out_copy(b, out);
    return rc;
}

// The same step stage by stage, then the per-step epilogue on the new state
// (largest signal speed for the CFL time step, conserved sums); counts[7][5]
// receive, per stage (prim, slopes, predictor, Riemann fluxes, update, CFL
// signal speed, sums), the operations summed over all groups.
int fc_hydro_stages(const double *in, int64_t n, double dt, double dh, double g, double theta,
                    double *out, uint64_t *counts) {
    const size_t in_sz = 5 * 20 * 20 * 20, out_sz = 5 * 16 * 16 * 16;
    const size_t s_sz = 5 * 18 * 18 * 18, face_sz = 3 * 5 * 17 * 16 * 16;
    auto a = in_copy(in, size_t(n) * in_sz);
    std::vector<cdouble> W(in_sz), dW(3 * s_sz), Ub(6 * s_sz), Fl(face_sz), b(size_t(n) * out_sz), sums(5);
    memset(counts, 0, 7 * 5 * sizeof(uint64_t));
    auto stage = [&](int k, auto &&fn) {
        memset(flopcount::ops, 0, sizeof flopcount::ops);
        fn();
        for (int q = 0; q < 5; ++q) counts[5 * k + q] += flopcount::ops[q];
    };
    for (int64_t gi = 0; gi < n; ++gi) {
        const cdouble *U = a.data() + size_t(gi) * in_sz;
        stage(0, [&] { gamer_oracle_group_prim(U, {g}, W.data()); });
        stage(1, [&] { gamer_oracle_group_slopes(W.data(), {theta}, dW.data()); });
        stage(2, [&] { gamer_oracle_group_predict(U, W.data(), dW.data(), {dt}, {dh}, {g}, Ub.data()); });
        stage(3, [&] { gamer_oracle_group_fluxes(Ub.data(), {g}, Fl.data()); });
        stage(4, [&] { gamer_oracle_group_update(U, Fl.data(), {dt}, {dh}, b.data() + size_t(gi) * out_sz,
                                                 nullptr); });
    }
    stage(5, [&] { gamer_oracle_max_speed(b.data(), n, {g}); });
    stage(6, [&] { gamer_oracle_conserved_sums(b.data(), n, {dh}, sums.data()); });
    out_copy(b, out);
    return 0;
}

int fc_ctu_solve(const double *in, int64_t n, double dt, double dh, double g, double theta, double *out,
                 long long *fallbacks, uint64_t *counts) {
    auto a = in_copy(in, size_t(n) * 5 * 20 * 20 * 20);
    std::vector<cdouble> b(size_t(n) * 5 * 16 * 16 * 16);
    memset(flopcount::ops, 0, sizeof flopcount::ops);
    int rc = gamer_oracle_ctu_solve(a.data(), n, {dt}, {dh}, {g}, {theta}, nullptr, b.data(), fallbacks);
    take(counts);
    out_copy(b, out);
    return rc;
}

int fc_rtvd_solve(const double *in, int64_t n, double dt, double dh, double g, int order, double *out,
                  long long *bad, uint64_t *counts) {
    auto a = in_copy(in, size_t(n) * 5 * 22 * 22 * 22);
    std::vector<cdouble> b(size_t(n) * 5 * 16 * 16 * 16);
    memset(flopcount::ops, 0, sizeof flopcount::ops);
    int rc = gamer_oracle_rtvd_solve(a.data(), n, {dt}, {dh}, {g}, order, b.data(), bad);
    take(counts);
    out_copy(b, out);
    return rc;
}
}
