// Operation count of the oracle's right-hand side (test infrastructure).
//
// The oracle's C source is compiled here as C++ with every `double` replaced
// by Counted: a double that also records whether it depends on the state.
// An arithmetic operation (+, -, *, /, sqrt) with a state-dependent operand
// is counted; one on material constants, grid constants and literals only is
// not (those values are computed once in any implementation).  Comparisons,
// min, max and |x| are not counted.  The program prints the counts per
// interior cell of one right-hand side on two periodic grids, the asymptotic
// per-cell count of an infinite grid, and the counts of the building blocks
// (conservative -> primitive, one WENO5 pair, one HLLC face, the stage
// combinations), as one line of JSON.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

namespace opc {
uint64_t n_add = 0, n_mul = 0, n_div = 0, n_sqrt = 0;
inline void reset() { n_add = n_mul = n_div = n_sqrt = 0; }
inline uint64_t total() { return n_add + n_mul + n_div + n_sqrt; }
}  // namespace opc

struct Counted {
    double v;
    bool dep;
    Counted() = default;
    Counted(double x) : v(x), dep(false) {}
    Counted(double x, bool d) : v(x), dep(d) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return (int)v; }
};

#define OPC_BIN(op, counter)                                                                  \
    inline Counted operator op(Counted a, Counted b)                                          \
    {                                                                                         \
        const bool d = a.dep || b.dep;                                                        \
        if (d) opc::counter++;                                                                \
        return Counted(a.v op b.v, d);                                                        \
    }                                                                                         \
    inline Counted operator op(Counted a, double b) { return a op Counted(b); }               \
    inline Counted operator op(double a, Counted b) { return Counted(a) op b; }               \
    inline Counted operator op(Counted a, int b) { return a op Counted((double)b); }          \
    inline Counted operator op(int a, Counted b) { return Counted((double)a) op b; }          \
    inline Counted &operator op##=(Counted &a, Counted b) { return a = a op b; }              \
    inline Counted &operator op##=(Counted &a, double b) { return a = a op Counted(b); }
OPC_BIN(+, n_add)
OPC_BIN(-, n_add)
OPC_BIN(*, n_mul)
OPC_BIN(/, n_div)
#undef OPC_BIN
inline Counted operator-(Counted a) { return Counted(-a.v, a.dep); }
inline Counted operator+(Counted a) { return a; }

#define OPC_CMP(op)                                                              \
    inline bool operator op(Counted a, Counted b) { return a.v op b.v; }         \
    inline bool operator op(Counted a, double b) { return a.v op b; }            \
    inline bool operator op(double a, Counted b) { return a op b.v; }            \
    inline bool operator op(Counted a, int b) { return a.v op (double)b; }       \
    inline bool operator op(int a, Counted b) { return (double)a op b.v; }
OPC_CMP(<)
OPC_CMP(>)
OPC_CMP(<=)
OPC_CMP(>=)
OPC_CMP(==)
OPC_CMP(!=)
#undef OPC_CMP

inline Counted sqrt(Counted a)
{
    if (a.dep) opc::n_sqrt++;
    return Counted(::sqrt(a.v), a.dep);
}
inline Counted fabs(Counted a) { return Counted(::fabs(a.v), a.dep); }
inline Counted fmax(Counted a, Counted b) { return Counted(::fmax(a.v, b.v), a.dep || b.dep); }
inline Counted fmin(Counted a, Counted b) { return Counted(::fmin(a.v, b.v), a.dep || b.dep); }
inline Counted pow(Counted a, Counted b)
{
    if (a.dep || b.dep) opc::n_mul++;
    return Counted(::pow(a.v, b.v), a.dep || b.dep);
}
inline bool opc_isfinite(Counted a) { return isfinite(a.v); }

// the oracle, with its doubles counted
#undef isfinite
#define isfinite opc_isfinite
#define double Counted
#include "../../oracle/mfc_oracle.c"
#undef double
#undef isfinite

static Counted dep(double x) { return Counted(x, true); }

// Smooth subsonic two-fluid state on a periodic box of n cells per
// dimension: every face is a subsonic Riemann problem (the star-state
// branches of HLLC).
static void state(const ora_grid *g, Counted *q)
{
    const int nd = g->ndim, n = g->n[0], nv = 4 + nd;
    const int kg = nd == 3 ? NG : 0;
    Counted w[7], qc[7];
    for (int k = -kg; k < (nd == 3 ? n + NG : 1); k++)
        for (int j = -NG; j < n + NG; j++)
            for (int i = -NG; i < n + NG; i++) {
                const double x = (i + 0.5) / n, y = (j + 0.5) / n, z = (k + 0.5) / n;
                const double s = sin(2 * M_PI * x) * cos(2 * M_PI * y) + 0.5 * sin(2 * M_PI * z);
                const double a = 0.5 + 0.2 * s;
                const double u[3] = {5.0 * s, 3.0 * cos(2 * M_PI * z + 1.0), -4.0 * sin(2 * M_PI * y)};
                w[0] = dep(a * 1000.0 * (1 + 0.01 * s));
                w[1] = dep((1 - a) * 1.2 * (1 + 0.1 * s));
                for (int m = 0; m < nd; m++) w[2 + m] = dep(u[m]);
                w[nv - 2] = dep(1e5 * (1 + 0.2 * s));
                w[nv - 1] = dep(a);
                ora_prim_to_cons(g, w, qc);
                for (int v = 0; v < nv; v++) q[at(g, v, i, j, k)] = qc[v];
            }
}

static ora_grid grid(int nd, int n)
{
    ora_grid g;
    memset(&g, 0, sizeof g);
    g.ndim = nd;
    for (int d = 0; d < 3; d++) {
        g.n[d] = d < nd ? n : 1;
        g.dx[d] = Counted(1.0 / n);
    }
    g.gamma[0] = Counted(4.4);
    g.gamma[1] = Counted(1.4);
    g.pi_inf[0] = Counted(6e8);
    g.pi_inf[1] = Counted(0.0);
    for (int f = 0; f < 6; f++) g.bc[f] = 1;
    g.weno_eps = Counted(1e-6);
    return g;
}

static double rhs_per_cell(int nd, int n)
{
    ora_grid g = grid(nd, n);
    const int64_t cells = ora_padded_cells(&g);
    Counted *q = (Counted *)calloc(cells * 7, sizeof(Counted));
    Counted *r = (Counted *)calloc(cells * 7, sizeof(Counted));
    state(&g, q);
    opc::reset();
    if (ora_rhs(&g, q, r) != ORA_OK) {
        fprintf(stderr, "rhs failed\n");
        exit(1);
    }
    double interior = 1.0;
    for (int d = 0; d < nd; d++) interior *= n;
    free(q);
    free(r);
    return (double)opc::total() / interior;
}

// c(n) = A + B/n per cell (halo reconstructions, faces and ghost
// conversions grow like the surface): A from two sizes
static double asymptotic(int nd, int n1, int n2)
{
    const double c1 = rhs_per_cell(nd, n1), c2 = rhs_per_cell(nd, n2);
    return (n2 * c2 - n1 * c1) / (n2 - n1);
}

int main()
{
    const double A3 = asymptotic(3, 24, 36), A2 = asymptotic(2, 96, 192);

    ora_grid g = grid(3, 8);
    Counted w[7], q[7], F[7], uf, sp[5], pl, mi;
    for (int v = 0; v < 7; v++) w[v] = dep(v == 6 ? 0.5 : (v == 5 ? 1e5 : (v < 2 ? 500.0 : 1.0)));
    ora_prim_to_cons(&g, w, q);
    opc::reset();
    ora_cons_to_prim(&g, q, w);
    const uint64_t c2p = opc::total();
    for (int t = 0; t < 5; t++) sp[t] = dep(1.0 + 0.1 * t * t);
    opc::reset();
    ora_weno5(sp, g.weno_eps, &pl, &mi, NULL);
    const uint64_t weno = opc::total();
    Counted wL[7], wR[7];
    for (int v = 0; v < 7; v++) {
        wL[v] = dep(w[v].v);
        wR[v] = dep(w[v].v * (v == 2 ? 1.0 : 1.01) + (v == 2 ? 3.0 : 0.0));
    }
    opc::reset();
    ora_hllc(&g, 0, wL, wR, F, &uf);
    const uint64_t hllc = opc::total();
    Counted q0 = dep(1.0), qs = dep(1.1), L = dep(0.3), out;
    uint64_t rk[3];
    for (int s = 1; s <= 3; s++) {
        opc::reset();
        ora_rk3_combine(s, 1, &q0, &qs, &L, dep(1e-3), &out);
        rk[s - 1] = opc::total();
    }
    printf("{\"rhs_per_cell_3d\": %.3f, \"rhs_per_cell_2d\": %.3f, \"cons_to_prim_3d\": %llu, \"weno5_pair\": %llu, "
           "\"hllc_face\": %llu, \"rk3_stage\": [%llu, %llu, %llu]}\n",
           A3, A2, (unsigned long long)c2p, (unsigned long long)weno, (unsigned long long)hllc,
           (unsigned long long)rk[0], (unsigned long long)rk[1], (unsigned long long)rk[2]);
    return 0;
}
