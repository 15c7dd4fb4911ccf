/*
 * pecc_oracle_types.h -- descent parameters and outcome shared by the
 * oracle's C files (test infrastructure only, like the files that use it).
 */
#ifndef PECC_ORACLE_TYPES_H
#define PECC_ORACLE_TYPES_H
#include <stdint.h>

typedef struct {
    int32_t m;            /* history pairs kept                               */
    int32_t max_iter;     /* accepted iterations at most                      */
    int32_t max_halvings; /* step halvings per line search at most            */
    int32_t ftol_window;  /* iterations spanned by the relative-decrease test */
    double c1;            /* sufficient-decrease constant                     */
    double eps_curv;      /* keep (s,y) only if s^T y > eps_curv * y^T y      */
    double e_feasible;    /* E below this is feasible                         */
    double g_tol;         /* ||g||_2 at or below this is stationary           */
    double ftol;          /* relative decrease over the window (0 = off)      */
    double rad;           /* circle radius used by the energy                 */
} oracle_params;

typedef struct {
    int32_t status;
    int32_t iters;
    int32_t evals;
    int32_t resets;
    double E;
    double gnorm;
} oracle_result;

int oracle_descend(int n, double *xy, double R, const oracle_params *P,
                   oracle_result *res, double *trace);

#endif
