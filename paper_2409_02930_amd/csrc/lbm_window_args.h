// Argument block of the fused 1-D kernel (lbm_window.h).  Included by the host
// code of the library and, as a header of the run-time compiled program, by the
// kernel itself, so both sides share one definition.
#ifndef LBM_WINDOW_ARGS_H
#define LBM_WINDOW_ARGS_H

struct WinArgs {
  int N;                          // nodes
  int nx;                         // plain 1-D grid: its x extent; packed columns: 0
  const signed char *colflag;     // packed columns: bit0 first node, bit1 last node of a column
  const double *pin;              // populations [L][3][N] after the last completed step
  double *pout;                   // populations after the launch's last step
  const double *rec_prev;         // node records of the last completed step (v, sources)
  double *rec_out;                // node records of the launch's last step
  const double *phi, *kfac, *Tf, *far;
  const double *theta_in;         // [K][N] coverages after the last completed step
  double *theta_out;              // [K][N] after the launch's last step
  double *rrho, *rRT, *rA, *rFk, *srcsum;   // intra-step records of the last step
  double *skg;                    // rate constants: [wave][2R][64]
  double dt, rho_unit;
  int fuel, product;
};

#endif
