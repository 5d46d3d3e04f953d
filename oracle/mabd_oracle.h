/*
 * FP64 CPU oracle for one time step of the co-rotated multi-affine-body
 * method with joints enforced through the KKT system (M-ABD, arXiv 2603.08079).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the GPU library and is deliberately plain: dense 12x12 algebra per body,
 * a Jacobi-eigenvalue polar decomposition, block Thomas for chains, a primal
 * leaf-to-root condensation for trees, dense Cholesky or PCG for graphs.
 *
 * State layout (same convention as the paper, Sec. 3.1): per body 12 doubles
 * q = [a1; a2; a3; t], a_c the c-th column of A, i.e. A(r,c) = q[3c + r].
 */
#ifndef MABD_ORACLE_H
#define MABD_ORACLE_H
#include <stdint.h>

typedef struct {
  int32_t n;
  const double *dims;      /* n*3 box edge lengths (rest frame at the COM)        */
  const double *density;   /* n                                                    */
  const double *k_orth;    /* n  k_A (material 0) or Young's modulus (material 1)  */
  const double *poisson;   /* n  (material 1 only; may be NULL otherwise)          */
  const uint8_t *pinned;   /* n  1 = kinematic body held at q0                     */
  const double *q0;        /* n*12 creation state: pinned poses, hinge axes       */
  int32_t m;
  const uint8_t *jtype;    /* m  0 ball, 1 hinge, 2 universal, 3 prismatic         */
  const int32_t *ja, *jb;  /* m  body indices, -1 = world                         */
  const double *pa, *pb;   /* m*3 CP1 in the rest frame of a / b (world if -1)    */
  const double *axis;      /* m*3 hinge / prismatic axis, universal first axis a1, in
                              a's rest frame (world if a = -1)                     */
  const double *cp_len;    /* m  spacing of the further control points            */
  double gravity[3];
  int32_t material;        /* 0: mu = 4 k_A, lambda = 0 ; 1: Lame from (E, nu)     */
  int32_t hinge_grad;      /* 0: frozen frame + A-linearized rotation term; 2: frozen only */
  int32_t newton_iters;    /* >= 1                                                 */
  const double *wrench;    /* n*6 external spatial wrench [tau; f] per body, world
                              frame, about the COM (Eq. module1-wrench-map); NULL:
                              none                                                 */
  const double *axis2;     /* m*3 universal joints: the second axis a2 (orthogonal
                              to axis, a's rest frame or world if a = -1); NULL if
                              there is no universal joint                          */
  int32_t body_solve;      /* 0: polar rotation (Eq. polar); 1: bodies without
                              joints take the polar-free solve of Alg. 1         */
} ora_system;

/* diag[] slots written by ora_step / ora_finish */
enum { ORA_RHO_P = 0, ORA_RHO_D = 1, ORA_KKT = 2, ORA_CBALL = 3, ORA_CHINGE = 4,
       ORA_ITERS = 5, ORA_SOLVER = 6, ORA_NDIAG = 8 };

/* solver selection */
enum { ORA_AUTO = 0, ORA_CHAIN = 1, ORA_TREE = 2, ORA_DENSE = 3, ORA_PCG = 4 };

/* status codes (same meaning as the library's, independent definitions) */
enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ETOPO = -2, ORA_ENONFINITE = -5,
       ORA_ENOTCONV = -6, ORA_ESINGULAR = -7 };

int32_t ora_polar(const double *A, double *R);
int32_t ora_rows(const ora_system *s);
int32_t ora_classify(const ora_system *s);
int32_t ora_step(const ora_system *s, double h, double *q, double *qd, int32_t solver,
                 double tol, int32_t max_iters, double *lam, double *diag);
int32_t ora_body_terms(const ora_system *s, double h, const double *q, const double *qd,
                       int32_t i, double *H, double *f, double *R);
int32_t ora_joint_terms(const ora_system *s, const double *q, int32_t k, double *C,
                        double *Ga, double *Gb);
int64_t ora_dual_coo(const ora_system *s, double h, const double *q, const double *qd,
                     int64_t cap, int64_t *I, int64_t *J, double *V, double *r);
int32_t ora_finish(const ora_system *s, double h, const double *q, const double *qd,
                   const double *lam, double *q_out, double *qd_out, double *diag);
int32_t ora_residual(const ora_system *s, double h, const double *q, const double *qd,
                     const double *dq, const double *lam, const double *q_new, double *diag);
int32_t ora_twists(const ora_system *s, const double *q, const double *qd, double *V);
int32_t ora_joint_wrenches(const ora_system *s, const double *q, const double *lam, double *W);
#endif
