// Descriptors of the generic (any topology) path of libmabd.
#pragma once
#include <cstdint>

namespace mabd {

// One joint in the generic path.  Side a/b: solver-order dynamic body index,
// or -1 when that side is the world or a pinned body, in which case p1*/p2*/p3b
// hold the constant world positions of its control points.  Joints other than
// the ball are rows of one rotated frame R_J = dR R_a^T owned by side a.
struct GJoint {
  int32_t type;       // 0 ball (3 rows), 1 hinge (5), 2 universal (4), 3 prismatic (5)
  int32_t flags;      // bit0: the frame owner (side a) is static -> dR holds R_J itself
  int32_t sa, sb;
  double p1a[3], p1b[3];  // P1 (rest frame of the side's body, or world)
  double p2a[3], p2b[3];  // P2: hinge (both sides), universal and prismatic (side b)
  double p3b[3];          // P3 of side b: prismatic
  double dR[9];           // the joint's frame at rest (hinge, prismatic: Rod(axis),
                          // rows r_x, axis, r_z; universal: rows a1 x a2, a1, a2),
                          // or the constant R_J of a static owner
};

// constraint rows per joint type (Eqs. ball, hinge, universal, prismatic)
__host__ __device__ inline int joint_rows(int type) { return type == 0 ? 3 : (type == 2 ? 4 : 5); }

// Rows of the rotated-frame joints: row i is local component comp of
// R_J (y_X - y_Y), y the world position of a control point; points 0 P1 of a,
// 1 P2 of a, 2 P1 of b, 3 P2 of b, 4 P3 of b (Secs. 4.3-4.5).
struct JointRow { int8_t comp, x, y; };
__host__ __device__ inline JointRow joint_row(int type, int i) {
  // hinge: x y z of P1a - P1b, x z of P2a - P2b
  // universal: x y z of P1a - P1b, y of P2b - P1b
  // prismatic: x z of P1a - P1b, x z of P2b - P1b, x of P3b - P1b
  constexpr int8_t T[3][5][3] = {{{0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {0, 1, 3}, {2, 1, 3}},
                                 {{0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {1, 3, 2}, {0, 0, 2}},
                                 {{0, 0, 2}, {2, 0, 2}, {0, 3, 2}, {2, 3, 2}, {0, 4, 2}}};
  const int8_t *r = T[type - 1][i];
  return JointRow{r[0], r[1], r[2]};
}
__host__ __device__ inline int point_side(int p) { return p >= 2 ? 1 : 0; }

constexpr int GJ_FLAG_STATIC_OWNER = 1;

// per-joint generic data: C (5), L_a (5x12), L_b (5x12), each block starting
// on a 128-byte line (a record is 9 lines), so that a gather of one side's
// rows touches only the lines it uses
constexpr int GL_STRIDE = 144;
enum { GL_C = 0, GL_LA = 16, GL_LB = 80 };

// per-joint tree data: Sigma (5x5), rho (5) of the condensed child side
constexpr int GT_STRIDE = 64;
enum { GT_SIG = 0, GT_RHO = 25, GT_A = 30, GT_E = 35 };

// absorbed-joint entry of a tree body: joint index << 4 | (rows - 3) << 2 |
// side << 1 | unary (the joint's rows, 3 to 5, without a lookup)
inline int32_t abs_pack(int32_t k, int rows, int side, int unary) {
  return (k << 4) | ((rows - 3) << 2) | (side << 1) | unary;
}
__host__ __device__ inline int abs_joint(int32_t t) { return t >> 4; }
__host__ __device__ inline int abs_rows(int32_t t) { return 3 + ((t >> 2) & 3); }

constexpr int TEAM = 16;              // lanes per body in the tree elimination
constexpr int TREE_KLDS = 16;         // cliques up to this many rows are factored in LDS
constexpr int TREE_KMAX = 64;         // largest clique (absorbed + parent rows) accepted

// per-body incidence entry: joint index << 1 | side

struct TreeArgs {
  const int32_t *comp_lvl;  // per component: levels [comp_lvl[c], comp_lvl[c+1])
  const int32_t *lvl_off;   // per level: slots [lvl_off[l], lvl_off[l+1])
  const int32_t *tbody;     // slot -> solver body
  const int32_t *tpk;       // slot -> parent joint << 1 | side (or -1)
  const int32_t *tabs_off;  // slot -> absorbed entries
  const int32_t *tabs;
  const double *gl;
  double *gt;
  const double *u;
  int64_t ns;
  const int32_t *shp;
  const double *hinv;
  double *glam;             // 5 per generic joint
  uint32_t *status;
  int step;
  const int32_t *tne;       // slot -> absorbed rows
  const int64_t *foff;      // slot -> offset of its factor in fac
  double *fac;              // per slot: K (LD x LD, LD = absorbed rows + 5), y (LD), scratch
  const struct TcOp *ops;   // contraction schedule
  double *crec;             // compress records
  int zero_c;               // 1: the joints' constraint values are taken as zero (the
                            // loop-breaker's solves with other right-hand sides)
  const double *cc;         // if set: constraint values read from cc (5 per joint)
                            // instead of the joint rows (refinement right-hand sides)
  int f32;                  // 1: the clique matrices K0 = L Hbar^{-1} L^T are formed in
                            // FP32 (precision form 1; the factorisation stays FP64)
  const uint8_t *jrows;     // rows per generic joint (a byte each, read instead of the
                            // joint record)
};

// A component with a few closed loops (Sec. 5, Case III): its joints split
// into a spanning tree A, solved by the tree contraction, and loop breakers
// D.  Loop rows (joint << 3 | row) of component c are lrow[off[c], off[c+1]).
constexpr int LOOP_MAX_ROWS = 48;  // rows of D per component (the dense Schur system)

// Offsets per round of the tree contraction plan: the round's first
// operation, the ends of the rake classes (cliques of <= 10, 16, 32, 64 rows)
// and of the compress classes (<= 10, 16, 32, 48 rows); the compresses from
// the last end to the next round's first operation have larger cliques.
constexpr int TC_NSEG = 9;

// One operation of the tree contraction.  rake: eliminate the private rows of
// slot v (absorbed joints: condensed children and one-sided joints) and pass
// the Schur complement on its current parent joint kcur up (none at a root).
// compress: v has exactly one uncondensed child c, joined by joint e (the
// last absorbed entry of v); eliminate v's private rows, then joint e, which
// merges v into c: c's parent rows become kcur.
struct TcOp {
  int32_t v, c;      // slot eliminated; compress: slot merged into (else -1)
  int32_t kcur, ck;  // current parent joint of v (generic index, -1 at a root) and its rows
  int32_t e, ce;     // compress: joint v-c and its rows
  int32_t nv;        // current rows of v's clique (absorbed + ck)
  int32_t av, ac;    // absorbed rows of v and (compress) of c
  int32_t ev0, ev1;  // v's absorbed list [ev0, ev1) in tabs
  int32_t ec0, ec1;  // compress: c's absorbed list
  int32_t pad;
  int64_t fv, fc;    // factor slot offsets of v and (compress) c
  int64_t rec;       // compress: offset of (Lp 5x5, X_o ce x a_c, X_k 5x5, z 5) in crec
};

struct PcgArgs {
  int nb;                    // generic bodies in [b0, b0 + nb)
  int b0;
  int mj;                    // generic joints (all, tree joints included but masked)
  const int32_t *jmask;      // 1 if the joint belongs to a graph component
  const int32_t *bmask;      // 1 if the body belongs to a graph component
  const GJoint *J;
  const double *gl;          // C, L_a, L_b per joint
  const double *ug;          // local unconstrained increments (SoA)
  int64_t ns;
  const int32_t *shp;
  const double *hinv;
  const int32_t *inc_off, *inc;
  double *lam;               // 5 per joint: in = warm start (or zero), out = solution
  double *r, *p, *z, *sp;    // 5 per joint
  double *bv;                // right-hand side, 5 per joint
  double *dinv;              // 25 per joint
  double *zb;                // 12 per body (SoA with stride ns)
  double *partial;           // 4 per block
  double tol;
  int max_iters;
  int warm;                  // lambda holds a start value
  int *iters_out;
  double *res_out;           // |r|/|b| reached
  uint32_t *status;
  int step;
};
// PCG for graph components whose joints are all ball joints.  A ball row
// block is s J(p) in world coordinates (s = +1 side a, -1 side b), so the
// operator needs only the anchors and the body rotations: the body pass forms
// z = H^{-1} sum s J(p)^T x in world coordinates, the joint pass y = sum s J(p) z.
struct PcgBallArgs {
  int nj, nbd;                     // graph joints, graph bodies (compact numbering)
  const int32_t *jid;              // compact joint -> generic joint (gl, glam)
  const int32_t *jba, *jbb;        // compact joint -> compact body of side a / b, or -1
  const double *jp;                // anchors, 8 per compact joint: p_a xyz, p_b xyz, pad
  const int32_t *bid;              // compact body -> solver body
  const int32_t *binc_off, *binc;  // compact body -> compact joint << 1 | side
  const double *gl;                // C at GL_C per generic joint
  const double *Rg, *ug;           // per solver body, SoA with stride ns
  int64_t ns;
  const int32_t *shp;
  const double *hinv;
  double *glam;                    // 5 per generic joint: warm start in, solution out
  double *x, *r, *z, *p0, *p1, *sp, *bv;  // 3 per compact joint
  double *dinv;                    // 6 per compact joint: S_kk^{-1} (00 01 02 11 12 22)
  double *zw;                      // 16 per compact body: world-frame H^{-1} G^T v, pad
  double *partial;                 // 4 per joint block
  int nblk;                        // joint blocks (ceil(nj / 256))
  double *sc;                      // scalars of the iteration (8)
  int32_t *si;                     // flags and counters of the iteration (8)
  double tol;
  int max_iters;
  int warm;
  int32_t *iters_out;
  double *res_out;
  uint32_t *status;
  int step;
};

}  // namespace mabd

namespace mabd {

// Paths: tree components whose bodies carry at most two joints each (chains
// with hinges, universal or prismatic joints, free-floating chains).  Their
// joints, in path order, are the units of a block-tridiagonal dual: unit i
// couples only with i-1 and i+1, through the body the two joints share.
// Every block is padded to 5 rows (identity on the padding), so the kernels
// work on fixed 5x5 blocks in registers.  A level splits each path into
// segments of at most T units; a segment eliminates its units but the last
// (its separator) in order, which leaves a block-tridiagonal system over the
// separators (the next level).  A path with one segment at a level solves
// its separator there; back-substitution runs the levels in reverse.
constexpr int PATH_MAXLEVEL = 32;
constexpr int PATH_TMAX = 16;  // longest level-0 segment (its unit records are staged in LDS)
constexpr int PATH_UREC = 65;  // level >= 1 unit: D (15, packed lower), y (5), F (25: coupling
                               // from the previous unit, its rows x ours), dD (15), dy (5)
constexpr int PATH_FREC = 70;  // per eliminated unit: L (15, the reciprocals of the pivots on
                               // its diagonal), z (5), W (25), G (25)
enum { PU_D = 0, PU_Y = 15, PU_F = 20, PU_DD = 45, PU_DY = 60 };
enum { PF_L = 0, PF_Z = 15, PF_W = 20, PF_G = 45 };

// a level-0 unit: one joint of a path, with the dynamic bodies before and
// after it on the path (solver index, -1: none) and its side of the joint
// there (0: a, 1: b), which selects the joint rows L_a or L_b
struct PathUnitF {
  int32_t gj, r;     // generic joint index (multipliers at 5 gj), rows
  int32_t bb, sb;    // body before, its side
  int32_t ba, sa;    // body after, its side
};

struct PathSeg {
  int32_t u0, t;     // first unit (index within the level) and unit count
  int32_t k;         // the separator's unit index at the next level
  int32_t flags;     // bit 0: a left separator (the previous segment's);
                     // bit 1: the path's last segment at this level;
                     // bit 2: the path's only segment (its separator is solved here)
};

struct PathPlan {
  int nlevel;                              // levels with segments
  int T0;                                  // segment length of level 0
  const PathUnitF *uf;
  const PathSeg *seg;                      // level l: [seg_off[l], seg_off[l+1])
  const int32_t *rows;                     // units of levels >= 1
  double *unit;                            // PATH_UREC per unit of levels >= 1
  double *lam;                             // 5 per unit of levels >= 1
  double *fac;                             // level l at fac_off[l]: (T-1) x PATH_FREC per segment,
                                           // level 0 segment-major, levels >= 1 interleaved
                                           // across the segments
  int32_t seg_off[PATH_MAXLEVEL + 1];
  int64_t unit_off[PATH_MAXLEVEL + 2];     // level l >= 1 units from unit_off[l]
  int64_t fac_off[PATH_MAXLEVEL + 1];
};

}  // namespace mabd
