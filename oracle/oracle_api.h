/*
 * FP64 CPU oracle for the grid-SDF Fast-Grasp'D grasp step.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, plain reference that
 * the GPU path is checked against. Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it. It shares no code, header,
 * table or constant with the GPU library; inputs arrive as plain arrays.
 *
 * Method (Fast-Grasp'D, Sec. III-C and Sec. IV-A): forward kinematics of the
 * hand, penetration constraints of hand points against the object SDF,
 * position-based-dynamics corrections of the object pose (Eq. (1)) summed
 * over constraints, the velocity-test stability loss over M = 7 simulations,
 * joint range/limit losses, the leaky contact gradient, and the optimizer.
 * The object is a dense vertex-centred SDF grid sampled trilinearly (the
 * representation of the paper's predecessor, Sec. III-A), or an analytic
 * sphere / plane / box for checks.
 *
 * The gradient is computed by forward-mode dual numbers (one tangent per
 * degree of freedom), a mechanism independent of the GPU's hand-written
 * reverse-mode adjoint.
 *
 * All functions return 0 on success and a negative value on bad arguments.
 */
#ifndef GRASP_ORACLE_API_H
#define GRASP_ORACLE_API_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_links;                 /* link 0 is the palm (root) */
  const int* parent;           /* [n_links]; parent[0] = -1, parent[l] < l */
  const double* joint_origin;  /* [n_links][12] row-major 3x4: parent frame -> joint l at q = 0 */
  const double* joint_axis;    /* [n_links][3] unit axis in the joint frame */
  const double* q_low;         /* [n_dof]; entries 0..5 (wrist) unused */
  const double* q_up;          /* [n_dof] */
  int n_contacts;
  const double* contact_local; /* [n_contacts][3] in the frame of contact_link[i] */
  const int* contact_link;     /* [n_contacts] */
} ohand;

/* A closed triangle mesh with outward (counter-clockwise) faces and unit
   vertex normals for the Phong surface (Sec. III-B). */
typedef struct {
  int n_vertices;
  const double* vertices;  /* [n_vertices][3] */
  const double* normals;   /* [n_vertices][3] */
  int n_faces;
  const int* faces;        /* [n_faces][3] */
  double alpha;            /* Phong blend: 0 flat, 1 curved */
} omesh;

enum { OBJ_GRID = 0, OBJ_SPHERE = 1, OBJ_PLANE = 2, OBJ_BOX = 3, OBJ_MESH = 4 };

typedef struct {
  int kind;
  /* grid: vertex (i,j,k) at lo + (i,j,k) h, value index (k*n + j)*n + i */
  int n;
  double lo[3];
  double h;
  const float* values;
  /* sphere: |r - center| - radius; box: axis-aligned, centred at center */
  double center[3];
  double radius;
  double half[3];
  /* plane: normal . r - offset (normal unit) */
  double normal[3];
  double offset;
  /* I/m of the isotropic object; <= 0 for a grid means 0.4 R_eq^2 with
     R_eq^3 = 3 V / (4 pi), V = h^3 * #{vertices with value < 0} */
  double inertia_over_mass;
  /* grid only: 0 = the analytic gradient of the trilinear blend; 1 = the
     normal by central differences of the sampled value at +-h along each
     axis, seven queries per sample (the earlier method's normal that
     Sec. III-A contrasts with, kept for comparison) */
  int fd_normal;
  /* mesh: the Phong signed distance of this mesh (Sec. III-B; brute force
     over its faces, sign by the winding number); inertia_over_mass must be
     given (> 0) */
  const omesh* mesh;
} oobject;

typedef struct {
  double dt;          /* time step (1e-3 s) */
  double v0;          /* test speed (m/s); velocities +x,-x,+y,-y,+z,-z,0 */
  int K;              /* projection iterations inside the one step */
  double omega;       /* relaxation of the summed corrections */
  double r_dil;       /* SDF dilation radius for this step */
  double alpha_leak;  /* leaky gradient factor */
  double w_stable, w_pen, w_range, w_limit;
  double w_min;       /* a constraint with J M^-1 J^T <= w_min is skipped */
  int projection;     /* 0: all corrections at one pose, averaged over the active
                         constraints; 1: Gauss-Seidel, one constraint after another
                         in link-major order (stable by link), each at the pose the
                         previous ones left */
  double mu;          /* Coulomb friction coefficient (0: frictionless): each
                         active contact's tangential displacement over the step
                         is removed up to mu C (static below, kinetic above) */
} oparams;


/* Phong signed distance at n points r [n][3] (mesh.cpp): rho [n], grad [n][3]
   = (r - p) / rho, closest [n][3] = closest point of the flat mesh, face [n]
   its face, dist_flat [n] = |r - closest|, gap [n] = how much farther the
   nearest different surface point is (0 on the medial axis), spread [n] =
   the largest difference of Phong distances over faces whose flat distance
   is within single-precision resolution of the best (4e-7 (|r - closest| +
   |r|)); each output but rho may be NULL. */
int oracle_mesh_sdf(const omesh* m, int n, const double* r, double* rho, double* grad, double* closest,
                    int* face, double* dist_flat, double* gap, double* spread);

/* Generalized winding number of the mesh at r: 1 inside, 0 outside. */
double oracle_winding_number(const omesh* m, const double* r);

/* Closest point of triangle (a, b, c) to r and its barycentric weights [3]. */
int oracle_closest_on_triangle(const double* a, const double* b, const double* c, const double* r, double* out,
                               double* bary);

/* Forward kinematics. p_out [B][Nc][3]; frames_out [B][L][12] or NULL. */
int oracle_fk(const ohand* hand, int B, const double* q, double* p_out, double* frames_out);

/* SDF sample at n points r [n][3]: phi [n], grad [n][3], hess [n][9] or NULL,
   face_margin [n] or NULL = distance (cell units) of the nearest coordinate to
   a cell face or the box boundary (grids only). */
int oracle_sample(const oobject* obj, int n, const double* r, double* phi, double* grad,
                  double* hess, double* face_margin);

double oracle_inertia_over_mass(const oobject* obj);

/* One grasp step for B candidates q [B][n_dof].
   loss [B]; terms [B][4] = (L_stable, L_pen, L_range, L_limit) or NULL;
   grad [B][n_dof] or NULL; margins [B][3] = (min |d + eps| over samples
   with w > w_min, the distance from the activation d = -eps; min face margin
   in cell units over the penetrating ones, d < -eps, whose gradient sets a
   correction; the same over every sample with w > w_min, whose gradient the
   leaky rule reaches) or NULL. A sample of the projection penetrates (is an
   active constraint) when d < -eps, eps = 5e-3 dt v0 (contact tolerance); the
   penetration energy L_pen counts d < 0. */
int oracle_step(const ohand* hand, const oobject* obj, const oparams* prm, int B,
                const double* q, double* loss, double* terms, double* grad, double* margins,
                int n_threads);

/* A reading of one sample that FP32 arithmetic may take instead of FP64's:
   sample (m, k, i) = velocity test m, projection iteration k, contact i. */
typedef struct {
  int m, k, i;
  int what;  /* 0: the other side of the activation d = -eps (counted active
                or not: the value of C and its derivative rule follow the
                side); 1, 2, 3: the cell on the other side of the
                cell face nearest to the sample along x, y, z (the value is
                continuous there, the gradient is the other cell's); 4: the
                other side of the friction cone (static or kinetic friction)
                for a contact whose slide |dp_t| lies within kink_d of mu C;
                5: the other side of the friction floor (no friction for a
                slide up to 1e-3 dt v0) for a slide within kink_d of it;
                6: the other side of a mesh's flat surface (the sign of the
                Phong distance) for a sample within kink_d of it; 7: the
                nearest different point of a mesh for a sample whose two
                nearest points lie within kink_d of each other's distance
                (near the medial axis); 8: the neighbouring region (face
                interior, edge, vertex) of a mesh's closest point lying
                within kink_d of it */
} oflip;

/* A sample with w > w_min within FP32 resolution of a decision: d within
   kink_d of the activation -eps (what 0), a coordinate within kink_face cell
   units of a cell face (what 1 + axis), a friction slide within kink_d of
   mu C (what 4) or of the friction floor (what 5), a mesh sample within
   kink_d of the flat surface (what 6), of the medial axis (what 7) or of
   another region of its closest point (what 8);
   margin = that distance;
   penetrating = the side of the activation the sample took. */
typedef struct {
  int m, k, i, what;
  double margin;
  int penetrating;
} oamb;

/* oracle_step with readings and a report of the ambiguous samples: the
   n_flips flips apply to candidates flip_b[j]; for every candidate up to
   max_amb ambiguous samples go to amb [B][max_amb] in the order the step
   meets them, and n_amb [B] gets their full count. amb/n_amb may be NULL.
   The flips of the rest test's first iteration (m = 6, k = 0) also apply to
   the rest-pose samples of L_pen, which are the same points. */
int oracle_step_ex(const ohand* hand, const oobject* obj, const oparams* prm, int B, const double* q,
                   double* loss, double* terms, double* grad, int n_flips, const int* flip_b, const oflip* flips,
                   double kink_d, double kink_face, int max_amb, oamb* amb, int* n_amb, int n_threads);

/* One candidate in detail. poses [M][K+1][6] = (x, theta) before each
   iteration and after the last; samples [M][K][Nc][6] = (d, g, w, lambda) or NULL;
   p_world [Nc][3] or NULL. */
int oracle_trace(const ohand* hand, const oobject* obj, const oparams* prm, const double* q,
                 double* poses, double* samples, double* p_world);

/* Central finite differences of the loss, step fd_h. excluded [B][n_dof] is
   set where the discrete state (cells, clamps, penetration and limit
   branches) differs between q - h e_j, q and q + h e_j. */
int oracle_fd_grad(const ohand* hand, const oobject* obj, const oparams* prm, int B,
                   const double* q, double fd_h, double* grad, int* excluded, int n_threads);

/* Bias-corrected Adam step (t >= 1) on n values, in place. */
int oracle_adam(int n, double* q, double* m, double* v, const double* g, int t, double lr,
                double b1, double b2, double eps);

/* rank[k] = index of the k-th smallest loss; ties keep index order. */
int oracle_rank(int B, const double* loss, int* rank);

/* T optimizer steps with the linear dilation schedule r(t) = r0 (1 - t/(T-1)),
   then one forward at r = 0 for the final loss and the ranking.
   q [B][n_dof] in/out; loss_hist [T][B] or NULL. use_gd selects plain
   gradient descent q -= lr g instead of Adam. */
int oracle_optimize(const ohand* hand, const oobject* obj, const oparams* prm, int B, double* q,
                    int T, double r0, double lr, double b1, double b2, double eps, int use_gd,
                    double* final_loss, double* final_terms, int* rank, double* loss_hist,
                    int n_threads);

/* Weighted samples of the hand for the evaluation metrics: surface samples
   with the area each stands for, volume samples with their volume; link-local
   coordinates. */
typedef struct {
  int n_surface;
  const int* surface_link;       /* [n_surface] */
  const double* surface_local;   /* [n_surface][3] */
  const double* surface_area;    /* [n_surface] */
  int n_volume;
  const int* volume_link;        /* [n_volume] */
  const double* volume_local;    /* [n_volume][3] */
  const double* volume_weight;   /* [n_volume] */
} oeval;

/* Post-synthesis metrics of B candidates q [B][n_dof] against the object at
   rest (Sec. V-A): out [B][n_thr + 1] = contact area at each threshold
   thr[t] (total area of surface samples whose signed distance is below
   thr[t]) and the intersection volume (total volume of volume samples whose
   signed distance is below 0). slack [B][n_thr + 1] (or NULL) = the weight of
   the samples whose signed distance lies within delta of the threshold (of 0
   for the volume). A candidate with a non-finite coordinate gets NaN. */
int oracle_evaluate(const ohand* hand, const oobject* obj, int B, const double* q, const oeval* ev, int n_thr,
                    const double* thr, double delta, double* out, double* slack, int n_threads);

/* The k best of B candidates by key (ascending, or descending when
   higher_is_better), NaN keys after all others, equal keys by index:
   top [k]; mean [M] = the average of metrics [B][M] over them, summed in
   rank order. */
int oracle_select_top(int B, const double* key, int higher_is_better, int k, int M, const double* metrics,
                      int* top, double* mean);

#ifdef __cplusplus
}
#endif
#endif
