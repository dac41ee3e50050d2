/*
 * Plain FP64 CPU oracle of the Shan-Chen D3Q19 lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path includes, links or calls this file:
 * only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py use it. It shares
 * no code, header, table or constant with the HIP library.
 *
 * What it follows (Lulli, Biferale, Falcucci, Sbragaglia, Shan, "A Mesoscale Perspective on the
 * Tolman Length", arXiv:2105.08772):
 *   - lattice transport with BGK collision and Guo forcing: Sec. 2, Eqs. (lbm), (sm:omega_i) and
 *     the unnumbered Guo-term, equilibrium and equilibrium-velocity equations that follow them;
 *   - the Shan-Chen force, Eq. (SCForce), with W(1)=1/6, W(2)=1/12;
 *   - the lattice pressure tensor, Eq. (sm:pt);
 *   - the two pseudopotentials of Sec. 4: exp(-1/n) and 1-exp(-n);
 *   - the tanh initial profile of Sec. 4.
 *
 * Readings taken where the paper is silent or garbled:
 *   - the quadratic term of the equilibrium carries the usual factor 1/2, (xi.u)^2/(2 c_s^4);
 *     without it the second moment is not n c_s^2 delta + n u u;
 *   - D3Q19 weights are the standard 1/3, 1/18, 1/36 (the paper cites textbooks for them);
 *   - the state at time t is the pre-collision (post-streaming) population set, and psi, F and
 *     u_eq are all taken from it;
 *   - the initial populations are the equilibrium at zero physical velocity, f = f_eq(n, -F/(2n));
 *   - the tanh profile has an explicit width w: tanh((r - R)/w);
 *   - the additive initial noise is SplitMix64 (Steele, Lea, Flood 2014) evaluated at
 *     (seed XOR linear node index), mapped to [0,1) with its top 53 bits.
 *
 * Layout of every population array: f[i][z][y][x], x fastest, no padding, FP64.
 * Fields: n[z][y][x]; vectors v[c][z][y][x] (c = 0,1,2 for x,y,z); pressure tensor
 * P[k][z][y][x] with k = 0..5 for xx, yy, zz, xy, xz, yz.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* D3Q19 velocity set (Sec. 2, Sec. 4): rest, the six axis vectors, the twelve face diagonals.
 * Every moving velocity is followed by its opposite. */
static const int XI[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};

static const double CS2 = 1.0 / 3.0; /* speed of sound squared, c_s^2 = 1/3 (Sec. 2) */

/* Lattice weight w_i of D3Q19 by squared speed. */
static double lattice_w(int i)
{
    int s = XI[i][0] * XI[i][0] + XI[i][1] * XI[i][1] + XI[i][2] * XI[i][2];
    if (s == 0) return 1.0 / 3.0;
    if (s == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* Forcing weight W(|xi_a|^2) of Eq. (SCForce): W(1) = 1/6, W(2) = 1/12. */
static double force_W(int a)
{
    int s = XI[a][0] * XI[a][0] + XI[a][1] * XI[a][1] + XI[a][2] * XI[a][2];
    return s == 1 ? 1.0 / 6.0 : 1.0 / 12.0;
}

static int wrap(int v, int L)
{
    v %= L;
    return v < 0 ? v + L : v;
}

static size_t node(int x, int y, int z, int nx, int ny)
{
    return ((size_t)z * ny + y) * nx + x;
}

/* Pseudopotential psi(n) of Sec. 4: kind 0 is exp(-1/n), kind 1 is 1 - exp(-n). */
double ora_psi(double n, int kind)
{
    return kind == 0 ? exp(-1.0 / n) : 1.0 - exp(-n);
}

/* Threads an OpenMP loop of the oracle uses. */
int ora_threads(void) { return omp_get_max_threads(); }

/* Set the number of threads of the oracle's loops (for timing it on a given core count). */
void ora_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

/* Exposed constants so that tests can check the tables themselves. */
void ora_tables(int* xi_out, double* w_out, double* W_out)
{
    for (int i = 0; i < Q; ++i) {
        for (int c = 0; c < 3; ++c) xi_out[3 * i + c] = XI[i][c];
        w_out[i] = lattice_w(i);
        W_out[i] = i == 0 ? 0.0 : force_W(i);
    }
}

/* Density n = sum_i f_i (Sec. 2) and psi(n) at every node. */
void ora_density(const double* f, int nx, int ny, int nz, int kind, double* n, double* psi)
{
    size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double acc = 0.0;
        for (int i = 0; i < Q; ++i) acc += f[(size_t)i * N + s];
        n[s] = acc;
        if (psi) psi[s] = ora_psi(acc, kind);
    }
}

/* Shan-Chen force, Eq. (SCForce):
 *   F^mu(x) = -G c_s^2 psi(x) sum_{a=1..18} W(|xi_a|^2) psi(x + xi_a) xi_a^mu
 * on a periodic box. F is [3][z][y][x]. */
void ora_force(const double* psi, int nx, int ny, int nz, double G, double* F)
{
    size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s[3] = {0.0, 0.0, 0.0};
                for (int a = 1; a < Q; ++a) {
                    double pn = psi[node(wrap(x + XI[a][0], nx), wrap(y + XI[a][1], ny),
                                         wrap(z + XI[a][2], nz), nx, ny)];
                    for (int c = 0; c < 3; ++c) s[c] += force_W(a) * pn * XI[a][c];
                }
                size_t k = node(x, y, z, nx, ny);
                for (int c = 0; c < 3; ++c) F[c * N + k] = -G * CS2 * psi[k] * s[c];
            }
}

/* Second-order equilibrium (Sec. 2), with the 1/2 on the quadratic term:
 *   f_eq_i = w_i n [1 + xi.u/c_s^2 + (xi.u)^2/(2 c_s^4) - u.u/(2 c_s^2)] */
static double f_equilibrium(int i, double n, const double u[3])
{
    double xu = XI[i][0] * u[0] + XI[i][1] * u[1] + XI[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return lattice_w(i) * n * (1.0 + xu / CS2 + xu * xu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Guo forcing term (Sec. 2):
 *   F_i = (1 - 1/(2 tau)) w_i [ xi_i^a / c_s^2 + (xi_i^a xi_i^b - c_s^2 delta^ab) u_b / c_s^4 ] F_a */
static double guo_term(int i, double tau, const double u[3], const double F[3])
{
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
        double coef = XI[i][a] / CS2;
        for (int b = 0; b < 3; ++b) {
            double d = (a == b) ? 1.0 : 0.0;
            coef += (XI[i][a] * XI[i][b] - CS2 * d) * u[b] / (CS2 * CS2);
        }
        acc += coef * F[a];
    }
    return (1.0 - 1.0 / (2.0 * tau)) * lattice_w(i) * acc;
}

/* Post-collision populations at one node from its pre-collision populations fl[19], its density,
 * and its force: u_eq = (sum_i xi_i f_i + F/2)/n, then BGK (Eq. sm:omega_i) plus the Guo term:
 *   f*_i = f_i - (f_i - f_eq_i)/tau + F_i.                                                     */
static void collide(const double fl[Q], double n, const double F[3], double tau, double fstar[Q])
{
    double u[3];
    for (int c = 0; c < 3; ++c) {
        double j = 0.0;
        for (int i = 0; i < Q; ++i) j += XI[i][c] * fl[i];
        u[c] = j / n + F[c] / (2.0 * n);
    }
    for (int i = 0; i < Q; ++i) {
        double feq = f_equilibrium(i, n, u);
        fstar[i] = fl[i] - (fl[i] - feq) / tau + guo_term(i, tau, u, F);
    }
}

/* One time step, Eq. (lbm): f_i(x + xi_i, t + 1) = f_i(x, t) + Omega_i(x, t) + F_i(x, t).
 * f is the pre-collision state at t, fout receives the pre-collision state at t + 1. */
void ora_step(const double* f, double* fout, int nx, int ny, int nz, double G, double tau, int kind)
{
    size_t N = (size_t)nx * ny * nz;
    double* n = (double*)malloc(N * sizeof(double));
    double* psi = (double*)malloc(N * sizeof(double));
    double* F = (double*)malloc(3 * N * sizeof(double));
    ora_density(f, nx, ny, nz, kind, n, psi);
    ora_force(psi, nx, ny, nz, G, F);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t k = node(x, y, z, nx, ny);
                double fl[Q], fs[Q], Fk[3] = {F[k], F[N + k], F[2 * N + k]};
                for (int i = 0; i < Q; ++i) fl[i] = f[(size_t)i * N + k];
                collide(fl, n[k], Fk, tau, fs);
                for (int i = 0; i < Q; ++i) {
                    size_t dst = node(wrap(x + XI[i][0], nx), wrap(y + XI[i][1], ny),
                                      wrap(z + XI[i][2], nz), nx, ny);
                    fout[(size_t)i * N + dst] = fs[i];
                }
            }
    free(n);
    free(psi);
    free(F);
}

/* Post-collision populations f*_i(x) at a single node, computed from the full pre-collision state
 * without building any whole-box field: the densities of the node and of its 18 neighbours are
 * summed directly. Used to check large boxes on sampled nodes. */
void ora_collide_at(const double* f, int nx, int ny, int nz, double G, double tau, int kind, int x,
                    int y, int z, double* fstar)
{
    size_t N = (size_t)nx * ny * nz;
    double psin[Q];
    for (int a = 0; a < Q; ++a) {
        size_t k = node(wrap(x + XI[a][0], nx), wrap(y + XI[a][1], ny), wrap(z + XI[a][2], nz), nx,
                        ny);
        double nn = 0.0;
        for (int i = 0; i < Q; ++i) nn += f[(size_t)i * N + k];
        psin[a] = ora_psi(nn, kind);
    }
    size_t k0 = node(x, y, z, nx, ny);
    double fl[Q], n0 = 0.0, F[3], s[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        fl[i] = f[(size_t)i * N + k0];
        n0 += fl[i];
    }
    for (int a = 1; a < Q; ++a)
        for (int c = 0; c < 3; ++c) s[c] += force_W(a) * psin[a] * XI[a][c];
    for (int c = 0; c < 3; ++c) F[c] = -G * CS2 * psin[0] * s[c];
    collide(fl, n0, F, tau, fstar);
}

/* Lattice pressure tensor, Eq. (sm:pt):
 *   P^{mu nu}(x) = n c_s^2 delta^{mu nu}
 *                  + (G c_s^2 / 2) psi(x) sum_a W(|xi_a|^2) psi(x + xi_a) xi_a^mu xi_a^nu
 * from the pre-collision state f. P is [6][z][y][x] (xx, yy, zz, xy, xz, yz). */
void ora_pressure_tensor(const double* f, int nx, int ny, int nz, double G, int kind, double* P)
{
    static const int MU[6] = {0, 1, 2, 0, 0, 1};
    static const int NU[6] = {0, 1, 2, 1, 2, 2};
    size_t N = (size_t)nx * ny * nz;
    double* n = (double*)malloc(N * sizeof(double));
    double* psi = (double*)malloc(N * sizeof(double));
    ora_density(f, nx, ny, nz, kind, n, psi);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t k = node(x, y, z, nx, ny);
                double s[6] = {0, 0, 0, 0, 0, 0};
                for (int a = 1; a < Q; ++a) {
                    double pn = psi[node(wrap(x + XI[a][0], nx), wrap(y + XI[a][1], ny),
                                         wrap(z + XI[a][2], nz), nx, ny)];
                    for (int c = 0; c < 6; ++c)
                        s[c] += force_W(a) * pn * XI[a][MU[c]] * XI[a][NU[c]];
                }
                for (int c = 0; c < 6; ++c) {
                    double iso = (MU[c] == NU[c]) ? n[k] * CS2 : 0.0;
                    P[(size_t)c * N + k] = iso + 0.5 * G * CS2 * psi[k] * s[c];
                }
            }
    free(n);
    free(psi);
}

/* SplitMix64 output for one counter value (Steele, Lea, Flood, OOPSLA 2014): the generator's
 * state advance by the golden-ratio increment followed by its finalising mix. */
static uint64_t splitmix64(uint64_t state)
{
    uint64_t z = state + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform noise in [-amp, amp) for one node: SplitMix64(seed ^ linear node index), top 53 bits. */
double ora_noise(uint64_t seed, uint64_t linear_index, double amp)
{
    double u = (double)(splitmix64(seed ^ linear_index) >> 11) * (1.0 / 9007199254740992.0);
    return amp * (2.0 * u - 1.0);
}

/* Signed minimum-image displacement of coordinate v from centre c on a periodic axis of length L. */
static double min_image(int v, int c, int L)
{
    int d = v - c;
    if (2 * d > L) d -= L;
    if (2 * d < -L) d += L;
    return (double)d;
}

/* Initial density field (Sec. 4):
 *   n(r) = (n_in + n_out)/2 - (n_in - n_out)/2 * tanh((r - R)/w) + noise,
 * with r the distance to the box centre floor(L/2) (minimum image). geom 0/1 (droplet/bubble):
 * r is the 3D distance; geom 2 (slab): r is |displacement| along slab_axis and R is the half
 * thickness. Writes n[z][y][x]. */
void ora_init_density(int nx, int ny, int nz, int geom, int slab_axis, double R, double w,
                      double n_in, double n_out, double noise_amp, uint64_t seed, double* n)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double d[3] = {min_image(x, cx, nx), min_image(y, cy, ny), min_image(z, cz, nz)};
                double r;
                if (geom == 2)
                    r = fabs(d[slab_axis]);
                else
                    r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                size_t k = node(x, y, z, nx, ny);
                double v = 0.5 * (n_in + n_out) - 0.5 * (n_in - n_out) * tanh((r - R) / w);
                if (noise_amp != 0.0) v += ora_noise(seed, (uint64_t)k, noise_amp);
                n[k] = v;
            }
}

/* Initial populations from a density field: the equilibrium at zero physical velocity,
 * f_i = f_eq_i(n, u) with u = -F/(2n), so that u_eq = (sum xi f + F/2)/n = 0. */
void ora_init_populations(const double* n, int nx, int ny, int nz, double G, int kind, double* f)
{
    size_t N = (size_t)nx * ny * nz;
    double* psi = (double*)malloc(N * sizeof(double));
    double* F = (double*)malloc(3 * N * sizeof(double));
    for (size_t k = 0; k < N; ++k) psi[k] = ora_psi(n[k], kind);
    ora_force(psi, nx, ny, nz, G, F);
#pragma omp parallel for schedule(static)
    for (long long k = 0; k < (long long)N; ++k) {
        double u[3];
        for (int c = 0; c < 3; ++c) u[c] = -F[(size_t)c * N + k] / (2.0 * n[k]);
        for (int i = 0; i < Q; ++i) f[(size_t)i * N + k] = f_equilibrium(i, n[k], u);
    }
    free(psi);
    free(F);
}

/* Momentum density sum_i xi_i f_i and physical velocity u_eq = (sum_i xi_i f_i + F/2)/n at
 * every node (Sec. 2). j and u are [3][z][y][x]; either may be NULL. */
void ora_velocity(const double* f, int nx, int ny, int nz, double G, int kind, double* j, double* u)
{
    size_t N = (size_t)nx * ny * nz;
    double* n = (double*)malloc(N * sizeof(double));
    double* psi = (double*)malloc(N * sizeof(double));
    double* F = (double*)malloc(3 * N * sizeof(double));
    ora_density(f, nx, ny, nz, kind, n, psi);
    ora_force(psi, nx, ny, nz, G, F);
#pragma omp parallel for schedule(static)
    for (long long k = 0; k < (long long)N; ++k)
        for (int c = 0; c < 3; ++c) {
            double jc = 0.0;
            for (int i = 0; i < Q; ++i) jc += XI[i][c] * f[(size_t)i * N + k];
            if (j) j[(size_t)c * N + k] = jc;
            if (u) u[(size_t)c * N + k] = (jc + 0.5 * F[(size_t)c * N + k]) / n[k];
        }
    free(n);
    free(psi);
    free(F);
}

/* Helper for the step loop used by long runs: nsteps applications of ora_step, ping-ponging
 * between f and a scratch buffer; the result is left in f. */
void ora_run(double* f, int nx, int ny, int nz, double G, double tau, int kind, long long nsteps)
{
    size_t N = (size_t)nx * ny * nz;
    double* g = (double*)malloc((size_t)Q * N * sizeof(double));
    double* cur = f;
    double* nxt = g;
    for (long long s = 0; s < nsteps; ++s) {
        ora_step(cur, nxt, nx, ny, nz, G, tau, kind);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != f) memcpy(f, cur, (size_t)Q * N * sizeof(double));
    free(g);
}
