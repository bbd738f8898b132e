// Drives the host-side model build (constraint tables, ordering, supernodal
// Cholesky factor) over good, bad and large inputs.  Built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py; any memory
// error or undefined behaviour aborts with a report, and each case checks the
// return code the C ABI documents.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "host_model.h"

namespace {

struct Grid {
    int n;
    std::vector<double> X, mass, k;
    std::vector<int32_t> tris, attach;
    explicit Grid(int n_) : n(n_) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                X.push_back(i / double(n - 1));
                X.push_back(0.5 + 0.001 * ((i * 7 + j * 3) % 5));
                X.push_back(j / double(n - 1));
            }
        for (int i = 0; i + 1 < n; ++i)
            for (int j = 0; j + 1 < n; ++j) {
                const int a = i * n + j, b = (i + 1) * n + j, c = i * n + j + 1, d = (i + 1) * n + j + 1;
                const int t[6] = {a, b, d, a, d, c};
                tris.insert(tris.end(), t, t + 6);
            }
        mass.assign(n * n, 0.1 / (n * n));
        const int E = 3 * (n - 1) * (n - 1) + 2 * (n - 1);   // unique edges of this triangulation
        k.assign(E, 1.0e3);
        attach = {0, n - 1};
    }
};

int run(Grid &g, void (*edit)(sim_mesh_t &, sim_params_t &, std::vector<sim_obstacle_t> &), int leaf = 32) {
    sim_mesh_t mesh{};
    mesh.n_nodes = g.n * g.n;
    mesh.X = g.X.data();
    mesh.n_tris = (int32_t)g.tris.size() / 3;
    mesh.tris = g.tris.data();
    mesh.n_attach = (int32_t)g.attach.size();
    mesh.attach = g.attach.data();
    mesh.attach_axis[1] = 1.0;
    sim_params_t p{};
    p.h = 1.0 / 120.0;
    p.pd_iters = 20;
    p.gravity[1] = -9.8;
    p.node_mass = g.mass.data();
    p.edge_stiffness = g.k.data();
    p.bend_weight = 1e-2;
    p.attach_weight = 1e5;
    p.adj_solver = SIM_ADJ_ITERATIVE;
    std::vector<sim_obstacle_t> obst(1);
    obst[0].type = SIM_SPHERE;
    obst[0].radius = 0.25;
    obst[0].mu = 0.4;
    p.n_obstacles = 1;
    p.obstacles = obst.data();
    if (edit) edit(mesh, p, obst);
    dc::HostModel hm;
    int rc = hm.build(&mesh, &p);
    if (!rc) rc = hm.order_and_factor(leaf);
    if (!rc && hm.m <= 200) {
        std::vector<double> L((size_t)hm.m * hm.m);
        hm.dense_L(L.data());
    }
    return rc;
}

int failures = 0;
void expect(const char *name, int got, int want) {
    std::printf("%-28s rc %3d (want %3d)%s\n", name, got, want, got == want ? "" : "  <-- MISMATCH");
    if (got != want) ++failures;
}

}  // namespace

int main() {
    Grid g10(10), g150(150);
    expect("valid 10x10", run(g10, nullptr), SIM_OK);
    expect("valid 10x10 small leaves", run(g10, nullptr, 4), SIM_OK);
    expect("valid 150x150", run(g150, nullptr), SIM_OK);
    expect("self-collision", run(g10, [](sim_mesh_t &, sim_params_t &p, std::vector<sim_obstacle_t> &) {
               p.self_thickness = 0.01; p.self_radius = 0.02; p.self_mu = 0.3; }), SIM_OK);
    expect("self with direct adjoint", run(g10, [](sim_mesh_t &, sim_params_t &p, std::vector<sim_obstacle_t> &) {
               p.self_thickness = 0.01; p.adj_solver = SIM_ADJ_DIRECT; }), SIM_EINVAL);
    expect("triangle out of range", run(g10, [](sim_mesh_t &m, sim_params_t &, std::vector<sim_obstacle_t> &) {
               const_cast<int32_t *>(m.tris)[5] = 100000; }), SIM_EINVAL);
    Grid g10b(10);
    expect("negative triangle index", run(g10b, [](sim_mesh_t &m, sim_params_t &, std::vector<sim_obstacle_t> &) {
               const_cast<int32_t *>(m.tris)[0] = -3; }), SIM_EINVAL);
    Grid g10c(10);
    expect("non-finite position", run(g10c, [](sim_mesh_t &m, sim_params_t &, std::vector<sim_obstacle_t> &) {
               const_cast<double *>(m.X)[7] = NAN; }), SIM_ENONFINITE);
    Grid g10d(10);
    expect("zero mass", run(g10d, [](sim_mesh_t &, sim_params_t &p, std::vector<sim_obstacle_t> &) {
               const_cast<double *>(p.node_mass)[3] = 0.0; }), SIM_ENOTSPD);
    Grid g10e(10);
    expect("negative stiffness", run(g10e, [](sim_mesh_t &, sim_params_t &p, std::vector<sim_obstacle_t> &) {
               const_cast<double *>(p.edge_stiffness)[2] = -1.0; }), SIM_EINVAL);
    expect("attachment out of range", run(g10, [](sim_mesh_t &m, sim_params_t &, std::vector<sim_obstacle_t> &) {
               static const int32_t bad[1] = {1000}; m.attach = bad; m.n_attach = 1; }), SIM_EINVAL);
    expect("too many obstacles", run(g10, [](sim_mesh_t &, sim_params_t &p, std::vector<sim_obstacle_t> &) {
               p.n_obstacles = 9; }), SIM_EINVAL);
    expect("mesh obstacle bad vertex", run(g10, [](sim_mesh_t &, sim_params_t &, std::vector<sim_obstacle_t> &o) {
               static const double v[9] = {0, 0, 0, 1, 0, 0, 0, 0, 1};
               static const int32_t t[3] = {0, 1, 7};
               o[0].type = SIM_MESH; o[0].n_verts = 3; o[0].verts = v; o[0].n_tris = 1; o[0].tris = t; }),
           SIM_EINVAL);
    expect("explicit bad edge", run(g10, [](sim_mesh_t &m, sim_params_t &, std::vector<sim_obstacle_t> &) {
               static const int32_t e[4] = {0, 1, 5, 5}; m.edges = e; m.n_edges = 2; }), SIM_EINVAL);
    expect("no triangles", run(g10, [](sim_mesh_t &m, sim_params_t &, std::vector<sim_obstacle_t> &) {
               m.n_tris = 0; }), SIM_EINVAL);
    expect("bad time step", run(g10, [](sim_mesh_t &, sim_params_t &p, std::vector<sim_obstacle_t> &) {
               p.h = -1.0; }), SIM_EINVAL);
    std::printf("failures: %d\n", failures);
    return failures ? 1 : 0;
}
