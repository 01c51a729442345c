// Builds host-only IFGF plans (no GPU use) through the C ABI, for the
// ThreadSanitizer run of the threaded host plan builder: an equiangular
// cube-sphere at two wavenumbers, a random cloud, and both again on an
// adaptive octree, printing the counts.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../include/ifgf.h"

static std::vector<double> cube_sphere(int n)
{
    std::vector<double> p;
    const double pi = 3.14159265358979323846;
    for (int f = 0; f < 6; ++f)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double u = std::tan(pi / 4.0 * (2.0 * (i + 0.5) / n - 1.0));
                double v = std::tan(pi / 4.0 * (2.0 * (j + 0.5) / n - 1.0));
                double s = (f & 1) ? -1.0 : 1.0;
                double x[3];
                if (f < 2) { x[0] = s; x[1] = u; x[2] = v; }
                else if (f < 4) { x[0] = u; x[1] = s; x[2] = v; }
                else { x[0] = u; x[1] = v; x[2] = s; }
                double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                for (int a = 0; a < 3; ++a) p.push_back(x[a] / r);
            }
    return p;
}

static int run(const std::vector<double>& p, double k, int levels, int leaf_max = 0)
{
    ifgf_options o{};
    o.host_only = 1;
    o.leaf_max = leaf_max;
    ifgf_plan_t plan = nullptr;
    ifgf_status s = ifgf_plan_create(p.data(), (int64_t)(p.size() / 3), k, levels, nullptr, &o, &plan);
    if (s != IFGF_OK) {
        std::printf("create failed: %s\n", ifgf_last_error());
        return 1;
    }
    ifgf_stats st;
    ifgf_plan_stats(plan, &st);
    long long cones = 0;
    for (int d = 1; d <= st.D; ++d) cones += st.n_cones[d];
    std::printf("N=%d D=%d cones=%lld near=%lld\n", st.n_points, st.D, cones, (long long)st.n_near_pairs);
    ifgf_plan_destroy(plan);
    return 0;
}

int main()
{
    int bad = 0;
    bad |= run(cube_sphere(48), 12.0 * 3.14159265358979323846, 0);
    bad |= run(cube_sphere(24), 0.0, 0);
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> u(-0.5, 0.5);
    std::vector<double> c(3 * 8000);
    for (double& x : c) x = u(g);
    bad |= run(c, 40.0, 6);
    bad |= run(cube_sphere(32), 8.0 * 3.14159265358979323846, 6, 12);
    bad |= run(c, 40.0, 6, 20);
    return bad;
}
