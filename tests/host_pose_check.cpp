// Host check of the bound that lets lbm_set_pose place a moving solid without
// waiting for the device's count of samples outside the domain (compiled and
// run by test_host_pose.py).  For random bodies and poses, many of them with
// the body grazing a face, whenever pose_inside_box accepts a pose every
// sample placed by place_coord (the kernel's own placement) must satisfy the
// device's test 0 <= x < top on every axis.  Also counts how often an inside
// pose is accepted (the bound's tightness, printed).  Prints "OK" at the end.
#include "lbm_internal.hpp"

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

using namespace lbm;

static void rotation(std::mt19937_64 &rng, double R[9])
{
    std::normal_distribution<double> n01(0.0, 1.0);
    double q[4], s = 0;
    for (double &v : q) {
        v = n01(rng);
        s += v * v;
    }
    s = std::sqrt(s);
    const double w = q[0] / s, x = q[1] / s, y = q[2] / s, z = q[3] / s;
    const double M[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                         2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                         2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
    for (int k = 0; k < 9; ++k) R[k] = M[k];
}

int main()
{
    std::mt19937_64 rng(2101);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    long accepted = 0, inside = 0, unsound = 0, trials = 0;
    for (int body = 0; body < 300; ++body) {
        // a point cloud: scale from tiny to large, offset from the origin, the
        // box corners included so that the box is tight
        const double scale = std::pow(10.0, -2.0 + 4.0 * u01(rng));
        const double off[3] = {scale * (u01(rng) - 0.5), scale * (u01(rng) - 0.5), scale * (u01(rng) - 0.5)};
        const int n = 64;
        std::vector<float> X(3 * n);
        for (int s = 0; s < n; ++s)
            for (int a = 0; a < 3; ++a) X[3 * s + a] = (float)(off[a] + scale * (u01(rng) - 0.5));
        for (int a = 0; a < 3; ++a) {
            X[3 * 0 + a] = (float)(off[a] - 0.5 * scale);
            X[3 * 1 + a] = (float)(off[a] + 0.5 * scale);
        }
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = hi[a] = X[a];
            for (int s = 1; s < n; ++s) {
                lo[a] = std::fmin(lo[a], X[3 * s + a]);
                hi[a] = std::fmax(hi[a], X[3 * s + a]);
            }
        }
        const double top[3] = {std::floor(8.0 + 3.0 * scale * (1.0 + u01(rng))), std::floor(8.0 + 3.0 * scale),
                               std::floor(8.0 + 3.0 * scale * u01(rng) + 3.0 * scale)};
        for (int pose = 0; pose < 400; ++pose) {
            double R[9], o[3];
            rotation(rng, R);
            // origins anywhere, and origins that put the body's reach right at a face
            for (int a = 0; a < 3; ++a) {
                double reach = std::fabs(R[3 * a] * off[0] + R[3 * a + 1] * off[1] + R[3 * a + 2] * off[2]);
                for (int b = 0; b < 3; ++b) reach += std::fabs(R[3 * a + b]) * 0.5 * scale;
                const double r = u01(rng);
                if (pose % 3 == 0) o[a] = top[a] * r;
                else if (pose % 3 == 1) o[a] = reach * (1.0 + 1e-7 * (r - 0.5));   // grazing the low face
                else o[a] = top[a] - reach * (1.0 + 1e-7 * (r - 0.5));             // grazing the high face
            }
            ++trials;
            bool all_in = true;
            for (int s = 0; s < n && all_in; ++s)
                for (int a = 0; a < 3; ++a) {
                    const float p = place_coord(R, o, a, X[3 * s], X[3 * s + 1], X[3 * s + 2]);
                    if (!(p >= 0.0f) || !(p < (float)top[a])) all_in = false;
                }
            const bool ok = pose_inside_box(R, o, lo, hi, top);
            inside += all_in;
            accepted += ok;
            if (ok && !all_in) {
                if (unsound++ < 5) std::printf("accepted a pose that places a sample outside (body %d pose %d)\n", body, pose);
            }
        }
    }
    std::printf("trials %ld, all samples inside %ld, accepted without waiting %ld\n", trials, inside, accepted);
    if (unsound) return 1;
    std::printf("OK\n");
    return 0;
}
