// Host-only sanitizer run: the einsum parser on valid, malformed and random
// specs, and the oracle on tiny shapes, built with AddressSanitizer and
// UndefinedBehaviorSanitizer (a report aborts the run).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

extern "C" {
int oracle_mttkrp(int N, const int64_t *dims, int n, int64_t R, const double *X, const double *const *U, double *M);
int oracle_ttmc(int N, const int64_t *dims, int n, const int64_t *ranks, const double *X, const double *const *U,
                double *Y);
}

int main()
{
    const char *specs[] = {"ijk,ja,ka->ia",
                           "ijk,ia,ka->ja",
                           "ijklm,jb,kc,ld,me->ibcde",
                           "ij,ja->ia",
                           "abcde,az,bz,dz,ez->cz",
                           "",
                           "->",
                           "ijk,ja,ka",
                           "ijk,ja,kb->ia",
                           "ijk,ja,ka->iaa",
                           "iik,ia,ka->ia",
                           "ijkabcdefghijklmnop,ja->ia",
                           "  i j k , j a , k a -> i a ",
                           "ijk,ja,ka->ia,",
                           ",,,->"};
    int accepted = 0;
    for (const char *t : specs) {
        deinsum_spec sp;
        if (deinsum::parse_spec(t, &sp) == DEINSUM_OK) ++accepted;
    }
    // random strings over the spec alphabet
    std::srand(11);
    const char alphabet[] = "ijklmabcz,->  ";
    for (int k = 0; k < 20000; ++k) {
        std::string t;
        const int len = std::rand() % 40;
        for (int i = 0; i < len; ++i) t += alphabet[std::rand() % (sizeof(alphabet) - 1)];
        deinsum_spec sp;
        (void)deinsum::parse_spec(t.c_str(), &sp);
    }
    (void)deinsum::parse_spec(nullptr, nullptr);
    // oracle on tiny shapes
    const int64_t dims[3] = {3, 4, 5};
    std::vector<double> X(60), B(4 * 2), C(5 * 2), M(3 * 2), Y(3 * 2 * 2);
    for (size_t i = 0; i < X.size(); ++i) X[i] = static_cast<double>(i % 7) - 3.0;
    for (size_t i = 0; i < B.size(); ++i) B[i] = 0.5 * static_cast<double>(i);
    for (size_t i = 0; i < C.size(); ++i) C[i] = 1.0 - 0.25 * static_cast<double>(i);
    const double *U[3] = {nullptr, B.data(), C.data()};
    int rc = oracle_mttkrp(3, dims, 0, 2, X.data(), U, M.data());
    const int64_t ranks[3] = {0, 2, 2};
    rc |= oracle_ttmc(3, dims, 0, ranks, X.data(), U, Y.data());
    const int64_t empty[3] = {3, 0, 5};  // rejected or summed to zero; either way no fault
    (void)oracle_mttkrp(3, empty, 0, 2, X.data(), U, M.data());
    std::printf("san: accepted %d, oracle rc %d\n", accepted, rc);
    return rc == 0 ? 0 : 1;
}
