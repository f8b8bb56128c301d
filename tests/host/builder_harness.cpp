// Host-side checks of two numerical routines of librad's builder
// (build.cpp), run on the CPU with no HIP call:
//   "svd":  stdin "l" then the l x l matrix column-major; prints the singular
//           values, then U*Sigma and V column-major (one-sided Jacobi SVD used
//           by the rank search on the host);
//   "geom": stdin "nv nf", vertices (nv x 3) and faces (nf x 3); prints each
//           facet's centroid, unit normal and area (section 3 geometry).
#include "build.cpp"

#include <cstdio>
#include <cstring>

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    if (!std::strcmp(argv[1], "svd")) {
        int l;
        if (scanf("%d", &l) != 1 || l < 1) return 3;
        std::vector<double> A((size_t)l * l), V, sv;
        for (auto &a : A)
            if (scanf("%lf", &a) != 1) return 4;
        rad::jacobi_svd(l, A, V, sv);
        for (double s : sv) printf("%.17g ", s);
        printf("\n");
        for (double a : A) printf("%.17g ", a);
        printf("\n");
        for (double v : V) printf("%.17g ", v);
        printf("\n");
        return 0;
    }
    long nv, nf;
    if (scanf("%ld %ld", &nv, &nf) != 2) return 3;
    std::vector<double> verts(3 * nv);
    std::vector<int32_t> faces(3 * nf);
    for (auto &v : verts)
        if (scanf("%lf", &v) != 1) return 4;
    for (auto &f : faces)
        if (scanf("%d", &f) != 1) return 5;
    std::vector<double> x, n, A;
    rad::facet_geometry(verts.data(), nv, faces.data(), nf, x, n, A);
    for (long i = 0; i < nf; ++i)
        printf("%.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", x[3 * i], x[3 * i + 1], x[3 * i + 2], n[3 * i],
               n[3 * i + 1], n[3 * i + 2], A[i]);
    return 0;
}
