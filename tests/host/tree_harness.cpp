// Host-side check of librad's tree builder (Algorithm 2, quadtree or octree).
// Compiled by tests/test_host_tree.py into a small CPU program: it includes
// the builder's translation unit, builds the tree of the centroids read from
// stdin and prints the leaf count, the tree permutation and the leaves'
// (start, size).  No HIP call is made.
//
// stdin: N leaf_size dims, then N x 3 centroid coordinates.
#include "build.cpp"

#include <cstdio>

int main() {
    long N;
    int leaf, dims;
    if (scanf("%ld %d %d", &N, &leaf, &dims) != 3) return 2;
    std::vector<double> x(3 * N);
    for (long i = 0; i < 3 * N; ++i)
        if (scanf("%lf", &x[i]) != 1) return 3;
    rad::QuadBuilder qb;
    qb.x = x.data();
    qb.leaf_size = leaf;
    qb.max_depth = 0;
    qb.dims = dims;
    qb.nodes.resize(1);
    std::vector<int32_t> all(N);
    for (long i = 0; i < N; ++i) all[i] = (int32_t)i;
    qb.split(0, std::move(all), 0);
    printf("%d\n", qb.nleaves);
    for (int32_t p : qb.perm) printf("%d ", p);
    printf("\n");
    for (const auto &nd : qb.nodes)
        if (nd.nchild == 0) printf("%d %d ", nd.start, nd.size);
    printf("\n");
    return 0;
}
