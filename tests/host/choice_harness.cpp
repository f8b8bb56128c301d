// Host-side check of librad's block choice (Algorithm 4: fewest bytes among
// zero / dense / CSR / low-rank / hierarchical, ties to the simpler form, then
// coalescing of uniform children), run on the CPU with no HIP call.
//   stdin: N leaf_size dims nearfield s, then N x 3 centroids.
//   "pairs":  prints the tree permutation, then every block pair as
//             "I_start I_size J_start J_size first_child nchild level".
//   "decide": then reads one line "nnz rank svd_bytes" per pair (in the order
//             "pairs" printed), decides every level bottom-up as the builder
//             does, and prints the final blocks "I_start I_size J_start J_size kind".
#include "build.cpp"

#include <cstdio>
#include <cstring>

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    long N;
    int leaf, dims, nearfield, s;
    if (scanf("%ld %d %d %d %d", &N, &leaf, &dims, &nearfield, &s) != 5) return 3;
    std::vector<double> x(3 * N);
    for (auto &v : x)
        if (scanf("%lf", &v) != 1) return 4;
    rad::QuadBuilder qb;
    qb.x = x.data();
    qb.leaf_size = leaf;
    qb.max_depth = 0;
    qb.dims = dims;
    qb.nodes.resize(1);
    std::vector<int32_t> all(N);
    for (long i = 0; i < N; ++i) all[i] = (int32_t)i;
    qb.split(0, std::move(all), 0);

    rad_hmat H;
    H.nodes = qb.nodes;
    H.perm = qb.perm;
    rad::Builder B;
    B.H = &H;
    rad_build_opts_default(&B.o);
    B.o.leaf_size = leaf;
    B.o.nearfield = nearfield;
    B.s = s;
    B.enumerate_pairs();
    if (!std::strcmp(argv[1], "pairs")) {
        for (int32_t p : H.perm) printf("%d ", p);
        printf("\n%zu\n", B.bp.size());
        for (const auto &b : B.bp)
            printf("%d %d %d %d %d %d %d\n", H.nodes[b.I].start, H.nodes[b.I].size, H.nodes[b.J].start,
                   H.nodes[b.J].size, b.first_child, b.nchild, b.level);
        return 0;
    }
    for (auto &b : B.bp) {
        long long nnz, rank, svd;
        if (scanf("%lld %lld %lld", &nnz, &rank, &svd) != 3) return 5;
        b.nnz = nnz;
        b.rank = (int32_t)rank;
        b.svd_bytes = svd;
    }
    int32_t max_level = 0;
    for (const auto &b : B.bp) max_level = std::max(max_level, b.level);
    for (int32_t L = max_level; L >= 0; --L)
        for (size_t p = 0; p < B.bp.size(); ++p)
            if (B.bp[p].level == L) B.decide((int64_t)p);
    std::vector<int64_t> stack;
    for (size_t p = 0; p < B.bp.size() && B.bp[p].level == 0; ++p) stack.push_back((int64_t)p);
    while (!stack.empty()) {
        const int64_t p = stack.back();
        stack.pop_back();
        const auto &b = B.bp[p];
        if (b.kind == rad::BK_HIER) {
            for (int k = 0; k < b.nchild; ++k) stack.push_back(b.first_child + k);
        } else {
            printf("%d %d %d %d %d\n", H.nodes[b.I].start, H.nodes[b.I].size, H.nodes[b.J].start, H.nodes[b.J].size,
                   (int)b.kind);
        }
    }
    return 0;
}
