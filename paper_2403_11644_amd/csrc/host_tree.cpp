// host_tree.cpp -- the paper's own method on the host's cores: the Pauli tree
// walk (Sec. III-A, Algorithms 1-4) and its multi-threaded forest (Sec. V-B),
// with the diagonal variant of Sec. IV-A.  It is a baseline of that method
// next to the device path, not a path of it: nothing else in the library
// calls it, and it makes no HIP call.
//
// The tree's first level below the root fixes qubit 0 (the rightmost
// Kronecker factor), its leaves qubit n - 1.  A node at depth q has chosen
// the letters of qubits 0 .. q - 1, and its state describes rows j < 2^q of
// the partial product P~ (Y replaced by iY, so that every nonzero is +1 or
// -1): the sign m[j] and the column offset k[j] = (j ^ x) - x, relative to
// the node's X-bits x.  Kept relative, a choice of X or Y on qubit q leaves
// rows below 2^q untouched, so the four children of a node differ only in
// rows 2^q .. 2^(q+1) - 1, and visiting them in the order I, X, Y, Z turns
// each into the next with one pass over that half:
//   I: copy the lower half up, columns + 2^q, signs unchanged;
//   X: columns - 2^(q+1) (the same values one block to the left);
//   Y: signs negated (iY has X's positions);
//   Z: columns + 2^(q+1) (Z has iY's values at I's positions).
// At a leaf, row j of P~ has its nonzero at column k[j] + x = j ^ x, and the
// coefficient is 2^-n (-i)^(number of Y) sum_j m[j] A[j ^ x][j] (Algorithm 2:
// the trace of P A).  With the diagonal flag only I and Z are visited, k is
// the identity and only m is kept (Sec. IV-A).
//
// Elementary operations are counted as the paper counts them: one per entry
// of k or m written by an update, plus the two of the root's initialisation.
// A whole tree (split 0) then costs 9/7 + 5/7 8^n (general) or 4/3 + 2/3 4^n
// (diagonal), the closed forms of Sec. III-B and IV-A.
//
// The forest cuts every branch at depth `split`: 4^split trees (2^split
// diagonal), numbered in the order the single walk would reach their roots
// (qubit 0's letter is the most significant base-4 digit).  Each tree builds
// its root's state by replaying the updates along its path from a fresh
// root, then walks on exactly as the whole tree would, so the arithmetic of
// every coefficient, and hence its value, is independent of the split and of
// the thread count.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <new>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/ptd.h"

namespace {

struct TreeTask {
    int n = 0;
    int split = 0;
    bool diag = false;
    const double* A = nullptr;  // complex128, interleaved, row pitch lda elements
    int64_t lda = 0;
    double* coeff = nullptr;    // complex128, interleaved, 2^n x 2^n, c[x][z]
};

class Walker {
public:
    explicit Walker(const TreeTask& t) : t_(t), N_((int64_t)1 << t.n), k_(N_), m_(N_) {}

    uint64_t ops() const { return ops_; }

    // Decompose every string of tree `tree` of the forest.
    void run_tree(int64_t tree)
    {
        k_[0] = 0;
        m_[0] = 1;
        ops_ += 2;
        const int radix_bits = t_.diag ? 1 : 2;
        uint32_t x = 0, z = 0;
        int ny = 0;
        for (int q = 0; q < t_.split; ++q) {
            const int letter = (int)((tree >> (radix_bits * (t_.split - 1 - q))) & (t_.diag ? 1 : 3));
            const int64_t h = (int64_t)1 << q;
            copy_up(h);
            if (t_.diag) {
                if (letter == 1) {
                    negate(h);
                    z |= (uint32_t)h;
                }
                continue;
            }
            // reach the letter through its elder siblings, as the walk does
            if (letter >= 1) shift_x(h);
            if (letter >= 2) negate(h);
            if (letter >= 3) shift_z(h);
            if (letter == 1 || letter == 2) x |= (uint32_t)h;
            if (letter >= 2) z |= (uint32_t)h;
            if (letter == 2) ++ny;
        }
        walk(t_.split, x, z, ny);
    }

private:
    void copy_up(int64_t h)
    {
        if (!t_.diag)
            for (int64_t j = 0; j < h; ++j) k_[h + j] = k_[j] + (int32_t)h;
        for (int64_t j = 0; j < h; ++j) m_[h + j] = m_[j];
        ops_ += (uint64_t)(t_.diag ? h : 2 * h);
    }
    void shift_x(int64_t h)
    {
        for (int64_t j = 0; j < h; ++j) k_[h + j] -= (int32_t)(2 * h);
        ops_ += (uint64_t)h;
    }
    void negate(int64_t h)
    {
        for (int64_t j = 0; j < h; ++j) m_[h + j] = (int8_t)-m_[h + j];
        ops_ += (uint64_t)h;
    }
    void shift_z(int64_t h)
    {
        for (int64_t j = 0; j < h; ++j) k_[h + j] += (int32_t)(2 * h);
        ops_ += (uint64_t)h;
    }

    void walk(int q, uint32_t x, uint32_t z, int ny)
    {
        if (q == t_.n) {
            leaf(x, z, ny);
            return;
        }
        const int64_t h = (int64_t)1 << q;
        copy_up(h);
        walk(q + 1, x, z, ny);  // I
        if (t_.diag) {
            negate(h);
            walk(q + 1, x, z | (uint32_t)h, ny);  // Z
            return;
        }
        shift_x(h);
        walk(q + 1, x | (uint32_t)h, z, ny);  // X
        negate(h);
        walk(q + 1, x | (uint32_t)h, z | (uint32_t)h, ny + 1);  // Y
        shift_z(h);
        walk(q + 1, x, z | (uint32_t)h, ny);  // Z
    }

    void leaf(uint32_t x, uint32_t z, int ny)
    {
        double re = 0.0, im = 0.0;
        const double* A = t_.A;
        const int64_t lda = t_.lda;
        if (t_.diag) {
            for (int64_t j = 0; j < N_; ++j) {
                const double s = (double)m_[j];
                const double* a = A + 2 * (j * lda + j);
                re += s * a[0];
                im += s * a[1];
            }
        } else {
            for (int64_t j = 0; j < N_; ++j) {
                const double s = (double)m_[j];
                const double* a = A + 2 * ((int64_t)(k_[j] + (int32_t)x) * lda + j);
                re += s * a[0];
                im += s * a[1];
            }
        }
        // P = (-i)^ny P~, and the 2^-n of the Hilbert-Schmidt normalisation
        double cr, ci;
        switch (ny & 3) {
            case 0: cr = re; ci = im; break;
            case 1: cr = im; ci = -re; break;
            case 2: cr = -re; ci = -im; break;
            default: cr = -im; ci = re; break;
        }
        double* out = t_.coeff + 2 * ((int64_t)x * N_ + z);
        out[0] = std::ldexp(cr, -t_.n);
        out[1] = std::ldexp(ci, -t_.n);
    }

    const TreeTask& t_;
    const int64_t N_;
    std::vector<int32_t> k_;
    std::vector<int8_t> m_;
    uint64_t ops_ = 0;
};

}  // namespace

extern "C" ptd_status ptd_host_tree_decompose(int n, unsigned flags, const void* A, int64_t lda, void* coeff_out,
                                              int split, int64_t tree_begin, int64_t tree_end, int threads,
                                              uint64_t* ops_out)
{
    if (n < 1 || n > 16 || !A || !coeff_out) return PTD_EINVAL;
    if ((flags & ~(unsigned)PTD_DIAGONAL) != 0u) return PTD_EINVAL;
    const int64_t N = (int64_t)1 << n;
    if (lda < N || split < 0 || split > n || threads < 0) return PTD_EINVAL;
    const bool diag = (flags & PTD_DIAGONAL) != 0u;
    const int64_t trees = (int64_t)1 << (diag ? split : 2 * split);
    if (tree_begin < 0 || tree_end < tree_begin || tree_end > trees) return PTD_EINVAL;

    TreeTask task;
    task.n = n;
    task.split = split;
    task.diag = diag;
    task.A = (const double*)A;
    task.lda = lda;
    task.coeff = (double*)coeff_out;

    const int64_t count = tree_end - tree_begin;
    int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = (int)std::min<int64_t>(nt, std::max<int64_t>(count, 1));

    std::atomic<int64_t> next{tree_begin};
    std::vector<uint64_t> ops(nt, 0);
    std::atomic<bool> failed{false};
    auto worker = [&](int w) {
        try {
            Walker walker(task);
            for (int64_t t = next.fetch_add(1); t < tree_end; t = next.fetch_add(1)) walker.run_tree(t);
            ops[w] = walker.ops();
        } catch (const std::bad_alloc&) {
            failed = true;
        }
    };

    std::vector<std::thread> pool;
    try {
        pool.reserve(nt > 1 ? nt - 1 : 0);
        for (int w = 1; w < nt; ++w) pool.emplace_back(worker, w);
    } catch (const std::exception&) {
        // fewer threads than asked: the ones started still drain the queue
    }
    worker(0);
    for (auto& th : pool) th.join();
    if (failed) return PTD_ENOMEM;
    if (ops_out) {
        uint64_t total = 0;
        for (uint64_t v : ops) total += v;
        *ops_out = total;
    }
    return PTD_OK;
}
