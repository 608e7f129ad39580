// parse.cpp -- restricted Einstein-notation parser for the MTTKRP and TTMc
// families (paper Sec. III-A notation; the benchmark strings of Tab. IV).
//
// An einsum lists the access indices of each input, then "->" and the output
// indices; repeated letters are summed, the others index the output.  The
// library accepts the two families the hot path implements:
//   MTTKRP  "<X>,<m1 r>,...,<m_{N-1} r>-><n r>"          (one shared rank letter)
//   TTMc    "<X>,<m1 r1>,...,<m_{N-1} r_{N-1}>-><X with each m_k -> r_k>"
//   MTTKRP followed by a matrix product (the paper's running example, Sec. II-A)
//           "<X>,<m1 r>,...,<m_{N-1} r>,<r l>-><n l>"
#include <cctype>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace deinsum {

namespace {

bool is_letter(char c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'); }

}  // namespace

deinsum_status parse_spec(const char *text, deinsum_spec *out)
{
    if (text == nullptr || out == nullptr)
        return fail(DEINSUM_ERR_INVALID_ARG, "parse: null argument");
    std::string s;
    for (const char *p = text; *p; ++p)
        if (!std::isspace(static_cast<unsigned char>(*p))) s.push_back(*p);
    if (s.size() > 256) return fail(DEINSUM_ERR_PARSE, "parse: spec longer than 256 characters");
    if (s.find("...") != std::string::npos)
        return fail(DEINSUM_ERR_PARSE, "parse: ellipsis (broadcast) is not supported");
    const size_t arrow = s.find("->");
    if (arrow == std::string::npos)
        return fail(DEINSUM_ERR_PARSE, "parse: missing '->' (implicit output is not supported)");
    if (s.find("->", arrow + 2) != std::string::npos)
        return fail(DEINSUM_ERR_PARSE, "parse: more than one '->'");
    const std::string lhs = s.substr(0, arrow), rhs = s.substr(arrow + 2);

    std::vector<std::string> ops;
    {
        size_t start = 0;
        for (;;) {
            size_t c = lhs.find(',', start);
            ops.push_back(lhs.substr(start, c == std::string::npos ? std::string::npos : c - start));
            if (c == std::string::npos) break;
            start = c + 1;
        }
    }
    for (const std::string &op : ops) {
        if (op.empty()) return fail(DEINSUM_ERR_PARSE, "parse: empty operand");
        for (char c : op)
            if (!is_letter(c))
                return fail(DEINSUM_ERR_PARSE, std::string("parse: invalid character '") + c + "'");
        for (size_t i = 0; i < op.size(); ++i)
            for (size_t j = i + 1; j < op.size(); ++j)
                if (op[i] == op[j])
                    return fail(DEINSUM_ERR_PARSE, "parse: letter '" + std::string(1, op[i]) +
                                                       "' repeated inside operand '" + op + "'");
    }
    for (char c : rhs)
        if (!is_letter(c))
            return fail(DEINSUM_ERR_PARSE, std::string("parse: invalid output character '") + c + "'");
    for (size_t i = 0; i < rhs.size(); ++i)
        for (size_t j = i + 1; j < rhs.size(); ++j)
            if (rhs[i] == rhs[j]) return fail(DEINSUM_ERR_PARSE, "parse: repeated output letter");

    const std::string &X = ops[0];
    const int N = static_cast<int>(X.size());
    if (N < 2 || N > DEINSUM_MAX_ORDER)
        return fail(DEINSUM_ERR_UNSUPPORTED, "parse: tensor order must be 2.." +
                                                 std::to_string(DEINSUM_MAX_ORDER));
    // One operand beyond the N-1 factors: the matrix of an MTTKRP-GEMM chain.
    const bool chain = static_cast<int>(ops.size()) == N + 1;
    if (static_cast<int>(ops.size()) != N && !chain)
        return fail(DEINSUM_ERR_UNSUPPORTED,
                    "parse: an order-N tensor needs exactly N-1 factor operands (plus one matrix for a chain)");

    deinsum_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.order = N;
    sp.n_factors = N - 1;
    for (int m = 0; m < DEINSUM_MAX_ORDER; ++m) sp.operand_of_mode[m] = -1;
    std::memcpy(sp.tensor_idx, X.data(), X.size());

    char rank_of_mode[DEINSUM_MAX_ORDER];
    for (int m = 0; m < N; ++m) rank_of_mode[m] = 0;
    for (int k = 1; k < N; ++k) {
        const std::string &f = ops[k];
        if (f.size() != 2)
            return fail(DEINSUM_ERR_UNSUPPORTED, "parse: factor operand '" + f +
                                                     "' must be two letters <mode><rank>");
        const size_t m = X.find(f[0]);
        if (m == std::string::npos) {
            if (X.find(f[1]) != std::string::npos)
                return fail(DEINSUM_ERR_UNSUPPORTED, "parse: factor '" + f +
                                                         "' is transposed; write <mode><rank>");
            return fail(DEINSUM_ERR_UNSUPPORTED, "parse: factor '" + f + "' contracts no mode of X");
        }
        if (X.find(f[1]) != std::string::npos)
            return fail(DEINSUM_ERR_UNSUPPORTED, "parse: factor '" + f +
                                                     "' has a tensor letter as its rank index");
        if (sp.operand_of_mode[m] >= 0)
            return fail(DEINSUM_ERR_UNSUPPORTED, "parse: mode '" + std::string(1, f[0]) +
                                                     "' is contracted by two factors");
        sp.operand_of_mode[m] = k - 1;
        sp.factor_mode[k - 1] = static_cast<int32_t>(m);
        rank_of_mode[m] = f[1];
    }
    int free_mode = -1;
    for (int m = 0; m < N; ++m)
        if (sp.operand_of_mode[m] < 0) free_mode = m;
    // N-1 factors on N-1 distinct modes leave exactly one free mode.
    sp.free_mode = free_mode;

    bool shared = true, distinct = true;
    for (int m = 0; m < N; ++m) {
        if (m == free_mode) continue;
        for (int p = m + 1; p < N; ++p) {
            if (p == free_mode) continue;
            if (rank_of_mode[m] != rank_of_mode[p]) shared = false;
            else distinct = false;
        }
    }
    for (int m = 0; m < N; ++m) sp.rank_idx[m] = (m == free_mode) ? '-' : rank_of_mode[m];

    // MTTKRP output: "<free letter><rank letter>" with a shared rank letter.
    const int first_contracted = (free_mode == 0) ? 1 : 0;
    const std::string mttkrp_out = std::string(1, X[free_mode]) + rank_of_mode[first_contracted];
    // TTMc output: X's letters with each contracted letter replaced in place.
    std::string ttmc_out = X;
    for (int m = 0; m < N; ++m)
        if (m != free_mode) ttmc_out[m] = rank_of_mode[m];

    if (chain) {
        const std::string &c = ops[N];
        const char r = rank_of_mode[first_contracted];
        if (!shared || c.size() != 2 || c[0] != r || X.find(c[1]) != std::string::npos || c[1] == r)
            return fail(DEINSUM_ERR_UNSUPPORTED, "parse: a chain is an MTTKRP (one shared rank letter) followed by "
                                                 "'<rank letter><new letter>'");
        const std::string chain_out = std::string(1, X[free_mode]) + c[1];
        if (rhs != chain_out)
            return fail(DEINSUM_ERR_UNSUPPORTED, "parse: output '" + rhs + "' is not '" + chain_out + "' (MTTKRP-GEMM)");
        sp.kind = DEINSUM_MTTKRP_MM;
    } else if (shared && rhs == mttkrp_out) {
        sp.kind = DEINSUM_MTTKRP;
    } else if (distinct && rhs == ttmc_out) {
        sp.kind = DEINSUM_TTMC;
    } else {
        std::string why = "parse: output '" + rhs + "' is not ";
        if (shared) why += "'" + mttkrp_out + "' (MTTKRP)";
        else if (distinct) why += "'" + ttmc_out + "' (TTMc)";
        else why = "parse: factors must share one rank letter (MTTKRP) or all differ (TTMc)";
        return fail(DEINSUM_ERR_UNSUPPORTED, why);
    }
    std::memcpy(sp.out_idx, rhs.data(), rhs.size());
    *out = sp;
    clear_error();
    return DEINSUM_OK;
}

}  // namespace deinsum
