"""The evaluation metrics of the learned part (host arithmetic, no GPU)."""
def test_class_scores_closed_forms():
    """Precision/recall/F1 and the column-normalised confusion matrix of the
    evaluation, on hand-counted matrices."""
    import numpy as np
    from paper_2403_13135_amd.learn import class_scores
    cm = np.array([[8, 2, 0], [1, 6, 3], [0, 0, 10]])  # rows true, columns predicted
    sc = class_scores(cm)
    assert np.allclose(sc["precision"], [8 / 9, 6 / 8, 10 / 13])
    assert np.allclose(sc["recall"], [8 / 10, 6 / 10, 10 / 10])
    p, r = 6 / 8, 6 / 10
    assert np.isclose(sc["f1"][1], 2 * p * r / (p + r))
    col = np.array(sc["confusion_col_normalised"])
    assert np.allclose(col.sum(axis=0), 1.0, atol=1e-3)
    perfect = class_scores(np.diag([5, 7, 9]))
    assert perfect["f1"] == [1.0, 1.0, 1.0]
    empty = class_scores(np.array([[3, 0, 0], [0, 0, 0], [0, 0, 4]]))
    assert empty["precision"][1] == 0.0 and empty["recall"][1] == 0.0
